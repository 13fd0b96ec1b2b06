"""Many small graphs in one launch: PageRank and BFS per graph against the oracle."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2010_16012_amd as pp
from tests import helpers as H
from tests.gpu_util import F, PR_L1_TOL, announce

pytestmark = pytest.mark.gpu


def _mixed_graphs():
    gs = gg.rmat_batch(24, 6, 12, seed=4)
    gs += [gg.from_edges(1, [], [], True), gg.from_edges(50, [1, 2], [2, 3], True), H.path(300), H.star(1000),
           H.full_grid(30, 40), H.complete(33)]
    return gs


def _check(gs, policies=(pp.PP_PUSH, pp.PP_PULL, pp.PP_SWITCH), dirs=(pp.PP_PULL, pp.PP_PUSH), iters=20):
    mg = pp.MultiGraph(gs)
    for d in dirs:
        for pol in policies:
            announce(f"multi graphs={len(gs)} pr_dir={d} bfs={pol}")
            x, lv, par = mg.run(pr_iters=iters, f=F, pr_dir=d, bfs_policy=pol)
            torch.cuda.synchronize()
            xs, lvs, pars = mg.split(x.cpu().numpy()), mg.split(lv.cpu().numpy()), mg.split(par.cpu().numpy())
            for h, xi, li, pi in zip(gs, xs, lvs, pars):
                want = oracle.pagerank(h.off, h.idx, F, iters)
                assert np.abs(xi.astype(np.float64) - want).sum() <= PR_L1_TOL, h.name
                wl, _, _ = oracle.bfs(h.off, h.idx, 0)
                assert np.array_equal(li, wl), h.name
                assert H.bfs_violations(h, 0, li, pi) == [], h.name


def test_mixed_batch_all_directions_and_policies():
    _check(_mixed_graphs())


def test_directed_batch():
    gs = [H.random_graph(n, 4 * n, s, symmetric=False) for s, n in enumerate([10, 500, 3000, 7000])]
    for h in gs:
        h.ensure_transpose()
    _check(gs, policies=(pp.PP_PULL, pp.PP_SWITCH, pp.PP_PUSH))


def test_pr_only_and_bfs_only():
    gs = gg.rmat_batch(6, 8, 10, seed=9)
    mg = pp.MultiGraph(gs)
    x, _, _ = mg.run(pr_iters=0, bfs_policy=pp.PP_SWITCH)
    _, lv, _ = mg.run(pr_iters=5, f=F, bfs_policy=-1)


def test_size_limit_and_errors():
    with pytest.raises(pp.PPError):
        pp.MultiGraph([gg.rmat(15, 2, seed=1)]).run()
    mg = pp.MultiGraph([H.path(5)])
    with pytest.raises(pp.PPError):
        mg.run(bfs_root=7)
    bad = H.path(5)
    bad.idx = bad.idx.copy()
    bad.idx[3] = 5  # an id past the graph's last vertex
    with pytest.raises(pp.PPError):
        pp.MultiGraph([bad])


@pytest.mark.slow
def test_batch_of_512_rmat_graphs():
    gs = gg.rmat_batch(512, 8, 14, seed=1)
    mg = pp.MultiGraph(gs)
    # every graph, the largest (whole-wavefront hub rows) included
    want_x = [oracle.pagerank(h.off, h.idx, F, 20) for h in gs]
    want_l = [oracle.bfs(h.off, h.idx, 0)[0] for h in gs]
    for d in (pp.PP_PULL, pp.PP_PUSH):
        x, lv, par = mg.run(pr_iters=20, f=F, pr_dir=d, bfs_policy=pp.PP_SWITCH)
        xs, lvs, ps = mg.split(x.cpu().numpy()), mg.split(lv.cpu().numpy()), mg.split(par.cpu().numpy())
        for i in range(len(gs)):
            assert np.abs(xs[i].astype(np.float64) - want_x[i]).sum() <= PR_L1_TOL
            assert np.array_equal(lvs[i], want_l[i])
            assert H.bfs_violations_fast(gs[i], 0, lvs[i], ps[i]) == []


def test_largest_ids_and_repeatable_pull():
    # ids up to 16383 (the 16-bit arena's top graph size): a star centred on the
    # last vertex, a long path, and a graph with an empty row 0; the pull sums
    # rows in a fixed order, so a second launch gives the same bits
    n = 16384
    star = gg.from_edges(n, np.full(n - 1, n - 1), np.arange(n - 1), True)
    gs = [star, H.path(n), gg.from_edges(40, [5, 6, 39], [6, 7, 1], True)]
    _check(gs, policies=(pp.PP_SWITCH, pp.PP_PULL))
    mg = pp.MultiGraph(gs)
    x1, _, _ = mg.run(pr_iters=20, f=F, pr_dir=pp.PP_PULL, bfs_policy=-1)
    x2, _, _ = mg.run(pr_iters=20, f=F, pr_dir=pp.PP_PULL, bfs_policy=-1)
    assert torch.equal(x1, x2)


def test_row_lists_that_overflow():
    # more rows of 512+ edges than the hub list holds (K_700), and more rows of
    # 64-511 edges than the middle-row list holds (5,000 vertices of degree
    # ~80): those rows fall back to the small groups, results unchanged
    dense = H.random_graph(5000, 200_000, 3, symmetric=True)
    deg = np.diff(dense.off)
    assert ((deg >= 64) & (deg < 512)).sum() > 4096
    _check([H.complete(700), dense, H.path(50)], policies=(pp.PP_SWITCH,))
