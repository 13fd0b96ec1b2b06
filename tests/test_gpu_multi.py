"""Many small graphs in one launch: PageRank and BFS per graph against the oracle."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2010_16012_amd as pp
from paper_2010_16012_amd import _lib
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
    # pr_iters = 0 runs the BFS alone, bfs_policy = -1 the PageRank alone
    gs = gg.rmat_batch(6, 8, 10, seed=9)
    mg = pp.MultiGraph(gs)
    _, lv, par = mg.run(pr_iters=0, bfs_policy=pp.PP_SWITCH)
    for h, li, pi in zip(gs, mg.split(lv.cpu().numpy()), mg.split(par.cpu().numpy())):
        assert np.array_equal(li, oracle.bfs(h.off, h.idx, 0)[0]), h.name
        assert H.bfs_violations(h, 0, li, pi) == [], h.name
    for d in (pp.PP_PULL, pp.PP_PUSH):
        x, _, _ = mg.run(pr_iters=5, f=F, pr_dir=d, bfs_policy=-1)
        for h, xi in zip(gs, mg.split(x.cpu().numpy())):
            want = oracle.pagerank(h.off, h.idx, F, 5)
            assert np.abs(xi.astype(np.float64) - want).sum() <= PR_L1_TOL, h.name


def _raw_run(n, nnz, off, idx, x, level, parent, ws):
    """pp_multi_run through the C ABI with the arena exactly as given (the
    Python MultiGraph would reject a bad id before the call)."""
    _lib.pp_multi_run(n, nnz, off, idx, off, idx, pp.PP_PULL, 5, F, x, pp.PP_SWITCH, 0, 14.0, 24.0, level, parent,
                      ws)


def test_malformed_arena_is_rejected_on_the_device():
    # Two graphs (a 5-path and a 4-cycle).  Each corruption is caught by the
    # device check before any sweep: PP_E_GRAPH, outputs untouched; the same
    # workspace then runs the intact arena correctly.
    gs = [H.path(5), H.cycle(4)]
    n = np.array([h.n for h in gs], dtype=np.int32)
    nnz = np.array([h.nnz for h in gs], dtype=np.int64)
    off0 = np.concatenate([h.off for h in gs]).astype(np.int32)
    idx0 = np.concatenate([h.idx for h in gs]).astype(np.int16)
    dev = torch.device("cuda")
    ws = torch.empty(_lib.pp_multi_workspace_bytes(2, int(n.sum())), dtype=torch.uint8, device=dev)
    cases = []
    o = off0.copy(); o[2] = o[3] + 1; cases.append(("offsets decrease", o, idx0))          # noqa: E702
    o = off0.copy(); o[6 + 4] += 1; cases.append(("end past nnz", o, idx0))                # noqa: E702
    o = off0.copy(); o[6] = 1; cases.append(("second graph starts at 1", o, idx0))         # noqa: E702
    i = idx0.copy(); i[3] = 5; cases.append(("id equals n", off0, i))                      # noqa: E702
    i = idx0.copy(); i[-1] = -1; cases.append(("id 65535 in 16 bits", off0, i))            # noqa: E702
    for name, o, i in cases:
        announce(f"multi malformed arena: {name}")
        x = torch.full((int(n.sum()),), -7.0, device=dev)
        lv = torch.full((int(n.sum()),), -9, dtype=torch.int32, device=dev)
        par = lv.clone()
        with pytest.raises(pp.PPError) as ei:
            _raw_run(n, nnz, torch.as_tensor(o).to(dev), torch.as_tensor(i).to(dev), x, lv, par, ws)
        assert ei.value.status == _lib.PP_E_GRAPH, name
        assert bool((x == -7.0).all()) and bool((lv == -9).all()) and bool((par == -9).all()), name
    x = torch.empty(int(n.sum()), device=dev)
    lv = torch.empty(int(n.sum()), dtype=torch.int32, device=dev)
    par = torch.empty_like(lv)
    _raw_run(n, nnz, torch.as_tensor(off0).to(dev), torch.as_tensor(idx0).to(dev), x, lv, par, ws)
    bounds = np.concatenate([[0], np.cumsum(n)])
    for k, h in enumerate(gs):
        xs = x.cpu().numpy()[bounds[k]:bounds[k + 1]].astype(np.float64)
        assert np.abs(xs - oracle.pagerank(h.off, h.idx, F, 5)).sum() <= PR_L1_TOL
        assert np.array_equal(lv.cpu().numpy()[bounds[k]:bounds[k + 1]], oracle.bfs(h.off, h.idx, 0)[0])


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


@pytest.mark.parametrize("big,mid,pg,ml", [(512, 64, 2, 16), (256, 32, 1, 8), (1024, 128, 4, 32), (64, 8, 4, 8)])
def test_every_tuned_mapping_matches_the_oracle(big, mid, pg, ml):
    # the autotuner's search space: wavefront rows from `big` edges, middle rows
    # from `mid` on `ml`-lane groups, short pull rows on `pg` lanes
    _lib.pp_set_multi_tuning(big, mid, pg, ml)
    try:
        gs = gg.rmat_batch(16, 8, 13, seed=6) + [H.star(3000), H.complete(70), H.full_grid(40, 40)]
        _check(gs, policies=(pp.PP_SWITCH,))
    finally:
        _lib.pp_set_multi_tuning(512, 64, 2, 16)
