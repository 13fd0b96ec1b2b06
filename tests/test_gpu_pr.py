"""PageRank push/pull sweeps on the GPU against the FP64 oracle.

Bar: L1 distance <= 1e-6 between the FP32 GPU iterate and the FP64 oracle
iterate after T steps (and per-element relative error reported), for push and
pull, on closed-form graphs, directed graphs (push walks CSR, pull walks CSC),
R-MAT scale 14, graphs forced through every degree bin, and at R-MAT scale 22
via one-step sampled checks and the mass balance that holds at any size.
"""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2010_16012_amd as pp
from paper_2010_16012_amd import _lib
from tests import helpers as H
from tests.gpu_util import F, PR_L1_TOL, announce, default_bins, pr_gpu, tiny_bins

pytestmark = pytest.mark.gpu

DIRS = [pp.PP_PULL, pp.PP_PUSH]
DIR_IDS = ["pull", "push"]


@pytest.fixture(autouse=True)
def _bins():
    default_bins()
    yield
    default_bins()


def _check(host, iters=20, bins=None, tol=PR_L1_TOL, relabel=(True, False)):
    if bins == "tiny":
        tiny_bins()
    want = oracle.pagerank(host.off, host.idx, F, iters)
    for rl in relabel:
        g = pp.Graph(host, relabel=rl)
        _check_graph(g, host, want, iters, tol, rl)
        g.close()


def _check_graph(g, host, want, iters, tol, rl):
    for d, name in zip(DIRS, DIR_IDS):
        announce(f"PR {name} {host.name} n={host.n} nnz={host.nnz} T={iters} relabel={rl}")
        got = pr_gpu(g, d, iters).astype(np.float64)
        l1 = np.abs(got - want).sum()
        assert l1 <= tol, f"{name} relabel={rl}: L1 {l1:.3e} > {tol}"


@pytest.mark.parametrize("maker", [lambda: H.star(50), lambda: H.complete(9), lambda: H.cycle(257),
                                   lambda: H.complete_bipartite(3, 70), lambda: H.full_grid(13, 17)],
                         ids=["star", "K9", "cycle", "K3_70", "grid"])
def test_closed_form_graphs(maker):
    _check(maker())


def test_rmat14_both_forms():
    _check(gg.workload("rmat14"))


@pytest.mark.parametrize("relabel", [True, False])
def test_rmat14_every_bin_including_split_rows(relabel):
    host = gg.workload("rmat14")
    tiny_bins()
    g = pp.Graph(host, relabel=relabel)
    bins = g.bins(pp.PP_PULL)
    assert all(b > 0 for b in bins), bins
    want = oracle.pagerank(host.off, host.idx, F, 20)
    for d in DIRS:
        got = pr_gpu(g, d, 20).astype(np.float64)
        assert np.abs(got - want).sum() <= PR_L1_TOL


@pytest.mark.parametrize("hot,blocks", [(0, 1024), (1, 7), (16384, 3), (4096, 100000 // 97)])
def test_push_privatisation_settings(hot, blocks):
    # LDS privatisation off, tiny, maximal; few or many persistent workgroups
    host = gg.workload("rmat14")
    want = oracle.pagerank(host.off, host.idx, F, 20)
    _lib.pp_set_push_tuning(hot, blocks)
    try:
        for rl in (True, False):
            g = pp.Graph(host, relabel=rl)
            got = pr_gpu(g, pp.PP_PUSH, 20).astype(np.float64)
            assert np.abs(got - want).sum() <= PR_L1_TOL, (hot, blocks, rl)
    finally:
        _lib.pp_set_push_tuning(8192, 1024)


@pytest.mark.parametrize("hot,blocks", [(8192, 1024), (0, 64), (1, 7), (16384, 100), (100000, 512)])
def test_hybrid_push_hot_pull_cold(hot, blocks):
    # edges into the first `hot` vertices pushed into LDS, the other rows pulled;
    # hot = 0 is a pure pull, hot >= n a pure (LDS-only) push
    host = gg.workload("rmat14")
    want = oracle.pagerank(host.off, host.idx, F, 20)
    _lib.pp_set_push_tuning(min(hot, 40960), blocks)
    try:
        for rl in (True, False):
            g = pp.Graph(host, relabel=rl)
            got = pr_gpu(g, pp.PP_SWITCH, 20).astype(np.float64)
            assert np.abs(got - want).sum() <= PR_L1_TOL, (hot, blocks, rl)
    finally:
        _lib.pp_set_push_tuning(8192, 1024)


def test_hybrid_wide_privatisation():
    # 40960 hot targets: 1024-thread workgroups holding 160 KB of LDS
    host = gg.rmat(16, 16, seed=3)
    want = oracle.pagerank(host.off, host.idx, F, 20)
    _lib.pp_set_push_tuning(40960, 256)
    try:
        g = pp.Graph(host)
        assert np.abs(pr_gpu(g, pp.PP_SWITCH, 20).astype(np.float64) - want).sum() <= PR_L1_TOL
    finally:
        _lib.pp_set_push_tuning(8192, 1024)


def test_hybrid_directed_weighted():
    # weighted uniform PageRank = mean over all sources of weighted PPR
    host = H.random_graph(2000, 12000, 6, symmetric=False, connected=True)
    gg.with_weights(host, seed=3)
    X, _ = oracle.ppr(host.off, host.idx, np.arange(host.n), F, T=15, weights=host.weights)
    want = X.mean(axis=1)
    _lib.pp_set_push_tuning(500, 37)
    try:
        for rl in (True, False):
            g = pp.Graph(host, relabel=rl)
            got = pr_gpu(g, pp.PP_SWITCH, 15).astype(np.float64)
            assert np.abs(got - want).sum() <= PR_L1_TOL, rl
    finally:
        _lib.pp_set_push_tuning(8192, 1024)


@pytest.mark.parametrize("hot,blocks", [(16385, 3), (40960, 256), (30000, 1000)])
def test_push_wide_privatisation(hot, blocks):
    # more than 16384 privatised targets: 1024-thread workgroups, up to 160 KB of LDS
    host = gg.rmat(16, 16, seed=3)
    want = oracle.pagerank(host.off, host.idx, F, 20)
    _lib.pp_set_push_tuning(hot, blocks)
    try:
        for rl in (True, False):
            g = pp.Graph(host, relabel=rl)
            got = pr_gpu(g, pp.PP_PUSH, 20).astype(np.float64)
            assert np.abs(got - want).sum() <= PR_L1_TOL, (hot, blocks, rl)
    finally:
        _lib.pp_set_push_tuning(8192, 1024)


@pytest.mark.parametrize("hot,block", [(0, 1024), (1, 256), (300, 512), (1 << 20, 1024)])
def test_pull_lds_staging_settings(hot, block):
    # no staging, a single staged entry, a partial prefix, everything that fits in LDS
    host = gg.workload("rmat14")
    want = oracle.pagerank(host.off, host.idx, F, 20)
    _lib.pp_set_pull_tuning(hot, block)
    try:
        for rl in (True, False):
            g = pp.Graph(host, relabel=rl)
            got = pr_gpu(g, pp.PP_PULL, 20).astype(np.float64)
            assert np.abs(got - want).sum() <= PR_L1_TOL, (hot, block, rl)
    finally:
        _lib.pp_set_pull_tuning(32768, 1024)


def test_relabel_map_is_a_degree_ordered_permutation():
    host = gg.workload("rmat14")
    g = pp.Graph(host, relabel=True)
    perm = g.relabel_map().cpu().numpy()
    assert np.array_equal(np.sort(perm), np.arange(host.n))
    deg = np.diff(host.off)
    cls = np.floor(np.log2(2 * deg[perm] + 1)).astype(int)  # d_out + d_in = 2d here
    assert np.all(np.diff(cls) <= 0)
    # ties keep caller order
    for c in np.unique(cls):
        ids = perm[cls == c]
        assert np.all(np.diff(ids) > 0)


@pytest.mark.parametrize("seed", [1, 2])
def test_directed_graph_push_uses_out_edges_pull_uses_in_edges(seed):
    host = H.random_graph(3000, 20000, seed, symmetric=False)
    host.ensure_transpose()
    _check(host, bins=None)
    _check(host, bins="tiny")
    # weighted directed graph through every path
    gg.with_weights(host, seed=seed)
    X, _ = oracle.ppr(host.off, host.idx, np.arange(host.n), F, T=10, weights=host.weights)
    want = X.mean(axis=1)
    for rl in (True, False):
        g = pp.Graph(host, relabel=rl)
        for d in DIRS:
            got = pr_gpu(g, d, 10).astype(np.float64)
            assert np.abs(got - want).sum() <= PR_L1_TOL, (rl, d)


def test_edge_cases_single_vertex_and_no_edges():
    one = gg.from_edges(1, [], [], True)
    _check(one, iters=5)
    empty = gg.from_edges(100, [], [], True)
    _check(empty, iters=3)
    # ragged: vertex count not a multiple of any tile, with a few isolated vertices
    _check(H.random_graph(1001, 1500, 3), iters=7)


def test_zero_iterations_is_identity():
    host = H.cycle(10)
    g = pp.Graph(host)
    x0 = torch.arange(10, dtype=torch.float32, device="cuda")
    for d in DIRS:
        x = pp.pagerank(g, 0, F, d, x0=x0)
        assert torch.equal(x, x0)


def test_pull_is_bit_reproducible_and_resumable():
    host = gg.workload("rmat14")
    g = pp.Graph(host)
    a = pr_gpu(g, pp.PP_PULL, 20)
    b = pr_gpu(g, pp.PP_PULL, 20)
    assert np.array_equal(a, b)
    half = pp.pagerank(g, 10, F, pp.PP_PULL)
    full = pp.pagerank(g, 10, F, pp.PP_PULL, x0=half)
    assert np.array_equal(full.cpu().numpy(), a)
    # push is order-dependent in the last bits but resumes within tolerance
    p_half = pp.pagerank(g, 10, F, pp.PP_PUSH)
    p_full = pp.pagerank(g, 10, F, pp.PP_PUSH, x0=p_half).cpu().numpy().astype(np.float64)
    assert np.abs(p_full - a).sum() <= PR_L1_TOL


@pytest.mark.parametrize("relabel", [True, False])
def test_step_api_matches_run_api(relabel):
    host = H.random_graph(5000, 40000, 5, symmetric=False)
    host.ensure_transpose()
    g = pp.Graph(host, relabel=relabel)
    x = torch.rand(g.n, device="cuda", dtype=torch.float32) / g.n
    want = oracle.pagerank(host.off, host.idx, F, 1, x0=x.cpu().numpy().astype(np.float64))
    for fn in (_lib.pp_pr_pull, _lib.pp_pr_push):
        y = torch.empty_like(x)
        fn(g.handle, x, y, F)
        torch.cuda.synchronize()
        assert np.abs(y.cpu().numpy() - want).sum() <= 1e-7
    y_run = pp.pagerank(g, 1, F, pp.PP_PULL, x0=x)
    y_step = torch.empty_like(x)
    _lib.pp_pr_pull(g.handle, x, y_step, F)
    assert torch.equal(y_run, y_step)


def test_weighted_pagerank_matches_oracle_ppr_average():
    # weighted uniform PageRank = mean over all sources of weighted PPR
    host = H.random_graph(300, 1500, 8, symmetric=True)
    gg.with_weights(host, seed=2)
    X, _ = oracle.ppr(host.off, host.idx, np.arange(host.n), F, T=15, weights=host.weights)
    want = X.mean(axis=1)
    for rl in (True, False):
        g = pp.Graph(host, relabel=rl)
        for d in DIRS:
            got = pr_gpu(g, d, 15).astype(np.float64)
            assert np.abs(got - want).sum() <= PR_L1_TOL


def test_argument_errors_raise():
    host = H.cycle(8)
    g = pp.Graph(host)
    x = torch.zeros(8, device="cuda")
    with pytest.raises(pp.PPError):
        _lib.pp_pr_pull(g.handle, x, x, F)        # aliasing
    with pytest.raises(pp.PPError):
        _lib.pp_pr_push(g.handle, x, torch.zeros(8, device="cuda"), 1.5)  # f out of range
    with pytest.raises(pp.PPError):
        _lib.pp_pr_run(g.handle, 7, 3, F, x)  # not a direction
    bad = gg.from_edges(4, [0, 1], [1, 2], True)
    bad.idx = bad.idx.copy()
    bad.idx[0] = 7  # out of range index
    with pytest.raises(pp.PPError):
        pp.Graph(bad)


@pytest.mark.slow
def test_rmat22_sampled_step_and_mass_balance():
    host = gg.workload("rmat22")
    announce(f"PR rmat22 n={host.n} nnz={host.nnz}")
    g = pp.Graph(host)
    deg = np.diff(host.off)
    rng = np.random.default_rng(0)
    verts = np.concatenate([np.arange(64), rng.integers(0, host.n, 4032)]).astype(np.int32)
    for d, name in zip(DIRS, DIR_IDS):
        x19 = pp.pagerank(g, 19, F, d)
        x20 = pp.pagerank(g, 1, F, d, x0=x19)
        torch.cuda.synchronize()
        x19h = x19.cpu().numpy()
        x20h = x20.cpu().numpy().astype(np.float64)
        want = oracle.pagerank_step_at(host.off, host.idx, x19h, verts, F)
        # FP32 bound for y = base + sum of d positive terms, each term rounded
        # about three times (1/d, two products), summed in any order:
        # |err| <= (d + 4) * 2^-24 * y.
        bound = (deg[verts] + 4) * 2.0**-24 * want
        err = np.abs(x20h[verts] - want)
        assert np.all(err <= bound), f"{name}: worst err/bound {np.max(err / bound):.2f}"
        # mass balance of one step, at every size
        lhs = x20h.sum()
        rhs = (1 - F) + F * x19h[deg > 0].astype(np.float64).sum()
        assert abs(lhs - rhs) <= 1e-5, f"{name}: mass {lhs} vs {rhs}"
        # isolated vertices sit exactly at the teleport value
        iso = np.nonzero(deg == 0)[0][:1000]
        assert np.all(x20h[iso] == np.float32((1 - F) / host.n))  # F is FP32-exact


# ---------------------------------------------------------------- tiled pull
@pytest.mark.parametrize("rows,width,pull_hot", [(4096, 512, 32768), (100000, 1024, 32768), (64, 64, 32768),
                                                 (16384, 32768, 40960), (2000, 256, 0), (300, 4096, 300)])
def test_tiled_pull_rmat14(rows, width, pull_hot):
    # the heavy rows pull slice by slice from LDS (many slices and tiles, a
    # ragged last slice), the rest as usual; against the oracle, repeatable
    # bit for bit, and within FP32 rounding of the plain pull
    host = gg.workload("rmat14")
    want = oracle.pagerank(host.off, host.idx, F, 20)
    _lib.pp_set_pull_tuning(pull_hot, 1024)
    plain = pr_gpu(pp.Graph(host), pp.PP_PULL, 20).astype(np.float64)
    _lib.pp_set_pull_slices(rows, width)
    g = pp.Graph(host)
    R, W, S, T = g.slices()
    announce(f"tiled pull rmat14 R={R} W={W} S={S} tiles={T} pull_hot={pull_hot}")
    assert R > 0 and W == width and S >= 1 and T >= 1
    got = pr_gpu(g, pp.PP_PULL, 20)
    assert np.abs(got.astype(np.float64) - want).sum() <= PR_L1_TOL
    assert np.array_equal(got, pr_gpu(g, pp.PP_PULL, 20))
    assert np.abs(got - plain).max() <= 1e-5 * plain.max()
    # the one-step entry point takes the same path
    x0 = torch.full((host.n,), 1.0 / host.n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x0)
    _lib.pp_pr_pull(g.handle, x0, y, F)
    want1 = oracle.pagerank(host.off, host.idx, F, 1)
    assert np.abs(y.cpu().numpy().astype(np.float64) - want1).sum() <= PR_L1_TOL


def test_tiled_pull_long_segments_in_chunks():
    # a star's hub row has 59,999 in-edges: its segments in slice 0 (32,767
    # sources) and slice 1 (27,232) are cut into 1,024-edge chunks whose
    # partials the combine adds in order
    host = H.star(60000)
    _lib.pp_set_pull_slices(8, 32768)
    g = pp.Graph(host)
    R, W, S, T = g.slices()
    assert R == 1 and S == 2 and T == 32 + 27
    want = oracle.pagerank(host.off, host.idx, F, 20)
    got = pr_gpu(g, pp.PP_PULL, 20).astype(np.float64)
    assert np.abs(got - want).sum() <= PR_L1_TOL


def _directed_rmat(scale, seed):
    """R-MAT with each directed edge kept with probability 0.6: hubs with
    different in- and out-degrees."""
    h = gg.rmat(scale, 16, seed=seed)
    src = np.repeat(np.arange(h.n), np.diff(h.off))
    keep = np.random.default_rng(seed).random(h.nnz) < 0.6
    d = gg.from_edges(h.n, src[keep], h.idx[keep], False, f"drmat{scale}_{seed}")
    d.ensure_transpose()
    return d


@pytest.mark.parametrize("seed", [1, 2])
def test_tiled_pull_directed_and_split_rest_rows(seed):
    # directed: rows pull over in-edges; tiny bins leave split rows (bin 5)
    # beyond the tiled prefix, which the plain part still sums in chunks
    host = _directed_rmat(14, seed)
    tiny_bins()
    _lib.pp_set_pull_slices(16, 128)
    g = pp.Graph(host)
    R, W, S, T = g.slices()
    announce(f"tiled pull directed R={R} S={S} tiles={T} bin5={g.bins(pp.PP_PULL)[5]}")
    assert R == 16 and g.bins(pp.PP_PULL)[5] > R
    want = oracle.pagerank(host.off, host.idx, F, 20)
    got = pr_gpu(g, pp.PP_PULL, 20).astype(np.float64)
    assert np.abs(got - want).sum() <= PR_L1_TOL


def test_tiled_pull_rows_without_in_edges_at_the_end():
    # Rows past the last vertex with in-edges get the teleport term from the
    # combine kernel instead of a unit of the plain part.  3,000 of them have
    # an out-edge into an R-MAT core, so their contributions feed the next
    # step and a wrong tail value shows in the core's ranks; the rest are
    # isolated.  Personalised runs (k_tile = 1: the same sweep) seeded on tail
    # rows put the teleport mass there.
    core = gg.rmat(12, 16, seed=5)
    K, M, Z = core.n, 3000, 500
    n = K + M + Z
    rng = np.random.default_rng(5)
    src = np.concatenate([np.repeat(np.arange(K), np.diff(core.off)), np.arange(K, K + M)])
    dst = np.concatenate([core.idx, rng.integers(0, K, M)])
    host = gg.from_edges(n, src, dst, False, "rmat12_core_plus_sources")
    host.ensure_transpose()
    _lib.pp_set_pull_slices(512, 256)
    g = pp.Graph(host)
    assert g.slices()[0] > 0
    # the premise: in internal ids the out-only vertices follow every vertex with in-edges
    perm = g.relabel_map().cpu().numpy().astype(np.int64)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    indeg = np.bincount(host.idx, minlength=n)
    assert inv[K:K + M].min() > inv[indeg > 0].max()
    announce(f"tiled pull tail rows={n - 1 - inv[indeg > 0].max()} R={g.slices()[0]}")
    want = oracle.pagerank(host.off, host.idx, F, 20)
    got = pr_gpu(g, pp.PP_PULL, 20).astype(np.float64)
    assert np.abs(got - want).sum() <= PR_L1_TOL
    seeds = np.array([K + 7, n - 1, int(np.argmax(indeg))], dtype=np.int32)
    wantp, _ = oracle.ppr(host.off, host.idx, seeds, F, T=20)
    X, _ = pp.ppr(g, seeds, iters=20, f=F, k_tile=1, direction=pp.PP_PULL)
    assert np.abs(X.cpu().numpy().astype(np.float64) - wantp).sum(axis=0).max() <= 1e-6


def test_tiled_pull_off_for_weighted_and_unrelabelled_graphs():
    host = gg.workload("rmat14")
    _lib.pp_set_pull_slices(4096, 1024)
    assert pp.Graph(host, relabel=False).slices()[0] == 0
    with pytest.raises(pp.PPError):
        _lib.pp_set_pull_slices(4096, 40960)  # offsets in a slice have 15 bits
    gw = gg.rmat(12, 16, seed=3)
    gg.with_weights(gw, seed=1)
    assert pp.Graph(gw).slices()[0] == 0
    # a grid has no heavy rows: nothing qualifies
    assert pp.Graph(H.full_grid(60, 60)).slices()[0] == 0


@pytest.mark.parametrize("hot,blocks", [(8192, 1024), (1, 7), (40960, 256), (100, 333)])
def test_binned_push_matches_oracle_and_atomic_push(hot, blocks):
    # Updates to targets past the privatised ones go to per-workgroup slices of
    # 16384-id bins (summed in LDS by a second kernel) instead of global
    # atomics.  R-MAT 17 spans several bins (uniform PageRank); a weighted
    # directed graph runs single-source PPR, whose first sweeps skip the rows
    # with zero contribution (slices left part-filled).  Both layouts agree
    # with the oracle and with each other.
    rmat = gg.rmat(17, 16, seed=1)
    wdir = H.random_graph(70000, 400000, 3, symmetric=False, connected=True)
    gg.with_weights(wdir, seed=2)
    src = gg.pick_vertices(wdir, 3, seed=5)
    want_r = oracle.pagerank(rmat.off, rmat.idx, F, 20)
    want_w, _ = oracle.ppr(wdir.off, wdir.idx, src, F, T=20, weights=wdir.weights)
    _lib.pp_set_push_tuning(hot, blocks)
    try:
        for rl in (True, False):
            got = {}
            for on in (1, 0):
                _lib.pp_set_push_bins(on)
                g = pp.Graph(rmat, relabel=rl)
                gw = pp.Graph(wdir, relabel=rl)
                for gr, host in ((g, rmat), (gw, wdir)):
                    info = gr.push_bins()
                    if on:
                        assert info[0] == -(-(host.n - info[1]) // 16384) >= (2 if host is rmat else 1), info
                    else:
                        assert info[0] == 0, info
                announce(f"binned push={on} hot={hot} blocks={blocks} relabel={rl}")
                x = pr_gpu(g, pp.PP_PUSH, 20).astype(np.float64)
                X, _ = pp.ppr(gw, src, iters=20, f=F, k_tile=1, direction=pp.PP_PUSH)
                X = X.cpu().numpy().astype(np.float64)
                g.close()
                gw.close()
                assert np.abs(x - want_r).sum() <= PR_L1_TOL, (hot, blocks, rl, on)
                assert np.abs(X - want_w).sum(axis=0).max() <= PR_L1_TOL, (hot, blocks, rl, on)
                got[on] = (x, X)
            assert np.abs(got[1][0] - got[0][0]).sum() <= PR_L1_TOL
            assert np.abs(got[1][1] - got[0][1]).sum(axis=0).max() <= PR_L1_TOL
    finally:
        _lib.pp_set_push_tuning(8192, 1024)
        _lib.pp_set_push_bins(1)
