"""Batched personalised PageRank and its adjoint on the GPU against the oracle.

Bars: every column within 1e-6 L1 of the FP64 oracle column (FP32 sweeps);
the adjoint gradient within 1e-5 relative (L2) of the FP64 oracle gradient
at the fixed point, and of FP64 central differences of the dense solve.
"""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2010_16012_amd as pp
from tests import helpers as H
from tests.gpu_util import F, announce, default_bins, tiny_bins

pytestmark = pytest.mark.gpu

DIRS = [pp.PP_PULL, pp.PP_PUSH]


@pytest.fixture(autouse=True)
def _bins():
    default_bins()
    yield
    default_bins()


def _cols_close(got, want, tol=1e-6):
    l1 = np.abs(got.astype(np.float64) - want).sum(axis=0)
    assert l1.max() <= tol, f"worst column L1 {l1.max():.3e}"


@pytest.mark.parametrize("kt,k", [(8, 64), (16, 64), (32, 64), (64, 64), (32, 45), (64, 3)])
def test_batched_ppr_matches_oracle_columns(kt, k):
    host = gg.workload("rmat14")
    src = gg.pick_vertices(host, k, seed=5)
    want, _ = oracle.ppr(host.off, host.idx, src, F, T=30)
    for rl in (True, False):
        g = pp.Graph(host, relabel=rl)
        for d in DIRS:
            announce(f"PPR kt={kt} relabel={rl} dir={d}")
            X, done = pp.ppr(g, src, iters=30, f=F, k_tile=kt, direction=d)
            assert done == 30
            _cols_close(X.cpu().numpy(), want)


@pytest.mark.parametrize("tiled", [False, True])
def test_sequential_single_vector_columns(tiled):
    # k_tile = 1: each column with the single-vector sweep (the sequential
    # baseline of the batched runs), tiled pull rows included
    host = gg.workload("rmat14")
    src = gg.pick_vertices(host, 12, seed=5)
    want, _ = oracle.ppr(host.off, host.idx, src, F, T=30)
    if tiled:
        pp._lib.pp_set_pull_slices(2048, 4096)
    try:
        g = pp.Graph(host)
        if tiled:
            assert g.slices()[0] > 0
        for d in DIRS:
            announce(f"PPR k_tile=1 tiled={tiled} dir={d}")
            X, done = pp.ppr(g, src, iters=30, f=F, k_tile=1, direction=d)
            assert done == 30
            _cols_close(X.cpu().numpy(), want)
            X0, _ = pp.ppr(g, src[:2], iters=0, f=F, k_tile=1, direction=d)
            e = np.zeros((host.n, 2), dtype=np.float32)
            e[src[:2], [0, 1]] = 1
            assert np.array_equal(X0.cpu().numpy(), e)
    finally:
        pp._lib.pp_set_pull_slices(0, 32768)


def test_sequential_single_vector_weighted_directed():
    host = H.random_graph(3000, 9000, 12, symmetric=False, connected=True)
    gg.with_weights(host, seed=2)
    src = np.array([3, 700, 2999], dtype=np.int32)
    want, _ = oracle.ppr(host.off, host.idx, src, F, T=25, weights=host.weights)
    g = pp.Graph(host)
    for d in DIRS:
        X, _ = pp.ppr(g, src, iters=25, f=F, k_tile=1, direction=d)
        _cols_close(X.cpu().numpy(), want)
    with pytest.raises(pp.PPError):
        pp.ppr(g, src, iters=25, f=F, k_tile=1, direction=pp.PP_SWITCH)
    with pytest.raises(pp.PPError):
        pp.ppr(g, src, iters=25, f=F, k_tile=1, tol=1e-6)
    with pytest.raises(pp.PPError):
        pp.ppr(g, np.array([3000], dtype=np.int32), iters=2, f=F, k_tile=1)


@pytest.mark.parametrize("name,kt,k", [("rmat14", 32, 64), ("grid64", 16, 20), ("grid200", 8, 8),
                                        ("star5000", 8, 3)])
def test_switch_sparse_push_then_dense_pull(name, kt, k):
    # rmat14 switches to dense after a sweep or two; the 64x64 grid part-way
    # through; on the 200x200 grid the 30-hop support stays sparse throughout
    host = {"rmat14": lambda: gg.workload("rmat14"), "grid64": lambda: H.full_grid(64, 64),
            "grid200": lambda: H.full_grid(200, 200), "star5000": lambda: H.star(5000)}[name]()
    src = gg.pick_vertices(host, k, seed=11)
    want, _ = oracle.ppr(host.off, host.idx, src, F, T=30)
    for rl in (True, False):
        g = pp.Graph(host, relabel=rl)
        announce(f"PPR switch {name} kt={kt} relabel={rl}")
        X, done = pp.ppr(g, src, iters=30, f=F, k_tile=kt, direction=pp.PP_SWITCH)
        assert done == 30
        _cols_close(X.cpu().numpy(), want)


def test_switch_weighted_directed_and_converged():
    host = H.random_graph(3000, 9000, 12, symmetric=False, connected=True)
    gg.with_weights(host, seed=2)
    src = np.array([3, 700, 2999], dtype=np.int32)
    want, _ = oracle.ppr(host.off, host.idx, src, F, T=25, weights=host.weights)
    g = pp.Graph(host)
    X, _ = pp.ppr(g, src, iters=25, f=F, k_tile=8, direction=pp.PP_SWITCH)
    _cols_close(X.cpu().numpy(), want)
    P = H.dense_transition(host, host.weights) if host.n <= 3000 else None
    Xc, done = pp.ppr(g, src, iters=5000, f=F, k_tile=8, direction=pp.PP_SWITCH, tol=1e-8)
    assert done < 5000
    for j, s in enumerate(src):
        e = np.zeros(host.n)
        e[s] = 1
        exact = np.linalg.solve(np.eye(host.n) - F * P, (1 - F) * e)
        assert np.abs(Xc[:, j].cpu().numpy() - exact).sum() <= 2e-6


def test_batched_ppr_directed_weighted_every_bin():
    host = H.random_graph(4000, 30000, 3, symmetric=False, connected=True)
    gg.with_weights(host, seed=8)
    src = np.array([0, 5, 77, 1234, 3999, 2, 3, 4], dtype=np.int32)
    want, _ = oracle.ppr(host.off, host.idx, src, F, T=25, weights=host.weights)
    for bins in ("default", "tiny"):
        (tiny_bins if bins == "tiny" else default_bins)()
        for rl in (True, False):
            g = pp.Graph(host, relabel=rl)
            for d in DIRS:
                X, _ = pp.ppr(g, src, iters=25, f=F, k_tile=8, direction=d)
                _cols_close(X.cpu().numpy(), want)


def test_pull_batched_is_deterministic_and_tile_independent():
    host = gg.workload("rmat14")
    src = gg.pick_vertices(host, 32, seed=6)
    g = pp.Graph(host)
    a, _ = pp.ppr(g, src, iters=20, f=F, k_tile=16)
    b, _ = pp.ppr(g, src, iters=20, f=F, k_tile=16)
    assert torch.equal(a, b)
    c, _ = pp.ppr(g, src, iters=20, f=F, k_tile=32)
    assert (a - c).abs().sum(dim=0).max().item() <= 1e-6
    # a batch equals its columns run one tile at a time
    d, _ = pp.ppr(g, src[:8], iters=20, f=F, k_tile=8)
    assert (a[:, :8] - d).abs().sum(dim=0).max().item() <= 1e-6


def test_converged_mode_matches_dense_solve():
    host = H.random_graph(300, 1500, 9, symmetric=False, connected=True)
    gg.with_weights(host, seed=1)
    src = np.arange(8, dtype=np.int32) * 7
    P = H.dense_transition(host, host.weights)
    g = pp.Graph(host)
    for d in DIRS:
        X, done = pp.ppr(g, src, iters=5000, f=F, k_tile=8, direction=d, tol=1e-8)
        assert done < 5000
        for j, s in enumerate(src):
            e = np.zeros(host.n)
            e[s] = 1
            want = np.linalg.solve(np.eye(host.n) - F * P, (1 - F) * e)
            assert np.abs(X[:, j].cpu().numpy() - want).sum() <= 2e-6


def test_ppr_edge_cases_and_errors():
    host = gg.from_edges(10, [0, 1, 2], [1, 2, 3], True)  # vertices 4..9 isolated
    g = pp.Graph(host)
    X, _ = pp.ppr(g, [5, 0, 1, 2, 3, 4, 6, 7], iters=3, f=F, k_tile=8)
    Xh = X.cpu().numpy()
    assert Xh[5, 0] == pytest.approx(1 - F, abs=1e-7) and np.abs(Xh[:, 0]).sum() == pytest.approx(1 - F, abs=1e-7)
    Z, done = pp.ppr(g, np.zeros(0, np.int32), iters=3, k_tile=8)
    assert Z.shape == (10, 0) and done == 0
    # a partial last tile: columns agree with a full-tile run
    P3, _ = pp.ppr(g, [1, 2, 3], iters=3, f=F, k_tile=8)
    assert torch.equal(P3, X[:, 2:5])
    with pytest.raises(pp.PPError):
        pp.ppr(g, [1] * 8, k_tile=12)
    with pytest.raises(pp.PPError):
        pp.ppr(g, [0, 1, 2, 3, 4, 5, 6, 10], k_tile=8)  # source out of range
    with pytest.raises(pp.PPError):  # not a direction
        pp.ppr_adjoint(g, X, torch.ones_like(X), iters=2, k_tile=8, direction=7)


# ----------------------------------------------------------------------- adjoint
def _forward_fixed_point(host, src):
    X, _ = oracle.ppr(host.off, host.idx, src, F, T=20000, tol=1e-15, weights=host.weights)
    return X


@pytest.mark.parametrize("symmetric", [True, False])
def test_adjoint_matches_oracle_gradient(symmetric):
    host = H.random_graph(600, 4000, 14, symmetric=symmetric, connected=True)
    gg.with_weights(host, seed=3)
    src = np.arange(16, dtype=np.int32) * 31
    Xo = _forward_fixed_point(host, src)
    c = gg.normal(host.n * len(src), seed=2).reshape(host.n, len(src)).astype(np.float64)
    lam_o, grad_o, _ = oracle.ppr_adjoint(host.off, host.idx, Xo, c, F, T=20000, tol=1e-15, weights=host.weights)
    for rl in (True, False):
        g = pp.Graph(host, relabel=rl)
        X, _ = pp.ppr(g, src, iters=3000, f=F, k_tile=16, tol=1e-9)
        for fd in DIRS:
            for ad in DIRS:
                announce(f"adjoint sym={symmetric} relabel={rl} fwd={fd} adj={ad}")
                Xf, _ = pp.ppr(g, src, iters=3000, f=F, k_tile=16, direction=fd, tol=1e-9)
                lam, grad, done = pp.ppr_adjoint(g, Xf, torch.as_tensor(c, dtype=torch.float32, device="cuda"),
                                                 iters=3000, f=F, k_tile=16, direction=ad, tol=1e-9)
                assert done < 3000
                gh = grad.cpu().numpy().astype(np.float64)
                rel = np.linalg.norm(gh - grad_o) / np.linalg.norm(grad_o)
                assert rel <= 1e-5, f"relative gradient error {rel:.2e}"
                lh = lam.cpu().numpy().astype(np.float64)
                assert np.abs(lh - lam_o).max() / np.abs(lam_o).max() <= 1e-5


def test_adjoint_against_finite_differences_tiny():
    host = H.random_graph(24, 80, 5, symmetric=True, connected=True)
    gg.with_weights(host, seed=6)
    src = np.arange(8, dtype=np.int32) * 3
    c = gg.normal(host.n * 8, seed=9).reshape(host.n, 8).astype(np.float64)
    w64 = host.weights.astype(np.float64)

    def loss(w):
        P = H.dense_transition(host, w)
        M = np.linalg.inv(np.eye(host.n) - F * P)
        L = 0.0
        for j, s in enumerate(src):
            L += c[:, j] @ ((1 - F) * M[:, s])
        return L

    h = 1e-6
    fd = np.array([(loss(w64 + h * np.eye(host.nnz)[e]) - loss(w64 - h * np.eye(host.nnz)[e])) / (2 * h)
                   for e in range(host.nnz)])
    g = pp.Graph(host)
    X, _ = pp.ppr(g, src, iters=3000, f=F, k_tile=8, tol=1e-10)
    _, grad, _ = pp.ppr_adjoint(g, X, torch.as_tensor(c, dtype=torch.float32, device="cuda"), iters=3000, f=F,
                                k_tile=8, tol=1e-10)
    gh = grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gh - fd) / np.linalg.norm(fd) <= 1e-5


def test_autograd_function():
    host = H.random_graph(200, 900, 21, symmetric=True, connected=True)
    gg.with_weights(host, seed=4)
    src = np.arange(8, dtype=np.int32) * 11
    w = torch.tensor(host.weights, device="cuda", requires_grad=True)
    X = pp.PPRFunction.apply(w, host, src)
    c = torch.as_tensor(gg.normal(host.n * 8, seed=1).reshape(host.n, 8), device="cuda")
    (X * c).sum().backward()
    Xo = _forward_fixed_point(host, src)
    _, grad_o, _ = oracle.ppr_adjoint(host.off, host.idx, Xo, c.cpu().numpy().astype(np.float64), F, T=20000,
                                      tol=1e-15, weights=host.weights)
    gh = w.grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gh - grad_o) / np.linalg.norm(grad_o) <= 1e-5


def test_adjoint_finite_differences_rmat10_sampled_edges_and_directions():
    # R-MAT scale 10 (n = 1024), weighted, 8 sources: the GPU gradient against
    # FP64 central differences of the dense solve on 256 sampled edges and on
    # 8 random directions (g . delta vs [L(w + h delta) - L(w - h delta)] / 2h)
    import scipy.linalg as sla

    host = gg.rmat(10, 16, seed=1)
    gg.with_weights(host, seed=5)
    n = host.n
    src = gg.pick_vertices(host, 8, seed=3)
    c = gg.normal(n * 8, seed=7).reshape(n, 8).astype(np.float64)
    w64 = host.weights.astype(np.float64)
    rows = np.repeat(np.arange(n), np.diff(host.off))
    E = np.zeros((n, 8))
    E[src, np.arange(8)] = 1.0 - F

    def transition(w):
        s = np.bincount(rows, weights=w, minlength=n)
        P = np.zeros((n, n))
        np.add.at(P, (host.idx, rows), w / s[rows])
        return P

    def loss(w):
        return float((c * np.linalg.solve(np.eye(n) - F * transition(w), E)).sum())

    P0 = transition(w64)
    lu = sla.lu_factor(np.eye(n) - F * P0)
    X0 = sla.lu_solve(lu, E)
    L0 = float((c * X0).sum())

    def loss_edge(e, dh):
        # one weight changes column v of P only: I - fP changes by a rank-one
        # term, so the solve is updated by Sherman-Morrison
        v = rows[e]
        w = w64.copy()
        w[e] += dh
        b, t = host.off[v], host.off[v + 1]
        col = np.zeros(n)
        np.add.at(col, host.idx[b:t], w[b:t] / w[b:t].sum())
        y = sla.lu_solve(lu, F * (col - P0[:, v]))
        return L0 + float((c.T @ y) @ X0[v]) / (1.0 - y[v])

    g = pp.Graph(host)
    X, _ = pp.ppr(g, src, iters=3000, f=F, k_tile=8, tol=1e-10)
    _, grad, _ = pp.ppr_adjoint(g, X, torch.as_tensor(c, dtype=torch.float32, device="cuda"), iters=3000, f=F,
                                k_tile=8, tol=1e-10)
    gh = grad.cpu().numpy().astype(np.float64)
    h = 1e-6
    edges = np.unique(gg.uniform_int(256, 0, host.nnz - 1, seed=9))
    fd = np.array([(loss_edge(e, h) - loss_edge(e, -h)) / (2 * h) for e in edges])
    assert abs(loss_edge(int(edges[0]), h) - loss(w64 + h * np.eye(1, host.nnz, int(edges[0]))[0])) <= 1e-10
    assert np.linalg.norm(gh[edges] - fd) / np.linalg.norm(fd) <= 1e-5
    for r in range(8):
        d = gg.normal(host.nnz, seed=100 + r).astype(np.float64)
        d /= np.linalg.norm(d)
        fdd = (loss(w64 + h * d) - loss(w64 - h * d)) / (2 * h)
        assert abs(gh @ d - fdd) <= 1e-5 * np.linalg.norm(gh), (r, gh @ d, fdd)


@pytest.mark.parametrize("sym,kt,k,T", [(True, 8, 8, 30), (False, 16, 20, 12), (True, 32, 3, 1), (False, 8, 5, 0)])
def test_unrolled_adjoint_matches_oracle(sym, kt, k, T):
    host = H.random_graph(3000, 15000, 30 + T, symmetric=sym, connected=True)
    gg.with_weights(host, seed=9)
    src = gg.pick_vertices(host, k, seed=4)
    c = gg.normal(host.n * k, seed=6).reshape(host.n, k).astype(np.float64)
    lam_o, grad_o = oracle.ppr_adjoint_unrolled(host.off, host.idx, src, c, F, T, weights=host.weights)
    for rl in (True, False):
        g = pp.Graph(host, relabel=rl)
        announce(f"unrolled adjoint sym={sym} kt={kt} k={k} T={T} relabel={rl}")
        lam, grad = pp.ppr_adjoint_unrolled(g, src, torch.as_tensor(c, dtype=torch.float32), T=T, f=F, k_tile=kt)
        gh = grad.cpu().numpy().astype(np.float64)
        lh = lam.cpu().numpy().astype(np.float64)
        if T == 0:
            assert np.abs(gh).max() == 0.0
        else:
            assert np.linalg.norm(gh - grad_o) / np.linalg.norm(grad_o) <= 1e-5
        assert np.abs(lh - lam_o).max() <= 1e-5 * max(np.abs(lam_o).max(), 1e-30)


def test_unrolled_adjoint_finite_differences_rmat10():
    # the T-step map itself: central differences of c . X_T(w) in FP64
    host = gg.rmat(10, 16, seed=2)
    gg.with_weights(host, seed=1)
    n, T = host.n, 20
    src = gg.pick_vertices(host, 4, seed=2)
    c = gg.normal(n * 4, seed=3).reshape(n, 4).astype(np.float64)
    w64 = host.weights.astype(np.float64)
    rows = np.repeat(np.arange(n), np.diff(host.off))

    def loss(w):
        s = np.bincount(rows, weights=w, minlength=n)
        P = np.zeros((n, n))
        np.add.at(P, (host.idx, rows), w / s[rows])
        X = np.zeros((n, 4))
        X[src, np.arange(4)] = 1.0
        E = (1 - F) * X.copy()
        for _ in range(T):
            X = E + F * (P @ X)
        return float((c * X).sum())

    g = pp.Graph(host)
    _, grad = pp.ppr_adjoint_unrolled(g, src, torch.as_tensor(c, dtype=torch.float32), T=T, f=F, k_tile=8)
    gh = grad.cpu().numpy().astype(np.float64)
    h = 1e-6
    edges = np.unique(gg.uniform_int(64, 0, host.nnz - 1, seed=11))
    fd = np.array([(loss(w64 + h * np.eye(1, host.nnz, e)[0]) - loss(w64 - h * np.eye(1, host.nnz, e)[0])) / (2 * h)
                   for e in edges])
    assert np.linalg.norm(gh[edges] - fd) / np.linalg.norm(fd) <= 1e-5


@pytest.mark.parametrize("relabel", [True, False])
def test_set_weights_in_place_matches_a_fresh_registration(relabel):
    # New weights on a registered graph give bit-identical pull results (and
    # push results within the bar) to registering the graph with them.
    host = H.random_graph(3000, 20000, 8, symmetric=False, connected=True)
    gg.with_weights(host, seed=1)
    w2 = gg.uniform(host.nnz, 0.1, 1.0, 99, stream=3).astype(np.float32)
    src = gg.pick_vertices(host, 16, seed=2)
    g = pp.Graph(host, relabel=relabel)
    g.set_weights(torch.as_tensor(w2, device="cuda"))
    import copy
    fresh_host = copy.copy(host)
    fresh_host.weights = w2
    fresh = pp.Graph(fresh_host, relabel=relabel)
    want, _ = oracle.ppr(host.off, host.idx, src, F, T=25, weights=w2)
    for d in (pp.PP_PULL, pp.PP_PUSH):
        a, _ = pp.ppr(g, src, iters=25, f=F, k_tile=16, direction=d)
        b, _ = pp.ppr(fresh, src, iters=25, f=F, k_tile=16, direction=d)
        if d == pp.PP_PULL:
            assert torch.equal(a, b)
        _cols_close(a.cpu().numpy(), want)
        _cols_close(b.cpu().numpy(), want)
    with pytest.raises(ValueError):
        g.set_weights(torch.ones(host.nnz + 1, device="cuda"))
    unweighted = pp.Graph(H.path(10))
    with pytest.raises(ValueError):
        unweighted.set_weights(torch.ones(18, device="cuda"))


def test_autograd_function_registers_once_and_keeps_each_forwards_weights():
    # Two forwards with different weights before either backward: the graph is
    # registered once, and each backward uses its own forward's weights.
    host = H.random_graph(200, 900, 21, symmetric=True, connected=True)
    gg.with_weights(host, seed=4)
    src = np.arange(8, dtype=np.int32) * 11
    c = torch.as_tensor(gg.normal(host.n * 8, seed=1).reshape(host.n, 8), device="cuda")
    w1 = torch.tensor(host.weights, device="cuda", requires_grad=True)
    w2 = torch.tensor(host.weights * 1.5 + 0.05, device="cuda", requires_grad=True)
    X1 = pp.PPRFunction.apply(w1, host, src)
    X2 = pp.PPRFunction.apply(w2, host, src)
    assert len(host._pp_graphs) == 1
    (X1 * c).sum().backward()
    (X2 * c).sum().backward()
    assert len(host._pp_graphs) == 1
    for w, Xg in ((w1, X1), (w2, X2)):
        wn = w.detach().cpu().numpy().astype(np.float32)
        Xo, _ = oracle.ppr(host.off, host.idx, src, F, T=20000, tol=1e-15, weights=wn)
        assert np.abs(Xg.detach().cpu().numpy() - Xo).sum(axis=0).max() <= 1e-6
        _, grad_o, _ = oracle.ppr_adjoint(host.off, host.idx, Xo, c.cpu().numpy().astype(np.float64), F, T=20000,
                                          tol=1e-15, weights=wn)
        gh = w.grad.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(gh - grad_o) / np.linalg.norm(grad_o) <= 1e-5


@pytest.mark.parametrize("name", ["grid", "directed"])
def test_adjoint_generic_switch_sparse_then_dense(name):
    # PP_SWITCH for the adjoint: Lambda's support starts at the nonzero rows of
    # dL/dX and grows along in-edges, pushed sparsely until it holds m/14
    # edges, then dense pulls.  A loss on a few vertices keeps the first sweeps
    # sparse; a dense loss switches at once.  Both match the oracle's Lambda
    # and gradient, and T fixed sweeps equal T pull sweeps.
    if name == "grid":
        host = H.full_grid(60, 60)
        gg.with_weights(host, seed=13)
    else:
        host = H.random_graph(2500, 7000, 17, symmetric=False, connected=True)
        gg.with_weights(host, seed=14)
    src = np.arange(8, dtype=np.int32) * 97
    Xo = _forward_fixed_point(host, src)
    sparse_c = np.zeros((host.n, 8))
    rows = np.array([5, 700, 1400, 2100, 2498])
    sparse_c[rows, :] = gg.normal(len(rows) * 8, seed=3).reshape(len(rows), 8)
    dense_c = gg.normal(host.n * 8, seed=4).reshape(host.n, 8).astype(np.float64)
    for rl in (True, False):
        g = pp.Graph(host, relabel=rl)
        X, _ = pp.ppr(g, src, iters=3000, f=F, k_tile=8, tol=1e-9)
        for which, c in (("sparse", sparse_c), ("dense", dense_c)):
            announce(f"adjoint switch {name} relabel={rl} loss={which}")
            lam_o, grad_o, _ = oracle.ppr_adjoint(host.off, host.idx, Xo, c, F, T=20000, tol=1e-15,
                                                  weights=host.weights)
            ct = torch.as_tensor(c, dtype=torch.float32, device="cuda")
            lam, grad, done = pp.ppr_adjoint(g, X, ct, iters=3000, f=F, k_tile=8, direction=pp.PP_SWITCH, tol=1e-9)
            # (FP32 sweeps on a grid with a dense loss can cycle just above a
            # 1e-9 relative change instead of stopping: accuracy is the bar)
            gh = grad.cpu().numpy().astype(np.float64)
            assert np.linalg.norm(gh - grad_o) / np.linalg.norm(grad_o) <= 1e-5
            lh = lam.cpu().numpy().astype(np.float64)
            assert np.abs(lh - lam_o).max() / np.abs(lam_o).max() <= 1e-5
            # a fixed number of sweeps: the sparse sweeps are exact iterations
            ls, _, _ = pp.ppr_adjoint(g, X, ct, iters=12, f=F, k_tile=8, direction=pp.PP_SWITCH)
            lp, _, _ = pp.ppr_adjoint(g, X, ct, iters=12, f=F, k_tile=8, direction=pp.PP_PULL)
            assert (ls - lp).abs().max().item() <= 1e-5 * lp.abs().max().item()
        g.close()
