"""Pins of the FP64 oracle against what the paper's definitions and mathematics fix.

Each test checks the oracle against something other than itself: closed forms
of the PageRank equation (Sec. 3.1) on regular, star and bipartite graphs, a
dense linear solve of the fixed point, the T-step matrix form, brute-force hop
distances, a library shortest-path routine, BFS invariants, and finite
differences for the adjoint.  Directed graphs are included so that a
transposed operand (in- vs out-neighbours) cannot pass unnoticed.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen as gg
import oracle
from tests import helpers as H

F = 0.85


# --------------------------------------------------------------------------- PageRank
@pytest.mark.parametrize("g", [H.complete(7), H.cycle(11), H.full_grid(1, 2)], ids=lambda g: g.name)
def test_pr_regular_graph_stays_uniform(g):
    # On a d-regular graph with x0 = 1/n every update returns 1/n exactly.
    for T in (1, 5, 20):
        x = oracle.pagerank(g.off, g.idx, F, T)
        np.testing.assert_allclose(x, 1.0 / g.n, rtol=0, atol=1e-15)


def _star_recurrence(n, f, T):
    xc, xl = 1.0 / n, 1.0 / n
    for _ in range(T):
        xc, xl = (1 - f) / n + f * (n - 1) * xl, (1 - f) / n + f * xc / (n - 1)
    return xc, xl


@pytest.mark.parametrize("n", [2, 5, 40])
def test_pr_star_two_state_recurrence_and_fixed_point(n):
    g = H.star(n)
    for T in (1, 2, 7, 20):
        x = oracle.pagerank(g.off, g.idx, F, T)
        xc, xl = _star_recurrence(n, F, T)
        assert abs(x[0] - xc) < 1e-15
        np.testing.assert_allclose(x[1:], xl, rtol=0, atol=1e-15)
    x = oracle.pagerank(g.off, g.idx, F, 400)
    xc = (1 + F * (n - 1)) / (n * (1 + F))
    xl = (1 + F / (n - 1)) / (n * (1 + F))
    assert abs(x[0] - xc) < 1e-14
    np.testing.assert_allclose(x[1:], xl, atol=1e-14)
    assert abs(x.sum() - 1.0) < 1e-13


def test_pr_complete_bipartite_closed_form():
    a, b = 3, 8
    g = H.complete_bipartite(a, b)
    n = a + b
    xa, xb = 1.0 / n, 1.0 / n
    for T in range(1, 15):
        xa, xb = (1 - F) / n + F * b * xb / a, (1 - F) / n + F * a * xa / b
        x = oracle.pagerank(g.off, g.idx, F, T)
        np.testing.assert_allclose(x[:a], xa, atol=1e-15)
        np.testing.assert_allclose(x[a:], xb, atol=1e-15)


@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pr_matches_dense_solve_and_matrix_power(symmetric, seed):
    g = H.random_graph(30, 90, seed, symmetric=symmetric, connected=True)
    P = H.dense_transition(g)
    n = g.n
    b = np.full(n, (1 - F) / n)
    # T-step matrix form x_T = (fP)^T x0 + sum_{k<T} (fP)^k b
    M = F * P
    x = np.full(n, 1.0 / n)
    for T in (1, 3, 20):
        xt = np.linalg.matrix_power(M, T) @ x + sum(np.linalg.matrix_power(M, k) @ b for k in range(T))
        np.testing.assert_allclose(oracle.pagerank(g.off, g.idx, F, T), xt, rtol=0, atol=1e-15)
    # converged iterate = fixed point of (I - fP) x = (1-f)/n
    xs = np.linalg.solve(np.eye(n) - M, b)
    np.testing.assert_allclose(oracle.pagerank(g.off, g.idx, F, 400), xs, rtol=0, atol=1e-14)


def test_pr_directed_transposed_operand_would_fail():
    # On a directed graph the pulling sum must run over IN-neighbours; using
    # out-neighbours gives a different vector, which the dense form rejects.
    g = H.random_graph(25, 70, 9, symmetric=False, connected=True)
    P = H.dense_transition(g)
    x = oracle.pagerank(g.off, g.idx, F, 3)
    M = F * P
    x0 = np.full(g.n, 1.0 / g.n)
    b = np.full(g.n, (1 - F) / g.n)
    want = M @ (M @ (M @ x0 + b) + b) + b
    np.testing.assert_allclose(x, want, atol=1e-15)
    wrong = F * P.T
    bad = wrong @ (wrong @ (wrong @ x0 + b) + b) + b
    assert np.abs(bad - want).sum() > 1e-4


def test_pr_push_and_pull_forms_agree():
    g = gg.rmat(10, 16, seed=3)
    a = oracle.pagerank(g.off, g.idx, F, 20)
    b = oracle.pagerank_push(g.off, g.idx, F, 20)
    assert np.abs(a - b).sum() < 1e-14
    d = H.random_graph(200, 900, 4, symmetric=False)
    assert np.abs(oracle.pagerank(d.off, d.idx, F, 20) - oracle.pagerank_push(d.off, d.idx, F, 20)).sum() < 1e-14


def test_pr_threaded_pull_is_the_same_iterate():
    # The multi-threaded pulling form (timed as the CPU baseline) matches the
    # T-step matrix form on a directed graph, and the sequential oracle bit for
    # bit on an R-MAT graph with isolated vertices and hubs.
    d = H.random_graph(25, 70, 11, symmetric=False, connected=True)
    M = F * H.dense_transition(d)
    b = np.full(d.n, (1 - F) / d.n)
    x = np.full(d.n, 1.0 / d.n)
    for _ in range(4):
        x = M @ x + b
    got, threads = oracle.pagerank_threads(d.off, d.idx, F, 4)
    assert threads >= 1
    np.testing.assert_allclose(got, x, rtol=0, atol=1e-15)
    g = gg.rmat(12, 16, seed=5)
    got, _ = oracle.pagerank_threads(g.off, g.idx, F, 20)
    assert np.array_equal(got, oracle.pagerank(g.off, g.idx, F, 20))
    got0, _ = oracle.pagerank_threads(g.off, g.idx, F, 0)
    assert np.array_equal(got0, np.full(g.n, 1.0 / g.n))


def test_pr_mass_balance_with_isolated_vertices():
    # Dangling/isolated vertices keep (1-f)/n and pass nothing on, so
    # sum x_{t+1} = (1-f) + f * sum_{d(v)>0} x_t(v).
    g = gg.rmat(12, 16, seed=5)
    deg = np.diff(g.off)
    assert (deg == 0).any()
    xt = oracle.pagerank(g.off, g.idx, F, 7)
    xt1 = oracle.pagerank(g.off, g.idx, F, 1, x0=xt)
    assert abs(xt1.sum() - ((1 - F) + F * xt[deg > 0].sum())) < 1e-13
    # isolated vertices (no in-edges either, symmetric graph) sit at (1-f)/n
    assert np.all(np.abs(xt1[deg == 0] - (1 - F) / g.n) < 1e-18)


def test_pr_step_at_matches_full_step():
    g = H.random_graph(300, 1500, 6, symmetric=False)
    x = (np.random.default_rng(0).random(g.n) / g.n).astype(np.float32)
    full = oracle.pagerank(g.off, g.idx, F, 1, x0=x.astype(np.float64))
    verts = np.array([0, 5, 17, 17, 299, 123], dtype=np.int32)
    np.testing.assert_allclose(oracle.pagerank_step_at(g.off, g.idx, x, verts, F), full[verts], atol=1e-16)


def test_pr_zero_iterations_returns_start():
    g = H.path(5)
    np.testing.assert_array_equal(oracle.pagerank(g.off, g.idx, F, 0), np.full(5, 0.2))


# --------------------------------------------------------------------------- PPR
@pytest.mark.parametrize("symmetric", [True, False])
def test_ppr_linearity_gives_uniform_pagerank(symmetric):
    # mean over all sources of PPR(e_s) = uniform PageRank, for every T.
    g = H.random_graph(40, 150, 11, symmetric=symmetric)
    X, _ = oracle.ppr(g.off, g.idx, np.arange(g.n), F, T=12)
    np.testing.assert_allclose(X.mean(axis=1), oracle.pagerank(g.off, g.idx, F, 12), atol=1e-16)


@pytest.mark.parametrize("weighted", [False, True])
def test_ppr_fixed_point_dense_solve(weighted):
    g = H.random_graph(35, 120, 12, symmetric=False, connected=True)
    w = gg.uniform(g.nnz, 0.1, 1.0, seed=3) if weighted else None
    P = H.dense_transition(g, w)
    src = np.array([0, 7, 20], dtype=np.int32)
    X, it = oracle.ppr(g.off, g.idx, src, F, T=5000, tol=1e-15, weights=w)
    assert np.all(it < 5000)
    for j, s in enumerate(src):
        e = np.zeros(g.n)
        e[s] = 1.0
        want = np.linalg.solve(np.eye(g.n) - F * P, (1 - F) * e)
        np.testing.assert_allclose(X[:, j], want, atol=1e-13)


def test_ppr_constant_weights_equal_unweighted():
    g = H.random_graph(50, 200, 13, symmetric=True)
    src = np.array([1, 2, 3], dtype=np.int32)
    a, _ = oracle.ppr(g.off, g.idx, src, F, T=15)
    b, _ = oracle.ppr(g.off, g.idx, src, F, T=15, weights=np.full(g.nnz, 0.37, np.float32))
    np.testing.assert_allclose(a, b, atol=1e-15)


# --------------------------------------------------------------------------- adjoint
def _loss_dense(g, w, src, c):
    P = H.dense_transition(g, w)
    X = np.zeros((g.n, len(src)))
    for j, s in enumerate(src):
        e = np.zeros(g.n)
        e[s] = 1.0
        X[:, j] = np.linalg.solve(np.eye(g.n) - F * P, (1 - F) * e)
    return float((c * X).sum()), X


@pytest.mark.parametrize("symmetric", [True, False])
def test_adjoint_matches_finite_differences_of_dense_solve(symmetric):
    g = H.random_graph(18, 60, 21, symmetric=symmetric, connected=True)
    w = gg.uniform(g.nnz, 0.1, 1.0, seed=4).astype(np.float64)
    src = np.array([0, 5], dtype=np.int32)
    c = np.random.default_rng(5).standard_normal((g.n, len(src)))
    L0, X = _loss_dense(g, w, src, c)
    lam, grad, it = oracle.ppr_adjoint(g.off, g.idx, X, c, F, T=5000, tol=1e-15, weights=w.astype(np.float32))
    # finite differences need the same float32-rounded weights the oracle saw
    w32 = w.astype(np.float32).astype(np.float64)
    h = 1e-6
    fd = np.empty(g.nnz)
    for e in range(g.nnz):
        wp, wm = w32.copy(), w32.copy()
        wp[e] += h
        wm[e] -= h
        fd[e] = (_loss_dense(g, wp, src, c)[0] - _loss_dense(g, wm, src, c)[0]) / (2 * h)
    assert np.linalg.norm(grad - fd) / np.linalg.norm(fd) < 1e-7
    # Lambda is the adjoint solve (I - f P^T) Lambda = c
    P = H.dense_transition(g, w32)
    np.testing.assert_allclose(lam, np.linalg.solve(np.eye(g.n) - F * P.T, c), atol=1e-12)


# --------------------------------------------------------------------------- BFS
def _hop_distance_brute_force(A, r):
    """Smallest k with (A^k)[r, v] > 0, by boolean matrix powers."""
    n = A.shape[0]
    dist = np.full(n, -1)
    reach = np.zeros(n, dtype=bool)
    reach[r] = True
    dist[r] = 0
    cur = reach.copy()
    for k in range(1, n + 1):
        cur = (cur.astype(float) @ A) > 0
        new = cur & ~reach
        dist[new] = k
        reach |= cur
        if not new.any():
            break
    return dist


@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("seed", range(6))
def test_bfs_levels_brute_force(symmetric, seed):
    g = H.random_graph(48, 70, 100 + seed, symmetric=symmetric)
    A = H.dense_adjacency(g)
    for r in (0, 7, 47):
        level, parent, nlev = oracle.bfs(g.off, g.idx, r)
        np.testing.assert_array_equal(level, _hop_distance_brute_force(A, r))
        assert nlev == level.max() + 1
        assert H.bfs_violations(g, r, level, parent) == []


def test_bfs_matches_library_shortest_path_mid_size():
    for sym in (True, False):
        g = H.random_graph(3000, 6000, 7, symmetric=sym)
        A = sp.csr_matrix((np.ones(g.nnz), g.idx, g.off), shape=(g.n, g.n))
        d = csg.shortest_path(A, directed=True, unweighted=True, indices=11)
        want = np.where(np.isinf(d), -1, d).astype(np.int64)
        level, parent, _ = oracle.bfs(g.off, g.idx, 11)
        np.testing.assert_array_equal(level, want)
        assert H.bfs_violations_fast(g, 11, level, parent) == []


def test_bfs_closed_forms():
    n = 13
    lv, _, _ = oracle.bfs(H.path(n).off, H.path(n).idx, 4)
    np.testing.assert_array_equal(lv, np.abs(np.arange(n) - 4))
    c = H.cycle(n)
    lv, _, _ = oracle.bfs(c.off, c.idx, 0)
    np.testing.assert_array_equal(lv, np.minimum(np.arange(n), n - np.arange(n)))
    s = H.star(9)
    lv, _, _ = oracle.bfs(s.off, s.idx, 3)
    np.testing.assert_array_equal(lv, [1, 2, 2, 0, 2, 2, 2, 2, 2])
    k = H.complete(6)
    lv, _, _ = oracle.bfs(k.off, k.idx, 2)
    np.testing.assert_array_equal(lv, [1, 1, 0, 1, 1, 1])
    gr = H.full_grid(7, 9)
    lv, par, nlev = oracle.bfs(gr.off, gr.idx, 0)
    r, q = np.divmod(np.arange(63), 9)
    np.testing.assert_array_equal(lv, r + q)
    assert nlev == 6 + 8 + 1


def test_bfs_unreachable_and_isolated():
    g = gg.from_edges(6, [0, 1, 3], [1, 2, 4], True)
    lv, par, nlev = oracle.bfs(g.off, g.idx, 0)
    np.testing.assert_array_equal(lv, [0, 1, 2, -1, -1, -1])
    np.testing.assert_array_equal(par, [0, 0, 1, -1, -1, -1])
    lv, par, nlev = oracle.bfs(g.off, g.idx, 5)
    np.testing.assert_array_equal(lv, [-1, -1, -1, -1, -1, 0])
    assert nlev == 1


def test_bfs_validator_rejects_corruption():
    g = H.random_graph(200, 600, 8)
    lv, par, _ = oracle.bfs(g.off, g.idx, 0)
    assert H.bfs_violations(g, 0, lv, par) == []
    assert H.bfs_violations_fast(g, 0, lv, par) == []
    reached = np.nonzero((lv > 0))[0]
    v = reached[len(reached) // 2]
    bad = lv.copy()
    bad[v] += 1
    assert H.bfs_violations(g, 0, bad, par) and H.bfs_violations_fast(g, 0, bad, par)
    badp = par.copy()
    badp[v] = v
    assert H.bfs_violations(g, 0, lv, badp) and H.bfs_violations_fast(g, 0, lv, badp)
    # a parent one level up but not adjacent
    cands = np.nonzero(lv == lv[v] - 1)[0]
    row = set(g.idx[g.off[v]:g.off[v + 1]].tolist())
    non = [u for u in cands if u not in row]
    if non:
        badp = par.copy()
        badp[v] = non[0]
        assert H.bfs_violations(g, 0, lv, badp) and H.bfs_violations_fast(g, 0, lv, badp)


def test_bfs_replay_counts():
    for sym in (True, False):
        g = H.random_graph(500, 2000, 31, symmetric=sym)
        lv, _, nlev = oracle.bfs(g.off, g.idx, 0)
        hist = np.bincount(lv[lv >= 0])
        deg = np.diff(g.off)
        # all top-down: each reached vertex's out-row is examined once
        fr, ex, di = oracle.bfs_replay(g.off, g.idx, 0, np.zeros(nlev + 2, np.int8))
        np.testing.assert_array_equal(fr, hist)
        np.testing.assert_array_equal(ex, [deg[lv == l].sum() for l in range(len(fr))])
        np.testing.assert_array_equal(di, list(hist[1:]) + [0])
        # all bottom-up: same frontiers; each unvisited vertex scans its in-row
        # up to the first frontier member (vectorised recount here)
        fr2, ex2, di2 = oracle.bfs_replay(g.off, g.idx, 0, np.ones(nlev + 2, np.int8))
        np.testing.assert_array_equal(fr2, hist)
        g.ensure_transpose()
        for l in range(len(fr2)):
            cnt = 0
            for v in np.nonzero((lv > l) | (lv == -1))[0]:
                row = g.in_idx[g.in_off[v]:g.in_off[v + 1]]
                hit = np.nonzero(lv[row] == l)[0]
                cnt += (hit[0] + 1) if len(hit) else len(row)
            assert ex2[l] == cnt


# --------------------------------------------------------------------------- triangles
def test_triangles_closed_form_and_trace():
    k = H.complete(7)
    np.testing.assert_array_equal(oracle.triangles(k.off, k.idx), np.full(7, 15))
    g = H.random_graph(60, 400, 17)
    A = H.dense_adjacency(g)
    tc = oracle.triangles(g.off, g.idx)
    np.testing.assert_array_equal(tc, np.diag(A @ A @ A).astype(np.int64) // 2)


# --------------------------------------------------------------------------- betweenness
def _bc_by_definition(g, sources=None):
    """bc(v) = sum over ordered s != v != t of sigma_st(v) / sigma_st (s in
    ``sources``, default all), with
    sigma_st(v) = sigma_sv * sigma_vt when d(s,v) + d(v,t) = d(s,t): all-pairs
    BFS path counts, no dependency recursion."""
    n = g.n
    A = H.dense_adjacency(g) > 0
    dist = np.full((n, n), -1, dtype=np.int64)
    sig = np.zeros((n, n))
    for s in range(n):
        dist[s, s], sig[s, s] = 0, 1.0
        frontier = [s]
        while frontier:
            nxt = set()
            for v in frontier:
                for w in np.nonzero(A[v])[0]:
                    if dist[s, w] < 0:
                        dist[s, w] = dist[s, v] + 1
                        nxt.add(int(w))
                    if dist[s, w] == dist[s, v] + 1:
                        sig[s, w] += sig[s, v]
            frontier = sorted(nxt)
    bc = np.zeros(n)
    for s in (range(n) if sources is None else sources):
        for t in range(n):
            if s == t or dist[s, t] < 0:
                continue
            for v in range(n):
                if v in (s, t) or dist[s, v] < 0 or dist[v, t] < 0:
                    continue
                if dist[s, v] + dist[v, t] == dist[s, t]:
                    bc[v] += sig[s, v] * sig[v, t] / sig[s, t]
    return bc


@pytest.mark.parametrize("sym", [True, False])
def test_bc_matches_definition_on_small_graphs(sym):
    for seed, (n, m) in enumerate([(12, 20), (25, 60), (40, 90)]):
        g = H.random_graph(n, m, 60 + seed, symmetric=sym)
        np.testing.assert_allclose(oracle.bc(g.off, g.idx, np.arange(n)), _bc_by_definition(g), rtol=1e-12,
                                   atol=1e-12)
        # a subset of sources (on a directed graph this also fixes the edge direction)
        sub = [0, n // 3, n - 1]
        np.testing.assert_allclose(oracle.bc(g.off, g.idx, sub), _bc_by_definition(g, sub), rtol=1e-12,
                                   atol=1e-12)


def test_bc_closed_forms():
    n = 9
    # path: vertex i separates i vertices from n-1-i, both directions
    i = np.arange(n)
    np.testing.assert_allclose(oracle.bc(H.path(n).off, H.path(n).idx, i), 2.0 * i * (n - 1 - i))
    st = H.star(n)
    want = np.zeros(n)
    want[0] = (n - 1) * (n - 2)
    np.testing.assert_allclose(oracle.bc(st.off, st.idx, i), want)
    k = H.complete(n)
    np.testing.assert_allclose(oracle.bc(k.off, k.idx, i), np.zeros(n))
    # even cycle C_2k: every vertex has the same score, and the scores sum to
    # the total excess path length sum_{s != t} (d(s,t) - 1)
    c = H.cycle(10)
    b = oracle.bc(c.off, c.idx, np.arange(10))
    d = np.minimum(np.arange(10), 10 - np.arange(10))
    np.testing.assert_allclose(b, np.full(10, b[0]))
    assert b.sum() == pytest.approx(10 * np.sum(np.maximum(d[1:] - 1, 0)))


def test_bc_is_additive_over_sources():
    g = H.random_graph(60, 200, 77)
    a = oracle.bc(g.off, g.idx, [0, 5, 9])
    b = oracle.bc(g.off, g.idx, [0]) + oracle.bc(g.off, g.idx, [5]) + oracle.bc(g.off, g.idx, [9])
    np.testing.assert_allclose(a, b, rtol=1e-13)


# --------------------------------------------------------------------------- unrolled adjoint
@pytest.mark.parametrize("sym,weighted,T", [(True, False, 5), (False, True, 12), (True, True, 1), (False, False, 0)])
def test_unrolled_adjoint_matches_finite_differences_of_the_T_step_map(sym, weighted, T):
    g = H.random_graph(30, 90, 90 + T, symmetric=sym, connected=True)
    if weighted:
        gg.with_weights(g, seed=3)
    w0 = g.weights.astype(np.float64) if weighted else np.ones(g.nnz)
    src = np.array([0, 7, 29], dtype=np.int32)
    c = gg.normal(g.n * 3, seed=5).reshape(g.n, 3).astype(np.float64)

    def xT(w):
        P = H.dense_transition(g, w)
        X = np.zeros((g.n, 3))
        X[src, np.arange(3)] = 1.0
        E = (1 - F) * X.copy()
        for _ in range(T):
            X = E + F * P @ X
        return X

    lam0, grad = oracle.ppr_adjoint_unrolled(g.off, g.idx, src, c, F, T, weights=w0.astype(np.float32))
    h = 1e-6
    fd = np.array([((c * xT(w0 + h * np.eye(1, g.nnz, e)[0])).sum() - (c * xT(w0 - h * np.eye(1, g.nnz, e)[0])).sum())
                   / (2 * h) for e in range(g.nnz)])
    scale = max(1.0, np.abs(fd).max())
    np.testing.assert_allclose(grad, fd, atol=1e-8 * scale, rtol=1e-6)
    # dL/dX_0 = (f P^T)^T ... = (f P)^T applied T times to c
    P = H.dense_transition(g, w0)
    want0 = c.copy()
    for _ in range(T):
        want0 = F * P.T @ want0
    np.testing.assert_allclose(lam0, want0, rtol=1e-12, atol=1e-14)


def test_unrolled_adjoint_approaches_the_implicit_one():
    g = H.random_graph(40, 160, 3, symmetric=True, connected=True)
    src = np.array([1, 2], dtype=np.int32)
    c = gg.normal(g.n * 2, seed=8).reshape(g.n, 2).astype(np.float64)
    X, _ = oracle.ppr(g.off, g.idx, src, F, T=3000, tol=1e-15)
    _, g_imp, _ = oracle.ppr_adjoint(g.off, g.idx, X, c, F, T=3000, tol=1e-15)
    _, g_unr = oracle.ppr_adjoint_unrolled(g.off, g.idx, src, c, F, 400)
    assert np.abs(g_unr - g_imp).max() <= 1e-9 * np.abs(g_imp).max()
