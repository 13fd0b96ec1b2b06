"""Full-size configurations, in the launch configuration the benchmark times:
batched PPR on R-MAT 20 (k = 256; every k-tile's first and last column
and one inside each), the Erdos-Renyi graph with n = 2^22, and
the PPR adjoint on weighted R-MAT 20 (k = 32).

Where the oracle finishes in seconds it is compared column by column (PPR on
sampled columns, BFS levels, PageRank); the adjoint is checked through
properties that hold at any size: the fixed-point residuals of X and Lambda
and the gradient's definition evaluated in FP64 on sampled CSR slots.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import graphgen as gg
import oracle
import paper_2010_16012_amd as pp
from paper_2010_16012_amd import autotune
from tests import helpers as H
from tests.gpu_util import F, announce, default_bins

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TUNED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2010_16012_amd",
                     "tuned.json")


@pytest.fixture(autouse=True)
def _bins():
    yield
    default_bins()


def test_ppr_rmat20_k256_sampled_columns():
    # the ppr20 workload: 256 seeded sources, 30 sweeps, tuned tile width
    host = gg.rmat(20, 16, seed=1)
    src = gg.pick_vertices(host, 256, seed=2)
    tuned = autotune.load(TUNED, host.n, host.nnz)
    autotune.apply(tuned)
    kt = tuned.get("k_tile", 32)
    # every k-tile's first and last lane, plus one seeded lane inside each tile
    rng = np.random.default_rng(11)
    cols = np.array(sorted({c for t in range(0, 256, kt) for c in (t, t + kt - 1, t + int(rng.integers(1, kt - 1)))}))
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        parts = list(ex.map(lambda s: oracle.ppr(host.off, host.idx, [s], F, T=30)[0][:, 0], src[cols]))
    want = np.stack(parts, axis=1)
    g = pp.Graph(host)
    for d in (pp.PP_PULL, pp.PP_PUSH, pp.PP_SWITCH):
        announce(f"PPR rmat20 k=256 kt={kt} dir={d}")
        X, done = pp.ppr(g, src, iters=30, f=F, k_tile=kt, direction=d)
        assert done == 30
        got = X[:, torch.as_tensor(cols, device=X.device)].cpu().numpy().astype(np.float64)
        l1 = np.abs(got - want).sum(axis=0)
        assert l1.max() <= 1e-6, f"dir {d}: worst sampled column L1 {l1.max():.3e} (column {cols[l1.argmax()]})"
        del X
        torch.cuda.empty_cache()


def test_er22_bfs_levels_and_pagerank():
    host = gg.workload("er22")
    autotune.apply(autotune.load(TUNED, host.n, host.nnz))
    g = pp.Graph(host)
    want, _, nlev = oracle.bfs(host.off, host.idx, 0)
    r = pp.BfsRun(g)
    for pol in (pp.PP_PUSH, pp.PP_PULL, pp.PP_SWITCH):
        announce(f"BFS er22 policy={pol}")
        st = r.run(0, pol)
        torch.cuda.synchronize()
        lv, par = r.level.cpu().numpy(), r.parent.cpu().numpy()
        assert np.array_equal(lv, want)
        assert st.levels == nlev
        assert H.bfs_violations_fast(host, 0, lv, par) == []
    want_x, _ = oracle.pagerank_threads(host.off, host.idx, F, 20)  # bit-identical to oracle.pagerank
    for d in (pp.PP_PULL, pp.PP_PUSH):
        announce(f"PageRank er22 dir={d}")
        x = pp.pagerank(g, 20, F, d).cpu().numpy().astype(np.float64)
        assert np.abs(x - want_x).sum() <= 1e-6


def _transition(host):
    """P (n x n, FP64): P[u, v] = w(v->u) / s(v), s(v) the out-strength."""
    n = host.n
    src = np.repeat(np.arange(n), np.diff(host.off))
    w = host.weights.astype(np.float64)
    s = np.bincount(src, weights=w, minlength=n)
    return sp.csr_matrix((w / s[src], (host.idx, src)), shape=(n, n)), s, src


@pytest.mark.parametrize("fwd,adj", [(pp.PP_PUSH, pp.PP_PULL), (pp.PP_PULL, pp.PP_PUSH)])
def test_adjoint_rmat20_k32_properties(fwd, adj):
    # the adjoint20 workload: weighted R-MAT 20, 32 sources, c ~ N(0, 1)
    host = gg.rmat(20, 16, seed=1)
    gg.with_weights(host, seed=5)
    src = gg.pick_vertices(host, 32, seed=3)
    g = pp.Graph(host)
    c = torch.as_tensor(gg.normal(host.n * 32, seed=1).reshape(host.n, 32), device="cuda")
    announce(f"adjoint rmat20 k=32 forward={fwd} adjoint={adj}")
    X, _ = pp.ppr(g, src, iters=300, f=F, k_tile=32, direction=fwd, tol=1e-6)
    lam, grad, _ = pp.ppr_adjoint(g, X, c, iters=300, f=F, k_tile=32, direction=adj, tol=1e-6)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy().astype(np.float64)
    L = lam.cpu().numpy().astype(np.float64)
    C = c.cpu().numpy().astype(np.float64)
    G = grad.cpu().numpy().astype(np.float64)
    P, s, src_of_slot = _transition(host)
    # forward fixed point: X = (1 - f) E + f P X, per column (L1 ~ 1)
    E = np.zeros_like(Xh)
    E[src, np.arange(len(src))] = 1.0
    res_x = np.abs(Xh - (1 - F) * E - F * (P @ Xh)).sum(axis=0)
    assert res_x.max() <= 2e-5, f"forward residual {res_x.max():.3e}"
    # adjoint fixed point: Lambda = C + f P^T Lambda
    PtL = P.T @ L
    res_l = np.linalg.norm(L - C - F * PtL) / np.linalg.norm(C)
    assert res_l <= 2e-5, f"adjoint residual {res_l:.3e}"
    # gradient on sampled slots: (f / s_v) sum_s X[v, s] (Lambda[u, s] - (P^T Lambda)[v, s])
    rng = np.random.default_rng(7)
    slots = rng.choice(host.nnz, size=4000, replace=False)
    v = src_of_slot[slots]
    u = host.idx[slots]
    want = F / s[v] * np.einsum("ij,ij->i", Xh[v], L[u] - PtL[v])
    rel = np.linalg.norm(G[slots] - want) / np.linalg.norm(want)
    assert rel <= 5e-5, f"gradient relative error {rel:.3e}"
