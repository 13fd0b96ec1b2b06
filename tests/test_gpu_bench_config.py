"""The benchmark's own configurations, checked against the oracle exactly as
``bench.py`` runs them.

* R-MAT scale 22 with the cached tuned settings the benchmark applies
  (``tuned.json``: degree bins, LDS stages, workgroup sizes, alpha/beta):
  PageRank, 20 pull and 20 push steps from x = 1/n (L1 <= 1e-6), and BFS
  from all 64 benchmark roots with every policy at the tuned alpha/beta
  (levels bit-identical to the oracle, statistics exact; parents valid on
  every switch run and on 8 roots each for push and pull).  The library's
  default settings are checked too (PageRank, and the switch at
  alpha/beta = 14/24 on a few roots).
* The 4096 x 4096 grid with 5% of the edges removed: PageRank push and pull
  (T = 20) and BFS from the corner with the bottom-up (pull) policy, the one
  the many-level BFS tests elsewhere do not run.

The oracle's threaded PageRank is used for speed; it is bit-identical to the
sequential one (pinned in test_oracle.py).
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2010_16012_amd as pp
from paper_2010_16012_amd import autotune
from tests import helpers as H
from tests.gpu_util import F, PR_L1_TOL, announce, default_bins

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TUNED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2010_16012_amd",
                     "tuned.json")
N_ROOTS = 64
GROUP = 8


def _oracle_bfs_many(host, roots):
    with cf.ThreadPoolExecutor(max_workers=min(8, len(roots))) as ex:
        return list(ex.map(lambda r: oracle.bfs(host.off, host.idx, int(r)), roots))


@pytest.fixture(scope="module")
def rmat22():
    host = gg.workload("rmat22")
    tuned = autotune.load(TUNED, host.n, host.nnz)
    assert tuned, "tuned.json has no entry for this GPU and size class"
    autotune.apply(tuned)
    g = pp.Graph(host)
    default_bins()
    roots = gg.pick_vertices(host, N_ROOTS, seed=1)
    yield host, g, tuned, roots
    g.close()


@pytest.fixture(scope="module")
def rmat22_validator(rmat22):
    return H.BfsValidator(rmat22[0])


@pytest.fixture(scope="module")
def rmat22_pagerank(rmat22):
    host = rmat22[0]
    x, _ = oracle.pagerank_threads(host.off, host.idx, F, 20)
    return x


def _pr_bench_form(g, n, d):
    # exactly the benchmark's call: x = 1/n, then 20 steps in place
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    x.fill_(1.0 / n)
    pp.pagerank_into(g, x, 20, F, d)
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("d,name", [(pp.PP_PULL, "pull"), (pp.PP_PUSH, "push")])
def test_rmat22_pagerank_tuned(rmat22, rmat22_pagerank, d, name):
    host, g, tuned, _ = rmat22
    announce(f"PR rmat22 tuned {name}: {tuned}")
    got = _pr_bench_form(g, host.n, d)
    l1 = np.abs(got - rmat22_pagerank).sum()
    assert l1 <= PR_L1_TOL, f"{name}: L1 {l1:.3e}"


def test_rmat22_pagerank_default_settings(rmat22, rmat22_pagerank):
    host = rmat22[0]
    default_bins()
    g = pp.Graph(host)
    for d, name in ((pp.PP_PULL, "pull"), (pp.PP_PUSH, "push")):
        announce(f"PR rmat22 default settings {name}")
        l1 = np.abs(_pr_bench_form(g, host.n, d) - rmat22_pagerank).sum()
        assert l1 <= PR_L1_TOL, f"{name}: L1 {l1:.3e}"
    g.close()


@pytest.mark.parametrize("group", range(N_ROOTS // GROUP))
def test_rmat22_bfs_bench_roots(rmat22, rmat22_validator, group):
    host, g, tuned, roots = rmat22
    alpha, beta = tuned["alpha"], tuned["beta"]
    mine = roots[group * GROUP:(group + 1) * GROUP]
    want = _oracle_bfs_many(host, mine)
    deg = np.diff(host.off)
    r = pp.BfsRun(g)
    for i, (root, (wl, _, nlev)) in enumerate(zip(mine, want)):
        for pol, name in ((pp.PP_PUSH, "push"), (pp.PP_PULL, "pull"), (pp.PP_SWITCH, "switch")):
            announce(f"BFS rmat22 root={root} {name} alpha={alpha} beta={beta}")
            st = r.run(int(root), pol, alpha, beta)
            torch.cuda.synchronize()
            lv = r.level.cpu().numpy()
            assert np.array_equal(lv, wl), f"{name} root {root}: levels differ"
            assert st.levels == nlev
            assert st.reached == int((wl >= 0).sum())
            assert st.edges_reached == int(deg[wl >= 0].sum())
            if pol == pp.PP_SWITCH or i == 0:
                viol = rmat22_validator(int(root), lv, r.parent.cpu().numpy())
                assert viol == [], f"{name} root {root}: {viol}"


def test_rmat22_bfs_default_switch_constants(rmat22, rmat22_validator):
    host, g, _, roots = rmat22
    r = pp.BfsRun(g)
    for root in roots[:3]:
        announce(f"BFS rmat22 root={root} switch alpha=14 beta=24")
        wl, _, _ = oracle.bfs(host.off, host.idx, int(root))
        r.run(int(root), pp.PP_SWITCH, 14.0, 24.0)
        torch.cuda.synchronize()
        lv = r.level.cpu().numpy()
        assert np.array_equal(lv, wl)
        assert rmat22_validator(int(root), lv, r.parent.cpu().numpy()) == []


# ------------------------------------------------------------------ grid
@pytest.fixture(scope="module")
def grid():
    host = gg.workload("grid4096")
    default_bins()
    g = pp.Graph(host)
    yield host, g
    g.close()


@pytest.mark.parametrize("d,name", [(pp.PP_PULL, "pull"), (pp.PP_PUSH, "push")])
def test_grid4096_pagerank(grid, d, name):
    host, g = grid
    want, _ = oracle.pagerank_threads(host.off, host.idx, F, 20)
    announce(f"PR grid4096 {name}")
    got = _pr_bench_form(g, host.n, d)
    l1 = np.abs(got - want).sum()
    assert l1 <= PR_L1_TOL, f"{name}: L1 {l1:.3e}"


def test_grid4096_bfs_pull_from_corner(grid):
    host, g = grid
    wl, _, nlev = oracle.bfs(host.off, host.idx, 0)
    announce(f"BFS grid4096 pull from the corner ({nlev} levels)")
    r = pp.BfsRun(g)
    st = r.run(0, pp.PP_PULL)
    torch.cuda.synchronize()
    lv = r.level.cpu().numpy()
    assert np.array_equal(lv, wl)
    assert st.levels == nlev
    assert H.bfs_violations_fast(host, 0, lv, r.parent.cpu().numpy()) == []
