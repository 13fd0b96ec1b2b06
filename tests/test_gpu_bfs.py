"""BFS top-down (push), bottom-up (pull) and direction-switching runs on the
GPU against the FP64 oracle's FIFO BFS.

Bar: levels bit-identical to the oracle; parents checked for validity (a
reached vertex's parent is an in-neighbour one level up), since several
parents are correct.
"""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2010_16012_amd as pp
from tests import helpers as H
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

POLICIES = [pp.PP_PUSH, pp.PP_PULL, pp.PP_SWITCH]
POL_IDS = ["push", "pull", "switch"]


def _run(g, root, policy):
    r = pp.BfsRun(g)
    st = r.run(root, policy)
    torch.cuda.synchronize()
    return r.level.cpu().numpy(), r.parent.cpu().numpy(), st


def _check(host, roots, policies=POLICIES, fast=False, relabel=(True, False)):
    for rl in relabel:
        g = pp.Graph(host, relabel=rl)
        _check_graph(g, host, roots, policies, fast)
        g.close()


def _check_graph(g, host, roots, policies, fast):
    for root in roots:
        want, _, nlev = oracle.bfs(host.off, host.idx, int(root))
        for pol, name in zip(POLICIES, POL_IDS):
            if pol not in policies:
                continue
            announce(f"BFS {name} {host.name} root={root}")
            lv, par, st = _run(g, int(root), pol)
            assert np.array_equal(lv, want), f"{name} root {root}: levels differ"
            viol = (H.bfs_violations_fast if fast else H.bfs_violations)(host, int(root), lv, par)
            assert viol == [], f"{name} root {root}: {viol}"
            assert st.levels == nlev
            assert st.reached == int((want >= 0).sum())
            deg = np.diff(host.off)
            assert st.edges_reached == int(deg[want >= 0].sum())


def test_vertices_without_in_edges():
    # Bottom-up levels (and frontiers read from a bitmap) stop at the last
    # bitmap word that holds a vertex with an in-edge: vertices past it can
    # never be discovered.  Directed graph: 300 sources with out-edges only,
    # 700 isolated vertices, and a 3,000-vertex random core the sources
    # point into; roots among the sources (in-degree 0, so past that word
    # after relabelling), isolated, and in the core, under every policy.
    rng = np.random.default_rng(7)
    core = H.random_graph(3000, 12000, 21, symmetric=False, connected=True)
    n = 3000 + 300 + 700
    src = [np.repeat(np.arange(core.n), np.diff(core.off)), 3000 + np.repeat(np.arange(300), 20)]
    dst = [core.idx, rng.integers(0, 3000, 300 * 20)]
    host = gg.from_edges(n, np.concatenate(src), np.concatenate(dst), False, "sources_core_isolated")
    host.ensure_transpose()
    assert np.diff(host.in_off)[3000:].max() == 0
    _check(host, [3000, 3299, 3400, n - 1, 0, 2999])


@pytest.mark.parametrize("maker", [lambda: H.path(300), lambda: H.star(100), lambda: H.cycle(129),
                                   lambda: H.complete(12), lambda: H.full_grid(20, 33)],
                         ids=["path", "star", "cycle", "K12", "grid"])
def test_small_graphs(maker):
    host = maker()
    _check(host, [0, host.n // 2, host.n - 1])


def test_rmat14_from_vertex0_and_random_roots():
    host = gg.workload("rmat14")
    roots = [0] + list(gg.pick_vertices(host, 5, seed=3))
    _check(host, roots)


def test_long_rows_take_the_chunked_top_down_pass():
    # rows longer than 1024 edges go through the second top-down kernel
    host = H.star(5000)
    _check(host, [0, 17])
    host = gg.from_edges(9002, np.concatenate([np.zeros(3000), np.ones(3000), np.arange(2, 3002)]),
                         np.concatenate([np.arange(2, 3002), np.arange(3002, 6002), np.arange(6002, 9002)]), True)
    _check(host, [0, 1, 5000])


def test_disconnected_isolated_root_and_ragged():
    host = gg.from_edges(1000, np.arange(0, 400), np.arange(1, 401), True)  # a path 0..400, rest isolated
    _check(host, [0, 200, 999])
    one = gg.from_edges(1, [], [], True)
    _check(one, [0])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_directed_graphs_td_uses_out_bu_uses_in(seed):
    host = H.random_graph(4000, 9000, seed, symmetric=False)
    host.ensure_transpose()
    _check(host, [0, 17])


@pytest.mark.parametrize("relabel", [True, False])
def test_step_api_any_direction_sequence(relabel):
    host = gg.workload("rmat14")
    g = pp.Graph(host, relabel=relabel)
    want, _, nlev = oracle.bfs(host.off, host.idx, 0)
    rng = np.random.default_rng(4)
    for trial in range(4):
        r = pp.BfsRun(g)
        r.init(0)
        lvl = 0
        while True:
            r.step(lvl, pp.PP_PUSH if rng.random() < 0.5 else pp.PP_PULL)
            lvl += 1
            if r.frontier() == 0:
                break
        assert lvl == nlev
        lv = r.level.cpu().numpy()
        par = r.parent.cpu().numpy()
        assert np.array_equal(lv, want)
        assert H.bfs_violations(host, 0, lv, par) == []
        # a step on an empty frontier changes nothing
        r.step(lvl, pp.PP_PULL)
        assert np.array_equal(r.level.cpu().numpy(), want)


def _streamed_levels(host, want):
    """Levels l whose bottom-up expansion streams the whole in-edge array: a
    sparse frontier (8 |F| < ceil(n/64)) with few out-edges (256 m_f <= nnz)
    while at least half the edges leave vertices not yet visited."""
    deg = np.diff(host.off).astype(np.int64)
    words = (host.n + 63) // 64
    out = set()
    for l in range(int(want.max()) + 1):
        nf = int(np.count_nonzero(want == l))
        mf = int(deg[want == l].sum())
        reached = (want >= 0) & (want <= l)
        mu = int(host.nnz - deg[reached].sum())
        if nf * 8 < words and 2 * mu >= host.nnz and 256 * mf <= host.nnz:
            out.add(l)
    return out


@pytest.mark.parametrize("relabel", [True, False])
def test_bottom_up_parents_are_first_in_stored_order(relabel):
    # pull scans in-neighbours in stored order and stops at the first frontier
    # member; in-rows of more than 256 edges are scanned in chunks, any of
    # which may claim the vertex, and a level that streams the in-edge array
    # takes any frontier in-neighbour (each still a valid parent)
    host = gg.workload("rmat14")
    g = pp.Graph(host, relabel=relabel)
    want, _, _ = oracle.bfs(host.off, host.idx, 0)
    lv, par, _ = _run(g, 0, pp.PP_PULL)
    deg = np.diff(host.off)
    streamed = _streamed_levels(host, want)
    checked = 0
    for v in np.nonzero(want > 0)[0]:
        row = host.idx[host.off[v]:host.off[v + 1]]
        hits = row[want[row] == want[v] - 1]
        if deg[v] <= 256 and (want[v] - 1) not in streamed:
            assert par[v] == hits[0]
            checked += 1
        else:
            assert par[v] in hits
    assert checked > 1000


def test_streamed_bottom_up_levels_on_sparse_frontiers():
    # pull BFS from low-degree roots: the first levels have tiny frontiers and
    # stream the in-edge array; levels and parents stay exact / valid
    host = gg.workload("rmat14")
    g = pp.Graph(host)
    deg = np.diff(host.off)
    roots = [int(r) for r in np.nonzero(deg == 1)[0][:3]]
    for root in roots:
        announce(f"bfs streamed pull rmat14 root={root}")
        want, _, _ = oracle.bfs(host.off, host.idx, root)
        assert 0 in _streamed_levels(host, want)
        lv, par, st = _run(g, root, pp.PP_PULL)
        np.testing.assert_array_equal(lv, want)
        assert H.bfs_violations_fast(host, root, lv, par) == []
        assert st.reached == int((want >= 0).sum())


def test_switch_policy_changes_direction_on_rmat():
    host = gg.workload("rmat14")
    g = pp.Graph(host)
    lv, par, st = _run(g, 0, pp.PP_SWITCH)
    dirs = [st.dir[i] for i in range(st.levels)]
    assert pp.PP_PUSH in dirs and pp.PP_PULL in dirs, dirs


def test_bad_root_raises():
    g = pp.Graph(H.path(5))
    with pytest.raises(pp.PPError):
        pp.bfs(g, 5)
    with pytest.raises(pp.PPError):
        pp.bfs(g, -1)


@pytest.mark.slow
def test_grid4096_corner_many_levels():
    host = gg.workload("grid4096")
    announce(f"BFS grid n={host.n}")
    _check(host, [0], policies=[pp.PP_PUSH, pp.PP_SWITCH], fast=True, relabel=(True,))


@pytest.mark.parametrize("maker,root", [(lambda: H.path(300), 0), (lambda: gg.workload("rmat14"), 0),
                                        (lambda: H.full_grid(40, 60), 0)], ids=["path300", "rmat14", "grid40x60"])
def test_level_log_covers_every_level(maker, root):
    # The caller-sized log holds every level, also past the 64 the stats keep:
    # n_f and m_f per level equal the level sizes and out-edge sums of the
    # oracle's levels, and the first 64 entries agree with the stats.
    host = maker()
    want, _, nlev = oracle.bfs(host.off, host.idx, root)
    deg = np.diff(host.off)
    g = pp.Graph(host)
    r = pp.BfsRun(g)
    for pol in POLICIES:
        announce(f"BFS level log {host.name} policy={pol}")
        st, dirs, nf, mf = r.run_logged(root, pol)
        assert st.levels == nlev == len(dirs)
        assert np.array_equal(nf, np.bincount(want[want >= 0], minlength=nlev))
        assert np.array_equal(mf, np.bincount(want[want >= 0], weights=deg[want >= 0], minlength=nlev).astype(np.int64))
        if pol != pp.PP_SWITCH:
            assert np.all(dirs == pol)
        assert set(np.unique(dirs)) <= {pp.PP_PUSH, pp.PP_PULL}
        m = min(nlev, 64)
        assert list(dirs[:m]) == [st.dir[i] for i in range(m)]
        assert list(nf[:m]) == [st.frontier[i] for i in range(m)]
        assert np.array_equal(r.level.cpu().numpy(), want)


# ----------------------------------------------------------------- deep graphs
# Small top-down frontiers run whole levels inside one one-workgroup launch and
# hand larger ones back to the grid-wide level kernels.  Levels, parents, the
# statistics and the per-level log must not depend on it: each case is run with
# the default caps, with the launch off (0, 0), with tiny caps (64 vertices,
# 256 out-edges) that force hand-overs in both directions and frontiers that
# outgrow the LDS sets part-way through a level, and with the largest sets.
MULTI_CAPS = [(256, 1024), (0, 0), (64, 256), (6144, 32768)]


def _directed(n, m, seed):
    host = H.random_graph(n, m, seed, symmetric=False, connected=True)
    host.ensure_transpose()
    return host


def _run_caps(host, root, policy, caps, relabel=True):
    from paper_2010_16012_amd import _lib
    _lib.pp_set_bfs_multi(*caps)
    try:
        g = pp.Graph(host, relabel=relabel)
    finally:
        _lib.pp_set_bfs_multi(*MULTI_CAPS[0])
    r = pp.BfsRun(g)
    st, dirs, nf, mf = r.run_logged(root, policy)
    torch.cuda.synchronize()
    out = (r.level.cpu().numpy(), r.parent.cpu().numpy(), st, dirs, nf, mf)
    g.close()
    return out


@pytest.mark.parametrize("maker", [lambda: H.path(5000), lambda: H.full_grid(200, 200),
                                   lambda: gg.grid(256, 256, 0.05, seed=3), lambda: gg.workload("rmat14"),
                                   lambda: _directed(3000, 9000, 4)],
                         ids=["path5000", "grid200", "grid256_holes", "rmat14", "directed3000"])
def test_multi_level_launch_matches_level_kernels(maker):
    host = maker()
    for root in (0, host.n // 3):
        want, _, nlev = oracle.bfs(host.off, host.idx, root)
        deg = np.diff(host.off)
        for pol, name in ((pp.PP_PUSH, "push"), (pp.PP_SWITCH, "switch")):
            ref = None
            for caps in MULTI_CAPS:
                announce(f"BFS multi {host.name} root={root} {name} caps={caps}")
                lv, par, st, dirs, nf, mf = _run_caps(host, root, pol, caps)
                assert np.array_equal(lv, want), f"{name} caps {caps}: levels differ"
                assert H.bfs_violations_fast(host, root, lv, par) == []
                assert st.levels == nlev == len(dirs)
                assert st.reached == int((want >= 0).sum())
                assert st.edges_reached == int(deg[want >= 0].sum())
                assert np.array_equal(nf, np.bincount(want[want >= 0], minlength=nlev))
                log = (list(dirs), list(nf), list(mf))
                if ref is None:
                    ref = log
                else:  # the switch rule sees the same statistics either way
                    assert log == ref, f"{name} caps {caps}: level log differs"


def test_multi_level_launch_budget_and_retake():
    # 40,000 levels: more than one launch takes (32,768), so the level kernels
    # run a few levels in between and the next batch's launch takes over again
    host = H.path(40000)
    want, _, nlev = oracle.bfs(host.off, host.idx, 0)
    for relabel in (True, False):
        announce(f"BFS multi path40000 relabel={relabel}")
        lv, par, st, dirs, nf, mf = _run_caps(host, 0, pp.PP_PUSH, MULTI_CAPS[0], relabel=relabel)
        assert np.array_equal(lv, want)
        assert H.bfs_violations_fast(host, 0, lv, par) == []
        assert st.levels == nlev == 40000
        assert np.all(dirs == pp.PP_PUSH) and np.all(nf == 1)


def _core_and_path():
    """A connected random core (depth ~10) and, as a component of its own, a
    60-vertex path (depth up to 59)."""
    core = H.random_graph(3000, 9000, 31, symmetric=True, connected=True)
    src = [np.repeat(np.arange(core.n), np.diff(core.off)), 3000 + np.arange(59)]
    dst = [core.idx, 3001 + np.arange(59)]
    host = gg.from_edges(3060, np.concatenate(src), np.concatenate(dst), True, "core_and_path")
    return host


@pytest.mark.parametrize("pol,name", list(zip(POLICIES, POL_IDS)), ids=POL_IDS)
def test_run_many_matches_run(pol, name):
    # Many roots with one host wait: each root's statistics are those of a
    # run on its own, and level/parent hold the last root's run.  The first
    # call runs its first root alone to size the batches; the path roots are
    # deeper than that batch and run again on their own (also as the last
    # root).
    host = _core_and_path()
    g = pp.Graph(host)
    core = [5, 900, 2999, 17]
    for roots in (core + [3000, 3030], core + [3059], [3059, 3000] + core, core):
        announce(f"BFS run_many {name} roots={roots}")
        r = pp.BfsRun(g)
        many = r.run_many(roots, pol)
        torch.cuda.synchronize()
        lv, par = r.level.cpu().numpy(), r.parent.cpu().numpy()
        want, _, nlev = oracle.bfs(host.off, host.idx, roots[-1])
        assert np.array_equal(lv, want)
        assert H.bfs_violations(host, roots[-1], lv, par) == []
        for root, st in zip(roots, many):
            one = pp.BfsRun(g).run(root, pol)
            _, _, nl = oracle.bfs(host.off, host.idx, root)
            assert st.levels == one.levels == nl
            assert st.reached == one.reached and st.edges_reached == one.edges_reached
            assert list(st.dir[:st.levels]) == list(one.dir[:one.levels])
            assert list(st.frontier[:st.levels]) == list(one.frontier[:one.levels])
    assert pp.BfsRun(g).run_many([], pol) == []
    with pytest.raises(pp.PPError):
        pp.BfsRun(g).run_many([0, host.n], pol)


def _star_of_stars(centres, leaves):
    """A hub joined to `centres` centres with `leaves` leaves each: rows of
    centres (hub), leaves + 1 (centre) and 1 (leaf) edges."""
    c = np.arange(1, centres + 1)
    first_leaf = centres + 1
    n = first_leaf + centres * leaves
    src = np.concatenate([np.zeros(centres, dtype=np.int64), np.repeat(c, leaves)])
    dst = np.concatenate([c, np.arange(first_leaf, n)])
    return gg.from_edges(n, src, dst, True, f"star_of_stars_{centres}x{leaves}")


@pytest.mark.parametrize("centres", [300, 200], ids=["hub300", "hub200"])
def test_small_levels_cut_rows_into_short_chunks(centres):
    # Top-down levels with fewer frontier out-edges than nnz/32 cut every row
    # longer than 32 edges into chunk items, when rows longer than 256 edges
    # exist (the chunk kernel then follows every level).  From a leaf, level 1
    # (its centre's 101-edge row) and level 2 (the hub's row) are such levels,
    # level 3 (the other centres) is not.  With 200 centres no row passes 256
    # edges, there is no chunk kernel and rows stay whole.  The one-workgroup
    # launch is off in one pass, so the level kernel takes the small levels.
    host = _star_of_stars(centres, 100)
    leaf = centres + 1 + 5 * 100 + 7
    want, _, nlev = oracle.bfs(host.off, host.idx, leaf)
    assert nlev == 5
    for pol, name in ((pp.PP_PUSH, "push"), (pp.PP_SWITCH, "switch")):
        for caps in ((0, 0), MULTI_CAPS[0]):
            announce(f"BFS {host.name} root={leaf} {name} caps={caps}")
            lv, par, st, dirs, nf, mf = _run_caps(host, leaf, pol, caps)
            assert np.array_equal(lv, want), f"{name} caps {caps}: levels differ"
            assert H.bfs_violations(host, leaf, lv, par) == []
            assert st.levels == nlev
            assert st.reached == host.n
