"""Shared test helpers: small named graphs, dense matrices, a BFS validator.

Nothing here computes PageRank or BFS the way the oracle or the library does;
the dense forms are built directly from edge lists with numpy.
"""
from __future__ import annotations

import numpy as np

import graphgen as gg


def star(n):
    return gg.from_edges(n, np.zeros(n - 1), np.arange(1, n), True, f"star{n}")


def cycle(n):
    a = np.arange(n)
    return gg.from_edges(n, a, (a + 1) % n, True, f"cycle{n}")


def path(n):
    a = np.arange(n - 1)
    return gg.from_edges(n, a, a + 1, True, f"path{n}")


def complete(n):
    s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return gg.from_edges(n, s.ravel(), t.ravel(), True, f"K{n}")


def complete_bipartite(a, b):
    s, t = np.meshgrid(np.arange(a), a + np.arange(b), indexing="ij")
    return gg.from_edges(a + b, s.ravel(), t.ravel(), True, f"K{a},{b}")


def full_grid(rows, cols):
    return gg.grid(rows, cols, 0.0, seed=0)


def random_graph(n, m, seed, symmetric=True, connected=False):
    """Seeded random graph from `m` uniform pairs; `connected` adds a ring."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, m)
    t = rng.integers(0, n, m)
    if connected:
        s = np.concatenate([s, np.arange(n)])
        t = np.concatenate([t, (np.arange(n) + 1) % n])
    return gg.from_edges(n, s, t, symmetric, f"rand{n}_{m}_{seed}")


def dense_adjacency(g):
    """A[v, u] = 1 iff edge v -> u."""
    A = np.zeros((g.n, g.n))
    for v in range(g.n):
        A[v, g.idx[g.off[v]:g.off[v + 1]]] = 1.0
    return A


def dense_transition(g, weights=None):
    """P[u, v] = w(v->u)/s(v): column v spreads the mass of v over its out-edges."""
    W = np.zeros((g.n, g.n))
    for v in range(g.n):
        for e in range(g.off[v], g.off[v + 1]):
            W[g.idx[e], v] = 1.0 if weights is None else float(weights[e])
    s = W.sum(axis=0)
    P = np.divide(W, s, out=np.zeros_like(W), where=s > 0)
    return P


def bfs_violations(g, root, level, parent):
    """List of violated BFS invariants (empty when level/parent form a valid
    BFS tree of `g` from `root`).  Uses out-edges for tree and level checks."""
    n = g.n
    level = np.asarray(level)
    parent = np.asarray(parent)
    errs = []
    if level[root] != 0:
        errs.append("level[root] != 0")
    if parent[root] != root:
        errs.append("parent[root] != root")
    reached = level >= 0
    if np.any(level < -1):
        errs.append("level below -1")
    if np.any(parent[~reached] != -1):
        errs.append("unreached vertex with a parent")
    src = np.repeat(np.arange(n), np.diff(g.off))
    dst = g.idx.astype(np.int64)
    # every edge from a reached vertex reaches its target within one level
    lr = level[src]
    lt = level[dst]
    bad = (lr >= 0) & ((lt < 0) | (lt > lr + 1))
    if np.any(bad):
        errs.append(f"{int(bad.sum())} edges leave the reached set or skip a level")
    # tree edges
    v = np.nonzero(reached & (np.arange(n) != root))[0]
    p = parent[v]
    if np.any((p < 0) | (p >= n)):
        errs.append("parent out of range")
        return errs
    if np.any(level[p] != level[v] - 1):
        errs.append("parent not one level up")
    # (p, v) must be an edge: binary search p's sorted row
    ok = np.ones(len(v), dtype=bool)
    for i in range(len(v)):
        row = g.idx[g.off[p[i]]:g.off[p[i] + 1]]
        j = np.searchsorted(row, v[i])
        ok[i] = j < len(row) and row[j] == v[i]
        if not ok[i]:
            break
    if not ok.all():
        errs.append("parent is not an in-neighbour")
    return errs


def bfs_violations_fast(g, root, level, parent):
    """Vectorised variant of ``bfs_violations`` for large graphs."""
    n = g.n
    level = np.asarray(level).astype(np.int64)
    parent = np.asarray(parent).astype(np.int64)
    errs = []
    if level[root] != 0 or parent[root] != root:
        errs.append("root not level 0 / own parent")
    reached = level >= 0
    if np.any(level < -1):
        errs.append("level below -1")
    if np.any(parent[~reached] != -1):
        errs.append("unreached vertex with a parent")
    deg = np.diff(g.off)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    dst = g.idx.astype(np.int64)
    lr = level[src]
    lt = level[dst]
    bad = (lr >= 0) & ((lt < 0) | (lt > lr + 1))
    if np.any(bad):
        errs.append(f"{int(bad.sum())} edges leave the reached set or skip a level")
    del src, lr, lt, bad
    v = np.nonzero(reached & (np.arange(n) != root))[0]
    p = parent[v]
    if np.any((p < 0) | (p >= n)):
        errs.append("parent out of range")
        return errs
    if np.any(level[p] != level[v] - 1):
        errs.append("parent not one level up")
    # edge test via sorted keys p*n+v among all edge keys
    keys = np.repeat(np.arange(n, dtype=np.int64), deg) * n + dst
    want = p * n + v
    pos = np.searchsorted(keys, want)
    pos = np.minimum(pos, len(keys) - 1)
    if np.any(keys[pos] != want):
        errs.append("parent is not an in-neighbour")
    return errs


class BfsValidator:
    """``bfs_violations_fast`` with the per-edge arrays of one graph built once
    (for many runs on a large graph).  Rows must be sorted ascending, as
    ``graphgen`` writes them, so the edge keys v*n+u are sorted."""

    def __init__(self, g):
        self.g = g
        n = g.n
        deg = np.diff(g.off)
        self.src = np.repeat(np.arange(n, dtype=np.int32), deg)
        self.dst = np.ascontiguousarray(g.idx, dtype=np.int32)
        self.keys = self.src.astype(np.int64) * n + self.dst
        if len(self.keys) > 1 and not np.all(self.keys[1:] > self.keys[:-1]):
            raise ValueError("rows must be strictly ascending")

    def __call__(self, root, level, parent):
        n = self.g.n
        level = np.asarray(level).astype(np.int64)
        parent = np.asarray(parent).astype(np.int64)
        errs = []
        if level[root] != 0 or parent[root] != root:
            errs.append("root not level 0 / own parent")
        reached = level >= 0
        if np.any(level < -1):
            errs.append("level below -1")
        if np.any(parent[~reached] != -1):
            errs.append("unreached vertex with a parent")
        lr = level[self.src]
        lt = level[self.dst]
        bad = (lr >= 0) & ((lt < 0) | (lt > lr + 1))
        if np.any(bad):
            errs.append(f"{int(bad.sum())} edges leave the reached set or skip a level")
        del lr, lt, bad
        v = np.nonzero(reached & (np.arange(n) != root))[0]
        p = parent[v]
        if np.any((p < 0) | (p >= n)):
            errs.append("parent out of range")
            return errs
        if np.any(level[p] != level[v] - 1):
            errs.append("parent not one level up")
        want = np.sort(p * n + v)
        pos = np.minimum(np.searchsorted(self.keys, want), len(self.keys) - 1)
        if len(want) and np.any(self.keys[pos] != want):
            errs.append("parent is not an in-neighbour")
        return errs
