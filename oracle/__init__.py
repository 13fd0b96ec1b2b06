"""CPU FP64 oracle for the push/pull sweeps -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it: the C source (``oracle.c``) derives degrees and the
in-adjacency itself from the out-adjacency array it is given.

Every function takes a graph as the adjacency array of Sec. 2.2 of the paper
(``off`` int64[n+1], ``idx`` int32[nnz]; row v = targets of edges leaving v).
The definitions followed, and the readings taken where the paper is silent,
are stated at the top of ``oracle.c``:

* ``pagerank`` / ``pagerank_push`` -- the PageRank equation of Sec. 3.1 as a
  Jacobi iteration in its pulling and pushing forms (Sec. 4.1);
* ``pagerank_threads`` -- the pulling form with its rows split over threads
  (bit-identical; times the oracle on all host cores);
* ``pagerank_step_at`` -- one update at chosen vertices from a given iterate;
* ``ppr`` / ``ppr_adjoint`` / ``ppr_adjoint_unrolled`` -- personalised (and
  weighted) PageRank and its adjoint with respect to edge weights, at the
  fixed point or exactly for T steps (not in the paper);
* ``bfs`` -- FIFO-queue BFS (Sec. 3.3; Sec. 4.3 with ready counters of one);
* ``bfs_replay`` -- what each top-down / bottom-up step examines (Sec. 4.3);
* ``triangles`` -- per-vertex triangle counts (Sec. 3.2);
* ``bc`` -- betweenness centrality over a set of sources (Sec. 3.5, Brandes).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain -O2; OpenMP only for
    ``pagerank_threads``, every other function is single-threaded)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-fopenmp", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sigs = {
        "orc_pagerank": [i64, P, P, f64, i32, P, P],
        "orc_pagerank_push": [i64, P, P, f64, i32, P, P],
        "orc_pagerank_threads": [i64, P, P, f64, i32, P, P, P],
        "orc_pagerank_step_at": [i64, P, P, f64, P, i64, P, P],
        "orc_ppr": [i64, P, P, P, i64, P, f64, i32, f64, P, P],
        "orc_ppr_adjoint": [i64, P, P, P, i64, P, P, f64, i32, f64, P, P, P],
        "orc_bfs": [i64, P, P, i64, P, P],
        "orc_bfs_replay": [i64, P, P, i64, i32, P, P, P, P],
        "orc_triangles": [i64, P, P, P],
        "orc_bc": [i64, P, P, P, i64, P],
        "orc_ppr_adjoint_unrolled": [i64, P, P, P, i64, P, f64, i32, P, P, P],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = i32
    _lib = lib
    return lib


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _graph(off, idx):
    off = _arr(off, np.int64)
    idx = _arr(idx, np.int32)
    if idx.size == 0:
        idx = np.zeros(1, dtype=np.int32)
    return len(off) - 1, off, idx


def _check(rc, name):
    if rc < 0:
        raise ValueError(f"{name} failed with code {rc}")
    return rc


def pagerank(off, idx, f=0.85, T=20, x0=None) -> np.ndarray:
    n, off, idx = _graph(off, idx)
    out = np.empty(n, dtype=np.float64)
    x0 = None if x0 is None else _arr(x0, np.float64)
    _check(_load().orc_pagerank(n, _p(off), _p(idx), f, T, _p(x0), _p(out)), "orc_pagerank")
    return out


def pagerank_threads(off, idx, f=0.85, T=20, x0=None):
    """``pagerank`` with its row loop split over OpenMP threads (bit-identical
    result).  Returns (x, threads used)."""
    n, off, idx = _graph(off, idx)
    out = np.empty(n, dtype=np.float64)
    x0 = None if x0 is None else _arr(x0, np.float64)
    th = np.zeros(1, dtype=np.int32)
    _check(_load().orc_pagerank_threads(n, _p(off), _p(idx), f, T, _p(x0), _p(out), _p(th)),
           "orc_pagerank_threads")
    return out, int(th[0])


def pagerank_push(off, idx, f=0.85, T=20, x0=None) -> np.ndarray:
    n, off, idx = _graph(off, idx)
    out = np.empty(n, dtype=np.float64)
    x0 = None if x0 is None else _arr(x0, np.float64)
    _check(_load().orc_pagerank_push(n, _p(off), _p(idx), f, T, _p(x0), _p(out)), "orc_pagerank_push")
    return out


def pagerank_step_at(off, idx, x_prev, verts, f=0.85) -> np.ndarray:
    n, off, idx = _graph(off, idx)
    x_prev = _arr(x_prev, np.float32)
    verts = _arr(verts, np.int32)
    out = np.empty(max(len(verts), 1), dtype=np.float64)
    _check(_load().orc_pagerank_step_at(n, _p(off), _p(idx), f, _p(x_prev), len(verts), _p(verts), _p(out)),
           "orc_pagerank_step_at")
    return out[: len(verts)]


def ppr(off, idx, sources, f=0.85, T=30, tol=0.0, weights=None):
    """Returns (X n*k, iterations per column)."""
    n, off, idx = _graph(off, idx)
    sources = _arr(sources, np.int32)
    k = len(sources)
    X = np.empty((n, max(k, 1)), dtype=np.float64)
    iters = np.zeros(max(k, 1), dtype=np.int32)
    w = None if weights is None else _arr(weights, np.float32)
    _check(_load().orc_ppr(n, _p(off), _p(idx), _p(w), k, _p(sources), f, T, tol, _p(X), _p(iters)), "orc_ppr")
    return X[:, :k], iters[:k]


def ppr_adjoint(off, idx, X, G, f=0.85, T=2000, tol=0.0, weights=None):
    """Returns (Lambda n*k, grad[nnz] in CSR slot order, iterations)."""
    n, off, idx = _graph(off, idx)
    X = _arr(X, np.float64)
    G = _arr(G, np.float64)
    k = X.shape[1]
    lam = np.empty_like(X)
    nnz = int(off[-1])
    grad = np.empty(max(nnz, 1), dtype=np.float64)
    it = np.zeros(1, dtype=np.int32)
    w = None if weights is None else _arr(weights, np.float32)
    _check(_load().orc_ppr_adjoint(n, _p(off), _p(idx), _p(w), k, _p(X), _p(G), f, T, tol, _p(lam), _p(grad), _p(it)),
           "orc_ppr_adjoint")
    return lam, grad[:nnz], int(it[0])


def ppr_adjoint_unrolled(off, idx, sources, G, f=0.85, T=30, weights=None):
    """Exact gradient of L(X_T) for T PPR steps from X_0 = e_s: returns
    (dL/dX_0 n*k, grad[nnz] in CSR slot order)."""
    n, off, idx = _graph(off, idx)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    G = _arr(G, np.float64)
    k = G.shape[1]
    lam = np.empty_like(G)
    nnz = int(off[-1])
    grad = np.empty(max(nnz, 1), dtype=np.float64)
    w = None if weights is None else _arr(weights, np.float32)
    _check(_load().orc_ppr_adjoint_unrolled(n, _p(off), _p(idx), _p(w), k, _p(src), f, T, _p(G), _p(lam), _p(grad)),
           "orc_ppr_adjoint_unrolled")
    return lam, grad[:nnz]


def bfs(off, idx, root):
    """Returns (level int32[n], parent int32[n], number of levels)."""
    n, off, idx = _graph(off, idx)
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    nlev = _check(_load().orc_bfs(n, _p(off), _p(idx), root, _p(level), _p(parent)), "orc_bfs")
    return level, parent, nlev


def bfs_replay(off, idx, root, dirs):
    """Per-step (frontier size, edges examined, vertices discovered) for a
    given direction schedule (0 = top-down, 1 = bottom-up)."""
    n, off, idx = _graph(off, idx)
    dirs = _arr(dirs, np.int8)
    s = len(dirs)
    fr = np.zeros(max(s, 1), dtype=np.int64)
    ex = np.zeros(max(s, 1), dtype=np.int64)
    di = np.zeros(max(s, 1), dtype=np.int64)
    steps = _check(_load().orc_bfs_replay(n, _p(off), _p(idx), root, s, _p(dirs), _p(fr), _p(ex), _p(di)),
                   "orc_bfs_replay")
    return fr[:steps], ex[:steps], di[:steps]


def triangles(off, idx) -> np.ndarray:
    n, off, idx = _graph(off, idx)
    tc = np.empty(n, dtype=np.int64)
    _check(_load().orc_triangles(n, _p(off), _p(idx), _p(tc)), "orc_triangles")
    return tc


def bc(off, idx, sources) -> np.ndarray:
    """Betweenness centrality summed over ``sources`` (ordered pairs)."""
    n, off, idx = _graph(off, idx)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    out = np.empty(n, dtype=np.float64)
    _check(_load().orc_bc(n, _p(off), _p(idx), _p(src), len(src), _p(out)), "orc_bc")
    return out
