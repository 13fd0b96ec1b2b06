"""Seeded synthetic graph inputs (R-MAT, Erdos-Renyi, 2D grid) in adjacency-array form.

This module only produces *inputs*: the adjacency array plus offsets of Sec. 2.2
of the paper (a CSR of out-neighbours), its transpose (in-neighbours), and seeded
vectors (edge weights, Gaussian coefficients, vertex picks).  It holds none of
the arithmetic of PageRank or BFS.  Both the HIP library and the CPU oracle take
what it returns; neither is imported here.

Randomness is one counter-based generator (SplitMix64's output function at
state = key + (ctr+1)*0x9E3779B97F4A7C15); see ``graphgen.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libgraphgen.so`` next to its source with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, u64, i32, f32, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_float, ctypes.c_double
    lib.gg_rand.argtypes = [u64, u64, u64]
    lib.gg_rand.restype = u64
    lib.gg_rmat_edges.argtypes = [i32, i64, f64, f64, f64, u64, P, P]
    lib.gg_rmat_edges.restype = i32
    lib.gg_er_edges.argtypes = [i64, i64, u64, P, P]
    lib.gg_er_edges.restype = i32
    lib.gg_build_adjacency.argtypes = [i64, i64, P, P, i32, P, P]
    lib.gg_build_adjacency.restype = i64
    lib.gg_grid.argtypes = [i64, i64, i64, u64, P, P]
    lib.gg_grid.restype = i64
    lib.gg_uniform_f32.argtypes = [u64, u64, i64, f32, f32, P]
    lib.gg_uniform_f32.restype = i32
    lib.gg_normal_f32.argtypes = [u64, u64, i64, P]
    lib.gg_normal_f32.restype = i32
    lib.gg_pick_vertices.argtypes = [u64, u64, i64, P, i64, i64, P]
    lib.gg_pick_vertices.restype = i32
    lib.gg_uniform_int.argtypes = [u64, u64, i64, i64, i64, P]
    lib.gg_uniform_int.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class HostGraph:
    """A directed graph as out-adjacency (CSR) and in-adjacency (CSC) arrays.

    ``off``/``idx``: row v lists the out-neighbours of v, ascending.
    ``in_off``/``in_idx``: row u lists the in-neighbours of u, ascending; for a
    symmetric graph these are the same arrays.  ``in_to_out`` maps each CSC slot
    to the CSR slot of the same directed edge (needed for per-edge weights).
    """

    n: int
    off: np.ndarray  # int64[n+1]
    idx: np.ndarray  # int32[nnz]
    symmetric: bool
    name: str = ""
    in_off: Optional[np.ndarray] = None
    in_idx: Optional[np.ndarray] = None
    in_to_out: Optional[np.ndarray] = None
    weights: Optional[np.ndarray] = None  # float32[nnz], CSR slot order
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.off[-1])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.off)

    def ensure_transpose(self) -> "HostGraph":
        """Fill in_off/in_idx/in_to_out (a stable counting sort by destination)."""
        if self.in_off is not None and self.in_to_out is not None:
            return self
        n, nnz = self.n, self.nnz
        src = np.repeat(np.arange(n, dtype=np.int32), np.diff(self.off))
        order = np.argsort(self.idx, kind="stable")
        in_idx = src[order].astype(np.int32)
        in_off = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(self.idx, minlength=n), out=in_off[1:])
        self.in_off, self.in_idx = in_off, in_idx
        self.in_to_out = order.astype(np.int32)
        assert in_off[-1] == nnz
        return self


def _adjacency_from_edges(n: int, src: np.ndarray, dst: np.ndarray, sym: bool):
    lib = _load()
    cap = 2 * len(src) if sym else len(src)
    work = np.empty(max(cap, 1), dtype=np.int32)
    off = np.empty(n + 1, dtype=np.int64)
    nnz = lib.gg_build_adjacency(n, len(src), _ptr(src), _ptr(dst), 1 if sym else 0, _ptr(off), _ptr(work))
    if nnz < 0:
        raise ValueError(f"gg_build_adjacency failed ({nnz})")
    idx = work[:nnz].copy()
    del work
    return off, idx


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, symmetric: bool = True) -> HostGraph:
    """R-MAT graph: edge_factor * 2^scale draws, self-loops and duplicates removed,
    symmetrised when ``symmetric``."""
    lib = _load()
    n = 1 << scale
    m = edge_factor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = lib.gg_rmat_edges(scale, m, a, b, c, seed, _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError(f"gg_rmat_edges failed ({rc})")
    off, idx = _adjacency_from_edges(n, src, dst, symmetric)
    g = HostGraph(n=n, off=off, idx=idx, symmetric=symmetric,
                  name=f"rmat{scale}_ef{edge_factor}_s{seed}",
                  meta=dict(kind="rmat", scale=scale, edge_factor=edge_factor, a=a, b=b, c=c, seed=seed))
    if symmetric:
        g.in_off, g.in_idx = off, idx
    return g


def erdos_renyi(n: int, num_draws: int, seed: int = 1) -> HostGraph:
    """Symmetric Erdos-Renyi graph from ``num_draws`` uniform vertex pairs."""
    lib = _load()
    src = np.empty(num_draws, dtype=np.int32)
    dst = np.empty(num_draws, dtype=np.int32)
    rc = lib.gg_er_edges(n, num_draws, seed, _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError(f"gg_er_edges failed ({rc})")
    off, idx = _adjacency_from_edges(n, src, dst, True)
    g = HostGraph(n=n, off=off, idx=idx, symmetric=True, name=f"er{n}_m{num_draws}_s{seed}",
                  meta=dict(kind="er", draws=num_draws, seed=seed))
    g.in_off, g.in_idx = off, idx
    return g


def grid(rows: int, cols: int, remove_frac: float = 0.05, seed: int = 1) -> HostGraph:
    """4-neighbour grid, row-major ids, round(remove_frac * #edges) edges removed."""
    lib = _load()
    n = rows * cols
    ne = rows * (cols - 1) + (rows - 1) * cols
    remove = int(round(remove_frac * ne))
    off = np.empty(n + 1, dtype=np.int64)
    idx = np.empty(max(4 * n, 1), dtype=np.int32)
    nnz = lib.gg_grid(rows, cols, remove, seed, _ptr(off), _ptr(idx))
    if nnz < 0:
        raise ValueError(f"gg_grid failed ({nnz})")
    idx = idx[:nnz].copy()
    g = HostGraph(n=n, off=off, idx=idx, symmetric=True, name=f"grid{rows}x{cols}_r{remove}_s{seed}",
                  meta=dict(kind="grid", rows=rows, cols=cols, removed=remove, seed=seed))
    g.in_off, g.in_idx = off, idx
    return g


def from_edges(n: int, src, dst, symmetric: bool = True, name: str = "edges") -> HostGraph:
    """Adjacency arrays of an explicit edge list (self-loops and duplicates dropped)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    off, idx = _adjacency_from_edges(n, src, dst, symmetric)
    g = HostGraph(n=n, off=off, idx=idx, symmetric=symmetric, name=name, meta=dict(kind="explicit"))
    if symmetric:
        g.in_off, g.in_idx = off, idx
    return g


def uniform(count: int, lo: float, hi: float, seed: int, stream: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.float32)
    rc = _load().gg_uniform_f32(seed, stream, count, lo, hi, _ptr(out))
    if rc != 0:
        raise ValueError("gg_uniform_f32 failed")
    return out


def normal(count: int, seed: int, stream: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.float32)
    rc = _load().gg_normal_f32(seed, stream, count, _ptr(out))
    if rc != 0:
        raise ValueError("gg_normal_f32 failed")
    return out


def pick_vertices(g: HostGraph, count: int, seed: int, stream: int = 0, min_deg: int = 1) -> np.ndarray:
    """``count`` distinct vertices with out-degree >= min_deg, seeded."""
    out = np.empty(max(count, 1), dtype=np.int32)
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    rc = _load().gg_pick_vertices(seed, stream, g.n, _ptr(off), min_deg, count, _ptr(out))
    if rc != 0:
        raise ValueError(f"gg_pick_vertices failed ({rc})")
    return out[:count].copy()


def uniform_int(count: int, lo: int, hi: int, seed: int, stream: int = 0) -> np.ndarray:
    out = np.empty(max(count, 1), dtype=np.int64)
    rc = _load().gg_uniform_int(seed, stream, count, lo, hi, _ptr(out))
    if rc != 0:
        raise ValueError("gg_uniform_int failed")
    return out[:count].copy()


def rand_u64(seed: int, stream: int, ctr: int) -> int:
    return int(_load().gg_rand(seed, stream, ctr))


def with_weights(g: HostGraph, seed: int, lo: float = 0.1, hi: float = 1.0) -> HostGraph:
    """Attach per-directed-slot weights ~ U(lo, hi) in CSR slot order."""
    g.weights = uniform(g.nnz, lo, hi, seed, stream=7)
    g.ensure_transpose()
    return g


def rmat_batch(num_graphs: int = 512, scale_lo: int = 8, scale_hi: int = 14, edge_factor: int = 16,
               seed: int = 1) -> List[HostGraph]:
    """Independent symmetric R-MAT graphs with scales uniform in [scale_lo, scale_hi]."""
    scales = uniform_int(num_graphs, scale_lo, scale_hi, seed, stream=11)
    seeds = [rand_u64(seed, 12, i) & 0x7FFFFFFFFFFFFFFF for i in range(num_graphs)]
    return [rmat(int(s), edge_factor, seed=int(sd)) for s, sd in zip(scales, seeds)]


# Named workloads -------------------------------------------------------------

def workload(name: str) -> HostGraph:
    """The seeded graphs used by tests and the benchmark, by name."""
    if name == "rmat14":
        return rmat(14, 16, seed=1)
    if name == "rmat22":
        return rmat(22, 16, seed=1)
    if name == "rmat20":
        return rmat(20, 16, seed=1)
    if name == "rmat10":
        return rmat(10, 16, seed=1)
    if name == "er22":
        return erdos_renyi(1 << 22, 8 << 22, seed=1)
    if name == "grid4096":
        return grid(4096, 4096, 0.05, seed=1)
    raise KeyError(name)
