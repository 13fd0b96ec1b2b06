"""Push/pull graph sweeps on MI355X (gfx950): PageRank and BFS steps in their
pushing and pulling forms (Besta et al., "To Push or To Pull", HPDC'17).

The compute lives in ``libpp.so`` (hand-written HIP kernels behind the C ABI of
``include/pp.h``).  ``_lib`` binds every entry point under its C name; this
module adds thin conveniences that own the device tensors a call needs.
PyTorch provides device memory and streams only.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import (PP_PULL, PP_PUSH, PP_SWITCH, PPError, BfsStats)  # noqa: F401
from ._lib import *  # noqa: F401,F403  (the C names)

__all__ = ["Graph", "BfsRun", "PPError", "PP_PUSH", "PP_PULL", "PP_SWITCH", "pagerank", "pagerank_into", "bfs",
           "ppr", "ppr_adjoint", "ppr_adjoint_unrolled", "PPRFunction", "MultiGraph", "triangles", "betweenness"]


class Graph:
    """A graph registered with libpp: device adjacency arrays, the workspace of
    derived data, and the library handle.

    ``host`` is a ``graphgen.HostGraph``-like object with ``n``, ``off`` and
    ``idx`` (CSR = out-adjacency), optional ``in_off``/``in_idx`` (CSC =
    in-adjacency; the CSR is reused when the graph is symmetric), and optional
    ``weights`` (per CSR slot) with ``in_to_out`` (CSR slot of each CSC slot).
    """

    def __init__(self, host, device="cuda", weighted=None, relabel=True, stream=None):
        n = int(host.n)
        nnz = int(host.off[-1])
        if nnz > 2**31 - 1:
            raise ValueError("nnz must fit in int32")
        self.n, self.nnz = n, nnz
        dev = torch.device(device)

        def up(a, dt):
            return torch.as_tensor(a).to(dtype=dt).to(dev).contiguous()

        self.csr_off = up(host.off, torch.int32)
        self.csr_idx = up(host.idx, torch.int32) if nnz else torch.zeros(1, dtype=torch.int32, device=dev)
        in_off = getattr(host, "in_off", None)
        if in_off is None or in_off is host.off:
            if in_off is None and not getattr(host, "symmetric", False):
                raise ValueError("a directed graph needs in_off/in_idx")
            self.csc_off, self.csc_idx = self.csr_off, self.csr_idx  # symmetric: CSC = CSR
        else:
            self.csc_off = up(host.in_off, torch.int32)
            self.csc_idx = up(host.in_idx, torch.int32) if nnz else self.csr_idx
        if weighted is None:
            weighted = getattr(host, "weights", None) is not None
        self.weighted = bool(weighted)
        flags = (_lib.PP_GRAPH_WEIGHTED if self.weighted else 0) | (_lib.PP_GRAPH_RELABEL if relabel else 0)
        self.relabel = bool(relabel)
        if self.weighted:
            self.csr_w = up(host.weights, torch.float32)
            self.csc_to_csr = up(host.in_to_out, torch.int32)
        else:
            self.csr_w = self.csc_to_csr = None
        ws_bytes = _lib.pp_graph_workspace_bytes(n, nnz, flags)
        if ws_bytes == 0:
            raise ValueError("graph size out of range")
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        self.handle = _lib.pp_graph_create(n, nnz, self.csr_off, self.csr_idx, self.csc_off, self.csc_idx,
                                           self.csr_w, self.csc_to_csr, flags, self.ws, stream)
        self.device = dev

    def relabel_map(self):
        """perm[i] = caller id of internal vertex i (graphs registered with relabel)."""
        perm = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _lib.pp_graph_relabel_map(self.handle, perm)
        return perm

    def slices(self):
        """(R, width, S, tiles) of the tiled pull (R = 0: plain pull only)."""
        return _lib.pp_graph_slices(self.handle)

    def push_bins(self):
        """(bins, first binned target, sweep workgroups, summing units); bins = 0
        when the push sweep uses global atomics."""
        return _lib.pp_graph_push_bins(self.handle)

    def bins(self, direction=PP_PULL):
        return _lib.pp_graph_bins(self.handle, direction)

    def set_weights(self, w, stream=None):
        """Replace the edge weights (float[nnz], CSR slot order, same structure)
        of a weighted graph in place.  The values are copied into a buffer the
        graph owns, so later changes to ``w`` do not reach it."""
        if not self.weighted:
            raise ValueError("graph was registered without weights")
        w = torch.as_tensor(w, device=self.device).reshape(-1)
        if w.numel() != self.nnz:
            raise ValueError(f"expected {self.nnz} weights, got {w.numel()}")
        if self.nnz:
            self.csr_w.copy_(w.detach().to(torch.float32))
        _lib.pp_graph_set_weights(self.handle, self.csr_w, stream)

    def close(self):
        if getattr(self, "handle", None) is not None:
            _lib.pp_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pagerank(g: Graph, iters=20, f=0.85, direction=PP_PULL, x0=None, stream=None):
    """``iters`` Jacobi steps of the PageRank equation from x0 (default 1/n)."""
    x = torch.full((g.n,), 1.0 / g.n, dtype=torch.float32, device=g.device) if x0 is None else x0.clone()
    _lib.pp_pr_run(g.handle, direction, iters, f, x, stream)
    return x


def pagerank_into(g: Graph, x, iters=20, f=0.85, direction=PP_PULL, stream=None):
    """In place: x (float32[n] on the device) holds x_0 on entry, x_iters on exit."""
    _lib.pp_pr_run(g.handle, direction, iters, f, x, stream)
    return x


class BfsRun:
    """Device buffers of one BFS: level, parent and the library's state."""

    def __init__(self, g: Graph):
        self.g = g
        self.level = torch.empty(g.n, dtype=torch.int32, device=g.device)
        self.parent = torch.empty(g.n, dtype=torch.int32, device=g.device)
        self.state = torch.empty(_lib.pp_bfs_state_bytes(g.handle), dtype=torch.uint8, device=g.device)

    def run(self, root, policy=PP_SWITCH, alpha=14.0, beta=24.0, stream=None) -> BfsStats:
        return _lib.pp_bfs_run(self.g.handle, root, policy, alpha, beta, self.level, self.parent, self.state, stream)

    def run_many(self, roots, policy=PP_SWITCH, alpha=14.0, beta=24.0, stream=None):
        """``run`` from every root in turn with one host wait (per-root
        stats; level and parent hold the last root's run)."""
        return _lib.pp_bfs_run_many(self.g.handle, roots, policy, alpha, beta, self.level, self.parent, self.state,
                                    stream)

    def run_logged(self, root, policy=PP_SWITCH, alpha=14.0, beta=24.0, stream=None):
        """``run`` with the whole per-level log: returns (stats, dirs, n_f, m_f),
        one entry per expanded frontier (numpy arrays)."""
        import numpy as np
        if getattr(self, "_log", None) is None:
            self._log_cap = self.g.n + 1
            self._log = torch.empty(2 * self._log_cap, dtype=torch.int64, device=self.g.device)
        st = _lib.pp_bfs_run_log(self.g.handle, root, policy, alpha, beta, self.level, self.parent, self.state,
                                 self._log, self._log_cap, stream)
        raw = self._log[:2 * st.levels].cpu().numpy()
        head = raw[0::2]
        dirs = (head & 0xFFFFFFFF).astype(np.int64).astype(np.int32)
        nf = (head >> 32).astype(np.int32)
        return st, dirs, nf, raw[1::2].copy()

    def init(self, root, stream=None):
        _lib.pp_bfs_init(self.g.handle, root, self.level, self.parent, self.state, stream)

    def step(self, cur_level, direction, stream=None):
        fn = _lib.pp_bfs_step_push if direction == PP_PUSH else _lib.pp_bfs_step_pull
        fn(self.g.handle, self.state, self.level, self.parent, cur_level, stream)

    def frontier(self, stream=None) -> int:
        return _lib.pp_bfs_frontier(self.g.handle, self.state, stream)


def bfs(g: Graph, root, policy=PP_SWITCH, alpha=14.0, beta=24.0):
    r = BfsRun(g)
    stats = r.run(root, policy, alpha, beta)
    return r.level, r.parent, stats


def _scratch(g: Graph, k: int, k_tile: int):
    nbytes = _lib.pp_ppr_scratch_bytes(g.handle, k, k_tile)
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=g.device)


def ppr(g: Graph, sources, iters=30, f=0.85, k_tile=32, direction=PP_PULL, tol=0.0, stream=None):
    """Personalised PageRank for every source (caller ids): returns X (n x k,
    column j = PageRank personalised on sources[j]) and the sweeps run."""
    src = torch.as_tensor(sources, dtype=torch.int32, device=g.device).contiguous()
    k = src.numel()
    X = torch.empty((g.n, k), dtype=torch.float32, device=g.device)
    done = _lib.pp_ppr_run(g.handle, direction, k, src, iters, tol, f, k_tile, X, _scratch(g, k, k_tile), stream)
    return X, done


def ppr_adjoint(g: Graph, X, dLdX, iters=2000, f=0.85, k_tile=32, direction=PP_PULL, tol=0.0, stream=None):
    """Adjoint solve and edge-weight gradient at the fixed point X:
    returns (Lambda n x k, grad[nnz] in CSR slot order, sweeps run)."""
    X = X.contiguous()
    dLdX = dLdX.contiguous()
    k = X.shape[1]
    lam = torch.empty_like(X)
    grad = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=g.device)
    done = _lib.pp_ppr_adjoint(g.handle, direction, k, X, dLdX, iters, tol, f, k_tile, lam, grad,
                               _scratch(g, k, k_tile), stream)
    return lam, grad[: g.nnz], done


def ppr_adjoint_unrolled(g: Graph, sources, dLdXT, T=30, f=0.85, k_tile=32, stream=None):
    """Exact gradient of a loss on the T-step PPR iterate: (dL/dX_0, dL/dw)."""
    src = torch.as_tensor(sources, dtype=torch.int32, device=g.device).contiguous()
    k = int(src.numel())
    G = dLdXT.to(device=g.device, dtype=torch.float32).contiguous()
    lam = torch.empty((g.n, k), dtype=torch.float32, device=g.device)
    grad = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=g.device)
    nbytes = _lib.pp_ppr_unrolled_scratch_bytes(g.handle, k, k_tile, T)
    scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=g.device)
    _lib.pp_ppr_adjoint_unrolled(g.handle, k, src, T, f, k_tile, G, lam, grad, scratch, stream)
    return lam, grad[:g.nnz]


class PPRFunction(torch.autograd.Function):
    """X = PPR(w): personalised PageRank at convergence as a function of the
    per-slot edge weights w (CSR slot order of `structure`).  backward() runs
    the library's adjoint: the transposed sweep solves (I - f P^T) Lambda =
    dL/dX and a per-slot kernel forms dL/dw.

    ``structure`` is a HostGraph-like object or a weighted ``Graph``.  A
    HostGraph is registered on the device once per (device, relabel) and kept
    on the object; every later call only replaces the weights in place
    (``Graph.set_weights``), so a training loop pays one pass over the edges
    per step, not a host round trip and a registration.  backward() puts the
    forward's weights back first if another forward changed them meanwhile.

    ``forward_dir`` / ``adjoint_dir`` pick push or pull for each solve (the
    adjoint of a forward push is a pull over the same CSR rows, and vice
    versa)."""

    @staticmethod
    def _graph(structure, w, relabel):
        if isinstance(structure, Graph):
            return structure
        cache = structure.__dict__.setdefault("_pp_graphs", {})
        key = (str(w.device), bool(relabel))
        g = cache.get(key)
        if g is None or g.handle is None:
            import copy
            host = copy.copy(structure)
            host.__dict__.pop("_pp_graphs", None)
            host.weights = w.detach().float().cpu().numpy()
            host.ensure_transpose()
            g = Graph(host, device=w.device, weighted=True, relabel=relabel)
            cache[key] = g
            g._pp_w_version = None
        return g

    @staticmethod
    def forward(ctx, w, structure, sources, f=0.85, iters=3000, tol=1e-9, k_tile=32,
                forward_dir=PP_PULL, adjoint_dir=PP_PULL, relabel=True):
        g = PPRFunction._graph(structure, w, relabel)
        wd = w.detach()
        g.set_weights(wd)
        g._pp_w_version = (wd.data_ptr(), wd._version)
        X, _ = ppr(g, sources, iters=iters, f=f, k_tile=k_tile, direction=forward_dir, tol=tol)
        ctx.g = g
        ctx.cfg = (f, iters, tol, k_tile, adjoint_dir)
        ctx.w_version = g._pp_w_version
        ctx.save_for_backward(X, wd)
        return X

    @staticmethod
    def backward(ctx, dX):
        X, wd = ctx.saved_tensors
        f, iters, tol, k_tile, adir = ctx.cfg
        g = ctx.g
        if getattr(g, "_pp_w_version", None) != ctx.w_version:
            g.set_weights(wd)
            g._pp_w_version = ctx.w_version
        _, grad, _ = ppr_adjoint(g, X, dX.float(), iters=iters, f=f, k_tile=k_tile, direction=adir, tol=tol)
        return grad, None, None, None, None, None, None, None, None, None


def triangles(g: Graph, direction=PP_PULL, stream=None):
    """Triangles per vertex (int64[n], caller ids) by the pulling or pushing
    form; the graph's rows must be in strictly ascending order."""
    dev = g.device if hasattr(g, "device") else torch.device("cuda")
    tc = torch.empty(g.n, dtype=torch.int64, device=dev)
    ws = torch.empty(max(_lib.pp_tc_workspace_bytes(g.handle), 1), dtype=torch.uint8, device=dev)
    _lib.pp_tc_run(g.handle, direction, tc, ws, stream)
    return tc


def betweenness(g: Graph, sources, fwd_dir=PP_PULL, bwd_dir=PP_PULL, stream=None):
    """Betweenness centrality summed over ``sources`` (float64[n], caller ids)."""
    bc = torch.empty(g.n, dtype=torch.float64, device=g.device)
    ws = torch.empty(max(_lib.pp_bc_workspace_bytes(g.handle), 1), dtype=torch.uint8, device=g.device)
    _lib.pp_bc_run(g.handle, fwd_dir, bwd_dir, sources, bc, ws, stream)
    return bc


class MultiGraph:
    """Many small symmetric (or directed, with in-adjacency) graphs in one
    device arena, for pp_multi_run."""

    def __init__(self, hosts, device="cuda"):
        import numpy as np
        self.hosts = hosts
        self.n = np.array([h.n for h in hosts], dtype=np.int32)
        self.nnz = np.array([int(h.off[-1]) for h in hosts], dtype=np.int64)
        dev = torch.device(device)
        for h in hosts:
            for ids in (h.idx, getattr(h, "in_idx", None)):
                if ids is not None and len(ids) and (int(ids.min()) < 0 or int(ids.max()) >= h.n):
                    raise PPError(PP_E_GRAPH, f"{getattr(h, 'name', 'graph')}: neighbour id outside 0..n-1")
        cat = lambda arrs: torch.as_tensor(np.concatenate(arrs).astype(np.int32)).to(dev)  # noqa: E731
        # local ids as 16 bits (graphs hold at most 16384 vertices); int16 storage, read as uint16
        cat16 = lambda arrs: torch.as_tensor(np.concatenate(arrs).astype(np.int16)).to(dev)  # noqa: E731
        self.off = cat([h.off for h in hosts])
        self.idx = cat16([h.idx for h in hosts] + [np.zeros(1, np.int16)])
        directed = [h for h in hosts if getattr(h, "in_off", None) is not None and h.in_off is not h.off]
        if directed:
            for h in hosts:
                if getattr(h, "in_off", None) is None:
                    h.ensure_transpose()
            self.in_off = cat([h.in_off for h in hosts])
            self.in_idx = cat16([h.in_idx for h in hosts] + [np.zeros(1, np.int16)])
        else:
            self.in_off, self.in_idx = self.off, self.idx
        self.total_n = int(self.n.sum())
        self.ws = torch.empty(max(_lib.pp_multi_workspace_bytes(len(hosts), self.total_n), 1), dtype=torch.uint8,
                              device=dev)
        self.device = dev

    def run(self, pr_iters=20, f=0.85, pr_dir=PP_PULL, bfs_policy=PP_SWITCH, bfs_root=0, alpha=14.0, beta=24.0,
            stream=None):
        x = torch.empty(max(self.total_n, 1), dtype=torch.float32, device=self.device)
        level = torch.empty(max(self.total_n, 1), dtype=torch.int32, device=self.device)
        parent = torch.empty_like(level)
        _lib.pp_multi_run(self.n, self.nnz, self.off, self.idx, self.in_off, self.in_idx, pr_dir, pr_iters, f, x,
                          bfs_policy, bfs_root, alpha, beta, level, parent, self.ws, stream)
        return x, level, parent

    def split(self, t):
        import numpy as np
        bounds = np.concatenate([[0], np.cumsum(self.n)])
        return [t[bounds[i]:bounds[i + 1]] for i in range(len(self.n))]
