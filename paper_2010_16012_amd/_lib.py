"""ctypes binding of libpp.so: the C ABI declared in include/pp.h, one Python
function per entry point with the same name.  Argument marshalling only --
every step of every sweep runs in the library's HIP kernels.  Arrays are torch
tensors on the GPU; streams default to torch's current stream.

There is no fallback: if libpp.so is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so libpp binds to the HIP runtime torch already uses

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2010_16012_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

PP_OK = 0
PP_E_NULL = -1
PP_E_SIZE = -2
PP_E_RANGE = -3
PP_E_GRAPH = -4
PP_E_WORKSPACE = -5
PP_E_HIP = -6
PP_E_UNSUPPORTED = -7
STATUS_NAMES = {0: "PP_OK", -1: "PP_E_NULL", -2: "PP_E_SIZE", -3: "PP_E_RANGE", -4: "PP_E_GRAPH",
                -5: "PP_E_WORKSPACE", -6: "PP_E_HIP", -7: "PP_E_UNSUPPORTED"}

PP_PUSH, PP_PULL, PP_SWITCH = 0, 1, 2
PP_GRAPH_WEIGHTED = 0x1
PP_GRAPH_RELABEL = 0x2
PP_NUM_BINS = 6
PP_BFS_MAX_LOG = 64


class PPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class BfsStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("reached", ctypes.c_int32), ("edges_reached", ctypes.c_int64),
                ("dir", ctypes.c_int8 * PP_BFS_MAX_LOG), ("frontier", ctypes.c_int32 * PP_BFS_MAX_LOG)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_F32 = ctypes.c_float
_SZ = ctypes.c_size_t

_SIGS = {
    "pp_abi_version": ([], ctypes.c_int),
    "pp_last_error": ([], ctypes.c_char_p),
    "pp_graph_workspace_bytes": ([_I32, _I64, _U32], _SZ),
    "pp_graph_create": ([_I32, _I64, _P, _P, _P, _P, _P, _P, _U32, _P, _SZ, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "pp_graph_destroy": ([_P], ctypes.c_int),
    "pp_graph_check": ([_P, _P], ctypes.c_int),
    "pp_graph_bins": ([_P, ctypes.c_int, ctypes.POINTER(_I32)], ctypes.c_int),
    "pp_set_bin_thresholds": ([ctypes.POINTER(_I32), _I32], ctypes.c_int),
    "pp_set_push_tuning": ([_I32, _I32], ctypes.c_int),
    "pp_set_pull_tuning": ([_I32, _I32], ctypes.c_int),
    "pp_graph_relabel_map": ([_P, _P, _P], ctypes.c_int),
    "pp_pr_push": ([_P, _P, _P, _F32, _P], ctypes.c_int),
    "pp_pr_pull": ([_P, _P, _P, _F32, _P], ctypes.c_int),
    "pp_pr_run": ([_P, ctypes.c_int, _I32, _F32, _P, _P], ctypes.c_int),
    "pp_bfs_state_bytes": ([_P], _SZ),
    "pp_bfs_init": ([_P, _I32, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "pp_bfs_step_push": ([_P, _P, _P, _P, _I32, _P], ctypes.c_int),
    "pp_bfs_step_pull": ([_P, _P, _P, _P, _I32, _P], ctypes.c_int),
    "pp_bfs_frontier": ([_P, _P, ctypes.POINTER(_I32), _P], ctypes.c_int),
    "pp_bfs_run": ([_P, _I32, ctypes.c_int, _F32, _F32, _P, _P, _P, _SZ, ctypes.POINTER(BfsStats), _P], ctypes.c_int),
    "pp_bfs_run_log": ([_P, _I32, ctypes.c_int, _F32, _F32, _P, _P, _P, _SZ, _P, _I32, ctypes.POINTER(BfsStats), _P],
                       ctypes.c_int),
    "pp_bfs_run_many": ([_P, _I32, _P, ctypes.c_int, _F32, _F32, _P, _P, _P, _SZ, ctypes.POINTER(BfsStats), _P],
                        ctypes.c_int),
    "pp_ppr_scratch_bytes": ([_P, _I32, _I32], _SZ),
    "pp_multi_workspace_bytes": ([_I32, _I64], _SZ),
    "pp_multi_run": ([_I32, _P, _P, _P, _P, _P, _P, ctypes.c_int, _I32, _F32, _P, _I32, _I32, _F32, _F32, _P, _P, _P,
                      _SZ, _P], ctypes.c_int),
    "pp_multi_run_static": ([_I32, _P, _P, _P, _P, _P, _P, ctypes.c_int, _I32, _F32, _P, _I32, _I32, _F32, _F32, _P,
                             _P, _P], ctypes.c_int),
    "pp_set_pull_slices": ([_I32, _I32], ctypes.c_int),
    "pp_set_bfs_multi": ([_I32, _I32], ctypes.c_int),
    "pp_set_push_bins": ([_I32], ctypes.c_int),
    "pp_set_multi_tuning": ([_I32, _I32, _I32, _I32], ctypes.c_int),
    "pp_graph_set_weights": ([_P, _P, _P], ctypes.c_int),
    "pp_graph_push_bins": ([_P, _P], ctypes.c_int),
    "pp_graph_slices": ([_P, _P], ctypes.c_int),
    "pp_ppr_run": ([_P, ctypes.c_int, _I32, _P, _I32, _F32, _F32, _I32, _P, _P, _SZ, ctypes.POINTER(_I32), _P],
                   ctypes.c_int),
    "pp_ppr_adjoint": ([_P, ctypes.c_int, _I32, _P, _P, _I32, _F32, _F32, _I32, _P, _P, _P, _SZ,
                        ctypes.POINTER(_I32), _P], ctypes.c_int),
    "pp_ppr_unrolled_scratch_bytes": ([_P, _I32, _I32, _I32], _SZ),
    "pp_ppr_adjoint_unrolled": ([_P, _I32, _P, _I32, _F32, _I32, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "pp_tc_workspace_bytes": ([_P], _SZ),
    "pp_tc_run": ([_P, ctypes.c_int, _P, _P, _SZ, _P], ctypes.c_int),
    "pp_bc_workspace_bytes": ([_P], _SZ),
    "pp_bc_run": ([_P, ctypes.c_int, ctypes.c_int, _I32, _P, _P, _P, _SZ, _P], ctypes.c_int),
}

EXPORTS = tuple(_SIGS)

for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


def _check(status: int) -> None:
    if status != PP_OK:
        raise PPError(status, _lib.pp_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("libpp takes device tensors")
        if not t.is_contiguous():
            raise ValueError("libpp takes contiguous tensors")
        return ctypes.c_void_p(t.data_ptr())
    return t


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _expect(t, dtype, numel=None, name="tensor"):
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {t.numel()}")


# ----------------------------------------------------------------------- ABI
def pp_abi_version() -> int:
    return _lib.pp_abi_version()


def pp_last_error() -> str:
    return _lib.pp_last_error().decode()


def pp_graph_workspace_bytes(n: int, nnz: int, flags: int = 0) -> int:
    return _lib.pp_graph_workspace_bytes(n, nnz, flags)


def pp_graph_create(n, nnz, csr_off, csr_idx, csc_off, csc_idx, csr_w, csc_to_csr, flags, ws, stream=None):
    h = _P()
    _check(_lib.pp_graph_create(n, nnz, _ptr(csr_off), _ptr(csr_idx), _ptr(csc_off), _ptr(csc_idx), _ptr(csr_w),
                                _ptr(csc_to_csr), flags, _ptr(ws), ws.numel() * ws.element_size(), _stream(stream),
                                ctypes.byref(h)))
    return h


def pp_graph_destroy(h) -> None:
    _check(_lib.pp_graph_destroy(h))


def pp_graph_check(h, stream=None) -> None:
    _check(_lib.pp_graph_check(h, _stream(stream)))


def pp_graph_bins(h, direction: int):
    out = (_I32 * PP_NUM_BINS)()
    _check(_lib.pp_graph_bins(h, direction, out))
    return list(out)


def pp_set_bin_thresholds(upper5, split_chunk: int) -> None:
    arr = (_I32 * 5)(*[int(u) for u in upper5])
    _check(_lib.pp_set_bin_thresholds(arr, split_chunk))


def pp_set_push_tuning(hot: int, push_blocks: int) -> None:
    _check(_lib.pp_set_push_tuning(hot, push_blocks))


def pp_set_pull_tuning(pull_hot: int, pull_block: int) -> None:
    _check(_lib.pp_set_pull_tuning(pull_hot, pull_block))


def pp_graph_relabel_map(h, perm, stream=None) -> None:
    _check(_lib.pp_graph_relabel_map(h, _ptr(perm), _stream(stream)))


def pp_pr_push(h, x, y, f: float, stream=None) -> None:
    _check(_lib.pp_pr_push(h, _ptr(x), _ptr(y), f, _stream(stream)))


def pp_pr_pull(h, x, y, f: float, stream=None) -> None:
    _check(_lib.pp_pr_pull(h, _ptr(x), _ptr(y), f, _stream(stream)))


def pp_pr_run(h, direction: int, iters: int, f: float, x, stream=None) -> None:
    _check(_lib.pp_pr_run(h, direction, iters, f, _ptr(x), _stream(stream)))


def pp_bfs_state_bytes(h) -> int:
    return _lib.pp_bfs_state_bytes(h)


def pp_bfs_init(h, root, level, parent, state, stream=None) -> None:
    _check(_lib.pp_bfs_init(h, root, _ptr(level), _ptr(parent), _ptr(state), state.numel(), _stream(stream)))


def pp_bfs_step_push(h, state, level, parent, cur_level, stream=None) -> None:
    _check(_lib.pp_bfs_step_push(h, _ptr(state), _ptr(level), _ptr(parent), cur_level, _stream(stream)))


def pp_bfs_step_pull(h, state, level, parent, cur_level, stream=None) -> None:
    _check(_lib.pp_bfs_step_pull(h, _ptr(state), _ptr(level), _ptr(parent), cur_level, _stream(stream)))


def pp_bfs_frontier(h, state, stream=None) -> int:
    out = _I32()
    _check(_lib.pp_bfs_frontier(h, _ptr(state), ctypes.byref(out), _stream(stream)))
    return out.value


def pp_bfs_run(h, root, policy, alpha, beta, level, parent, state, stream=None) -> BfsStats:
    st = BfsStats()
    _check(_lib.pp_bfs_run(h, root, policy, alpha, beta, _ptr(level), _ptr(parent), _ptr(state), state.numel(),
                           ctypes.byref(st), _stream(stream)))
    return st


def pp_bfs_run_many(h, roots, policy, alpha, beta, level, parent, state, stream=None):
    import numpy as np
    r = np.ascontiguousarray(roots, dtype=np.int32)
    stats = (BfsStats * max(len(r), 1))()
    _check(_lib.pp_bfs_run_many(h, len(r), r.ctypes.data_as(ctypes.c_void_p), policy, alpha, beta, _ptr(level),
                                _ptr(parent), _ptr(state), state.numel(), stats, _stream(stream)))
    return list(stats)[:len(r)]


def pp_set_pull_slices(rows: int, width: int) -> None:
    _check(_lib.pp_set_pull_slices(rows, width))


def pp_graph_set_weights(h, csr_w, stream=None) -> None:
    _check(_lib.pp_graph_set_weights(h, _ptr(csr_w), _stream(stream)))


def pp_set_multi_tuning(big: int, mid: int, pull_group: int, mid_lanes: int) -> None:
    _check(_lib.pp_set_multi_tuning(big, mid, pull_group, mid_lanes))


def pp_set_push_bins(on: int) -> None:
    _check(_lib.pp_set_push_bins(on))


def pp_graph_push_bins(h):
    """(bins, first binned target, sweep workgroups, summing units) of a
    registered graph (bins = 0: the push uses global atomics)."""
    info = (_I32 * 4)()
    _check(_lib.pp_graph_push_bins(h, info))
    return tuple(info)


def pp_set_bfs_multi(max_frontier: int, max_edges: int) -> None:
    _check(_lib.pp_set_bfs_multi(max_frontier, max_edges))


def pp_graph_slices(h):
    """(R, width, S, tiles) of the tiled pull of a registered graph (R = 0: off)."""
    info = (_I32 * 4)()
    _check(_lib.pp_graph_slices(h, info))
    return tuple(info)


# pp_bfs_level: int32 dir, int32 frontier, int64 frontier_edges (16 bytes)
BFS_LEVEL_BYTES = 16


def pp_bfs_run_log(h, root, policy, alpha, beta, level, parent, state, log, log_cap, stream=None) -> BfsStats:
    """log: device tensor of at least log_cap * 16 bytes (pp_bfs_level entries)."""
    if log is not None and log.numel() * log.element_size() < log_cap * BFS_LEVEL_BYTES:
        raise ValueError("log tensor smaller than log_cap entries")
    st = BfsStats()
    _check(_lib.pp_bfs_run_log(h, root, policy, alpha, beta, _ptr(level), _ptr(parent), _ptr(state), state.numel(),
                               _ptr(log), log_cap, ctypes.byref(st), _stream(stream)))
    return st


def pp_ppr_scratch_bytes(h, k: int, k_tile: int) -> int:
    return _lib.pp_ppr_scratch_bytes(h, k, k_tile)


def pp_ppr_run(h, direction, k, sources, iters, tol, f, k_tile, X, scratch, stream=None) -> int:
    done = _I32()
    _check(_lib.pp_ppr_run(h, direction, k, _ptr(sources), iters, tol, f, k_tile, _ptr(X), _ptr(scratch),
                           scratch.numel(), ctypes.byref(done), _stream(stream)))
    return done.value


def pp_ppr_adjoint(h, direction, k, X, dLdX, iters, tol, f, k_tile, Lambda, grad_w, scratch, stream=None) -> int:
    done = _I32()
    _check(_lib.pp_ppr_adjoint(h, direction, k, _ptr(X), _ptr(dLdX), iters, tol, f, k_tile, _ptr(Lambda),
                               _ptr(grad_w), _ptr(scratch), scratch.numel(), ctypes.byref(done), _stream(stream)))
    return done.value


def pp_multi_workspace_bytes(num_graphs: int, total_vertices: int) -> int:
    return _lib.pp_multi_workspace_bytes(num_graphs, total_vertices)


def pp_multi_run(graph_n, graph_nnz, off, idx, in_off, in_idx, pr_dir, pr_iters, f, x, bfs_policy, bfs_root,
                 alpha, beta, level, parent, ws, stream=None) -> None:
    """graph_n (int32) and graph_nnz (int64) are host numpy arrays; the rest device tensors."""
    import numpy as np
    gn = np.ascontiguousarray(graph_n, dtype=np.int32)
    ge = np.ascontiguousarray(graph_nnz, dtype=np.int64)
    _check(_lib.pp_multi_run(len(gn), ctypes.c_void_p(gn.ctypes.data), ctypes.c_void_p(ge.ctypes.data), _ptr(off),
                             _ptr(idx), _ptr(in_off), _ptr(in_idx), pr_dir, pr_iters, f, _ptr(x), bfs_policy,
                             bfs_root, alpha, beta, _ptr(level), _ptr(parent), _ptr(ws), ws.numel(), _stream(stream)))


PP_MULTI_STATIC_BYTES = 16 << 20


def pp_multi_run_static(graph_n, graph_nnz, off, idx, in_off, in_idx, pr_dir, pr_iters, f, x, bfs_policy, bfs_root,
                        alpha, beta, level, parent, stream=None) -> None:
    """pp_multi_run with the library's fixed scratch (no workspace argument)."""
    import numpy as np
    gn = np.ascontiguousarray(graph_n, dtype=np.int32)
    ge = np.ascontiguousarray(graph_nnz, dtype=np.int64)
    _check(_lib.pp_multi_run_static(len(gn), ctypes.c_void_p(gn.ctypes.data), ctypes.c_void_p(ge.ctypes.data),
                                    _ptr(off), _ptr(idx), _ptr(in_off), _ptr(in_idx), pr_dir, pr_iters, f, _ptr(x),
                                    bfs_policy, bfs_root, alpha, beta, _ptr(level), _ptr(parent), _stream(stream)))


def pp_tc_workspace_bytes(h) -> int:
    return _lib.pp_tc_workspace_bytes(h)


def pp_tc_run(h, direction, tc, ws, stream=None) -> None:
    _check(_lib.pp_tc_run(h, direction, _ptr(tc), _ptr(ws), ws.numel(), _stream(stream)))


def pp_bc_workspace_bytes(h) -> int:
    return _lib.pp_bc_workspace_bytes(h)


def pp_bc_run(h, fwd_dir, bwd_dir, sources, bc, ws, stream=None) -> None:
    """sources: host int32 array (caller ids); bc, ws: device tensors."""
    import numpy as np
    src = np.ascontiguousarray(sources, dtype=np.int32)
    _check(_lib.pp_bc_run(h, fwd_dir, bwd_dir, len(src), ctypes.c_void_p(src.ctypes.data), _ptr(bc), _ptr(ws),
                          ws.numel(), _stream(stream)))


def pp_ppr_adjoint_unrolled(h, k, sources, T, f, k_tile, dLdXT, Lambda0, grad_w, scratch, stream=None) -> None:
    _check(_lib.pp_ppr_adjoint_unrolled(h, k, _ptr(sources), T, f, k_tile, _ptr(dLdXT), _ptr(Lambda0), _ptr(grad_w),
                                        _ptr(scratch), scratch.numel(), _stream(stream)))


def pp_ppr_unrolled_scratch_bytes(h, k, k_tile, T) -> int:
    return _lib.pp_ppr_unrolled_scratch_bytes(h, k, k_tile, T)
