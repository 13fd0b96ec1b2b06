"""The C ABI library loads and exports every symbol include/pp.h declares;
host-side argument validation works without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_core_calls():
    syms = declared_symbols()
    for s in ["pp_graph_create", "pp_pr_push", "pp_pr_pull", "pp_bfs_step_push", "pp_bfs_step_pull", "pp_bfs_run"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2010_16012_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert missing == []
    assert sorted(_lib.EXPORTS) == declared_symbols()


def test_host_side_queries_and_validation():
    from paper_2010_16012_amd import _lib
    assert _lib.pp_abi_version() == 1
    assert _lib.pp_graph_workspace_bytes(0, 10, 0) == 0
    assert _lib.pp_graph_workspace_bytes(10, -1, 0) == 0
    assert _lib.pp_graph_workspace_bytes(1000, 5000, 0) > 0
    assert _lib.pp_graph_workspace_bytes(1000, 5000, 1) > _lib.pp_graph_workspace_bytes(1000, 5000, 0)
    h = ctypes.c_void_p()
    lib = _lib._lib
    # NULL arrays are rejected before anything reaches the GPU
    rc = lib.pp_graph_create(10, 20, None, None, None, None, None, None, 0, None, 0, None, ctypes.byref(h))
    assert rc == _lib.PP_E_NULL and "required" in _lib.pp_last_error()
    rc = lib.pp_graph_create(0, 20, None, None, None, None, None, None, 0, None, 0, None, ctypes.byref(h))
    assert rc == _lib.PP_E_SIZE
    assert lib.pp_pr_push(None, None, None, ctypes.c_float(0.85), None) == _lib.PP_E_NULL
    assert lib.pp_bfs_run(None, 0, 2, ctypes.c_float(14), ctypes.c_float(24), None, None, None, 0, None, None) \
        == _lib.PP_E_NULL
    assert lib.pp_bfs_run(None, 0, 7, ctypes.c_float(14), ctypes.c_float(24), None, None, None, 0, None, None) \
        == _lib.PP_E_RANGE
    with pytest.raises(_lib.PPError):
        _lib.pp_set_bin_thresholds([5, 4, 3, 2, 1], 1024)
    with pytest.raises(_lib.PPError):
        _lib.pp_set_bin_thresholds([1, 2, 3, 4, 5], 10)


def test_binding_has_a_function_for_every_export():
    from paper_2010_16012_amd import _lib
    assert [n for n in _lib.EXPORTS if not callable(getattr(_lib, n, None))] == []


def test_many_graph_arena_checks_ids_on_the_host():
    # the arena stores 16-bit local ids; an id outside 0..n-1 is refused while
    # the arena is built, before anything reaches a device
    import numpy as np
    import graphgen as gg
    import paper_2010_16012_amd as pp
    bad = gg.from_edges(6, [0, 1], [1, 2], True)
    bad.idx = bad.idx.copy()
    bad.idx[0] = 6
    with pytest.raises(pp.PPError):
        pp.MultiGraph([bad], device="cpu")
    good = gg.from_edges(6, [0, 1], [1, 2], True)
    mg = pp.MultiGraph([good, good], device="cpu")
    assert mg.idx.dtype.itemsize == 2 and int(mg.idx.max()) < 6
    assert np.array_equal(mg.off.numpy(), np.concatenate([good.off, good.off]))
