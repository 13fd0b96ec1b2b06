"""Host logic of the autotuner: size classes, cache keys and entries, and
that applying a cached entry reaches the library's tuning entry points."""
import json

import pytest

from paper_2010_16012_amd import _lib, autotune


def test_size_class_rounds_to_powers_of_two():
    assert autotune.size_class(4194304, 128305266) == "n2^22_m2^27"
    assert autotune.size_class(1048576, 31406614) == "n2^20_m2^25"
    assert autotune.size_class(1, 0) == "n2^0_m2^0"


def test_load_picks_the_entry_of_the_architecture_and_size(tmp_path):
    path = tmp_path / "t.json"
    path.write_text(json.dumps({"gfx950|n2^22_m2^27": {"hot": 40960}, "gfx942|n2^22_m2^27": {"hot": 1}}))
    assert autotune.load(str(path), 4194304, 128305266, "gfx950") == {"hot": 40960}
    assert autotune.load(str(path), 1024, 20000, "gfx950") == {}
    assert autotune.load(str(tmp_path / "missing.json"), 4194304, 128305266, "gfx950") == {}


def test_committed_cache_is_valid():
    import os
    path = os.path.join(os.path.dirname(autotune.__file__), "tuned.json")
    with open(path) as fh:
        cache = json.load(fh)
    for k, cfg in cache.items():
        arch, size = k.split("|")
        assert arch.startswith("gfx") and (size.startswith("n2^") or size.startswith("multi"))
        assert set(cfg) <= set(autotune.DEFAULTS)
        autotune.apply(cfg)  # every value is accepted by the library
    autotune.apply({})


def test_apply_rejects_out_of_range_values():
    with pytest.raises(_lib.PPError):
        autotune.apply({"hot": 10**6})
    with pytest.raises(_lib.PPError):
        autotune.apply({"upper": [64, 16, 4, 1024, 4096]})  # not increasing
    autotune.apply({})


def test_bin_candidates_are_increasing():
    for upper, chunk in autotune.BIN_CANDIDATES:
        assert all(a < b for a, b in zip(upper, upper[1:])) and chunk > 0


def test_multi_key_and_mapping_settings():
    assert autotune.multi_key(512, 2917543, 61503090, "gfx950") == "gfx950|multi512_n2^21_m2^26"
    for big, mid, pg, ml in autotune.MULTI_GRID:
        autotune.apply({"multi_big": big, "multi_mid": mid, "multi_pull_group": pg, "multi_mid_lanes": ml})
    for bad in ({"multi_pull_group": 3}, {"multi_mid_lanes": 64}, {"multi_mid": 600}, {"multi_mid": 0}):
        with pytest.raises(_lib.PPError):
            autotune.apply(bad)
    autotune.apply({})


def test_bfs_multi_caps_candidates_and_range():
    # every caps setting the switch search tries is accepted (0 switches the
    # one-workgroup launch off); negative caps are rejected
    for n_cap, m_cap in autotune.BFS_MULTI_CAPS:
        assert n_cap >= 0 and m_cap >= 0
        autotune.apply({"bfs_multi_n": n_cap, "bfs_multi_m": m_cap})
    assert (autotune.DEFAULTS["bfs_multi_n"], autotune.DEFAULTS["bfs_multi_m"]) in autotune.BFS_MULTI_CAPS
    for bad in ({"bfs_multi_n": -1}, {"bfs_multi_m": -5}):
        with pytest.raises(_lib.PPError):
            autotune.apply(bad)
    autotune.apply({})
