"""Input generators: determinism, the adjacency-array invariants (Sec. 2.2),
the R-MAT / grid / Erdos-Renyi recipes, and the counter-based PRNG."""
import hashlib

import numpy as np
import pytest

import graphgen as gg

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def test_splitmix64_published_first_output():
    # SplitMix64 seeded with 0 first returns 0xE220A8397B1DCDAF.
    assert _mix(GAMMA) == 0xE220A8397B1DCDAF


def test_counter_generator_definition():
    for seed, stream, ctr in [(1, 0, 0), (1, 2, 99), (123456789, 7, 2**40 + 3)]:
        key = _mix(seed ^ _mix((stream + GAMMA) & MASK))
        want = _mix((key + (ctr + 1) * GAMMA) & MASK)
        assert gg.rand_u64(seed, stream, ctr) == want


def _digest(g):
    h = hashlib.sha256()
    h.update(g.off.tobytes())
    h.update(g.idx.tobytes())
    return h.hexdigest()


def _check_adjacency(g, symmetric=True):
    off, idx = g.off, g.idx
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == len(idx)
    assert idx.dtype == np.int32 and (len(idx) == 0 or (idx.min() >= 0 and idx.max() < g.n))
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(off))
    assert not np.any(src == idx), "self-loop"
    keys = src * g.n + idx
    assert np.all(np.diff(keys) > 0), "rows not strictly ascending (duplicate or unsorted)"
    if symmetric:
        rkeys = np.sort(idx.astype(np.int64) * g.n + src)
        np.testing.assert_array_equal(rkeys, keys)


def test_rmat_deterministic_and_canonical():
    a = gg.rmat(12, 16, seed=1)
    b = gg.rmat(12, 16, seed=1)
    c = gg.rmat(12, 16, seed=2)
    assert _digest(a) == _digest(b) != _digest(c)
    _check_adjacency(a)


def test_rmat_quadrant_probabilities():
    # Top-level bits of source/destination follow (a, b, c, d).
    n_e = 1 << 18
    src = np.empty(n_e, np.int32)
    dst = np.empty(n_e, np.int32)
    lib = gg._load()
    assert lib.gg_rmat_edges(10, n_e, 0.57, 0.19, 0.19, 5, gg._ptr(src), gg._ptr(dst)) == 0
    for bit in (9, 0):
        s = (src >> bit) & 1
        t = (dst >> bit) & 1
        q = np.bincount(s * 2 + t, minlength=4) / n_e
        np.testing.assert_allclose(q, [0.57, 0.19, 0.19, 0.05], atol=4e-3)


def test_rmat14_statistics():
    g = gg.rmat(14, 16, seed=1)
    deg = np.diff(g.off)
    assert g.n == 16384
    assert 400_000 < g.nnz < 450_000
    assert 0.2 < (deg == 0).mean() < 0.27
    assert deg.argmax() == 0


def test_grid_counts_and_structure():
    g = gg.grid(40, 50, 0.05, seed=3)
    ne = 40 * 49 + 39 * 50
    assert g.nnz == 2 * (ne - round(0.05 * ne))
    _check_adjacency(g)
    v = np.repeat(np.arange(g.n), np.diff(g.off))
    d = np.abs(g.idx - v)
    assert set(np.unique(d)) <= {1, 50}
    full = gg.grid(40, 50, 0.0, seed=3)
    assert full.nnz == 2 * ne
    assert _digest(gg.grid(40, 50, 0.05, seed=3)) == _digest(g)


def test_grid4096_recipe_counts():
    # 4096 x 4096 grid: 33,546,240 edges, 1,677,312 removed -> 63,737,856 entries.
    ne = 4096 * 4095 * 2
    assert ne == 33_546_240
    assert round(0.05 * ne) == 1_677_312
    assert 2 * (ne - 1_677_312) == 63_737_856


def test_er_and_from_edges():
    g = gg.erdos_renyi(1 << 12, 8 << 12, seed=1)
    _check_adjacency(g)
    assert abs(g.nnz / g.n - 16) < 0.5
    h = gg.from_edges(5, [0, 0, 1, 2, 2, 4], [1, 1, 1, 0, 3, 4], True)
    np.testing.assert_array_equal(h.off, [0, 2, 3, 5, 6, 6])
    np.testing.assert_array_equal(h.idx, [1, 2, 0, 0, 3, 2])


def test_directed_transpose():
    g = gg.from_edges(4, [0, 0, 1, 3], [1, 2, 2, 0], False)
    g.ensure_transpose()
    np.testing.assert_array_equal(g.in_off, [0, 1, 2, 4, 4])
    np.testing.assert_array_equal(g.in_idx, [3, 0, 0, 1])
    # each CSC slot maps to the CSR slot of the same edge
    src = np.repeat(np.arange(4), np.diff(g.off))
    dst_of_in = np.repeat(np.arange(4), np.diff(g.in_off))
    np.testing.assert_array_equal(src[g.in_to_out], g.in_idx)
    np.testing.assert_array_equal(g.idx[g.in_to_out], dst_of_in)


def test_vectors_and_picks():
    u = gg.uniform(100000, 0.1, 1.0, seed=4)
    assert u.min() >= 0.1 and u.max() < 1.0 and abs(u.mean() - 0.55) < 0.01
    z = gg.normal(200000, seed=4)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    g = gg.rmat(10, 16, seed=1)
    p = gg.pick_vertices(g, 64, seed=9)
    assert len(set(p.tolist())) == 64 and np.all(np.diff(g.off)[p] >= 1)
    np.testing.assert_array_equal(p, gg.pick_vertices(g, 64, seed=9))
    with pytest.raises(ValueError):
        gg.pick_vertices(gg.from_edges(4, [0], [1], True), 3, seed=1)


def test_batch_scales():
    gs = gg.rmat_batch(12, 8, 10, seed=3)
    assert len(gs) == 12
    assert {g.meta["scale"] for g in gs} <= {8, 9, 10}
    for g in gs[:3]:
        _check_adjacency(g)
