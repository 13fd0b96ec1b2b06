"""Triangle counting, pushing and pulling forms, against the oracle (exact)."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2010_16012_amd as pp
from tests import helpers as H
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

DIRS = [pp.PP_PULL, pp.PP_PUSH]


def _tc(host, d):
    g = pp.Graph(host, relabel=False)
    out = pp.triangles(g, d)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _same(host):
    want = oracle.triangles(host.off, host.idx)
    for d in DIRS:
        announce(f"tc {host.name} n={host.n} nnz={host.nnz} dir={d}")
        got = _tc(host, d)
        np.testing.assert_array_equal(got, want)
    return want


def test_closed_forms():
    k = H.complete(40)
    np.testing.assert_array_equal(_same(k), np.full(40, 39 * 38 // 2))
    assert _same(H.star(500)).sum() == 0
    assert _same(H.cycle(3)).tolist() == [1, 1, 1]
    assert _same(H.cycle(50)).sum() == 0
    assert _same(H.full_grid(20, 30)).sum() == 0


def test_random_graphs_and_rmat14():
    for s, (n, m) in enumerate([(10, 30), (300, 3000), (5000, 60000)]):
        _same(H.random_graph(n, m, 40 + s, symmetric=True))
    _same(gg.workload("rmat14"))


def test_rows_across_many_slices_and_heavy_pairs():
    # a hub adjacent to everything plus a dense core: the hub row spans many
    # 256-edge slices, hub-core pairs need the wavefront-wide intersection
    n = 6000
    src = list(range(1, n))
    dst = [0] * (n - 1)
    rng = np.random.default_rng(3)
    core = rng.choice(np.arange(1, n), size=120, replace=False)
    for i in range(len(core)):
        for j in range(i + 1, len(core)):
            src.append(int(core[i]))
            dst.append(int(core[j]))
    extra = rng.integers(1, n, size=(20000, 2))
    src += extra[:, 0].tolist()
    dst += extra[:, 1].tolist()
    _same(gg.from_edges(n, src, dst, True, name="hub+core"))


def test_empty_and_isolated():
    _same(gg.from_edges(7, [], [], True, name="empty"))
    _same(gg.from_edges(9, [0, 1, 2], [1, 2, 0], True, name="triangle+isolated"))


def test_push_equals_pull_on_rmat16():
    host = gg.rmat(16, 16, seed=2)
    g = pp.Graph(host, relabel=False)
    a = pp.triangles(g, pp.PP_PULL)
    b = pp.triangles(g, pp.PP_PUSH)
    assert torch.equal(a, b)
    want = oracle.triangles(host.off, host.idx)
    np.testing.assert_array_equal(a.cpu().numpy(), want)


def test_unsorted_rows_are_rejected():
    host = gg.from_edges(6, [0, 0, 0, 1, 2], [1, 2, 3, 2, 3], True)
    idx = host.idx.copy()
    r0, r1 = int(host.off[0]), int(host.off[1])
    idx[r0:r1] = idx[r0:r1][::-1].copy()  # row 0 descending
    bad = gg.HostGraph(host.n, host.off.copy(), idx, True, name="unsorted")
    g = pp.Graph(bad, relabel=False)
    with pytest.raises(pp.PPError):
        pp.triangles(g, pp.PP_PULL)
