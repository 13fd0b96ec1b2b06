"""pp_multi_run_static (the many-graph launch with the library's fixed scratch,
for callers that cannot allocate) against pp_multi_run on the same arenas:
two calls in a row, the second on a smaller batch, so the second call runs on
scratch the first one left behind.  PageRank pull is summed in a fixed order
on both paths (bit-identical); push adds in atomic order (L1 <= 1e-6);
BFS levels are exact and parents valid.
"""
import numpy as np
import pytest
import torch

import graphgen as gg
import paper_2010_16012_amd as pp
from paper_2010_16012_amd import _lib
from tests import helpers as H
from tests.gpu_util import F, PR_L1_TOL, announce

pytestmark = pytest.mark.gpu


def _static_run(mg, pr_dir, pr_iters, bfs_policy):
    dev = mg.device
    x = torch.full((max(mg.total_n, 1),), -1.0, dtype=torch.float32, device=dev)
    level = torch.full((max(mg.total_n, 1),), -5, dtype=torch.int32, device=dev)
    parent = torch.full_like(level, -5)
    _lib.pp_multi_run_static(mg.n, mg.nnz, mg.off, mg.idx, mg.in_off, mg.in_idx, pr_dir, pr_iters, F, x, bfs_policy,
                             0, 14.0, 24.0, level, parent)
    torch.cuda.synchronize()
    return x, level, parent


def _compare(gs):
    mg = pp.MultiGraph(gs)
    for d, name in ((pp.PP_PULL, "pull"), (pp.PP_PUSH, "push")):
        announce(f"static scratch: {len(gs)} graphs, {mg.total_n} vertices, PageRank {name} + BFS switch")
        x0, l0, p0 = mg.run(pr_iters=20, f=F, pr_dir=d, bfs_policy=pp.PP_SWITCH)
        x1, l1, p1 = _static_run(mg, d, 20, pp.PP_SWITCH)
        xs0, xs1 = mg.split(x0.cpu().numpy()), mg.split(x1.cpu().numpy())
        ls0, ls1, ps1 = mg.split(l0.cpu().numpy()), mg.split(l1.cpu().numpy()), mg.split(p1.cpu().numpy())
        for h, a, b, la, lb, pb in zip(gs, xs0, xs1, ls0, ls1, ps1):
            if d == pp.PP_PULL:
                assert np.array_equal(a, b), h.name
            assert np.abs(a.astype(np.float64) - b).sum() <= PR_L1_TOL, h.name
            assert np.array_equal(la, lb), h.name
            assert H.bfs_violations(h, 0, lb, pb) == [], h.name


def test_static_scratch_matches_the_workspace_call():
    big = gg.rmat_batch(40, 8, 13, seed=21) + [H.star(3000), H.full_grid(50, 60)]
    small = gg.rmat_batch(6, 5, 8, seed=22) + [gg.from_edges(1, [], [], True), H.path(40)]
    _compare(big)
    _compare(small)  # smaller than the first call: stale scratch beyond its end


def test_static_scratch_refuses_batches_beyond_its_size():
    n = np.full(300, 16384, dtype=np.int32)  # 4.9 million vertices: more than 16 MiB of scratch
    nnz = np.zeros(300, dtype=np.int64)
    dev = torch.device("cuda")
    off = torch.zeros(int(n.sum()) + 300, dtype=torch.int32, device=dev)
    x = torch.empty(int(n.sum()), dtype=torch.float32, device=dev)
    level = torch.empty(int(n.sum()), dtype=torch.int32, device=dev)
    with pytest.raises(pp.PPError) as ei:
        _lib.pp_multi_run_static(n, nnz, off, None, off, None, pp.PP_PULL, 5, F, x, pp.PP_SWITCH, 0, 14.0, 24.0,
                                 level, level.clone())
    assert ei.value.status == _lib.PP_E_WORKSPACE
    assert _lib.pp_multi_workspace_bytes(300, int(n.sum())) > _lib.PP_MULTI_STATIC_BYTES
