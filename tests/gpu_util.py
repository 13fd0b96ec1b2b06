"""Helpers for the GPU parity tests (import only from tests marked gpu)."""
import numpy as np
import torch

import paper_2010_16012_amd as pp
from paper_2010_16012_amd import _lib

# the damping factor as the FP32 kernels see it; the oracle is run at the same value
F = float(np.float32(0.85))
PR_L1_TOL = 1e-6  # FP32 sweep vs FP64 oracle, L1 over the whole vector


def default_bins():
    _lib.pp_set_bin_thresholds([4, 16, 64, 1024, 4096], 4096)
    _lib.pp_set_push_tuning(8192, 1024)
    _lib.pp_set_pull_tuning(32768, 1024)
    _lib.pp_set_pull_slices(0, 32768)
    _lib.pp_set_bfs_multi(256, 1024)
    _lib.pp_set_push_bins(1)


def tiny_bins():
    """Thresholds that push small test graphs through every bin, bin 5 included."""
    _lib.pp_set_bin_thresholds([1, 2, 8, 32, 300], 256)


def pr_gpu(g, direction, iters, f=F, x0=None):
    x = pp.pagerank(g, iters, f, direction, x0=x0)
    torch.cuda.synchronize()
    return x.cpu().numpy()


def announce(msg):
    print(msg, flush=True)
