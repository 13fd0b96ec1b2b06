// Work units of the degree-binned sweeps, shared by the pull and push
// kernels: every bin owns a contiguous range of work units, heaviest bin
// first (units run bin 5, 4, ..., 0).
#pragma once

#include "pp_common.h"

namespace pp {

struct SweepPlan {
    int32_t block_off[PP_NUM_BINS + 1];
    int32_t list_off[PP_NUM_BINS + 1];
};

static SweepPlan sweep_plan(const BinPlan& p) {
    SweepPlan s;
    for (int b = 0; b <= PP_NUM_BINS; ++b) {
        s.block_off[b] = p.block_off[b];
        s.list_off[b] = p.list_off[b];
    }
    return s;
}

// Which bin does work unit `blk` belong to?  Units run bin 5, 4, ..., 0.
__device__ __forceinline__ int unit_bin(const SweepPlan& sp, int32_t blk) {
    int b = PP_NUM_BINS - 1;
#pragma unroll
    for (int i = PP_NUM_BINS - 1; i > 0; --i)
        if (blk >= sp.block_off[i - 1]) b = i - 1;
    return b;
}

// loads in flight per lane for a group of G lanes
template <int G>
constexpr int unroll_for() {
    return G >= 64 ? 8 : 4;
}

}  // namespace pp
