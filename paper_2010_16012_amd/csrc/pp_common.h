// Internal definitions shared by the libpp translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "pp.h"

#define PP_EXPORT extern "C" __attribute__((visibility("default")))

namespace pp {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup for the sweep kernels

// Degree bins: bin b holds vertices with degree in (upper[b-1], upper[b]];
// bin 0 starts at degree 0, bin PP_NUM_BINS-1 is unbounded.  Lanes per vertex:
//   bin 0: 1 lane   bin 1: 4 lanes   bin 2: 16 lanes   bin 3: one wavefront
//   bin 4: one workgroup   bin 5: the row is split into chunks, one workgroup each
constexpr int kBinLanes[PP_NUM_BINS] = {1, 4, 16, 64, kBlock, kBlock};

struct Tuning {
    int32_t upper[PP_NUM_BINS - 1] = {4, 16, 64, 1024, 16384};
    int32_t split_chunk = 16384;
};
Tuning& tuning();

// Work decomposition of one binned sweep launch: every bin owns a contiguous
// range of workgroups; heavy bins come first so the longest rows start first.
struct BinPlan {
    int32_t count[PP_NUM_BINS] = {};      // vertices per bin
    int32_t list_off[PP_NUM_BINS + 1] = {};  // start of each bin in the vertex list
    int32_t block_off[PP_NUM_BINS + 1] = {}; // first workgroup of each bin (launch order)
    int32_t split_chunks = 0;             // workgroups used by bin 5
    int32_t total_blocks = 0;
};

struct GraphDev {
    int32_t n;
    int64_t nnz;
    const int32_t* csr_off;
    const int32_t* csr_idx;
    const int32_t* csc_off;
    const int32_t* csc_idx;
    const float* csr_w;       // weights in CSR slot order (nullable)
    float* csc_w;             // weights in CSC slot order (workspace; nullable)
    float* inv_s;             // 1/d(v) or 1/s(v); 0 when nothing leaves v
    int32_t* out_deg;         // d(v)
    int32_t* pull_list;       // vertices grouped by in-degree bin
    int32_t* push_list;       // vertices grouped by out-degree bin
    int32_t* split_tab;       // bin-5 chunk table: (vertex-list position, chunk) pairs
    float* split_part;        // bin-5 partial sums (pull)
    float* buf0;              // PageRank scratch vectors, n floats each
    float* buf1;
    float* buf2;
    int32_t* err;             // device error word / counters
};

}  // namespace pp

struct pp_graph_s {
    pp::GraphDev d;
    uint32_t flags;
    bool weighted;
    pp::BinPlan pull_plan;
    pp::BinPlan push_plan;
    int32_t split_pull_entries;  // rows of the pull split table
    int32_t split_push_entries;
    int32_t split_cap;           // capacity of each split table
    pp::Tuning tune;
};

namespace pp {

pp_status set_error(pp_status s, const std::string& msg);
pp_status hip_error(hipError_t e, const char* what);
void clear_error();

#define PP_HIP(call)                                          \
    do {                                                      \
        hipError_t _e = (call);                               \
        if (_e != hipSuccess) return ::pp::hip_error(_e, #call); \
    } while (0)

#define PP_LAUNCH_CHECK(what)                                 \
    do {                                                      \
        hipError_t _e = hipGetLastError();                    \
        if (_e != hipSuccess) return ::pp::hip_error(_e, what); \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline int32_t ceil_div(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

pp_status check_graph_handle(pp_graph g);

}  // namespace pp
