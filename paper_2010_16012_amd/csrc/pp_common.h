// Internal definitions shared by the libpp translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

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

// The persistent pull sweep gives each row fewer lanes and each lane more
// loads in flight: lanes per row and loads per lane for bins 0..5 (bin 5 =
// one split chunk).  A wavefront therefore keeps 64 / lanes rows in flight.
constexpr int kPullLanes[PP_NUM_BINS] = {1, 1, 4, 16, 64, 64};
constexpr int kPullLoads[PP_NUM_BINS] = {4, 16, 16, 16, 16, 16};

// Push privatisation: the first kHotMax internal vertices can be accumulated
// in LDS by each workgroup of the persistent push sweep (160 KB of LDS).
constexpr int kHotMax = 40960;

// A slice of the tiled pull holds at most kSliceMax sources (15-bit offsets);
// besides it the kernel keeps a zero word and 1 KB per wavefront in LDS.
constexpr int kSliceMax = 32768;
constexpr int kTiledWaveLds = 1024;
// Wavefront-uniform descriptors (work-unit tables written before the kernel
// starts) are read through the constant address space, so they become scalar
// loads.  Vector memory operations complete in issue order, so a vector load
// here would make the wait on its value also wait for every vector load,
// store and atomic issued before it; a scalar load waits on its own counter.
template <typename T>
__device__ __forceinline__ T uniform_load(const T* p, int32_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) T* cptr;
    return ((cptr)p)[i];
#else
    return p[i];  // host pass: never executed
#endif
}

inline size_t tiled_lds_bytes(int32_t width, int32_t waves) {
    return (size_t)width * 4 + 16 + (size_t)waves * kTiledWaveLds;
}

struct Tuning {
    int32_t upper[PP_NUM_BINS - 1] = {4, 16, 64, 1024, 4096};
    int32_t split_chunk = 4096;
    int32_t hot = 8192;          // vertices privatised in LDS by the push sweep (0 = off)
    int32_t push_blocks = 1024;  // workgroups of the persistent push sweep
    int32_t pull_hot = 32768;    // contributions staged in LDS by the pull sweep (0 = off)
    int32_t pull_block = 1024;   // threads per workgroup of the persistent pull sweep
    int32_t slice_rows = 0;      // rows of the tiled pull (0 = off); see SlicePlan
    int32_t slice_width = kSliceMax; // sources per slice of the tiled pull
    int32_t push_bins = 1;       // binned push for targets past the privatised ones (0 = global atomics)
    // many-graph launch: rows of at least multi_big edges take a wavefront,
    // rows of multi_mid..multi_big-1 a group of multi_mid_lanes lanes, the
    // other pull rows multi_pull_group lanes
    int32_t multi_big = 512;
    int32_t multi_mid = 64;
    int32_t multi_pull_group = 2;
    int32_t multi_mid_lanes = 16;
    int32_t bfs_multi_n = 256;   // frontier vertices a one-workgroup BFS launch takes on (0 = off)
    int32_t bfs_multi_m = 1024;  // frontier out-edges per level it takes on
};
Tuning& tuning();

// Tiled pull sweep (relabelled unweighted graphs).  The in-edges of rows
// [0, rows) -- the heaviest rows -- are regrouped by source slice: slice s
// holds sources [s*width, (s+1)*width), and segment (s, u) lists the sources
// of row u that fall in slice s as offsets from s*width.  A workgroup stages
// one slice's contributions in LDS and its wavefronts sum segments into one
// partial per (slice, row); a combine kernel adds the partials of each row in
// slice order.  The other rows are pulled as usual ("rest").
//
// Index layout (16 bits per edge): the non-empty segments of a slice, rows
// ascending, packed into wavefront units of at most kUnitEdges edges and
// kUnitPairs segments, each unit starting 8-aligned; bit 15 marks the first
// edge of a segment, bits 0-14 hold the source offset (width <= 2^15).
// Segments of kSegLong or more edges are cut into chunks of kSegChunk edges,
// stored 8-aligned after all units.
constexpr int32_t kUnitEdges = 1024;  // 16 per lane
constexpr int32_t kUnitPairs = 256;   // 4 per lane
constexpr int32_t kSegLong = 1024;
constexpr int32_t kSegChunk = 1024;
constexpr uint32_t kSegHead = 0x8000u;

// One wavefront's work: edges [a, b) of slice `slice`; p0 >= 0: a unit whose
// segments are pairs p0, p0 + 1, ... of the pair list (their rows in
// prow[]); p0 < 0: chunk -p0-1 of a long segment.
struct SliceUnit {
    int32_t slice;
    int32_t a, b;
    int32_t p0;
};

// A workgroup's units of one slice: [u0, u1).
struct SliceSeg {
    int32_t slice;
    int32_t u0, u1;
    int32_t pad;
};

struct SlicePlan {
    int32_t rows = 0;    // R (0: the tiled pull is off)
    int32_t width = 0;   // W
    int32_t slices = 0;  // S
    int32_t tiles = 0;   // work units
    int32_t pairs = 0;   // non-empty segments
    int32_t chunks = 0;  // chunks of long segments
    int32_t idx_size = 0;  // 16-bit entries of the layout (a multiple of 8, 16 spare at the end)
    int32_t groups = 0;  // workgroups the units are divided among (the launch's grid)
    // the pull plan restricted to rows >= R: per bin, rows to skip at the
    // front of the bin's list; split-table entries and split rows to skip
    int32_t list_skip[PP_NUM_BINS] = {};
    int32_t tab0 = 0;
    int32_t fix0 = 0;
    int32_t wave_off[PP_NUM_BINS + 1] = {};
    int32_t units = 0;
    int32_t nsplit = 0;
    // rows [n - tail, n) have no in-edges and close bin 0's list: the combine
    // kernel gives them the teleport term instead of a wavefront unit each
    int32_t tail = 0;
};

// Binned push (pr.hip).  Updates to targets past the privatised ones (ids >=
// hot, "cold") are not global atomics: the push sweep appends them as
// (target offset, value) pairs to its workgroup's slice of the target's bin
// (kPushBinW consecutive ids), and a second kernel sums each bin in LDS.  The
// slices are sized at registration by walking the sweep's static work
// assignment once, so a sweep needs no global atomic at all.
constexpr int32_t kPushBinShift = 14;
constexpr int32_t kPushBinW = 1 << kPushBinShift;
constexpr int32_t kPushBinUnits = 512;  // target number of second-kernel units
constexpr int32_t kPushBinMinUnit = 4096;  // pairs a unit takes at least

struct PushBins {
    int32_t nbins = 0;   // 0: the push sweep uses global atomics
    int32_t hot = 0;     // first binned target id
    int32_t sub = 0;     // push launch shape the slices were sized for
    int32_t groups = 0;
    int32_t units = 0;   // units of the bin-summing kernel
};

// Most bins the binned push keeps in LDS state for (pp_graph_workspace_bytes
// sizes its tables with it).
inline int32_t push_bins_cap(int32_t n) { return (int32_t)(((int64_t)n + kPushBinW - 1) / kPushBinW) + 1; }
inline int32_t push_units_cap(int32_t n, int64_t nnz) {
    return (int32_t)std::min<int64_t>(kPushBinUnits, nnz / kPushBinMinUnit + 1) + push_bins_cap(n);
}

// Work decomposition of one binned sweep launch: every bin owns a contiguous
// range of work units; heavy bins come first so the longest rows start first.
struct BinPlan {
    int32_t count[PP_NUM_BINS] = {};         // vertices per bin
    int32_t list_off[PP_NUM_BINS + 1] = {};  // start of each bin in the vertex list
    int32_t block_off[PP_NUM_BINS + 1] = {}; // first work unit of each bin (launch order)
    int32_t split_chunks = 0;                // units used by bin 5
    int32_t total_blocks = 0;
    // the same work cut into wavefront-sized units (bins 3 and 4: one row per
    // wavefront; bin 5: one chunk per wavefront), heaviest bin first
    int32_t wave_off[PP_NUM_BINS + 1] = {};
    int32_t total_wave_units = 0;
};

struct GraphDev {
    int32_t n;
    int64_t nnz;
    // Adjacency arrays the kernels walk: the caller's, or the relabelled copy.
    const int32_t* csr_off;
    const int32_t* csr_idx;
    const int32_t* csc_off;
    const int32_t* csc_idx;
    const float* csr_w;       // weights in CSR slot order (nullable)
    float* csc_w;             // weights in CSC slot order (workspace; nullable)
    // Degree-ordered relabelling (both NULL when off): internal vertex i is
    // caller vertex perm[i]; caller vertex v is internal vertex iperm[v].
    const int32_t* perm;
    const int32_t* iperm;
    // The caller's arrays, as given.
    const int32_t* user_csr_off;
    const int32_t* user_csr_idx;
    const int32_t* user_csc_off;
    const int32_t* user_csc_idx;
    const int32_t* user_csc_to_csr;  // weighted: CSR slot of each caller CSC slot
    bool aliased;             // CSC given as the CSR arrays (symmetric graph)
    int32_t* csc_row;         // the row (in-row owner) of every CSC slot
    float* inv_s;             // 1/d(v) or 1/s(v); 0 when nothing leaves v
    int32_t* out_deg;         // d(v)
    int32_t* pull_list;       // vertices grouped by in-degree bin
    int32_t* push_list;       // vertices grouped by out-degree bin
    int32_t* split_tab;       // bin-5 chunk tables (pull, then push)
    float* split_part;        // bin-5 partial sums (pull)
    float* hot_part;          // push privatisation partials [push_blocks][hot]
    // binned push: per (workgroup, bin) slice start and size (pairs), pairs
    // written by the last sweep, second-kernel units (bin, first and end
    // workgroup), first unit of each bin [nbins+1], the pairs, unit partials
    int32_t* pb_base;
    int32_t* pb_cnt;
    int32_t* pb_fill;
    int32_t* pb_units;
    int32_t* pb_ulo;
    int2* pb_pairs;
    float* pb_part;
    float* buf0;              // PageRank scratch vectors, n floats each
    float* buf1;
    float* buf2;
    int32_t* err;             // device error word / counters
    // tiled pull (SlicePlan): 16-bit sources, the row of every unit segment,
    // work units, per-workgroup slice runs [groups+1 firsts], partial sums
    // [S*R] (zero where a segment is empty or chunked), chunk partials and
    // each row's first chunk [R+1]
    uint16_t* sl_idx;
    int32_t* sl_prow;
    SliceUnit* sl_units;
    SliceSeg* sl_segs;
    int32_t* sl_wg;
    float* sl_part;
    float* sl_cpart;
    int32_t* sl_cbeg;
};

// Caller id of internal vertex i.
__device__ __forceinline__ int32_t user_id(const int32_t* perm, int32_t i) { return perm ? perm[i] : i; }

}  // namespace pp

struct pp_graph_s {
    pp::GraphDev d;
    uint32_t flags;
    bool weighted;
    bool relabelled;
    pp::BinPlan pull_plan;
    pp::BinPlan push_plan;
    pp::SlicePlan slices;
    pp::PushBins pbins;
    int32_t split_pull_entries;  // rows of the pull split table
    int32_t split_push_entries;
    int32_t split_cap;           // capacity of each split table
    int32_t max_out_deg;
    int32_t max_in_deg;
    // every vertex with an in-edge lies below this id (after degree
    // relabelling, the vertices without in-edges form the tail of the ids)
    int32_t in_active;
    int32_t num_cu;              // compute units of the device the graph lives on
    int32_t max_lds;             // LDS bytes one workgroup may allocate
    int32_t lds_per_cu;          // LDS bytes of one compute unit
    pp::Tuning tune;
    // Instantiated HIP graphs of BFS level batches, keyed by their arguments
    // (released by pp_graph_destroy).
    struct BfsGraph {
        const void* state;
        const int32_t* level;
        const int32_t* parent;
        int32_t policy;
        float alpha, beta;
        int32_t batch;
        const void* log;
        int32_t log_cap;
        hipGraphExec_t exec;
        hipGraph_t graph;
    };
    std::vector<BfsGraph> bfs_graphs;
    // pinned host buffer a BFS run reads its state header into (a copy to
    // pageable memory goes through a staging buffer: slower per run)
    static constexpr size_t kBfsHdrHost = 4096;
    void* bfs_hdr_host = nullptr;
    void* bfs_hdrs_host = nullptr;  // pinned headers of pp_bfs_run_many (grown on demand)
    size_t bfs_hdrs_cap = 0;
    // level-kernel launches that found a frontier, per policy, over the last
    // kBfsHist runs on this graph (their maximum sizes a run's first batch)
    static constexpr int kBfsHist = 64;
    int32_t bfs_hist[3][kBfsHist] = {};
    int32_t bfs_hist_pos[3] = {};
    ~pp_graph_s() {
        for (auto& e : bfs_graphs) {
            (void)hipGraphExecDestroy(e.exec);
            (void)hipGraphDestroy(e.graph);
        }
        if (bfs_hdr_host) (void)hipHostFree(bfs_hdr_host);
        if (bfs_hdrs_host) (void)hipHostFree(bfs_hdrs_host);
    }
};

namespace pp {

// Teleport term and output layout of a pull sweep: y[u] = base + [u == vertex]
// * extra + f * (gathered sum), written to y[caller id * y_stride].  PageRank:
// base (1-f)/n, no vertex; one personalised column of an n x k matrix: base
// 0, vertex the source, extra 1-f, stride k.
struct Teleport {
    float base;
    int32_t vertex;  // internal id, -1: none
    float extra;
    int64_t y_stride;
};
Teleport uniform_teleport(int32_t n, float f);

// Pull and push sweeps of one vector (pr.hip).  c: contributions (internal
// ids); pull writes the next contributions and/or y; push accumulates into y
// (internal ids, pre-set to the teleport).
pp_status launch_pull(pp_graph g, const float* c, float* c_next, float* y, float f, hipStream_t st,
                      int32_t skip_below = 0, const Teleport* tp = nullptr);
pp_status launch_push(pp_graph g, const float* c, float* y, hipStream_t st);
// Sizes the binned push's slices (registration; sets g->pbins).
pp_status build_push_bins(pp_graph g, hipStream_t st);
// One personalised PageRank column with the single-vector sweeps (pr.hip):
// x_0 = e_s (s internal), iters steps, x written to x_out[caller id * x_stride].
pp_status run_single_ppr(pp_graph g, pp_dir dir, int32_t s, int32_t iters, float f, float* x_out, int64_t x_stride,
                         hipStream_t st);

pp_status set_error(pp_status s, const std::string& msg);
pp_status hip_error(hipError_t e, const char* what);
void clear_error();

// Lets kernel `fn` take `bytes` of dynamic LDS beyond the default 64 KiB on
// the current device.  The attribute is raised once per kernel and device
// (to the largest size asked for so far), so launch loops pay for it once.
void allow_dynamic_lds(const void* fn, size_t bytes);

#define PP_HIP(call)                                             \
    do {                                                         \
        hipError_t _e = (call);                                  \
        if (_e != hipSuccess) return ::pp::hip_error(_e, #call); \
    } while (0)

#define PP_LAUNCH_CHECK(what)                                    \
    do {                                                         \
        hipError_t _e = hipGetLastError();                       \
        if (_e != hipSuccess) return ::pp::hip_error(_e, what);  \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline int32_t ceil_div(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

}  // namespace pp
