// Graph registration: error state, workspace layout, device-derived degree
// data and the degree-binned vertex lists the sweeps are launched over.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "pp_common.h"

namespace pp {

static thread_local std::string g_last_error;

pp_status set_error(pp_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

pp_status hip_error(hipError_t e, const char* what) {
    g_last_error = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    return PP_E_HIP;
}

void clear_error() { g_last_error.clear(); }

Tuning& tuning() {
    static Tuning t;
    return t;
}

pp_status check_graph_handle(pp_graph g) {
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    return PP_OK;
}

// ------------------------------------------------------------------ kernels
// Degree of v in an adjacency array.
__device__ __forceinline__ int32_t row_len(const int32_t* off, int32_t v) { return off[v + 1] - off[v]; }

struct BinBounds {
    int32_t upper[PP_NUM_BINS - 1];
};

__device__ __forceinline__ int bin_of(int32_t d, const BinBounds& bb) {
    int b = 0;
#pragma unroll
    for (int i = 0; i < PP_NUM_BINS - 1; ++i) b += (d > bb.upper[i]);
    return b;
}

// d(v), and the reciprocal of d(v) (or of the out-strength s(v) when
// weighted).  Vertices with nothing leaving them get 0: they pass no mass on.
__global__ void k_degrees(int32_t n, const int32_t* __restrict__ csr_off, const float* __restrict__ csr_w,
                          int32_t* __restrict__ out_deg, float* __restrict__ inv_s) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t b = csr_off[v], e = csr_off[v + 1];
    out_deg[v] = e - b;
    float r = 0.f;
    if (csr_w) {
        double s = 0.0;  // once per graph: accumulate the strength in double
        for (int32_t j = b; j < e; ++j) s += (double)csr_w[j];
        r = s > 0.0 ? (float)(1.0 / s) : 0.f;
    } else {
        r = (e > b) ? 1.0f / (float)(e - b) : 0.f;
    }
    inv_s[v] = r;
}

// Weights gathered into CSC slot order: csc_w[j] = csr_w[csc_to_csr[j]].
__global__ void k_gather_weights(int64_t nnz, const float* __restrict__ csr_w, const int32_t* __restrict__ map,
                                 float* __restrict__ csc_w) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nnz) csc_w[j] = csr_w[map[j]];
}

// Stable partition of the vertices by degree bin: per-tile counts ...
constexpr int kTile = 256;

__global__ __launch_bounds__(kTile) void k_bin_count(int32_t n, const int32_t* __restrict__ off, BinBounds bb,
                                                     int32_t* __restrict__ tile_counts) {
    __shared__ int32_t cnt[PP_NUM_BINS];
    if (threadIdx.x < PP_NUM_BINS) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int32_t v = blockIdx.x * kTile + threadIdx.x;
    const int b = (v < n) ? bin_of(row_len(off, v), bb) : -1;
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int i = 0; i < PP_NUM_BINS; ++i) {
        const uint64_t m = __ballot(b == i);
        if (lane == 0 && m) atomicAdd(&cnt[i], __popcll(m));
    }
    __syncthreads();
    if (threadIdx.x < PP_NUM_BINS) tile_counts[blockIdx.x * PP_NUM_BINS + threadIdx.x] = cnt[threadIdx.x];
}

// ... an exclusive scan of the tile counts, bin-major (one workgroup) ...
__global__ __launch_bounds__(1024) void k_bin_scan(int32_t tiles, int32_t* __restrict__ tile_counts,
                                                   int32_t* __restrict__ totals) {
    __shared__ int32_t part[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int per = (tiles + 1023) / 1024;
    for (int b = 0; b < PP_NUM_BINS; ++b) {
        const int t0 = threadIdx.x * per;
        int32_t s = 0;
        for (int t = t0; t < t0 + per && t < tiles; ++t) s += tile_counts[t * PP_NUM_BINS + b];
        part[threadIdx.x] = s;
        __syncthreads();
        // Hillis-Steele inclusive scan over 1024 partial sums
        for (int d = 1; d < 1024; d <<= 1) {
            int32_t add = (threadIdx.x >= d) ? part[threadIdx.x - d] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        int32_t run = carry + part[threadIdx.x] - s;  // exclusive prefix of this thread's range
        for (int t = t0; t < t0 + per && t < tiles; ++t) {
            const int32_t c = tile_counts[t * PP_NUM_BINS + b];
            tile_counts[t * PP_NUM_BINS + b] = run;
            run += c;
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            totals[b] = part[1023];
            carry += part[1023];
        }
        __syncthreads();
    }
}

// ... and a scatter that keeps vertex order inside each bin.
__global__ __launch_bounds__(kTile) void k_bin_scatter(int32_t n, const int32_t* __restrict__ off, BinBounds bb,
                                                       const int32_t* __restrict__ tile_base,
                                                       int32_t* __restrict__ list) {
    __shared__ int32_t wave_cnt[kTile / kWave][PP_NUM_BINS];
    const int32_t v = blockIdx.x * kTile + threadIdx.x;
    const int b = (v < n) ? bin_of(row_len(off, v), bb) : -1;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    int rank = 0;
#pragma unroll
    for (int i = 0; i < PP_NUM_BINS; ++i) {
        const uint64_t m = __ballot(b == i);
        if (b == i) rank = __popcll(m & below);
        if (lane == 0) wave_cnt[w][i] = __popcll(m);
    }
    __syncthreads();
    if (b >= 0) {
        int pos = tile_base[blockIdx.x * PP_NUM_BINS + b] + rank;
        for (int ww = 0; ww < w; ++ww) pos += wave_cnt[ww][b];
        list[pos] = v;
    }
}

// Validation of one adjacency array: err[0] counts bad offsets, err[1] bad
// indices.
__global__ void k_check_offsets(int32_t n, int64_t nnz, const int32_t* __restrict__ off, int32_t* __restrict__ err) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    bool bad = false;
    if (v == 0) bad = off[0] != 0;
    else bad = off[v] < off[v - 1];
    if (v == n) bad = bad || ((int64_t)off[n] != nnz);
    if (bad) atomicAdd(&err[0], 1);
}

__global__ void k_check_indices(int32_t n, int64_t nnz, const int32_t* __restrict__ idx, int32_t* __restrict__ err) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nnz) return;
    const int32_t u = idx[j];
    if (u < 0 || u >= n) atomicAdd(&err[1], 1);
}

// ------------------------------------------------------------------ host side
struct WsLayout {
    size_t inv_s, out_deg, pull_list, push_list, buf0, buf1, buf2, csc_w, split_tab, split_part, err, tiles,
        total;
    int32_t split_cap;
};

static int32_t split_capacity(int64_t nnz, const Tuning& t) {
    int64_t cap = (nnz + t.split_chunk - 1) / t.split_chunk + nnz / ((int64_t)t.upper[PP_NUM_BINS - 2] + 1) + 1;
    return (int32_t)std::min<int64_t>(cap, INT32_MAX / 4);
}

static WsLayout layout(int32_t n, int64_t nnz, uint32_t flags, const Tuning& t) {
    WsLayout L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p = align_up(p + bytes, 256);
        return at;
    };
    const size_t nn = (size_t)n;
    L.split_cap = split_capacity(nnz, t);
    L.inv_s = take(nn * 4);
    L.out_deg = take(nn * 4);
    L.pull_list = take(nn * 4);
    L.push_list = take(nn * 4);
    L.buf0 = take(nn * 4);
    L.buf1 = take(nn * 4);
    L.buf2 = take(nn * 4);
    L.csc_w = (flags & PP_GRAPH_WEIGHTED) ? take((size_t)nnz * 4) : 0;
    // split table: per entry (vertex, begin, end) + per split vertex first entry, for pull and push
    L.split_tab = take((size_t)2 * (3 * (size_t)L.split_cap + (size_t)L.split_cap + 1) * 4);
    L.split_part = take((size_t)L.split_cap * 4);
    L.err = take(64 * 4);
    L.tiles = take(((size_t)ceil_div(n, kTile) + 1) * PP_NUM_BINS * 4);
    L.total = p;
    return L;
}

static void make_plan(BinPlan& p, const int32_t* counts, int32_t split_chunks) {
    p.list_off[0] = 0;
    for (int b = 0; b < PP_NUM_BINS; ++b) {
        p.count[b] = counts[b];
        p.list_off[b + 1] = p.list_off[b] + counts[b];
    }
    p.split_chunks = split_chunks;
    // launch order: bin 5 (chunks), 4, 3, 2, 1, 0; block_off indexed by bin
    int32_t blocks[PP_NUM_BINS];
    blocks[5] = split_chunks;
    blocks[4] = counts[4];
    for (int b = 0; b < 4; ++b) blocks[b] = ceil_div(counts[b], kBlock / kBinLanes[b]);
    int32_t at = 0;
    for (int b = PP_NUM_BINS - 1; b >= 0; --b) {
        p.block_off[b] = at;
        at += blocks[b];
    }
    p.block_off[PP_NUM_BINS] = at;  // unused sentinel
    p.total_blocks = at;
}

}  // namespace pp

using namespace pp;

PP_EXPORT int pp_abi_version(void) { return PP_ABI_VERSION; }

PP_EXPORT const char* pp_last_error(void) { return g_last_error.c_str(); }

PP_EXPORT size_t pp_graph_workspace_bytes(int32_t n, int64_t nnz, uint32_t flags) {
    if (n < 1 || nnz < 0 || nnz > INT32_MAX) return 0;
    return layout(n, nnz, flags, tuning()).total;
}

PP_EXPORT pp_status pp_set_bin_thresholds(const int32_t* upper5, int32_t split_chunk) {
    if (!upper5) return set_error(PP_E_NULL, "upper5 is NULL");
    for (int i = 0; i < PP_NUM_BINS - 1; ++i) {
        if (upper5[i] < 0 || (i > 0 && upper5[i] < upper5[i - 1]))
            return set_error(PP_E_RANGE, "bin thresholds must be non-negative and non-decreasing");
    }
    if (split_chunk < kBlock) return set_error(PP_E_RANGE, "split_chunk must be at least 256");
    for (int i = 0; i < PP_NUM_BINS - 1; ++i) tuning().upper[i] = upper5[i];
    tuning().split_chunk = split_chunk;
    return PP_OK;
}

namespace pp {
static pp_status bins_for(pp_graph g, const int32_t* off, int32_t* list, int32_t* tab, int32_t split_cap,
                          int32_t* tile_counts, BinPlan& plan, int32_t& entries, hipStream_t st) {
    const int32_t n = g->d.n;
    const int32_t tiles = ceil_div(n, kTile);
    BinBounds bb;
    for (int i = 0; i < PP_NUM_BINS - 1; ++i) bb.upper[i] = g->tune.upper[i];
    int32_t* totals = g->d.err + 8;
    hipLaunchKernelGGL(k_bin_count, dim3(tiles), dim3(kTile), 0, st, n, off, bb, tile_counts);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, tiles, tile_counts, totals);
    hipLaunchKernelGGL(k_bin_scatter, dim3(tiles), dim3(kTile), 0, st, n, off, bb, tile_counts, list);
    PP_LAUNCH_CHECK("degree binning");
    int32_t counts[PP_NUM_BINS];
    PP_HIP(hipMemcpyAsync(counts, totals, sizeof(counts), hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    // bin 5: split every row into chunks of split_chunk edges (host-built table)
    const int32_t n5 = counts[5];
    std::vector<int32_t> verts(n5), offs((size_t)2 * n5);
    if (n5 > 0) {
        const int32_t start5 = n - n5;  // bin 5 is last in the list
        std::vector<int32_t> all_off((size_t)n + 1);
        PP_HIP(hipMemcpyAsync(verts.data(), list + start5, sizeof(int32_t) * n5, hipMemcpyDeviceToHost, st));
        PP_HIP(hipMemcpyAsync(all_off.data(), off, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, st));
        PP_HIP(hipStreamSynchronize(st));
        for (int32_t i = 0; i < n5; ++i) {
            offs[2 * i] = all_off[verts[i]];
            offs[2 * i + 1] = all_off[verts[i] + 1];
        }
    }
    std::vector<int32_t> ev, eb, ee, first;
    first.reserve(n5 + 1);
    const int32_t chunk = g->tune.split_chunk;
    for (int32_t i = 0; i < n5; ++i) {
        first.push_back((int32_t)ev.size());
        for (int64_t b = offs[2 * i]; b < offs[2 * i + 1]; b += chunk) {
            ev.push_back(verts[i]);
            eb.push_back((int32_t)b);
            ee.push_back((int32_t)std::min<int64_t>(b + chunk, offs[2 * i + 1]));
        }
    }
    first.push_back((int32_t)ev.size());
    entries = (int32_t)ev.size();
    if (entries > split_cap) return set_error(PP_E_WORKSPACE, "split table exceeds its capacity");
    // table layout: v[cap] | begin[cap] | end[cap] | first[cap+1]
    if (entries > 0) {
        PP_HIP(hipMemcpyAsync(tab, ev.data(), entries * 4, hipMemcpyHostToDevice, st));
        PP_HIP(hipMemcpyAsync(tab + split_cap, eb.data(), entries * 4, hipMemcpyHostToDevice, st));
        PP_HIP(hipMemcpyAsync(tab + 2 * (size_t)split_cap, ee.data(), entries * 4, hipMemcpyHostToDevice, st));
    }
    PP_HIP(hipMemcpyAsync(tab + 3 * (size_t)split_cap, first.data(), first.size() * 4, hipMemcpyHostToDevice, st));
    PP_HIP(hipStreamSynchronize(st));
    make_plan(plan, counts, entries);
    return PP_OK;
}
}  // namespace pp

PP_EXPORT pp_status pp_graph_check(pp_graph g, void* stream);

PP_EXPORT pp_status pp_graph_create(int32_t n, int64_t nnz, const int32_t* csr_off, const int32_t* csr_idx,
                                    const int32_t* csc_off, const int32_t* csc_idx, const float* csr_w,
                                    const int32_t* csc_to_csr, uint32_t flags, void* ws, size_t ws_bytes,
                                    void* stream, pp_graph* out) {
    clear_error();
    if (!out) return set_error(PP_E_NULL, "out handle pointer is NULL");
    *out = nullptr;
    if (n < 1) return set_error(PP_E_SIZE, "n must be >= 1");
    if (nnz < 0 || nnz > INT32_MAX) return set_error(PP_E_SIZE, "nnz must be in [0, 2^31-1]");
    if (!csr_off || !csc_off || !ws) return set_error(PP_E_NULL, "csr_off, csc_off and ws are required");
    if (nnz > 0 && (!csr_idx || !csc_idx)) return set_error(PP_E_NULL, "csr_idx and csc_idx are required when nnz > 0");
    const bool weighted = (flags & PP_GRAPH_WEIGHTED) != 0;
    if (weighted && nnz > 0 && (!csr_w || !csc_to_csr))
        return set_error(PP_E_NULL, "weighted graph needs csr_w and csc_to_csr");
    if (flags & ~PP_GRAPH_WEIGHTED) return set_error(PP_E_UNSUPPORTED, "unknown graph flag");
    const Tuning t = tuning();
    const WsLayout L = layout(n, nnz, flags, t);
    if (ws_bytes < L.total) return set_error(PP_E_WORKSPACE, "graph workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return set_error(PP_E_RANGE, "workspace must be 256-byte aligned");

    pp_graph g = new (std::nothrow) pp_graph_s();
    if (!g) return set_error(PP_E_SIZE, "host allocation of the graph handle failed");
    g->flags = flags;
    g->weighted = weighted;
    g->tune = t;
    char* base = static_cast<char*>(ws);
    GraphDev& d = g->d;
    d.n = n;
    d.nnz = nnz;
    d.csr_off = csr_off;
    d.csr_idx = csr_idx;
    d.csc_off = csc_off;
    d.csc_idx = csc_idx;
    d.csr_w = weighted ? csr_w : nullptr;
    d.inv_s = reinterpret_cast<float*>(base + L.inv_s);
    d.out_deg = reinterpret_cast<int32_t*>(base + L.out_deg);
    d.pull_list = reinterpret_cast<int32_t*>(base + L.pull_list);
    d.push_list = reinterpret_cast<int32_t*>(base + L.push_list);
    d.buf0 = reinterpret_cast<float*>(base + L.buf0);
    d.buf1 = reinterpret_cast<float*>(base + L.buf1);
    d.buf2 = reinterpret_cast<float*>(base + L.buf2);
    d.csc_w = weighted ? reinterpret_cast<float*>(base + L.csc_w) : nullptr;
    d.split_tab = reinterpret_cast<int32_t*>(base + L.split_tab);
    d.split_part = reinterpret_cast<float*>(base + L.split_part);
    d.err = reinterpret_cast<int32_t*>(base + L.err);
    int32_t* tile_counts = reinterpret_cast<int32_t*>(base + L.tiles);
    hipStream_t st = static_cast<hipStream_t>(stream);

    auto fail = [&](pp_status s) {
        delete g;
        return s;
    };
    {
        // The sweeps trust the arrays, so malformed ones are rejected here.
        pp_status s = pp_graph_check(g, stream);
        if (s != PP_OK) return fail(s);
    }
    hipLaunchKernelGGL(k_degrees, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, csr_off, d.csr_w, d.out_deg, d.inv_s);
    if (weighted && nnz > 0)
        hipLaunchKernelGGL(k_gather_weights, dim3(ceil_div(nnz, 256)), dim3(256), 0, st, nnz, csr_w, csc_to_csr,
                           d.csc_w);
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(hip_error(e, "graph degree kernels"));
    }
    const int32_t cap = L.split_cap;
    g->split_cap = cap;
    int32_t* tab_pull = d.split_tab;
    int32_t* tab_push = d.split_tab + 4 * (size_t)cap + 1;
    pp_status s = bins_for(g, csc_off, d.pull_list, tab_pull, cap, tile_counts, g->pull_plan, g->split_pull_entries, st);
    if (s != PP_OK) return fail(s);
    s = bins_for(g, csr_off, d.push_list, tab_push, cap, tile_counts, g->push_plan, g->split_push_entries, st);
    if (s != PP_OK) return fail(s);
    *out = g;
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_destroy(pp_graph g) {
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    delete g;
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_bins(pp_graph g, pp_dir dir, int32_t* counts) {
    if (!g || !counts) return set_error(PP_E_NULL, "graph or counts is NULL");
    const BinPlan& p = (dir == PP_PUSH) ? g->push_plan : g->pull_plan;
    if (dir != PP_PUSH && dir != PP_PULL) return set_error(PP_E_RANGE, "dir must be PP_PUSH or PP_PULL");
    for (int b = 0; b < PP_NUM_BINS; ++b) counts[b] = p.count[b];
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_check(pp_graph g, void* stream) {
    clear_error();
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const GraphDev& d = g->d;
    int32_t h[4] = {0, 0, 0, 0};
    for (int pass = 0; pass < 2; ++pass) {
        const int32_t* off = pass ? d.csc_off : d.csr_off;
        const int32_t* idx = pass ? d.csc_idx : d.csr_idx;
        PP_HIP(hipMemsetAsync(d.err, 0, 2 * sizeof(int32_t), st));
        hipLaunchKernelGGL(k_check_offsets, dim3(ceil_div((int64_t)d.n + 1, 256)), dim3(256), 0, st, d.n, d.nnz, off,
                           d.err);
        if (d.nnz > 0)
            hipLaunchKernelGGL(k_check_indices, dim3(ceil_div(d.nnz, 256)), dim3(256), 0, st, d.n, d.nnz, idx, d.err);
        PP_LAUNCH_CHECK("graph check");
        PP_HIP(hipMemcpyAsync(h + 2 * pass, d.err, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        PP_HIP(hipStreamSynchronize(st));
    }
    if (h[0] || h[2]) return set_error(PP_E_GRAPH, "offsets are not monotone from 0 to nnz");
    if (h[1] || h[3]) return set_error(PP_E_GRAPH, "an index lies outside [0, n)");
    return PP_OK;
}
