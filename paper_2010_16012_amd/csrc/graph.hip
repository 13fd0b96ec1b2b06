// Graph registration: error state, workspace layout, validation, the
// optional degree-ordered relabelling, device-derived degree data and the
// degree-binned vertex lists the sweeps are launched over.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <utility>
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

void allow_dynamic_lds(const void* fn, size_t bytes) {
    if (bytes <= 65536) return;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> done;  // (kernel, device) -> bytes allowed
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;  // the launch will report the error
    std::lock_guard<std::mutex> lock(mu);
    size_t& have = done[{fn, dev}];
    if (have >= bytes) return;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess) have = bytes;
}

Tuning& tuning() {
    static Tuning t;
    return t;
}

// ------------------------------------------------------------------ kernels
constexpr int kTile = 256;      // vertices per partition tile
constexpr int kMaxKeys = 32;    // partition keys are 0..31
constexpr int kScanTile = 1024; // elements per scan tile

__device__ __forceinline__ int32_t row_len(const int32_t* off, int32_t v) { return off[v + 1] - off[v]; }

// Degree bin of every vertex (keys for the bin partition).
struct BinBounds {
    int32_t upper[PP_NUM_BINS - 1];
};

__global__ void k_bin_keys(int32_t n, const int32_t* __restrict__ off, BinBounds bb, uint8_t* __restrict__ key) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t d = row_len(off, v);
    int b = 0;
#pragma unroll
    for (int i = 0; i < PP_NUM_BINS - 1; ++i) b += (d > bb.upper[i]);
    key[v] = (uint8_t)b;
}

// Relabel key: heaviest vertices first, by floor(log2(d_out + d_in + 1)).
__global__ void k_relabel_keys(int32_t n, const int32_t* __restrict__ off, const int32_t* __restrict__ in_off,
                               uint8_t* __restrict__ key) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint32_t d = (uint32_t)row_len(off, v) + (uint32_t)row_len(in_off, v) + 1u;
    key[v] = (uint8_t)(__clz(d));  // 31 - floor(log2 d): larger degree -> smaller key
}

// Stable partition of 0..n-1 by key: per-tile counts ...
__global__ __launch_bounds__(kTile) void k_part_count(int32_t n, int nkeys, const uint8_t* __restrict__ key,
                                                      int32_t* __restrict__ tile_counts) {
    __shared__ int32_t cnt[kMaxKeys];
    if (threadIdx.x < kMaxKeys) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int32_t v = blockIdx.x * kTile + threadIdx.x;
    const int b = (v < n) ? key[v] : -1;
    const int lane = threadIdx.x & (kWave - 1);
    for (int i = 0; i < nkeys; ++i) {
        const uint64_t m = __ballot(b == i);
        if (lane == 0 && m) atomicAdd(&cnt[i], __popcll(m));
    }
    __syncthreads();
    if (threadIdx.x < nkeys) tile_counts[blockIdx.x * nkeys + threadIdx.x] = cnt[threadIdx.x];
}

// ... an exclusive scan of the tile counts, key-major (one workgroup) ...
__global__ __launch_bounds__(1024) void k_part_scan(int32_t tiles, int nkeys, int32_t* __restrict__ tile_counts,
                                                    int32_t* __restrict__ totals) {
    __shared__ int32_t part[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int per = (tiles + 1023) / 1024;
    for (int b = 0; b < nkeys; ++b) {
        const int t0 = threadIdx.x * per;
        int32_t s = 0;
        for (int t = t0; t < t0 + per && t < tiles; ++t) s += tile_counts[t * nkeys + b];
        part[threadIdx.x] = s;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            int32_t add = (threadIdx.x >= d) ? part[threadIdx.x - d] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        int32_t run = carry + part[threadIdx.x] - s;
        for (int t = t0; t < t0 + per && t < tiles; ++t) {
            const int32_t c = tile_counts[t * nkeys + b];
            tile_counts[t * nkeys + b] = run;
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

// ... and a scatter that keeps vertex order within each key.
__global__ __launch_bounds__(kTile) void k_part_scatter(int32_t n, int nkeys, const uint8_t* __restrict__ key,
                                                        const int32_t* __restrict__ tile_base,
                                                        int32_t* __restrict__ list) {
    __shared__ int32_t wave_cnt[kTile / kWave][kMaxKeys];
    const int32_t v = blockIdx.x * kTile + threadIdx.x;
    const int b = (v < n) ? key[v] : -1;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    int rank = 0;
    for (int i = 0; i < nkeys; ++i) {
        const uint64_t m = __ballot(b == i);
        if (b == i) rank = __popcll(m & below);
        if (lane == 0) wave_cnt[w][i] = __popcll(m);
    }
    __syncthreads();
    if (b >= 0) {
        int pos = tile_base[blockIdx.x * nkeys + b] + rank;
        for (int ww = 0; ww < w; ++ww) pos += wave_cnt[ww][b];
        list[pos] = v;
    }
}

// Exclusive scan of n int32 values into out[0..n] (out[n] = total):
// per-tile scans ...
__global__ __launch_bounds__(256) void k_scan_tiles(int32_t n, const int32_t* __restrict__ in,
                                                    int32_t* __restrict__ out, int32_t* __restrict__ tsum) {
    __shared__ int32_t part[256];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
    int32_t v[4];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        int32_t add = (threadIdx.x >= d) ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) tsum[blockIdx.x] = part[255];
}

// ... a scan of the tile sums (one workgroup) ...
__global__ __launch_bounds__(1024) void k_scan_sums(int32_t tiles, int32_t* __restrict__ tsum,
                                                    int32_t* __restrict__ total) {
    __shared__ int32_t part[1024];
    const int per = (tiles + 1023) / 1024;
    const int t0 = threadIdx.x * per;
    int32_t s = 0;
    for (int t = t0; t < t0 + per && t < tiles; ++t) s += tsum[t];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int32_t add = (threadIdx.x >= d) ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - s;
    for (int t = t0; t < t0 + per && t < tiles; ++t) {
        const int32_t c = tsum[t];
        tsum[t] = run;
        run += c;
    }
    if (threadIdx.x == 1023) *total = part[1023];
}

// ... and the tile offsets added back.
__global__ void k_scan_add(int32_t n, int32_t* __restrict__ out, const int32_t* __restrict__ tsum,
                           const int32_t* __restrict__ total) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tsum[i / kScanTile];
    if (i == n) out[n] = *total;
}

__global__ void k_invert_perm(int32_t n, const int32_t* __restrict__ perm, int32_t* __restrict__ iperm) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) iperm[perm[i]] = i;
}

__global__ void k_perm_degrees(int32_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ off,
                               int32_t* __restrict__ deg) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) deg[i] = row_len(off, perm[i]);
}

// Row i of the relabelled array is row perm[i] of the caller's array with
// every neighbour renamed (stored order kept).  Optional weights follow their
// slots: wsrc is indexed by slot, or by map[slot] when map is given.
__global__ __launch_bounds__(256) void k_relabel_rows(int32_t n, const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ iperm,
                                                      const int32_t* __restrict__ off, const int32_t* __restrict__ idx,
                                                      const int32_t* __restrict__ off_new, int32_t* __restrict__ idx_new,
                                                      const float* __restrict__ wsrc, const int32_t* __restrict__ map,
                                                      float* __restrict__ w_new) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t nw = gridDim.x * (blockDim.x / kWave);
    for (int32_t i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < n; i += nw) {
        const int32_t v = perm[i];
        const int32_t b = off[v], e = off[v + 1], o = off_new[i];
        for (int32_t j = b + lane; j < e; j += kWave) {
            if (idx_new) idx_new[o + (j - b)] = iperm[idx[j]];
            if (w_new) w_new[o + (j - b)] = map ? wsrc[map[j]] : wsrc[j];
        }
    }
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

// Largest out- and in-row length.
__global__ void k_max_deg(int32_t n, const int32_t* __restrict__ off, const int32_t* __restrict__ in_off,
                          int32_t* __restrict__ out) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t a = 0, b = 0, c = 0;  // c: v + 1 for a vertex with in-edges
    if (v < n) {
        a = row_len(off, v);
        b = row_len(in_off, v);
        c = (b > 0) ? v + 1 : 0;
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
        a = max(a, __shfl_xor(a, s));
        b = max(b, __shfl_xor(b, s));
        c = max(c, __shfl_xor(c, s));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&out[0], a);
        atomicMax(&out[1], b);
        atomicMax(&out[2], c);
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

// row[j] = v for every slot j of the row of v (rows of more than 64 slots
// are written by the whole wavefront).
__global__ void k_row_owner(int32_t n, const int32_t* off, int32_t* row) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gw = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
    const int32_t nw = (int32_t)(gridDim.x * blockDim.x / kWave);
    for (int32_t base = gw * kWave; base < n; base += nw * kWave) {
        const int32_t v = base + lane;
        const int32_t b = v < n ? off[v] : 0, e = v < n ? off[v + 1] : 0;
        const bool longrow = e - b > kWave;
        if (!longrow)
            for (int32_t j = b; j < e; ++j) row[j] = v;
        uint64_t m = __ballot(longrow);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int32_t lb = __shfl(b, src), le = __shfl(e, src);
            for (int32_t j = lb + lane; j < le; j += kWave) row[j] = base + src;
        }
    }
}

__global__ void k_zero_i32(int32_t n, int32_t* p) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ------------------------------------------------------------------ host side
struct WsLayout {
    size_t inv_s, out_deg, pull_list, push_list, buf0, buf1, buf2, csc_w, csc_row, split_tab, split_part, hot_part, err,
        tiles, keys, perm, iperm, r_csr_off, r_csc_off, r_csr_idx, r_csc_idx, r_csr_w, sl_idx, sl_prow,
        sl_units, sl_segs, sl_wg, sl_part, sl_cpart, sl_cbeg, pb_base, pb_cnt, pb_fill, pb_units, pb_ulo, pb_pairs,
        pb_part, total;
    int32_t split_cap;
    int64_t sl_rows_cap, sl_slices_cap, sl_pairs_cap, sl_units_cap, sl_chunks_cap, sl_idx_cap;
};

// Tiled pull: rows qualify while their in-degree is at least
// max(kTileMinDeg, S/2) (the partial sums cost 8 bytes per slice and row).
constexpr int32_t kTileMinDeg = 16;
constexpr int32_t kTileMaxGroups = 4096;

static bool sliced_layout(uint32_t flags, const Tuning& t) {
    return (flags & PP_GRAPH_RELABEL) && !(flags & PP_GRAPH_WEIGHTED) && t.slice_rows > 0 && t.slice_width > 0;
}

// The binned push needs privatised targets (its bins start past them).
static bool push_binned(const Tuning& t, int32_t n) { return t.push_bins && t.hot > 0 && n > t.hot; }

static int32_t split_capacity(int64_t nnz, const Tuning& t) {
    int64_t cap = (nnz + t.split_chunk - 1) / t.split_chunk + nnz / ((int64_t)t.upper[PP_NUM_BINS - 2] + 1) + 1;
    return (int32_t)std::min<int64_t>(cap, INT32_MAX / 4);
}

// `aliased`: the caller passes one array pair for CSR and CSC (symmetric graph).
static WsLayout layout(int32_t n, int64_t nnz, uint32_t flags, const Tuning& t, bool aliased) {
    WsLayout L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p = align_up(p + bytes, 256);
        return at;
    };
    const size_t nn = (size_t)n;
    const bool relabel = (flags & PP_GRAPH_RELABEL) != 0;
    const bool weighted = (flags & PP_GRAPH_WEIGHTED) != 0;
    const size_t nz = (size_t)std::max<int64_t>(nnz, 1);
    L.split_cap = split_capacity(nnz, t);
    L.inv_s = take(nn * 4);
    L.out_deg = take(nn * 4);
    L.pull_list = take(nn * 4);
    L.push_list = take(nn * 4);
    L.buf0 = take(nn * 4);
    L.buf1 = take(nn * 4);
    L.buf2 = take(nn * 4);
    L.csc_w = weighted ? take(nz * 4) : 0;
    L.csc_row = take(nz * 4);
    // split tables: per entry (vertex, begin, end) + per split vertex first entry, for pull and push
    L.split_tab = take((size_t)2 * (4 * (size_t)L.split_cap + 1) * 4);
    L.split_part = take((size_t)L.split_cap * 4);
    L.hot_part = take((size_t)t.push_blocks * (size_t)std::max(t.hot, 1) * 4);
    if (push_binned(t, n)) {
        const size_t slices = (size_t)t.push_blocks * push_bins_cap(n);
        const size_t units = push_units_cap(n, nnz);
        L.pb_base = take(slices * 4);
        L.pb_cnt = take(slices * 4);
        L.pb_fill = take(slices * 4);
        L.pb_units = take(units * 3 * 4);
        L.pb_ulo = take(((size_t)push_bins_cap(n) + 1) * 4);
        L.pb_pairs = take(nz * 8);
        L.pb_part = take(units * kPushBinW * 4);
    }
    L.err = take(64 * 4);
    const size_t tiles = std::max<size_t>((size_t)ceil_div(n, kTile) * kMaxKeys, (size_t)ceil_div(n, kScanTile) + 1);
    L.tiles = take(tiles * 4);
    L.keys = take(nn);
    if (relabel) {
        L.perm = take(nn * 4);
        L.iperm = take(nn * 4);
        L.r_csr_off = take((nn + 1) * 4);
        L.r_csr_idx = take(nz * 4);
        if (!aliased) {
            L.r_csc_off = take((nn + 1) * 4);
            L.r_csc_idx = take(nz * 4);
        }
        if (weighted) L.r_csr_w = take(nz * 4);
    }
    if (sliced_layout(flags, t)) {
        // rows that qualify have at least kTileMinDeg in-edges: at most nnz / kTileMinDeg of them
        const int64_t R = std::min<int64_t>(std::min<int64_t>(t.slice_rows, n), std::max<int64_t>(nnz / kTileMinDeg, 1));
        const int64_t S = ceil_div(n, t.slice_width);
        const int64_t P = std::min<int64_t>(S * R, std::max<int64_t>(nnz, 1));
        L.sl_rows_cap = R;
        L.sl_slices_cap = S;
        L.sl_pairs_cap = P;
        L.sl_chunks_cap = 2 * (nnz / kSegChunk) + 1;
        // a unit closes when the next segment does not fit: two consecutive
        // units hold more than kUnitEdges edges or the first kUnitPairs pairs
        L.sl_units_cap = 2 * (nnz / kUnitEdges) + P / kUnitPairs + 2 * S + 8;
        // every unit and chunk starts 8-aligned; 16 spare entries past the end
        L.sl_idx_cap = nz + 8 * (L.sl_units_cap + L.sl_chunks_cap) + 16;
        L.sl_idx = take((size_t)L.sl_idx_cap * 2);
        L.sl_prow = take((size_t)P * 4);
        L.sl_units = take((size_t)(L.sl_units_cap + L.sl_chunks_cap) * sizeof(SliceUnit));
        L.sl_segs = take((size_t)(kTileMaxGroups + S) * sizeof(SliceSeg));
        L.sl_wg = take((size_t)(kTileMaxGroups + 1) * 4);
        L.sl_part = take((size_t)(S * R) * 4);
        L.sl_cpart = take((size_t)L.sl_chunks_cap * 4);
        L.sl_cbeg = take((size_t)(R + 1) * 4);
    }
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
    int32_t waves[PP_NUM_BINS];
    waves[5] = split_chunks;
    for (int b = 0; b < PP_NUM_BINS - 1; ++b) waves[b] = ceil_div(counts[b], kWave / kPullLanes[b]);
    at = 0;
    for (int b = PP_NUM_BINS - 1; b >= 0; --b) {
        p.wave_off[b] = at;
        at += waves[b];
    }
    p.wave_off[PP_NUM_BINS] = at;
    p.total_wave_units = at;
}

// Stable partition of the vertices by key (keys already computed); writes
// list[] and, when host_totals is given, the per-key totals (host).
static pp_status partition(int32_t n, int nkeys, const uint8_t* keys, int32_t* tile_counts, int32_t* dev_totals,
                           int32_t* list, int32_t* host_totals, hipStream_t st) {
    const int32_t tiles = ceil_div(n, kTile);
    hipLaunchKernelGGL(k_part_count, dim3(tiles), dim3(kTile), 0, st, n, nkeys, keys, tile_counts);
    hipLaunchKernelGGL(k_part_scan, dim3(1), dim3(1024), 0, st, tiles, nkeys, tile_counts, dev_totals);
    hipLaunchKernelGGL(k_part_scatter, dim3(tiles), dim3(kTile), 0, st, n, nkeys, keys, tile_counts, list);
    PP_LAUNCH_CHECK("vertex partition");
    if (host_totals) {
        PP_HIP(hipMemcpyAsync(host_totals, dev_totals, sizeof(int32_t) * nkeys, hipMemcpyDeviceToHost, st));
        PP_HIP(hipStreamSynchronize(st));
    }
    return PP_OK;
}

static pp_status exclusive_scan(int32_t n, const int32_t* in, int32_t* out, int32_t* tsum, int32_t* total,
                                hipStream_t st) {
    const int32_t tiles = std::max(ceil_div(n, kScanTile), 1);
    hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(256), 0, st, n, in, out, tsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, tiles, tsum, total);
    hipLaunchKernelGGL(k_scan_add, dim3(ceil_div((int64_t)n + 1, 256)), dim3(256), 0, st, n, out, tsum, total);
    PP_LAUNCH_CHECK("exclusive scan");
    return PP_OK;
}

// Degree-binned vertex list and plan for one adjacency array; for bin 5 also
// the chunk table (built on the host from the bin-5 rows).
static pp_status bins_for(pp_graph g, const int32_t* off, int32_t* list, int32_t* tab, int32_t split_cap,
                          int32_t* tile_counts, uint8_t* keys, BinPlan& plan, int32_t& entries, hipStream_t st) {
    const int32_t n = g->d.n;
    BinBounds bb;
    for (int i = 0; i < PP_NUM_BINS - 1; ++i) bb.upper[i] = g->tune.upper[i];
    hipLaunchKernelGGL(k_bin_keys, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, off, bb, keys);
    int32_t counts[PP_NUM_BINS];
    pp_status s = partition(n, PP_NUM_BINS, keys, tile_counts, g->d.err + 8, list, counts, st);
    if (s != PP_OK) return s;
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

// Runs fn(lo, hi) over [0, count) split into contiguous ranges on a few host threads.
template <typename F>
static void parallel_ranges(int64_t count, const F& fn) {
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(std::thread::hardware_concurrency(), 16));
    if (count < 4096 || nt == 1) {
        fn((int64_t)0, count);
        return;
    }
    std::vector<std::thread> th;
    for (int64_t i = 0; i < nt; ++i) th.emplace_back([&, i] { fn(count * i / nt, count * (i + 1) / nt); });
    for (auto& t : th) t.join();
}

// Builds the tiled-pull plan (SlicePlan) from the relabelled in-adjacency on
// the host (once, at registration) and uploads it into the workspace.
static pp_status build_slices(pp_graph g, const WsLayout& L, char* base, hipStream_t st) {
    SlicePlan& sp = g->slices;
    sp = SlicePlan{};
    const Tuning& t = g->tune;
    if (!sliced_layout(g->flags, t) || L.sl_rows_cap <= 0) return PP_OK;
    const int32_t n = g->d.n;
    const int32_t W = t.slice_width;
    const int32_t waves = std::max(t.pull_block / kWave, 1);
    if (tiled_lds_bytes(W, waves) > (size_t)g->max_lds) return PP_OK;  // does not fit this device's LDS
    const int64_t Rc = L.sl_rows_cap;
    std::vector<int32_t> roff((size_t)Rc + 1);
    PP_HIP(hipMemcpyAsync(roff.data(), g->d.csc_off, roff.size() * 4, hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    const int64_t E_cap = roff[Rc];
    std::vector<int32_t> idx((size_t)std::max<int64_t>(E_cap, 1));
    if (E_cap > 0) PP_HIP(hipMemcpyAsync(idx.data(), g->d.csc_idx, (size_t)E_cap * 4, hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    // slices that hold a source of the candidate rows
    int32_t maxv = 0;
    for (int64_t j = 0; j < E_cap; ++j) maxv = std::max(maxv, idx[j]);
    const int32_t S = std::min<int32_t>(maxv / W + 1, (int32_t)L.sl_slices_cap);
    // the qualifying prefix of rows
    const int32_t min_deg = std::max(kTileMinDeg, S / 2);
    int32_t R = 0;
    while (R < Rc && roff[R + 1] - roff[R] >= min_deg) ++R;
    if (R == 0) return PP_OK;
    // segment lengths, slice-major (s * R + u), and every row's sources
    // grouped by slice in stored order (row-major scratch)
    std::vector<int32_t> seg((size_t)S * R, 0);
    parallel_ranges(R, [&](int64_t lo, int64_t hi) {
        for (int64_t u = lo; u < hi; ++u)
            for (int64_t j = roff[u]; j < roff[u + 1]; ++j) ++seg[(size_t)(idx[j] / W) * R + u];
    });
    std::vector<int32_t> rstart((size_t)R * S);  // where segment (s, u) starts in the row-major scratch
    std::vector<uint16_t> scratch((size_t)std::max<int64_t>(roff[R], 1));
    parallel_ranges(R, [&](int64_t lo, int64_t hi) {
        for (int64_t u = lo; u < hi; ++u) {
            int32_t at = roff[u];
            for (int32_t s2 = 0; s2 < S; ++s2) {
                rstart[(size_t)u * S + s2] = at;
                at += seg[(size_t)s2 * R + u];
            }
            std::vector<int32_t> cur(rstart.begin() + u * S, rstart.begin() + (u + 1) * S);
            for (int64_t j = roff[u]; j < roff[u + 1]; ++j) {
                const int32_t v = idx[j], s2 = v / W;
                scratch[cur[s2]++] = (uint16_t)(v - s2 * W);
            }
        }
    });
    // chunks of long segments, numbered row by row (the combine adds a row's
    // chunks [cbeg[u], cbeg[u+1]) after its slice partials)
    std::vector<int32_t> cbeg((size_t)R + 1, 0);
    int64_t nchunks = 0;
    for (int32_t u = 0; u < R; ++u) {
        cbeg[u] = (int32_t)nchunks;
        for (int32_t s2 = 0; s2 < S; ++s2) {
            const int32_t len = seg[(size_t)s2 * R + u];
            if (len >= kSegLong) nchunks += (len + kSegChunk - 1) / kSegChunk;
        }
    }
    cbeg[R] = (int32_t)nchunks;
    if (nchunks > L.sl_chunks_cap) return set_error(PP_E_WORKSPACE, "tiled pull: chunk table overflow");
    // units, slice by slice: segments packed whole into units of at most
    // kUnitEdges edges and kUnitPairs segments, each unit 8-aligned
    std::vector<uint16_t> out;
    out.reserve((size_t)roff[R] + 8 * 1024);
    std::vector<int32_t> prow;
    std::vector<SliceUnit> units;
    std::vector<int64_t> cost;
    constexpr int64_t kUnitCost = 64;  // fixed cost of a unit, in edges
    for (int32_t s2 = 0; s2 < S; ++s2) {
        const int32_t* sg = seg.data() + (size_t)s2 * R;
        int32_t u = 0;
        while (u < R) {
            if (sg[u] == 0 || sg[u] >= kSegLong) {
                ++u;
                continue;
            }
            while (out.size() % 8) out.push_back(0);  // pads sit past the previous unit's end
            const int32_t a = (int32_t)out.size(), p0 = (int32_t)prow.size();
            int32_t edges = 0, pairs = 0;
            for (; u < R; ++u) {
                const int32_t len = sg[u];
                if (len == 0 || len >= kSegLong) continue;
                if (edges + len > kUnitEdges || pairs == kUnitPairs) break;
                const uint16_t* src = scratch.data() + rstart[(size_t)u * S + s2];
                out.push_back((uint16_t)(src[0] | kSegHead));
                out.insert(out.end(), src + 1, src + len);
                prow.push_back(u);
                edges += len;
                ++pairs;
            }
            units.push_back(SliceUnit{s2, a, a + edges, p0});
            cost.push_back(kUnitCost + edges + 4 * pairs);
        }
    }
    const int64_t unit_count = (int64_t)units.size();
    // chunk units, slice by slice after all units (each chunk 8-aligned)
    std::vector<int32_t> cnext(cbeg.begin(), cbeg.end() - 1);
    std::vector<SliceUnit> cunits;
    for (int32_t u = 0; u < R; ++u)
        for (int32_t s2 = 0; s2 < S; ++s2) {
            const int32_t len = seg[(size_t)s2 * R + u];
            if (len < kSegLong) continue;
            const uint16_t* src = scratch.data() + rstart[(size_t)u * S + s2];
            for (int32_t c0 = 0; c0 < len; c0 += kSegChunk) {
                const int32_t c1 = std::min(c0 + kSegChunk, len);
                while (out.size() % 8) out.push_back(0);
                const int32_t a = (int32_t)out.size();
                out.insert(out.end(), src + c0, src + c1);
                cunits.push_back(SliceUnit{s2, a, a + (c1 - c0), -(cnext[u]++) - 1});
            }
        }
    // merge: per slice, its chunk units then its units (both were built in
    // slice order)
    std::vector<SliceUnit> all;
    std::vector<int64_t> all_cost;
    {
        std::stable_sort(cunits.begin(), cunits.end(),
                         [](const SliceUnit& x, const SliceUnit& y) { return x.slice < y.slice; });
        size_t i = 0, j = 0;
        for (int32_t s2 = 0; s2 < S; ++s2) {
            for (; j < cunits.size() && cunits[j].slice == s2; ++j) {
                all.push_back(cunits[j]);
                all_cost.push_back(kUnitCost + (cunits[j].b - cunits[j].a));
            }
            for (; i < units.size() && units[i].slice == s2; ++i) {
                all.push_back(units[i]);
                all_cost.push_back(cost[i]);
            }
        }
    }
    while (out.size() % 8) out.push_back(0);
    for (int k = 0; k < 16; ++k) out.push_back(0);  // wide loads may read past the last unit
    if ((int64_t)out.size() > L.sl_idx_cap || (int64_t)prow.size() > L.sl_pairs_cap ||
        unit_count > L.sl_units_cap || (int64_t)cunits.size() > L.sl_chunks_cap)
        return set_error(PP_E_WORKSPACE, "tiled pull: unit table overflow");
    // contiguous unit ranges of about equal cost, one per workgroup, split
    // into runs of one slice each
    const int32_t groups = std::max(1, std::min(g->num_cu, kTileMaxGroups));
    int64_t total = 0;
    for (int64_t c : all_cost) total += c;
    std::vector<int32_t> wg((size_t)groups + 1, 0);
    std::vector<SliceSeg> segs;
    {
        int64_t run = 0;
        size_t k = 0;
        for (int32_t w = 0; w < groups; ++w) {
            wg[w] = (int32_t)segs.size();
            const size_t k0 = k;
            const int64_t goal = total * (w + 1) / groups;
            while (k < all.size() && (w == groups - 1 || run + all_cost[k] / 2 <= goal)) run += all_cost[k++];
            for (size_t a = k0; a < k;) {
                size_t b = a;
                while (b < k && all[b].slice == all[a].slice) ++b;
                segs.push_back(SliceSeg{all[a].slice, (int32_t)a, (int32_t)b, 0});
                a = b;
            }
        }
        wg[groups] = (int32_t)segs.size();
    }
    if ((int64_t)segs.size() > kTileMaxGroups + S) return set_error(PP_E_WORKSPACE, "tiled pull: run table overflow");
    // upload; the dense partials start (and, where no unit writes, stay) zero
    GraphDev& d = g->d;
    d.sl_idx = reinterpret_cast<uint16_t*>(base + L.sl_idx);
    d.sl_prow = reinterpret_cast<int32_t*>(base + L.sl_prow);
    d.sl_units = reinterpret_cast<SliceUnit*>(base + L.sl_units);
    d.sl_segs = reinterpret_cast<SliceSeg*>(base + L.sl_segs);
    d.sl_wg = reinterpret_cast<int32_t*>(base + L.sl_wg);
    d.sl_part = reinterpret_cast<float*>(base + L.sl_part);
    d.sl_cpart = reinterpret_cast<float*>(base + L.sl_cpart);
    d.sl_cbeg = reinterpret_cast<int32_t*>(base + L.sl_cbeg);
    PP_HIP(hipMemcpyAsync(d.sl_idx, out.data(), out.size() * 2, hipMemcpyHostToDevice, st));
    if (!prow.empty()) PP_HIP(hipMemcpyAsync(d.sl_prow, prow.data(), prow.size() * 4, hipMemcpyHostToDevice, st));
    if (!all.empty())
        PP_HIP(hipMemcpyAsync(d.sl_units, all.data(), all.size() * sizeof(SliceUnit), hipMemcpyHostToDevice, st));
    if (!segs.empty())
        PP_HIP(hipMemcpyAsync(d.sl_segs, segs.data(), segs.size() * sizeof(SliceSeg), hipMemcpyHostToDevice, st));
    PP_HIP(hipMemcpyAsync(d.sl_wg, wg.data(), wg.size() * 4, hipMemcpyHostToDevice, st));
    PP_HIP(hipMemcpyAsync(d.sl_cbeg, cbeg.data(), cbeg.size() * 4, hipMemcpyHostToDevice, st));
    PP_HIP(hipMemsetAsync(d.sl_part, 0, (size_t)S * R * sizeof(float), st));
    // the pull plan without rows < R: they come first within each bin's list
    // (the partition is stable and ids ascend), and bin-5 rows < R own the
    // first split-table entries
    const BinPlan& pp_ = g->pull_plan;
    std::vector<int32_t> list((size_t)n);
    PP_HIP(hipMemcpyAsync(list.data(), d.pull_list, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    std::vector<int32_t> first((size_t)pp_.count[5] + 1);
    const int32_t* tab_first = d.split_tab + 3 * (size_t)g->split_cap;
    PP_HIP(hipMemcpyAsync(first.data(), tab_first, first.size() * 4, hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    int32_t counts[PP_NUM_BINS];
    for (int b = 0; b < PP_NUM_BINS; ++b) {
        int32_t k = 0;
        while (k < pp_.count[b] && list[pp_.list_off[b] + k] < R) ++k;
        for (int32_t i = k; i < pp_.count[b]; ++i)
            if (list[pp_.list_off[b] + i] < R) return set_error(PP_E_UNSUPPORTED, "tiled pull: bin lists out of order");
        sp.list_skip[b] = k;
        counts[b] = pp_.count[b] - k;
    }
    // rows past the last one with in-edges: the list is ascending within a
    // bin, so they are bin 0's last entries (checked entry by entry)
    int32_t tail = std::min(n - g->in_active, counts[0]);
    for (int32_t i = 0; i < tail; ++i)
        if (list[pp_.list_off[0] + pp_.count[0] - tail + i] != n - tail + i) {
            tail = 0;
            break;
        }
    counts[0] -= tail;
    sp.tail = tail;
    sp.fix0 = sp.list_skip[5];
    sp.tab0 = first[sp.fix0];
    sp.nsplit = pp_.count[5] - sp.fix0;
    int32_t waves_b[PP_NUM_BINS];
    waves_b[5] = g->split_pull_entries - sp.tab0;
    for (int b = 0; b < PP_NUM_BINS - 1; ++b) waves_b[b] = ceil_div(counts[b], kWave / kPullLanes[b]);
    int32_t at = 0;
    for (int b = PP_NUM_BINS - 1; b >= 0; --b) {
        sp.wave_off[b] = at;
        at += waves_b[b];
    }
    sp.wave_off[PP_NUM_BINS] = at;
    sp.units = at;
    sp.rows = R;
    sp.width = W;
    sp.slices = S;
    sp.tiles = (int32_t)all.size();
    sp.pairs = (int32_t)prow.size();
    sp.chunks = (int32_t)nchunks;
    sp.idx_size = (int32_t)out.size();
    sp.groups = groups;
    return PP_OK;
}

static pp_status check_arrays(int32_t n, int64_t nnz, const int32_t* off, const int32_t* idx, int32_t* err,
                              int32_t* host, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, 2, err);
    hipLaunchKernelGGL(k_check_offsets, dim3(ceil_div((int64_t)n + 1, 256)), dim3(256), 0, st, n, nnz, off, err);
    if (nnz > 0) hipLaunchKernelGGL(k_check_indices, dim3(ceil_div(nnz, 256)), dim3(256), 0, st, n, nnz, idx, err);
    PP_LAUNCH_CHECK("graph check");
    PP_HIP(hipMemcpyAsync(host, err, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    return PP_OK;
}

static pp_status check_graph(pp_graph g, hipStream_t st) {
    const GraphDev& d = g->d;
    int32_t h[4] = {0, 0, 0, 0};
    pp_status s = check_arrays(d.n, d.nnz, d.user_csr_off, d.user_csr_idx, d.err, h, st);
    if (s != PP_OK) return s;
    if (d.user_csc_off != d.user_csr_off || d.user_csc_idx != d.user_csr_idx) {
        s = check_arrays(d.n, d.nnz, d.user_csc_off, d.user_csc_idx, d.err, h + 2, st);
        if (s != PP_OK) return s;
    }
    if (h[0] || h[2]) return set_error(PP_E_GRAPH, "offsets are not monotone from 0 to nnz");
    if (h[1] || h[3]) return set_error(PP_E_GRAPH, "an index lies outside [0, n)");
    return PP_OK;
}

constexpr uint32_t kKnownFlags = PP_GRAPH_WEIGHTED | PP_GRAPH_RELABEL;

}  // namespace pp

using namespace pp;

PP_EXPORT int pp_abi_version(void) { return PP_ABI_VERSION; }

PP_EXPORT const char* pp_last_error(void) { return g_last_error.c_str(); }

PP_EXPORT size_t pp_graph_workspace_bytes(int32_t n, int64_t nnz, uint32_t flags) {
    if (n < 1 || nnz < 0 || nnz > INT32_MAX) return 0;
    if (flags & ~kKnownFlags) return 0;
    // sized for distinct CSR and CSC arrays, which also covers the aliased case
    return layout(n, nnz, flags, tuning(), false).total;
}

PP_EXPORT pp_status pp_set_bin_thresholds(const int32_t* upper5, int32_t split_chunk) {
    clear_error();
    if (!upper5) return set_error(PP_E_NULL, "upper5 is NULL");
    for (int i = 0; i < PP_NUM_BINS - 1; ++i) {
        if (upper5[i] < 0 || (i > 0 && upper5[i] < upper5[i - 1]))
            return set_error(PP_E_RANGE, "bin thresholds must be non-negative and non-decreasing");
    }
    if (split_chunk < kBlock) return set_error(PP_E_RANGE, "split_chunk must be at least 256");
    if (upper5[PP_NUM_BINS - 2] < upper5[PP_NUM_BINS - 3])
        return set_error(PP_E_RANGE, "bin thresholds must be non-decreasing");
    for (int i = 0; i < PP_NUM_BINS - 1; ++i) tuning().upper[i] = upper5[i];
    tuning().split_chunk = split_chunk;
    return PP_OK;
}

PP_EXPORT pp_status pp_set_push_tuning(int32_t hot, int32_t push_blocks) {
    clear_error();
    if (hot < 0 || hot > kHotMax) return set_error(PP_E_RANGE, "hot must lie in [0, 40960]");
    if (push_blocks < 1 || push_blocks > 65536) return set_error(PP_E_RANGE, "push_blocks must lie in [1, 65536]");
    tuning().hot = hot;
    tuning().push_blocks = push_blocks;
    return PP_OK;
}

PP_EXPORT pp_status pp_set_pull_tuning(int32_t pull_hot, int32_t pull_block) {
    clear_error();
    if (pull_hot < 0 || pull_hot > (1 << 20)) return set_error(PP_E_RANGE, "pull_hot must lie in [0, 2^20]");
    if (pull_block != 256 && pull_block != 512 && pull_block != 1024)
        return set_error(PP_E_RANGE, "pull_block must be 256, 512 or 1024");
    tuning().pull_hot = pull_hot;
    tuning().pull_block = pull_block;
    return PP_OK;
}

PP_EXPORT pp_status pp_set_pull_slices(int32_t rows, int32_t width) {
    clear_error();
    if (rows < 0) return set_error(PP_E_RANGE, "rows must be >= 0");
    if (width < 64 || width > kSliceMax || width % 64 != 0)
        return set_error(PP_E_RANGE, "width must be a multiple of 64 in [64, 32768]");
    tuning().slice_rows = rows;
    tuning().slice_width = width;
    return PP_OK;
}

PP_EXPORT pp_status pp_set_push_bins(int32_t on) {
    clear_error();
    if (on != 0 && on != 1) return set_error(PP_E_RANGE, "push bins: 0 or 1");
    tuning().push_bins = on;
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_push_bins(pp_graph g, int32_t* info) {
    clear_error();
    if (!g || !info) return set_error(PP_E_NULL, "graph or info is NULL");
    info[0] = g->pbins.nbins;
    info[1] = g->pbins.hot;
    info[2] = g->pbins.groups;
    info[3] = g->pbins.units;
    return PP_OK;
}

PP_EXPORT pp_status pp_set_multi_tuning(int32_t big, int32_t mid, int32_t pull_group, int32_t mid_lanes) {
    clear_error();
    if (mid < 1 || big < mid) return set_error(PP_E_RANGE, "many-graph tuning: need 1 <= mid <= big");
    if (pull_group != 1 && pull_group != 2 && pull_group != 4)
        return set_error(PP_E_RANGE, "many-graph tuning: pull_group must be 1, 2 or 4");
    if (mid_lanes != 8 && mid_lanes != 16 && mid_lanes != 32)
        return set_error(PP_E_RANGE, "many-graph tuning: mid_lanes must be 8, 16 or 32");
    tuning().multi_big = big;
    tuning().multi_mid = mid;
    tuning().multi_pull_group = pull_group;
    tuning().multi_mid_lanes = mid_lanes;
    return PP_OK;
}

PP_EXPORT pp_status pp_set_bfs_multi(int32_t max_frontier, int32_t max_edges) {
    clear_error();
    if (max_frontier < 0 || max_edges < 0) return set_error(PP_E_RANGE, "BFS multi-level caps must be >= 0");
    tuning().bfs_multi_n = max_frontier;
    tuning().bfs_multi_m = max_edges;
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_slices(pp_graph g, int32_t* info) {
    clear_error();
    if (!g || !info) return set_error(PP_E_NULL, "graph or info is NULL");
    info[0] = g->slices.rows;
    info[1] = g->slices.width;
    info[2] = g->slices.slices;
    info[3] = g->slices.tiles;
    return PP_OK;
}

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
    const bool relabel = (flags & PP_GRAPH_RELABEL) != 0;
    if (weighted && nnz > 0 && (!csr_w || !csc_to_csr))
        return set_error(PP_E_NULL, "weighted graph needs csr_w and csc_to_csr");
    if (flags & ~kKnownFlags) return set_error(PP_E_UNSUPPORTED, "unknown graph flag");
    const bool aliased = (csc_off == csr_off) && (csc_idx == csr_idx);
    const Tuning t = tuning();
    const WsLayout L = layout(n, nnz, flags, t, aliased);
    if (ws_bytes < L.total) return set_error(PP_E_WORKSPACE, "graph workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return set_error(PP_E_RANGE, "workspace must be 256-byte aligned");

    pp_graph g = new (std::nothrow) pp_graph_s();
    if (!g) return set_error(PP_E_SIZE, "host allocation of the graph handle failed");
    g->flags = flags;
    g->weighted = weighted;
    g->relabelled = relabel;
    g->tune = t;
    char* base = static_cast<char*>(ws);
    auto at = [&](size_t off) { return static_cast<void*>(base + off); };
    GraphDev& d = g->d;
    d.n = n;
    d.nnz = nnz;
    d.user_csr_off = csr_off;
    d.user_csr_idx = csr_idx;
    d.user_csc_off = csc_off;
    d.user_csc_idx = csc_idx;
    d.csr_off = csr_off;
    d.csr_idx = csr_idx;
    d.csc_off = csc_off;
    d.csc_idx = csc_idx;
    d.csr_w = weighted ? csr_w : nullptr;
    d.user_csc_to_csr = weighted ? csc_to_csr : nullptr;
    d.aliased = aliased;
    d.perm = d.iperm = nullptr;
    d.inv_s = static_cast<float*>(at(L.inv_s));
    d.out_deg = static_cast<int32_t*>(at(L.out_deg));
    d.pull_list = static_cast<int32_t*>(at(L.pull_list));
    d.push_list = static_cast<int32_t*>(at(L.push_list));
    d.buf0 = static_cast<float*>(at(L.buf0));
    d.buf1 = static_cast<float*>(at(L.buf1));
    d.buf2 = static_cast<float*>(at(L.buf2));
    d.csc_w = weighted ? static_cast<float*>(at(L.csc_w)) : nullptr;
    d.csc_row = static_cast<int32_t*>(at(L.csc_row));
    d.split_tab = static_cast<int32_t*>(at(L.split_tab));
    d.split_part = static_cast<float*>(at(L.split_part));
    d.hot_part = static_cast<float*>(at(L.hot_part));
    if (push_binned(t, n)) {
        d.pb_base = static_cast<int32_t*>(at(L.pb_base));
        d.pb_cnt = static_cast<int32_t*>(at(L.pb_cnt));
        d.pb_fill = static_cast<int32_t*>(at(L.pb_fill));
        d.pb_units = static_cast<int32_t*>(at(L.pb_units));
        d.pb_ulo = static_cast<int32_t*>(at(L.pb_ulo));
        d.pb_pairs = static_cast<int2*>(at(L.pb_pairs));
        d.pb_part = static_cast<float*>(at(L.pb_part));
    } else {
        d.pb_base = d.pb_cnt = d.pb_fill = d.pb_units = d.pb_ulo = nullptr;
        d.pb_pairs = nullptr;
        d.pb_part = nullptr;
    }
    d.err = static_cast<int32_t*>(at(L.err));
    d.sl_idx = nullptr;
    d.sl_prow = nullptr;
    d.sl_units = nullptr;
    d.sl_segs = nullptr;
    d.sl_wg = nullptr;
    d.sl_part = nullptr;
    d.sl_cpart = nullptr;
    d.sl_cbeg = nullptr;
    int32_t* tiles = static_cast<int32_t*>(at(L.tiles));
    uint8_t* keys = static_cast<uint8_t*>(at(L.keys));
    hipStream_t st = static_cast<hipStream_t>(stream);

    auto fail = [&](pp_status s) {
        delete g;
        return s;
    };
    // The sweeps trust the arrays, so malformed ones are rejected here.
    pp_status s = check_graph(g, st);
    if (s != PP_OK) return fail(s);

    if (relabel) {
        int32_t* perm = static_cast<int32_t*>(at(L.perm));
        int32_t* iperm = static_cast<int32_t*>(at(L.iperm));
        const dim3 vb(ceil_div(n, 256)), vt(256);
        hipLaunchKernelGGL(k_relabel_keys, vb, vt, 0, st, n, csr_off, csc_off, keys);
        s = partition(n, kMaxKeys, keys, tiles, d.err + 8, perm, nullptr, st);
        if (s != PP_OK) return fail(s);
        hipLaunchKernelGGL(k_invert_perm, vb, vt, 0, st, n, perm, iperm);
        int32_t* r_off = static_cast<int32_t*>(at(L.r_csr_off));
        int32_t* r_idx = static_cast<int32_t*>(at(L.r_csr_idx));
        int32_t* tmp_deg = d.out_deg;  // scratch until k_degrees fills it
        float* r_w = weighted ? static_cast<float*>(at(L.r_csr_w)) : nullptr;
        const int32_t row_blocks = std::max(std::min<int32_t>(ceil_div(n, 4), 16384), 1);
        hipLaunchKernelGGL(k_perm_degrees, vb, vt, 0, st, n, perm, csr_off, tmp_deg);
        s = exclusive_scan(n, tmp_deg, r_off, tiles, d.err + 40, st);
        if (s != PP_OK) return fail(s);
        hipLaunchKernelGGL(k_relabel_rows, dim3(row_blocks), dim3(256), 0, st, n, perm, iperm, csr_off, csr_idx,
                           r_off, r_idx, csr_w, (const int32_t*)nullptr, r_w);
        d.csr_off = r_off;
        d.csr_idx = r_idx;
        d.csr_w = r_w;
        if (aliased) {
            d.csc_off = r_off;
            d.csc_idx = r_idx;
            if (weighted)  // same slots as the CSR rows; weights arrive through the slot map
                hipLaunchKernelGGL(k_relabel_rows, dim3(row_blocks), dim3(256), 0, st, n, perm, iperm, csc_off,
                                   csc_idx, r_off, (int32_t*)nullptr, csr_w, csc_to_csr, d.csc_w);
        } else {
            int32_t* rc_off = static_cast<int32_t*>(at(L.r_csc_off));
            int32_t* rc_idx = static_cast<int32_t*>(at(L.r_csc_idx));
            hipLaunchKernelGGL(k_perm_degrees, vb, vt, 0, st, n, perm, csc_off, tmp_deg);
            s = exclusive_scan(n, tmp_deg, rc_off, tiles, d.err + 40, st);
            if (s != PP_OK) return fail(s);
            hipLaunchKernelGGL(k_relabel_rows, dim3(row_blocks), dim3(256), 0, st, n, perm, iperm, csc_off, csc_idx,
                               rc_off, rc_idx, csr_w, csc_to_csr, d.csc_w);
            d.csc_off = rc_off;
            d.csc_idx = rc_idx;
        }
        PP_LAUNCH_CHECK("relabel");
        d.perm = perm;
        d.iperm = iperm;
    } else if (weighted && nnz > 0) {
        hipLaunchKernelGGL(k_gather_weights, dim3(ceil_div(nnz, 256)), dim3(256), 0, st, nnz, csr_w, csc_to_csr,
                           d.csc_w);
    }
    hipLaunchKernelGGL(k_row_owner, dim3(std::max(std::min<int32_t>(ceil_div(n, 256), 4096), 1)), dim3(256), 0, st, n,
                       d.csc_off, d.csc_row);
    hipLaunchKernelGGL(k_degrees, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, d.csr_off, d.csr_w, d.out_deg,
                       d.inv_s);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, 3, d.err + 48);
    hipLaunchKernelGGL(k_max_deg, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, d.csr_off, d.csc_off, d.err + 48);
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(hip_error(e, "graph degree kernels"));
    }
    int32_t maxd[3];
    {
        hipError_t e = hipMemcpyAsync(maxd, d.err + 48, sizeof(maxd), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(hip_error(e, "reading degrees"));
    }
    g->max_out_deg = maxd[0];
    g->max_in_deg = maxd[1];
    g->in_active = maxd[2];
    {
        int dev = 0, cus = 0, lds = 0, lds_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
        if (e != hipSuccess) return fail(hip_error(e, "device attributes"));
        g->num_cu = std::max(cus, 1);
        g->max_lds = lds;
        g->lds_per_cu = std::max(lds_cu, lds);
    }
    const int32_t cap = L.split_cap;
    g->split_cap = cap;
    int32_t* tab_pull = d.split_tab;
    int32_t* tab_push = d.split_tab + 4 * (size_t)cap + 1;
    s = bins_for(g, d.csc_off, d.pull_list, tab_pull, cap, tiles, keys, g->pull_plan, g->split_pull_entries, st);
    if (s != PP_OK) return fail(s);
    s = bins_for(g, d.csr_off, d.push_list, tab_push, cap, tiles, keys, g->push_plan, g->split_push_entries, st);
    if (s != PP_OK) return fail(s);
    s = build_slices(g, L, base, st);
    if (s != PP_OK) return fail(s);
    {
        const hipError_t e = hipHostMalloc(&g->bfs_hdr_host, pp_graph_s::kBfsHdrHost, hipHostMallocDefault);
        if (e != hipSuccess) return fail(hip_error(e, "pinned BFS header buffer"));
    }
    if (d.pb_base) {
        s = build_push_bins(g, st);
        if (s != PP_OK) return fail(s);
    }
    *out = g;
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_set_weights(pp_graph g, const float* csr_w, void* stream) {
    clear_error();
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (!g->weighted) return set_error(PP_E_UNSUPPORTED, "graph was registered without PP_GRAPH_WEIGHTED");
    GraphDev& d = g->d;
    const int32_t n = d.n;
    const int64_t nnz = d.nnz;
    if (nnz > 0 && !csr_w) return set_error(PP_E_NULL, "csr_w is required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (nnz > 0) {
        if (g->relabelled) {
            // the relabelled CSR rows keep their stored order, so the new
            // weights follow their slots exactly as at registration
            const int32_t row_blocks = std::max(std::min<int32_t>(ceil_div(n, 4), 16384), 1);
            float* r_w = const_cast<float*>(d.csr_w);
            hipLaunchKernelGGL(k_relabel_rows, dim3(row_blocks), dim3(256), 0, st, n, d.perm, d.iperm, d.user_csr_off,
                               d.user_csr_idx, d.csr_off, (int32_t*)nullptr, csr_w, (const int32_t*)nullptr, r_w);
            hipLaunchKernelGGL(k_relabel_rows, dim3(row_blocks), dim3(256), 0, st, n, d.perm, d.iperm, d.user_csc_off,
                               d.user_csc_idx, d.csc_off, (int32_t*)nullptr, csr_w, d.user_csc_to_csr, d.csc_w);
        } else {
            d.csr_w = csr_w;
            hipLaunchKernelGGL(k_gather_weights, dim3(ceil_div(nnz, 256)), dim3(256), 0, st, nnz, csr_w,
                               d.user_csc_to_csr, d.csc_w);
        }
    }
    hipLaunchKernelGGL(k_degrees, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, d.csr_off, d.csr_w, d.out_deg, d.inv_s);
    PP_LAUNCH_CHECK("pp_graph_set_weights");
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_destroy(pp_graph g) {
    clear_error();
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    delete g;
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_bins(pp_graph g, pp_dir dir, int32_t* counts) {
    clear_error();
    if (!g || !counts) return set_error(PP_E_NULL, "graph or counts is NULL");
    if (dir != PP_PUSH && dir != PP_PULL) return set_error(PP_E_RANGE, "dir must be PP_PUSH or PP_PULL");
    const BinPlan& p = (dir == PP_PUSH) ? g->push_plan : g->pull_plan;
    for (int b = 0; b < PP_NUM_BINS; ++b) counts[b] = p.count[b];
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_relabel_map(pp_graph g, int32_t* perm, void* stream) {
    clear_error();
    if (!g || !perm) return set_error(PP_E_NULL, "graph or perm is NULL");
    if (!g->relabelled) return set_error(PP_E_UNSUPPORTED, "graph was registered without PP_GRAPH_RELABEL");
    PP_HIP(hipMemcpyAsync(perm, g->d.perm, sizeof(int32_t) * g->d.n, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(stream)));
    return PP_OK;
}

PP_EXPORT pp_status pp_graph_check(pp_graph g, void* stream) {
    clear_error();
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    return check_graph(g, static_cast<hipStream_t>(stream));
}
