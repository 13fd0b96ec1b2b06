// Triangle counting in its pushing and pulling forms (Sec. 3.2; Sec. 4.2
// listing).  For every vertex v and every pair of neighbours (w1, w2) with w2
// adjacent to w1, the pulling form credits v and the pushing form credits w1
// (an integer fetch-and-add on another vertex's counter); halving gives the
// triangles per vertex.  Here the pairs of one (v, w1) edge are counted
// together: |N(v) ∩ N(w1)| over sorted rows.
//
// Work decomposition: the edge array is cut into slices of kTcSlice edges,
// one wavefront each, so the load is balanced whatever the degrees.  A lane
// owns one (v, w1) edge; intersections whose shorter row has at most
// kTcLight entries run in the lane (binary search with a rising lower bound),
// longer ones are done by the whole wavefront (the shorter row is cut into 64
// pieces, each located in the longer row once and merged from there).
//
// Pull writes each vertex's counter exactly once: counts are reduced over the
// lanes of a row inside the slice (segmented scan); a row that crosses slice
// boundaries leaves partial sums (the last segment of its first slice, the
// first segment of each later slice) that k_tc_fix adds in a fixed order.
#include <hip/hip_runtime.h>

#include "pp_common.h"

namespace pp {

constexpr int32_t kTcSlice = 256;  // edges per wavefront
constexpr int32_t kTcLight = 16;   // lane-serial intersections up to this shorter row

struct TcArgs {
    int32_t n;
    int64_t nnz;
    int32_t slices;
    const int32_t* off;  // caller's CSR (rows sorted ascending)
    const int32_t* idx;
    int64_t* tc;         // [n] output (push: accumulator)
    int64_t* head;       // [slices] first segment of each slice (pull)
    int64_t* tail;       // [slices] last segment of each slice (pull)
    int32_t* flag;       // bit 0: a row is not strictly ascending
};

// Index of the row holding edge j: largest v in [lo, hi) with off[v] <= j.
__device__ __forceinline__ int32_t row_of(const int32_t* off, int32_t lo, int32_t hi, int64_t j) {
    while (hi - lo > 1) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (off[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

// |idx[a0, a1) ∩ idx[b0, b1)| for ascending rows, in one lane: every entry of
// the shorter row is searched in the longer one above the previous match.
__device__ __forceinline__ int64_t isect_lane(const int32_t* idx, int32_t a0, int32_t a1, int32_t b0, int32_t b1) {
    if (a1 - a0 > b1 - b0) {
        int32_t t = a0; a0 = b0; b0 = t;
        t = a1; a1 = b1; b1 = t;
    }
    int64_t cnt = 0;
    int32_t lo = b0;
    for (int32_t i = a0; i < a1 && lo < b1; ++i) {
        const int32_t x = idx[i];
        int32_t hi = b1;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (idx[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        if (lo < b1 && idx[lo] == x) {
            ++cnt;
            ++lo;
        }
    }
    return cnt;
}

// The same count by the whole wavefront (a0..b1 wave-uniform).  Lane l takes
// the l-th piece of the shorter row, finds its first entry's place in the
// longer row by binary search and merges forward.
__device__ __forceinline__ int64_t isect_wave(const int32_t* idx, int32_t a0, int32_t a1, int32_t b0, int32_t b1,
                                              int lane) {
    if (a1 - a0 > b1 - b0) {
        int32_t t = a0; a0 = b0; b0 = t;
        t = a1; a1 = b1; b1 = t;
    }
    const int32_t len = a1 - a0;
    const int32_t per = (len + kWave - 1) / kWave;
    const int32_t p0 = a0 + min(len, lane * per), p1 = a0 + min(len, (lane + 1) * per);
    int64_t cnt = 0;
    if (p0 < p1) {
        const int32_t x0 = idx[p0];
        int32_t lo = b0, hi = b1;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (idx[mid] < x0) lo = mid + 1;
            else hi = mid;
        }
        int32_t i = p0;
        while (i < p1 && lo < b1) {
            const int32_t x = idx[i], y = idx[lo];
            if (x < y) ++i;
            else if (x > y) ++lo;
            else {
                ++cnt;
                ++i;
                ++lo;
            }
        }
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) cnt += __shfl_xor(cnt, s);
    return cnt;
}

template <bool PUSH>
__global__ __launch_bounds__(kBlock) void k_tc_slices(TcArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int32_t nwaves = gridDim.x * (kBlock / kWave);
    for (int32_t s = gwave; s < a.slices; s += nwaves) {
        const int64_t e0 = (int64_t)s * kTcSlice;
        const int64_t e1 = min(e0 + kTcSlice, a.nnz);
        // rows holding the first and last edge of the slice bound every search
        int32_t v0 = 0, v1 = 0;
        if (lane == 0) v0 = row_of(a.off, 0, a.n, e0);
        if (lane == 1) v1 = row_of(a.off, 0, a.n, e1 - 1);
        v0 = __shfl(v0, 0);
        v1 = __shfl(v1, 1);
        int64_t carry = 0;  // running sum of the open segment (row carry_v)
        int32_t carry_v = -1;
        for (int64_t jb = e0; jb < e1; jb += kWave) {
            const int64_t j = jb + lane;
            const bool live = j < e1;
            int32_t v = -1, w = -1, rb = 0, re = 0;
            int64_t cnt = 0;
            bool heavy = false;
            if (live) {
                v = row_of(a.off, v0, v1 + 1, j);
                w = a.idx[j];
                rb = a.off[v];
                re = a.off[v + 1];
                if (j + 1 < re && a.idx[j + 1] <= w) atomicOr(a.flag, 1);
                const int32_t wb = a.off[w], we = a.off[w + 1];
                heavy = min(re - rb, we - wb) > kTcLight;
                if (!heavy) cnt = isect_lane(a.idx, rb, re, wb, we);
            }
            uint64_t hm = __ballot(heavy);
            while (hm) {
                const int src = __ffsll((long long)hm) - 1;
                hm &= hm - 1;
                const int32_t hv_b = __shfl(rb, src), hv_e = __shfl(re, src);
                const int32_t hw = __shfl(w, src);
                const int64_t c = isect_wave(a.idx, hv_b, hv_e, a.off[hw], a.off[hw + 1], lane);
                if (lane == src) cnt = c;
            }
            if (PUSH) {
                if (live && cnt) atomicAdd(reinterpret_cast<unsigned long long*>(&a.tc[w]), (unsigned long long)cnt);
                continue;
            }
            // pull: segmented inclusive sum over lanes of the same row (the
            // open segment of the previous round enters through lane 0)
            if (lane == 0 && v == carry_v) cnt += carry;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const int64_t y = __shfl_up(cnt, d);
                const int32_t yv = __shfl_up(v, d);
                if (lane >= d && yv == v) cnt += y;
            }
            // a segment ends where its row or the slice ends; one that reaches
            // lane 63 otherwise stays open into the next round
            const bool seg_end = live && (j + 1 >= e1 || j + 1 >= re);
            if (seg_end) {
                const bool starts_here = rb >= e0, ends_here = re <= e1;
                if (starts_here && ends_here) {
                    a.tc[v] = cnt / 2;
                } else {
                    if (!starts_here) a.head[s] = cnt;  // the slice's first segment
                    if (!ends_here) a.tail[s] = cnt;    // the slice's last segment
                }
            }
            const int src = min(kWave - 1, (int)(e1 - 1 - jb));
            carry = __shfl(cnt, src);
            carry_v = __shfl(v, src);
        }
    }
}

// Pull: counters of rows that cross slices, and of empty rows.
__global__ __launch_bounds__(kBlock) void k_tc_fix(TcArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t base = t - lane; base < a.n; base += stride) {
        const int32_t v = base + lane;
        int64_t rb = 0, re = 0;
        if (v < a.n) {
            rb = a.off[v];
            re = a.off[v + 1];
        }
        const int32_t s0 = (int32_t)(rb / kTcSlice), s1 = (int32_t)((re - 1) / kTcSlice);
        const bool span = v < a.n && re > rb && s1 > s0;
        if (v < a.n && re == rb) a.tc[v] = 0;
        // short spans in the lane, long ones (hub rows) by the wavefront
        const bool longspan = span && (s1 - s0) > 8;
        if (span && !longspan) {
            int64_t sum = a.tail[s0];
            for (int32_t s = s0 + 1; s <= s1; ++s) sum += a.head[s];
            a.tc[v] = sum / 2;
        }
        uint64_t lm = __ballot(longspan);
        while (lm) {
            const int src = __ffsll((long long)lm) - 1;
            lm &= lm - 1;
            const int32_t b = __shfl(s0, src), e = __shfl(s1, src);
            int64_t sum = 0;
            for (int32_t s = b + 1 + lane; s <= e; s += kWave) sum += a.head[s];
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) sum += __shfl_xor(sum, d);
            if (lane == src) a.tc[v] = (sum + a.tail[b]) / 2;
        }
    }
}

__global__ void k_tc_zero(int32_t n, int64_t* tc, int32_t* flag) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) tc[v] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
}

__global__ void k_tc_halve(int32_t n, int64_t* tc) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) tc[v] /= 2;
}

struct TcLayout {
    size_t flag, head, tail, total;
    int32_t slices;
};

static TcLayout tc_layout(int64_t nnz) {
    TcLayout L{};
    L.slices = (int32_t)((nnz + kTcSlice - 1) / kTcSlice);
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p = align_up(p + bytes, 256);
        return at;
    };
    L.flag = take(sizeof(int32_t));
    L.head = take((size_t)std::max(L.slices, 1) * 8);
    L.tail = take((size_t)std::max(L.slices, 1) * 8);
    L.total = p;
    return L;
}

}  // namespace pp

using namespace pp;

PP_EXPORT size_t pp_tc_workspace_bytes(pp_graph g) { return g ? tc_layout(g->d.nnz).total : 0; }

PP_EXPORT pp_status pp_tc_run(pp_graph g, pp_dir dir, int64_t* tc, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (!tc || !ws) return set_error(PP_E_NULL, "tc and ws are required");
    if (dir != PP_PUSH && dir != PP_PULL) return set_error(PP_E_RANGE, "dir must be PP_PUSH or PP_PULL");
    const TcLayout L = tc_layout(g->d.nnz);
    if (ws_bytes < L.total) return set_error(PP_E_WORKSPACE, "TC workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return set_error(PP_E_RANGE, "ws must be 256-byte aligned");
    char* w = static_cast<char*>(ws);
    TcArgs a;
    a.n = g->d.n;
    a.nnz = g->d.nnz;
    a.slices = L.slices;
    a.off = g->d.user_csr_off;
    a.idx = g->d.user_csr_idx;
    a.tc = tc;
    a.head = reinterpret_cast<int64_t*>(w + L.head);
    a.tail = reinterpret_cast<int64_t*>(w + L.tail);
    a.flag = reinterpret_cast<int32_t*>(w + L.flag);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t vb = std::max(1, std::min(ceil_div(a.n, kBlock), 4096));
    hipLaunchKernelGGL(k_tc_zero, dim3(vb), dim3(kBlock), 0, st, a.n, a.tc, a.flag);
    if (a.slices > 0) {
        const int32_t blocks = std::min(ceil_div(a.slices, kBlock / kWave), g->num_cu * 8);
        if (dir == PP_PUSH) hipLaunchKernelGGL(k_tc_slices<true>, dim3(blocks), dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL(k_tc_slices<false>, dim3(blocks), dim3(kBlock), 0, st, a);
    }
    if (dir == PP_PUSH) hipLaunchKernelGGL(k_tc_halve, dim3(vb), dim3(kBlock), 0, st, a.n, a.tc);
    else hipLaunchKernelGGL(k_tc_fix, dim3(vb), dim3(kBlock), 0, st, a);
    PP_LAUNCH_CHECK("k_tc_slices");
    int32_t flag = 0;
    PP_HIP(hipMemcpyAsync(&flag, a.flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    if (flag) return set_error(PP_E_GRAPH, "triangle counting needs rows in strictly ascending order");
    return PP_OK;
}
