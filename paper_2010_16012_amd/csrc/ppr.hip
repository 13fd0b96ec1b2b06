// Batched personalised PageRank (k source columns) and its adjoint with
// respect to the edge weights, on the push/pull sweeps.
//
// Forward, per column j with source s_j (the PageRank equation of Sec. 3.1
// with the teleport term concentrated on s_j):
//   x_{t+1}(u) = (1-f)[u == s_j] + f * sum over edges (v,u) of P_uv x_t(v),
//   P_uv = w(v->u)/s(v),  x_0 = e_{s_j}.
// Adjoint of L(X) at the fixed point (not in the paper): Lambda solves
// Lambda = dL/dX + f P^T Lambda, with (P^T z)(v) = (1/s(v)) sum over
// out-edges (v,u) of w(v->u) z(u) -- a gather along the CSR rows, i.e. the
// transposed sweep: the forward pull gathers along CSC and pushes along CSR;
// the adjoint pull gathers along CSR and pushes along CSC.  The gradient of
// the weight of slot (v->u) is
//   g = (f/s(v)) sum_j X[v,j] (Lambda[u,j] - (P^T Lambda)[v,j]).
//
// Columns are processed in tiles of KT (8, 16, 32 or 64) columns; a tile's
// state is stored tile-major (row u holds its KT values contiguously), so one
// neighbour costs one coalesced KT-float read.  A group of KT lanes owns a
// row (lane = column).  Rows are distributed with the degree bins of the
// graph: short rows one group each, long rows one workgroup each (groups take
// strided neighbours, reduced through LDS in a fixed order), and the longest
// rows in chunks finished by a fix-up kernel.  Pull sweeps use no atomics
// and are deterministic; push sweeps use FP32 atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "pp_common.h"

namespace pp {

constexpr int kKtMax = 64;

struct KPlan {
    int32_t unit_off[PP_NUM_BINS + 1];  // units per bin, launch order 5, 4, ..., 0
    int32_t list_off[PP_NUM_BINS + 1];
    int32_t units;
};

// Units of a KT-column sweep over a binned vertex list: bins 0-2 put
// kBlock/KT rows in a unit, bins 3-4 one row, bin 5 one chunk.
static KPlan kplan(const BinPlan& p, int kt) {
    KPlan k;
    int32_t u[PP_NUM_BINS];
    for (int b = 0; b < 3; ++b) u[b] = ceil_div(p.count[b], kBlock / kt);
    u[3] = p.count[3];
    u[4] = p.count[4];
    u[5] = p.split_chunks;
    int32_t at = 0;
    for (int b = PP_NUM_BINS - 1; b >= 0; --b) {
        k.unit_off[b] = at;
        at += u[b];
    }
    k.unit_off[PP_NUM_BINS] = at;
    k.units = at;
    for (int b = 0; b <= PP_NUM_BINS; ++b) k.list_off[b] = p.list_off[b];
    return k;
}

__device__ __forceinline__ int kunit_bin(const KPlan& kp, int32_t u) {
    int b = PP_NUM_BINS - 1;
#pragma unroll
    for (int i = PP_NUM_BINS - 1; i > 0; --i)
        if (u >= kp.unit_off[i - 1]) b = i - 1;
    return b;
}

enum EpiKind { kEpiForward = 0, kEpiAdjoint = 1, kEpiPtl = 2 };

// Everything a k-column gather sweep needs.  `src` is the tile being gathered
// (n x KT); the epilogue turns a row's gathered sums into the next state.
struct KArgs {
    KPlan kp;
    const int32_t* off;
    const int32_t* idx;
    const float* wt;        // per-slot weight in the walked order (nullable)
    const int32_t* list;
    const int32_t* tab;     // bin-5 chunk table (v | begin | end | first)
    int32_t tab_cap;
    float* part;            // bin-5 partials, entries x KT
    const float* src;       // gathered tile
    // epilogue
    int32_t kind;
    const float* inv_s;
    const int32_t* perm;    // internal -> caller id (nullable)
    float f;
    int32_t k;              // total columns (caller layout row length)
    int32_t col0;           // first column of the tile
    const int32_t* src_int; // forward: internal id of each column's source (length k)
    const float* prev;      // previous iterate (residual), tile layout (nullable)
    float* out_tile;        // new iterate, tile layout
    float* out_scaled;      // forward: c = f * x / s (tile layout, nullable)
    const float* g_caller;  // adjoint: dL/dX, caller layout n x k
    float* out_caller;      // last iteration: caller layout n x k (nullable)
    float* resid_part;      // per-unit-group residual partials (nullable)
};

// Returns (|new - previous|, |new|) for the relative convergence test.
template <int KT>
__device__ __forceinline__ float2 kt_epilogue(const KArgs& a, int32_t u, int lane, float acc) {
    float val;
    if (a.kind == kEpiForward) {
        val = acc + ((a.src_int[a.col0 + lane] == u) ? 1.0f - a.f : 0.f);
        if (a.out_scaled) a.out_scaled[(size_t)u * KT + lane] = a.f * val * a.inv_s[u];
    } else if (a.kind == kEpiAdjoint) {
        const int32_t uc = user_id(a.perm, u);
        const float gv = (a.col0 + lane < a.k) ? a.g_caller[(size_t)uc * a.k + a.col0 + lane] : 0.f;
        val = gv + a.f * a.inv_s[u] * acc;
    } else {
        val = a.inv_s[u] * acc;  // (P^T Lambda)(u)
    }
    a.out_tile[(size_t)u * KT + lane] = val;
    if (a.out_caller && a.col0 + lane < a.k) a.out_caller[(size_t)user_id(a.perm, u) * a.k + a.col0 + lane] = val;
    return a.prev ? make_float2(fabsf(val - a.prev[(size_t)u * KT + lane]), fabsf(val)) : make_float2(0.f, 0.f);
}

// Fixed-order workgroup sum of (difference, norm) pairs into out[2*slot].
__device__ __forceinline__ void resid_flush(float2 r, float* red, float* out, int32_t slot) {
    red[threadIdx.x] = r.x;
    red[kBlock + threadIdx.x] = r.y;
    __syncthreads();
    if (threadIdx.x == 0) {
        float d = 0.f, m = 0.f;
        for (int i = 0; i < kBlock; ++i) {
            d += red[i];
            m += red[kBlock + i];
        }
        out[2 * slot] = d;
        out[2 * slot + 1] = m;
    }
}

// One group of KT lanes sums src[idx[j]] (x wt[j]) over j = b + g, b + g + stride, ...
template <int KT, bool W>
__device__ __forceinline__ float kt_gather(const KArgs& a, int32_t b, int32_t e, int32_t g, int32_t stride, int lane) {
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    int32_t j = b + g;
    for (; j + 3 * stride < e; j += 4 * stride) {
        const int32_t v0 = a.idx[j], v1 = a.idx[j + stride], v2 = a.idx[j + 2 * stride], v3 = a.idx[j + 3 * stride];
        float x0 = a.src[(size_t)v0 * KT + lane], x1 = a.src[(size_t)v1 * KT + lane];
        float x2 = a.src[(size_t)v2 * KT + lane], x3 = a.src[(size_t)v3 * KT + lane];
        if (W) {
            x0 *= a.wt[j];
            x1 *= a.wt[j + stride];
            x2 *= a.wt[j + 2 * stride];
            x3 *= a.wt[j + 3 * stride];
        }
        a0 += x0;
        a1 += x1;
        a2 += x2;
        a3 += x3;
    }
    for (; j < e; j += stride) {
        float x = a.src[(size_t)a.idx[j] * KT + lane];
        if (W) x *= a.wt[j];
        a0 += x;
    }
    return (a0 + a1) + (a2 + a3);
}

// Sum over the groups of a workgroup, in group order (thread (0, lane) holds it).
template <int KT>
__device__ __forceinline__ float kt_block_sum(float v, float* red) {
    constexpr int G = kBlock / KT;
    red[threadIdx.x] = v;
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x < KT) {
#pragma unroll
        for (int g = 0; g < G; ++g) t += red[g * KT + threadIdx.x];
    }
    __syncthreads();
    return t;
}

// The pull sweep moves float4s: a row is owned by KT/4 lanes, lane q holding
// columns 4q..4q+3, so one neighbour costs one 16-byte load per lane (a
// KT-float row per group) and a wavefront keeps 256/KT rows going at once.
template <int KT>
constexpr int kq_lanes() { return KT / 4; }

__device__ __forceinline__ float4 f4_add(float4 x, float4 y) {
    return make_float4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
}

__device__ __forceinline__ float4 f4_scale(float4 x, float s) { return make_float4(x.x * s, x.y * s, x.z * s, x.w * s); }

// One group of KT/4 lanes sums src[idx[j]] (x wt[j]) over j = b + g,
// b + g + stride, ...: U index loads, then U float4 gathers in flight, summed
// pairwise before they join the running sum (fixed order, and a hub row of
// thousands of slots keeps its FP32 rounding error near log2(U) + slots/U
// steps).  Loads past the row's end are exec-masked, not clamped: a clamped
// gather would still move KT floats.
template <int KT, int U, bool W>
__device__ __forceinline__ float4 kt_gather4(const KArgs& a, int32_t b, int32_t e, int32_t g, int32_t stride,
                                             int q) {
    const float4* __restrict__ src4 = reinterpret_cast<const float4*>(a.src);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int32_t j0 = b + g; j0 < e; j0 += U * stride) {
        int32_t vv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) vv[k] = a.idx[min(j0 + k * stride, e - 1)];
        float4 x[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            x[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j0 + k * stride < e) x[k] = src4[(size_t)vv[k] * kq_lanes<KT>() + q];
        }
        if (W) {
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (j0 + k * stride < e) x[k] = f4_scale(x[k], a.wt[j0 + k * stride]);
        }
#pragma unroll
        for (int w = 1; w < U; w <<= 1) {
#pragma unroll
            for (int k = 0; k + w < U; k += 2 * w) x[k] = f4_add(x[k], x[k + w]);
        }
        acc = f4_add(acc, x[0]);
    }
    return acc;
}

// Sum over the groups of a workgroup as a fixed binary tree (thread q < KT/4
// holds it): log2(G) rounding steps instead of G - 1 for a row spread over all
// G groups.
template <int KT>
__device__ __forceinline__ float4 kt_block_sum4(float4 v, float4* red) {
    constexpr int Q = kq_lanes<KT>();
    constexpr int G = kBlock / Q;
    static_assert((G & (G - 1)) == 0, "group count must be a power of two");
    const int grp = threadIdx.x / Q;
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = G / 2; s >= 1; s >>= 1) {
        if (grp < s) red[threadIdx.x] = f4_add(red[threadIdx.x], red[threadIdx.x + s * Q]);
        __syncthreads();
    }
    const float4 t = (threadIdx.x < Q) ? red[threadIdx.x] : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    return t;
}

// kt_epilogue for columns 4q..4q+3 of row u.
template <int KT>
__device__ __forceinline__ float2 kt_epilogue4(const KArgs& a, int32_t u, int q, float4 acc) {
    const float in[4] = {acc.x, acc.y, acc.z, acc.w};
    float val[4];
    const int c0 = a.col0 + 4 * q;
    if (a.kind == kEpiForward) {
#pragma unroll
        for (int c = 0; c < 4; ++c) val[c] = in[c] + ((a.src_int[c0 + c] == u) ? 1.0f - a.f : 0.f);
        if (a.out_scaled) {
            const float sc = a.f * a.inv_s[u];
            reinterpret_cast<float4*>(a.out_scaled)[(size_t)u * kq_lanes<KT>() + q] =
                make_float4(sc * val[0], sc * val[1], sc * val[2], sc * val[3]);
        }
    } else if (a.kind == kEpiAdjoint) {
        const int32_t uc = user_id(a.perm, u);
        const float sc = a.f * a.inv_s[u];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float gv = (c0 + c < a.k) ? a.g_caller[(size_t)uc * a.k + c0 + c] : 0.f;
            val[c] = gv + sc * in[c];
        }
    } else {
        const float is = a.inv_s[u];
#pragma unroll
        for (int c = 0; c < 4; ++c) val[c] = is * in[c];  // (P^T Lambda)(u)
    }
    reinterpret_cast<float4*>(a.out_tile)[(size_t)u * kq_lanes<KT>() + q] = make_float4(val[0], val[1], val[2], val[3]);
    if (a.out_caller) {
        const int32_t uc = user_id(a.perm, u);
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c0 + c < a.k) a.out_caller[(size_t)uc * a.k + c0 + c] = val[c];
    }
    float2 r = make_float2(0.f, 0.f);
    if (a.prev) {
        const float4 p4 = reinterpret_cast<const float4*>(a.prev)[(size_t)u * kq_lanes<KT>() + q];
        const float pv[4] = {p4.x, p4.y, p4.z, p4.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            r.x += fabsf(val[c] - pv[c]);
            r.y += fabsf(val[c]);
        }
    }
    return r;
}

// Units of bin b in a plan: bins run 5, 4, ..., 0, so bin b ends where bin
// b - 1 starts (bin 0 at the end of the plan).
static int32_t kplan_bin_units(const KPlan& kp, int b) {
    return (b == 0 ? kp.units : kp.unit_off[b - 1]) - kp.unit_off[b];
}

// Units of the float4 pull over the row-unit plan kp: bins 0-2 put
// kBlock/(KT/4) rows in a unit, bins 3-4 one row, bin 5 one chunk.
static KPlan kplan_pull4(const KPlan& kp, int kt) {
    KPlan k = kp;
    int32_t at = 0;
    for (int b = PP_NUM_BINS - 1; b >= 0; --b) {
        const int32_t rows = kp.list_off[b + 1] - kp.list_off[b];
        const int32_t units = (b <= 2) ? ceil_div(rows, kBlock / (kt / 4)) : kplan_bin_units(kp, b);
        k.unit_off[b] = at;
        at += units;
    }
    k.unit_off[PP_NUM_BINS] = at;
    k.units = at;
    return k;
}

// A plan's bins must tile [0, units) in launch order with no negative count.
static bool kplan_valid(const KPlan& kp) {
    int32_t at = 0;
    for (int b = PP_NUM_BINS - 1; b >= 0; --b) {
        if (kp.unit_off[b] != at || kplan_bin_units(kp, b) < 0) return false;
        at += kplan_bin_units(kp, b);
    }
    return at == kp.units && kp.unit_off[PP_NUM_BINS] == kp.units;
}

template <int KT, bool W>
__global__ __launch_bounds__(kBlock) void k_kcol_pull(KArgs a) {
    __shared__ float4 red4[kBlock];
    constexpr int Q = kq_lanes<KT>();
    constexpr int G = kBlock / Q;
    const int q = threadIdx.x % Q;
    const int grp = threadIdx.x / Q;
    const int32_t unit = blockIdx.x;
    const int bin = kunit_bin(a.kp, unit);
    const int32_t lu = unit - a.kp.unit_off[bin];
    float2 res = make_float2(0.f, 0.f);
    if (bin <= 2) {
        const int32_t i = lu * G + grp;
        if (i < a.kp.list_off[bin + 1] - a.kp.list_off[bin]) {
            const int32_t u = a.list[a.kp.list_off[bin] + i];
            const float4 acc = (bin == 0) ? kt_gather4<KT, 4, W>(a, a.off[u], a.off[u + 1], 0, 1, q)
                                          : kt_gather4<KT, 8, W>(a, a.off[u], a.off[u + 1], 0, 1, q);
            res = kt_epilogue4<KT>(a, u, q, acc);
        }
    } else if (bin <= 4) {
        const int32_t u = a.list[a.kp.list_off[bin] + lu];
        float4 acc = kt_gather4<KT, 8, W>(a, a.off[u], a.off[u + 1], grp, G, q);
        acc = kt_block_sum4<KT>(acc, red4);
        if (threadIdx.x < Q) res = kt_epilogue4<KT>(a, u, q, acc);
    } else {
        const int32_t b = a.tab[a.tab_cap + lu], e = a.tab[2 * a.tab_cap + lu];
        float4 acc = kt_gather4<KT, 8, W>(a, b, e, grp, G, q);
        acc = kt_block_sum4<KT>(acc, red4);
        if (threadIdx.x < Q) reinterpret_cast<float4*>(a.part)[(size_t)lu * Q + q] = acc;
    }
    if (a.resid_part) resid_flush(res, reinterpret_cast<float*>(red4), a.resid_part, unit);
}

// Finishes the chunked rows: partials in chunk order, then the epilogue.
template <int KT>
__global__ __launch_bounds__(kBlock) void k_kcol_fix(KArgs a, int32_t nsplit, float* resid_fix) {
    const int lane = threadIdx.x % KT;
    const int32_t i = blockIdx.x * (kBlock / KT) + threadIdx.x / KT;
    float2 res = make_float2(0.f, 0.f);
    if (i < nsplit) {
        const int32_t* first = a.tab + 3 * a.tab_cap;
        float acc = 0.f;
        for (int32_t e = first[i]; e < first[i + 1]; ++e) acc += a.part[(size_t)e * KT + lane];
        res = kt_epilogue<KT>(a, a.tab[first[i]], lane, acc);
    }
    if (resid_fix) {
        __shared__ float red[2 * kBlock];
        resid_flush(res, red, resid_fix, blockIdx.x);
    }
}

// ------------------------------------------------------------------ push
struct KPushArgs {
    KPlan kp;
    const int32_t* off;
    const int32_t* idx;
    const float* wt;
    const int32_t* list;
    const int32_t* tab;
    int32_t tab_cap;
    const float* src;   // tile being scattered
    double* acc;        // accumulator tile, FP64 so the unordered atomic sum keeps FP32 accuracy
};

template <int KT, bool W>
__device__ __forceinline__ void kt_scatter(const KPushArgs& a, int32_t v, int32_t b, int32_t e, int32_t g,
                                           int32_t stride, int lane) {
    const float x = a.src[(size_t)v * KT + lane];
    if (x == 0.f) return;  // per-lane: a zero contributes nothing
    for (int32_t j = b + g; j < e; j += stride) {
        const int32_t u = a.idx[j];
        unsafeAtomicAdd(&a.acc[(size_t)u * KT + lane], (double)(W ? x * a.wt[j] : x));
    }
}

template <int KT, bool W>
__global__ __launch_bounds__(kBlock) void k_kcol_push(KPushArgs a) {
    constexpr int G = kBlock / KT;
    const int lane = threadIdx.x % KT;
    const int grp = threadIdx.x / KT;
    const int32_t unit = blockIdx.x;
    const int bin = kunit_bin(a.kp, unit);
    const int32_t lu = unit - a.kp.unit_off[bin];
    if (bin <= 2) {
        const int32_t i = lu * G + grp;
        if (i < a.kp.list_off[bin + 1] - a.kp.list_off[bin]) {
            const int32_t v = a.list[a.kp.list_off[bin] + i];
            kt_scatter<KT, W>(a, v, a.off[v], a.off[v + 1], 0, 1, lane);
        }
    } else if (bin <= 4) {
        const int32_t v = a.list[a.kp.list_off[bin] + lu];
        kt_scatter<KT, W>(a, v, a.off[v], a.off[v + 1], grp, G, lane);
    } else {
        const int32_t v = a.tab[lu];
        kt_scatter<KT, W>(a, v, a.tab[a.tab_cap + lu], a.tab[2 * a.tab_cap + lu], grp, G, lane);
    }
}

// After a push sweep, per (row, column): the epilogue on the accumulated sum,
// then the accumulator is reset for the next sweep (to zero plus, for the
// forward, nothing: the teleport is added by the epilogue).
template <int KT>
__global__ __launch_bounds__(kBlock) void k_kcol_push_epi(KArgs a, int32_t n, double* accum) {
    __shared__ float red[2 * kBlock];
    const int lane = threadIdx.x % KT;
    const int32_t u = blockIdx.x * (kBlock / KT) + threadIdx.x / KT;
    float2 res = make_float2(0.f, 0.f);
    if (u < n) {
        const float acc = (float)accum[(size_t)u * KT + lane];
        accum[(size_t)u * KT + lane] = 0.0;
        res = kt_epilogue<KT>(a, u, lane, acc);
    }
    if (a.resid_part) resid_flush(res, red, a.resid_part, blockIdx.x);
}

// ------------------------------------------------------------------ helpers
// Start of a forward tile: x0 = e_s per column (prev), c0 = f x0 / s.
template <int KT>
__global__ void k_kcol_forward_init(int32_t n, const int32_t* __restrict__ src_int, int32_t col0, float f,
                                    const float* __restrict__ inv_s, float* __restrict__ prev,
                                    float* __restrict__ c, double* __restrict__ accum) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * KT) return;
    const int32_t u = (int32_t)(t / KT);
    const int lane = (int)(t % KT);
    const float x0 = (src_int[col0 + lane] == u) ? 1.f : 0.f;
    prev[t] = x0;
    c[t] = f * x0 * inv_s[u];
    if (accum) accum[t] = 0.0;
}

// Start of an adjoint tile: Lambda_0 = G (caller layout -> tile layout).
template <int KT>
__global__ void k_kcol_adjoint_init(int32_t n, int32_t k, int32_t col0, const int32_t* __restrict__ perm,
                                    const float* __restrict__ g, float* __restrict__ lam, double* __restrict__ accum) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * KT) return;
    const int32_t u = (int32_t)(t / KT);
    const int lane = (int)(t % KT);
    lam[t] = (col0 + lane < k) ? g[(size_t)user_id(perm, u) * k + col0 + lane] : 0.f;
    if (accum) accum[t] = 0.0;
}

// Internal source ids, padded with -1 (no source) up to a whole tile.
__global__ void k_sources_internal(int32_t k, int32_t k_pad, const int32_t* __restrict__ sources,
                                   const int32_t* __restrict__ iperm, int32_t n, int32_t* __restrict__ out,
                                   int32_t* __restrict__ bad) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k_pad) return;
    if (j >= k) {
        out[j] = -1;
        return;
    }
    const int32_t s = sources[j];
    if (s < 0 || s >= n) {
        atomicOr(bad, 1);
        out[j] = -1;
        return;
    }
    out[j] = iperm ? iperm[s] : s;
}

// Fixed-order sum of m (difference, norm) partial pairs (one workgroup).
__global__ __launch_bounds__(1024) void k_sum_partials(int32_t m, const float* __restrict__ p, float* __restrict__ out) {
    __shared__ float red[2][1024];
    float d = 0.f, q = 0.f;
    for (int32_t i = threadIdx.x; i < m; i += 1024) {
        d += p[2 * i];
        q += p[2 * i + 1];
    }
    red[0][threadIdx.x] = d;
    red[1][threadIdx.x] = q;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

// Edge gradient of one tile, added into grad (caller CSR slot order):
// slot (v -> u): f/s(v) * sum_j X[v,j] (Lambda[u,j] - ptl[v,j]).  One group
// of KT lanes per slot of the row; slots of long rows spread over the groups
// of a workgroup.  Each slot has one writer.
struct GradArgs {
    KPlan kp;  // over the CSR (out-degree) lists
    const int32_t* off;
    const int32_t* idx;
    const int32_t* list;
    const int32_t* tab;
    int32_t tab_cap;
    const float* lam;       // tile layout
    const float* ptl;       // tile layout
    const float* x_caller;  // caller layout n x k (used when x_tile is NULL)
    const float* x_tile;    // tile layout n x KT, internal ids (nullable)
    const float* inv_s;
    const int32_t* perm;
    const int32_t* user_off;  // caller CSR offsets (slot mapping)
    int32_t k, col0;
    float f;
    float* grad;
};

template <int KT>
__device__ __forceinline__ void grad_row(const GradArgs& a, int32_t v, int32_t b, int32_t e, int32_t g,
                                         int32_t stride, int lane) {
    const int32_t vc = user_id(a.perm, v);
    const float xv = a.x_tile ? a.x_tile[(size_t)v * KT + lane]
                              : ((a.col0 + lane < a.k) ? a.x_caller[(size_t)vc * a.k + a.col0 + lane] : 0.f);
    const float pv = a.ptl[(size_t)v * KT + lane];
    const float scale = a.f * a.inv_s[v];
    const int32_t row0 = a.off[v], crow0 = a.user_off[vc];
    for (int32_t j = b + g; j < e; j += stride) {
        const int32_t u = a.idx[j];
        float t = xv * (a.lam[(size_t)u * KT + lane] - pv);
#pragma unroll
        for (int s = KT / 2; s > 0; s >>= 1) t += __shfl_xor(t, s);
        if (lane == 0) a.grad[crow0 + (j - row0)] += scale * t;
    }
}

template <int KT>
__global__ __launch_bounds__(kBlock) void k_kcol_grad(GradArgs a) {
    constexpr int G = kBlock / KT;
    const int lane = threadIdx.x % KT;
    const int grp = threadIdx.x / KT;
    const int32_t unit = blockIdx.x;
    const int bin = kunit_bin(a.kp, unit);
    const int32_t lu = unit - a.kp.unit_off[bin];
    if (bin <= 2) {
        const int32_t i = lu * G + grp;
        if (i < a.kp.list_off[bin + 1] - a.kp.list_off[bin]) {
            const int32_t v = a.list[a.kp.list_off[bin] + i];
            grad_row<KT>(a, v, a.off[v], a.off[v + 1], 0, 1, lane);
        }
    } else if (bin <= 4) {
        const int32_t v = a.list[a.kp.list_off[bin] + lu];
        grad_row<KT>(a, v, a.off[v], a.off[v + 1], grp, G, lane);
    } else {
        const int32_t v = a.tab[lu];
        grad_row<KT>(a, v, a.tab[a.tab_cap + lu], a.tab[2 * a.tab_cap + lu], grp, G, lane);
    }
}

__global__ void k_scale_f32(int64_t m, float s, float* __restrict__ p) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        p[i] *= s;
}

__global__ void k_zero_f32(int64_t m, float* __restrict__ p) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// ------------------------------------------------------------------ host side
// ------------------------------------------------- sparse phase (PP_SWITCH)
// The Generic-Switch strategy (Sec. 5) for PPR: the iterate of a one-hot
// start is supported on the ball of radius t around the sources, so the first
// sweeps push from the support only (a sparse matrix - sparse vector product
// along CSR, Sec. 7.1) and the run switches to the dense pull sweep once the
// support's out-edges exceed m / kSwAlpha.  The support grows monotonically;
// it is kept as a list of all its vertices (epilogue), a list of its vertices
// with at most kSwChunk out-edges and (v, begin, end) chunk items of the longer
// rows (scatter work units), all cumulative.
constexpr int32_t kSwChunk = 64;
constexpr int32_t kSwAlpha = 14;
constexpr int32_t kSwEpiBlocks = 4096;  // workgroups of the sparse epilogue (upper bound)

struct SwState {
    uint64_t* bits;   // support membership
    int32_t* all;     // support vertices
    int32_t* small;   // support vertices with <= kSwChunk out-edges
    int32_t* items;   // chunk items of the longer rows
    int32_t* cnt;     // [0] |all|, [1] |small|, [2] items, [3] overflow; [4..5] out-edges (int64)
    int32_t item_cap;
    const int32_t* off;
};

// Adds u to the support (first caller only).
__device__ __forceinline__ void sw_claim(const SwState& w, int32_t u) {
    const uint64_t bit = 1ull << (u & 63);
    if (w.bits[u >> 6] & bit) return;
    const uint64_t old = atomicOr(reinterpret_cast<unsigned long long*>(&w.bits[u >> 6]), (unsigned long long)bit);
    if (old & bit) return;
    w.all[atomicAdd(&w.cnt[0], 1)] = u;
    const int32_t b = w.off[u], e = w.off[u + 1];
    atomicAdd(reinterpret_cast<unsigned long long*>(&w.cnt[4]), (unsigned long long)(e - b));
    if (e - b <= kSwChunk) {
        w.small[atomicAdd(&w.cnt[1], 1)] = u;
    } else {
        const int32_t nch = (e - b + kSwChunk - 1) / kSwChunk;
        const int32_t first = atomicAdd(&w.cnt[2], nch);
        for (int32_t c = 0; c < nch; ++c) {
            const int32_t it = first + c;
            if (it >= w.item_cap) {
                atomicOr(&w.cnt[3], 1);
                break;
            }
            w.items[3 * it] = u;
            w.items[3 * it + 1] = b + c * kSwChunk;
            w.items[3 * it + 2] = min(e, b + (c + 1) * kSwChunk);
        }
    }
}

__global__ void k_sw_seed(SwState w, const int32_t* __restrict__ src_int, int32_t col0, int32_t kt) {
    const int32_t c = threadIdx.x;
    if (c < kt && src_int[col0 + c] >= 0) sw_claim(w, src_int[col0 + c]);
}

// Adjoint: the support of Lambda_0 = dL/dX, i.e. every vertex whose row of
// the tile's columns of g (caller layout n x k) holds a nonzero.
__global__ void k_sw_seed_rhs(SwState w, int32_t n, int32_t k, int32_t col0, int32_t kt,
                              const int32_t* __restrict__ perm, const float* __restrict__ g) {
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        const float* row = g + (size_t)user_id(perm, u) * k;
        bool nz = false;
        for (int32_t c = 0; c < kt && col0 + c < k; ++c) nz |= (row[col0 + c] != 0.f);
        if (nz) sw_claim(w, u);
    }
}

// One sparse push sweep: a group of KT lanes (one per column) per work unit
// scatters c[v] along the unit's edges into the FP64 accumulator and claims
// the targets for the next support.  The unit counts are read at launch.
template <int KT, bool W>
__global__ __launch_bounds__(kBlock) void k_sw_scatter(SwState w, const int32_t* __restrict__ idx,
                                                       const float* __restrict__ wt, const float* __restrict__ c,
                                                       double* __restrict__ acc, int32_t n_small, int32_t n_items) {
    constexpr int G = kBlock / KT;
    const int lane = threadIdx.x % KT;
    const int32_t grp = blockIdx.x * G + threadIdx.x / KT;
    const int32_t ngrp = gridDim.x * G;
    for (int32_t unit = grp; unit < n_small + n_items; unit += ngrp) {
        int32_t v, b, e;
        if (unit < n_small) {
            v = w.small[unit];
            b = w.off[v];
            e = w.off[v + 1];
        } else {
            const int32_t it = unit - n_small;
            v = w.items[3 * it];
            b = w.items[3 * it + 1];
            e = w.items[3 * it + 2];
        }
        const float x = c[(size_t)v * KT + lane];
        for (int32_t j = b; j < e; ++j) {
            const int32_t u = idx[j];
            if (x != 0.f) unsafeAtomicAdd(&acc[(size_t)u * KT + lane], (double)(W ? x * wt[j] : x));
            if (lane == 0) sw_claim(w, u);
        }
    }
}

// Epilogue of a sparse sweep over the support (count read on the device).
template <int KT>
__global__ __launch_bounds__(kBlock) void k_sw_epi(KArgs a, SwState w, double* accum) {
    __shared__ float red[2 * kBlock];
    constexpr int G = kBlock / KT;
    const int lane = threadIdx.x % KT;
    const int32_t count = w.cnt[0];
    float2 res = make_float2(0.f, 0.f);
    for (int32_t i = blockIdx.x * G + threadIdx.x / KT; i < count; i += gridDim.x * G) {
        const int32_t u = w.all[i];
        const float acc = (float)accum[(size_t)u * KT + lane];
        accum[(size_t)u * KT + lane] = 0.0;
        const float2 r = kt_epilogue<KT>(a, u, lane, acc);
        res.x += r.x;
        res.y += r.y;
    }
    if (a.resid_part) resid_flush(res, red, a.resid_part, blockIdx.x);
}

__global__ void k_sw_clear(int32_t words, uint64_t* bits, int32_t* cnt) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) bits[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x < 16) cnt[threadIdx.x] = 0;
}

struct PprLayout {
    size_t t0, t1, t2, t3, t4, part, resid, scal, srcs, hist;  // hist: T iterates (unrolled adjoint)
    size_t sw_bits, sw_all, sw_small, sw_items, sw_cnt;  // sparse-phase support (PP_SWITCH)
    int32_t sw_item_cap;
    size_t total;
};

static PprLayout ppr_layout(int32_t n, int64_t nnz, int32_t split_cap, int32_t k, int32_t kt, int32_t max_units,
                            int32_t hist_tiles = 0) {
    PprLayout L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p = align_up(p + bytes, 256);
        return at;
    };
    const size_t tile = (size_t)n * kt * 4;
    L.t0 = take(tile);
    L.t1 = take(tile);
    L.t2 = take(tile);
    L.t3 = take(tile);
    L.t4 = take(2 * tile);  // FP64 push accumulator
    L.part = take((size_t)split_cap * kt * 4);
    // residual pairs: one per work unit of a dense sweep, or one per
    // workgroup of the sparse epilogue (at most kSwEpiBlocks)
    L.resid = take((size_t)(std::max<int64_t>((int64_t)max_units + ceil_div(n, 4), kSwEpiBlocks) + 64) * 8);
    L.scal = take(64);
    L.srcs = take((size_t)(ceil_div(std::max(k, 1), kt) * kt) * 4);
    L.sw_bits = take((size_t)ceil_div(n, 64) * 8);
    L.sw_all = take((size_t)n * 4);
    L.sw_small = take((size_t)n * 4);
    L.sw_item_cap = (int32_t)std::min<int64_t>((int64_t)nnz / kSwChunk + n + 64, INT32_MAX / 4);
    L.sw_items = take((size_t)L.sw_item_cap * 3 * 4);
    L.sw_cnt = take(64);
    L.hist = take(tile * (size_t)std::max(hist_tiles, 0));
    L.total = p;
    return L;
}

static int32_t max_units(pp_graph g, int kt) {
    const KPlan a = kplan(g->pull_plan, kt), b = kplan(g->push_plan, kt);
    return std::max(a.units, b.units);
}

static bool valid_kt(int32_t kt) { return kt == 8 || kt == 16 || kt == 32 || kt == 64; }

// Launches a pull sweep over the row-unit plan a.kp; returns the residual
// slots written (units, then the fix-up's blocks) when a.resid_part is set.
template <int KT>
static int32_t launch_kpull(const KArgs& a_rows, int32_t nsplit, hipStream_t st, bool weighted) {
    KArgs a = a_rows;
    a.kp = kplan_pull4(a_rows.kp, KT);
    if (!kplan_valid(a_rows.kp) || !kplan_valid(a.kp) || kplan_bin_units(a.kp, 5) != kplan_bin_units(a_rows.kp, 5))
        return -1;  // never launch over an inconsistent plan
    if (a.kp.units > 0) {
        if (weighted) hipLaunchKernelGGL((k_kcol_pull<KT, true>), dim3(a.kp.units), dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_kcol_pull<KT, false>), dim3(a.kp.units), dim3(kBlock), 0, st, a);
    }
    float* resid_fix = a.resid_part ? a.resid_part + 2 * (size_t)a.kp.units : nullptr;
    if (nsplit > 0)
        hipLaunchKernelGGL((k_kcol_fix<KT>), dim3(ceil_div(nsplit, kBlock / KT)), dim3(kBlock), 0, st, a, nsplit,
                           resid_fix);
    return a.kp.units + (nsplit > 0 ? ceil_div(nsplit, kBlock / KT) : 0);
}

template <int KT>
static void launch_kpush(const KPushArgs& a, hipStream_t st, bool weighted) {
    if (a.kp.units == 0) return;
    if (weighted) hipLaunchKernelGGL((k_kcol_push<KT, true>), dim3(a.kp.units), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_kcol_push<KT, false>), dim3(a.kp.units), dim3(kBlock), 0, st, a);
}

// Pieces of the graph a k-column sweep walks: forward pull and adjoint push
// walk the CSC (pull lists); forward push and adjoint pull walk the CSR.
struct Walk {
    KPlan kp;
    const int32_t *off, *idx, *list, *tab;
    const float* wt;
    int32_t nsplit;
};

static Walk walk_csc(pp_graph g, int kt) {
    Walk w;
    w.kp = kplan(g->pull_plan, kt);
    w.off = g->d.csc_off;
    w.idx = g->d.csc_idx;
    w.list = g->d.pull_list;
    w.tab = g->d.split_tab;
    w.wt = g->d.csc_w;
    w.nsplit = g->pull_plan.count[5];
    return w;
}

static Walk walk_csr(pp_graph g, int kt) {
    Walk w;
    w.kp = kplan(g->push_plan, kt);
    w.off = g->d.csr_off;
    w.idx = g->d.csr_idx;
    w.list = g->d.push_list;
    w.tab = g->d.split_tab + 4 * (size_t)g->split_cap + 1;
    w.wt = g->d.csr_w;
    w.nsplit = g->push_plan.count[5];
    return w;
}

// Copies a tile (tile layout, internal ids) into caller layout columns.
template <int KT>
__global__ void k_tile_to_caller(int32_t n, int32_t k, int32_t col0, const int32_t* __restrict__ perm,
                                 const float* __restrict__ tile, float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * KT) return;
    const int32_t u = (int32_t)(t / KT);
    const int lane = (int)(t % KT);
    if (col0 + lane < k) out[(size_t)user_id(perm, u) * k + col0 + lane] = tile[t];
}

// Runs one tile for `iters` sweeps, or until the L1 change of a sweep falls
// below tol.  Forward state: t0/t1 iterates, t2/t3 scaled contributions;
// adjoint state: t0/t1 Lambda; t4 is the push accumulator.  On return
// *latest points at the newest iterate and *done holds the sweeps run.
// Sparse sweeps of a tile while the support is small (PP_SWITCH).  Forward:
// the support starts at the sources and grows along out-edges; the sweep
// pushes the scaled contributions along the CSR.  Adjoint: Lambda's support
// starts at the nonzero rows of dL/dX and grows along in-edges (the
// transposed sweep); the sweep pushes Lambda along the CSC and the epilogue
// forms dL/dX + f/s(u) * sum.  On return *done = sweeps taken (negative if
// the tolerance was met, then no dense sweep follows).  Buffers rotate as in
// the dense loop.
template <int KT>
static pp_status sparse_phase(pp_graph g, bool adjoint, int32_t k, int32_t col0, int32_t iters, float tol, float f,
                              const int32_t* src_int, const float* g_caller, char* base, const PprLayout& L,
                              float* prev, float* next, float* c_cur, float* c_nxt, double* t4, float* resid,
                              float* scal, int32_t* done, hipStream_t st) {
    const int32_t n = g->d.n;
    SwState w;
    w.bits = reinterpret_cast<uint64_t*>(base + L.sw_bits);
    w.all = reinterpret_cast<int32_t*>(base + L.sw_all);
    w.small = reinterpret_cast<int32_t*>(base + L.sw_small);
    w.items = reinterpret_cast<int32_t*>(base + L.sw_items);
    w.cnt = reinterpret_cast<int32_t*>(base + L.sw_cnt);
    w.item_cap = L.sw_item_cap;
    const Walk csr = adjoint ? walk_csc(g, KT) : walk_csr(g, KT);  // the rows the sweep scatters along
    w.off = csr.off;
    // the other tiles start at zero: cells outside the support stay zero
    const int64_t cells = (int64_t)n * KT;
    hipLaunchKernelGGL(k_zero_f32, dim3(std::min<int64_t>(ceil_div(cells, 256), 65536)), dim3(256), 0, st, cells, next);
    if (!adjoint)
        hipLaunchKernelGGL(k_zero_f32, dim3(std::min<int64_t>(ceil_div(cells, 256), 65536)), dim3(256), 0, st, cells,
                           c_nxt);
    hipLaunchKernelGGL(k_sw_clear, dim3(std::max(1, std::min(ceil_div(ceil_div(n, 64), 256), 4096))), dim3(256), 0,
                       st, ceil_div(n, 64), w.bits, w.cnt);
    if (adjoint)
        hipLaunchKernelGGL(k_sw_seed_rhs, dim3(std::max(1, std::min(ceil_div(n, 256), 4096))), dim3(256), 0, st, w, n,
                           k, col0, KT, g->d.perm, g_caller);
    else
        hipLaunchKernelGGL(k_sw_seed, dim3(1), dim3(64), 0, st, w, src_int, col0, KT);
    PP_LAUNCH_CHECK("ppr sparse seed");
    int32_t h[8] = {};
    PP_HIP(hipMemcpyAsync(h, w.cnt, sizeof(h), hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    const int64_t m_switch = g->d.nnz / kSwAlpha;
    const int32_t eb = std::min(g->num_cu * 4, kSwEpiBlocks);
    *done = 0;
    for (int32_t t = 0; t < iters; ++t) {
        const int64_t m_s = (int64_t)((uint64_t)(uint32_t)h[4] | ((uint64_t)(uint32_t)h[5] << 32));
        if (m_s > m_switch) break;  // dense from here on
        const int32_t units = h[1] + std::min(h[2], w.item_cap);
        // forward: the scaled contributions; adjoint: Lambda itself (the
        // epilogue applies f / s(u))
        const float* moved = adjoint ? prev : c_cur;
        if (units > 0) {
            const int32_t blocks = std::max(1, std::min(eb, ceil_div(units, kBlock / KT)));
            if (g->weighted)
                hipLaunchKernelGGL((k_sw_scatter<KT, true>), dim3(blocks), dim3(kBlock), 0, st, w, csr.idx, csr.wt,
                                   moved, t4, h[1], std::min(h[2], w.item_cap));
            else
                hipLaunchKernelGGL((k_sw_scatter<KT, false>), dim3(blocks), dim3(kBlock), 0, st, w, csr.idx, csr.wt,
                                   moved, t4, h[1], std::min(h[2], w.item_cap));
        }
        KArgs a{};
        a.kind = adjoint ? kEpiAdjoint : kEpiForward;
        a.inv_s = g->d.inv_s;
        a.perm = g->d.perm;
        a.f = f;
        a.k = k;
        a.col0 = col0;
        a.src_int = src_int;
        a.g_caller = g_caller;
        a.prev = prev;
        a.out_tile = next;
        a.out_scaled = adjoint ? nullptr : c_nxt;
        a.resid_part = resid;
        hipLaunchKernelGGL(k_sw_epi<KT>, dim3(eb), dim3(kBlock), 0, st, a, w, t4);
        PP_LAUNCH_CHECK("ppr sparse sweep");
        ++*done;
        std::swap(prev, next);
        std::swap(c_cur, c_nxt);
        if (tol > 0.f && t + 1 < iters)
            hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, eb, (const float*)resid, scal);
        PP_HIP(hipMemcpyAsync(h, w.cnt, sizeof(h), hipMemcpyDeviceToHost, st));
        float r[2] = {0.f, 0.f};
        if (tol > 0.f && t + 1 < iters) PP_HIP(hipMemcpyAsync(r, scal, sizeof(r), hipMemcpyDeviceToHost, st));
        PP_HIP(hipStreamSynchronize(st));
        if (h[3]) return set_error(PP_E_WORKSPACE, "sparse PPR item capacity exceeded");
        if (tol > 0.f && t + 1 < iters && r[0] <= tol * r[1]) {
            *done = -*done;
            return PP_OK;
        }
    }
    return PP_OK;
}

template <int KT>
static pp_status run_tile(pp_graph g, bool adjoint, pp_dir dir, int32_t k, int32_t col0, int32_t iters, float tol,
                          float f, const int32_t* src_int, const float* g_caller, char* base, const PprLayout& L,
                          float** latest, int32_t* done, hipStream_t st) {
    const int32_t n = g->d.n;
    float* t0 = reinterpret_cast<float*>(base + L.t0);
    float* t1 = reinterpret_cast<float*>(base + L.t1);
    float* t2 = reinterpret_cast<float*>(base + L.t2);
    float* t3 = reinterpret_cast<float*>(base + L.t3);
    double* t4 = reinterpret_cast<double*>(base + L.t4);
    float* part = reinterpret_cast<float*>(base + L.part);
    float* resid = reinterpret_cast<float*>(base + L.resid);
    float* scal = reinterpret_cast<float*>(base + L.scal);
    const int64_t cells = (int64_t)n * KT;
    const dim3 cb(ceil_div(cells, 256)), ct(256);
    if (adjoint) hipLaunchKernelGGL(k_kcol_adjoint_init<KT>, cb, ct, 0, st, n, k, col0, g->d.perm, g_caller, t0, t4);
    else hipLaunchKernelGGL(k_kcol_forward_init<KT>, cb, ct, 0, st, n, src_int, col0, f, g->d.inv_s, t0, t2, t4);
    PP_LAUNCH_CHECK("ppr tile init");
    float* prev = t0;   // current iterate
    float* next = t1;
    float* c_cur = t2;  // forward: scaled contributions of prev
    float* c_nxt = t3;
    *done = 0;
    int32_t t0_dense = 0;  // first dense sweep
    if (dir == PP_SWITCH) {
        pp_status s = sparse_phase<KT>(g, adjoint, k, col0, iters, tol, f, src_int, g_caller, base, L, prev, next,
                                       c_cur, c_nxt, t4, resid, scal, done, st);
        if (s != PP_OK) return s;
        t0_dense = *done;
        if (*done & 1) {  // the sparse sweeps swapped the buffers an odd number of times
            std::swap(prev, next);
            std::swap(c_cur, c_nxt);
        }
        if (*done < 0) {  // converged during the sparse phase
            *done = -*done;
            *latest = ((*done) & 1) ? t1 : t0;
            return PP_OK;
        }
    }
    const bool pull = (dir != PP_PUSH);
    for (int32_t t = t0_dense; t < iters; ++t) {
        KArgs a{};
        a.kind = adjoint ? kEpiAdjoint : kEpiForward;
        a.inv_s = g->d.inv_s;
        a.perm = g->d.perm;
        a.f = f;
        a.k = k;
        a.col0 = col0;
        a.src_int = src_int;
        a.prev = prev;
        a.out_tile = next;
        a.out_scaled = adjoint ? nullptr : c_nxt;
        a.g_caller = g_caller;
        a.out_caller = nullptr;
        a.resid_part = resid;
        const float* moved = adjoint ? prev : c_cur;
        int32_t nres = 0;
        if (pull) {
            // forward pull gathers along CSC; the adjoint pull gathers along CSR
            const Walk w = adjoint ? walk_csr(g, KT) : walk_csc(g, KT);
            a.kp = w.kp;
            a.off = w.off;
            a.idx = w.idx;
            a.wt = w.wt;
            a.list = w.list;
            a.tab = w.tab;
            a.tab_cap = g->split_cap;
            a.part = part;
            a.src = moved;
            nres = launch_kpull<KT>(a, w.nsplit, st, g->weighted);
            if (nres < 0) return set_error(PP_E_GRAPH, "inconsistent k-column sweep plan");
        } else {
            // forward push scatters along CSR; the adjoint push scatters along CSC
            const Walk w = adjoint ? walk_csc(g, KT) : walk_csr(g, KT);
            KPushArgs p{};
            p.kp = w.kp;
            p.off = w.off;
            p.idx = w.idx;
            p.wt = w.wt;
            p.list = w.list;
            p.tab = w.tab;
            p.tab_cap = g->split_cap;
            p.src = moved;
            p.acc = t4;
            launch_kpush<KT>(p, st, g->weighted);
            hipLaunchKernelGGL(k_kcol_push_epi<KT>, dim3(ceil_div(n, kBlock / KT)), dim3(kBlock), 0, st, a, n, t4);
            nres = ceil_div(n, kBlock / KT);
        }
        PP_LAUNCH_CHECK("ppr sweep");
        ++*done;
        std::swap(prev, next);
        std::swap(c_cur, c_nxt);
        if (tol > 0.f && t + 1 < iters) {
            float r[2] = {0.f, 0.f};
            hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, nres, (const float*)resid, scal);
            PP_HIP(hipMemcpyAsync(r, scal, sizeof(r), hipMemcpyDeviceToHost, st));
            PP_HIP(hipStreamSynchronize(st));
            if (r[0] <= tol * r[1]) break;  // L1 change relative to the L1 norm of the tile
        }
    }
    *latest = prev;
    return PP_OK;
}

// (P^T Lambda) of one tile by a CSR gather, then the tile's edge gradient
// added into grad (caller CSR slot order).
template <int KT>
static pp_status adjoint_grad(pp_graph g, int32_t k, int32_t col0, float f, const float* lam, float* ptl,
                              float* part, const float* x_caller, float* grad, hipStream_t st,
                              const float* x_tile = nullptr) {
    const Walk w = walk_csr(g, KT);
    KArgs a{};
    a.kind = kEpiPtl;
    a.inv_s = g->d.inv_s;
    a.perm = g->d.perm;
    a.f = f;
    a.k = k;
    a.col0 = col0;
    a.out_tile = ptl;
    a.kp = w.kp;
    a.off = w.off;
    a.idx = w.idx;
    a.wt = w.wt;
    a.list = w.list;
    a.tab = w.tab;
    a.tab_cap = g->split_cap;
    a.part = part;
    a.src = lam;
    if (launch_kpull<KT>(a, w.nsplit, st, g->weighted) < 0)
        return set_error(PP_E_GRAPH, "inconsistent k-column sweep plan");
    GradArgs ga{};
    ga.kp = w.kp;
    ga.off = w.off;
    ga.idx = w.idx;
    ga.list = w.list;
    ga.tab = w.tab;
    ga.tab_cap = g->split_cap;
    ga.lam = lam;
    ga.ptl = ptl;
    ga.x_caller = x_caller;
    ga.x_tile = x_tile;
    ga.inv_s = g->d.inv_s;
    ga.perm = g->d.perm;
    ga.user_off = g->d.user_csr_off;
    ga.k = k;
    ga.col0 = col0;
    ga.f = f;
    ga.grad = grad;
    if (w.kp.units > 0) hipLaunchKernelGGL(k_kcol_grad<KT>, dim3(w.kp.units), dim3(kBlock), 0, st, ga);
    PP_LAUNCH_CHECK("ppr adjoint gradient");
    return PP_OK;
}

// Unrolled adjoint of one tile: the T-step forward iterates X_0..X_{T-1}
// (pull sweeps, kept in `hist`), then T reverse steps.  With Lambda =
// dL/dX_{t+1}: the edge gradient of step t from X_t (CSR gather of
// P^T Lambda, then k_kcol_grad), and Lambda <- f P^T Lambda.
template <int KT>
static pp_status unrolled_tile(pp_graph g, int32_t k, int32_t col0, int32_t T, float f, const int32_t* src_int,
                               const float* g_caller, char* base, const PprLayout& L, float* lambda0, float* grad,
                               hipStream_t st) {
    const int32_t n = g->d.n;
    const int64_t cells = (int64_t)n * KT;
    const size_t tile = (size_t)cells;
    float* t0 = reinterpret_cast<float*>(base + L.t0);
    float* t1 = reinterpret_cast<float*>(base + L.t1);
    float* c_cur = reinterpret_cast<float*>(base + L.t2);
    float* c_nxt = reinterpret_cast<float*>(base + L.t3);
    float* part = reinterpret_cast<float*>(base + L.part);
    float* hist = reinterpret_cast<float*>(base + L.hist);
    const dim3 cb(ceil_div(cells, 256)), ct(256);
    if (T > 0) {
        hipLaunchKernelGGL(k_kcol_forward_init<KT>, cb, ct, 0, st, n, src_int, col0, f, g->d.inv_s, hist, c_cur,
                           (double*)nullptr);
        const Walk w = walk_csc(g, KT);
        for (int32_t t = 0; t + 1 < T; ++t) {
            KArgs a{};
            a.kind = kEpiForward;
            a.inv_s = g->d.inv_s;
            a.perm = g->d.perm;
            a.f = f;
            a.k = k;
            a.col0 = col0;
            a.src_int = src_int;
            a.out_tile = hist + (size_t)(t + 1) * tile;
            a.out_scaled = c_nxt;
            a.kp = w.kp;
            a.off = w.off;
            a.idx = w.idx;
            a.wt = w.wt;
            a.list = w.list;
            a.tab = w.tab;
            a.tab_cap = g->split_cap;
            a.part = part;
            a.src = c_cur;
            if (launch_kpull<KT>(a, w.nsplit, st, g->weighted) < 0)
                return set_error(PP_E_GRAPH, "inconsistent k-column sweep plan");
            std::swap(c_cur, c_nxt);
        }
        PP_LAUNCH_CHECK("ppr unrolled forward");
    }
    float* lam = t0;
    float* ptl = t1;
    hipLaunchKernelGGL(k_kcol_adjoint_init<KT>, cb, ct, 0, st, n, k, col0, g->d.perm, g_caller, lam, (double*)nullptr);
    for (int32_t t = T - 1; t >= 0; --t) {
        pp_status s = adjoint_grad<KT>(g, k, col0, f, lam, ptl, part, nullptr, grad, st, hist + (size_t)t * tile);
        if (s != PP_OK) return s;
        hipLaunchKernelGGL(k_scale_f32, dim3(std::min<int64_t>(ceil_div(cells, 256), 65536)), dim3(256), 0, st, cells,
                           f, ptl);
        std::swap(lam, ptl);
    }
    hipLaunchKernelGGL(k_tile_to_caller<KT>, cb, ct, 0, st, n, k, col0, g->d.perm, (const float*)lam, lambda0);
    PP_LAUNCH_CHECK("ppr unrolled adjoint");
    return PP_OK;
}

template <int KT>
static pp_status unrolled_call(pp_graph g, int32_t k, const int32_t* sources, int32_t T, float f,
                               const float* dLdXT, float* lambda0, float* grad, char* base, const PprLayout& L,
                               hipStream_t st) {
    const int32_t n = g->d.n;
    int32_t* src_int = reinterpret_cast<int32_t*>(base + L.srcs);
    int32_t* flag = reinterpret_cast<int32_t*>(base + L.scal) + 8;
    int32_t bad = 0;
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, st, (int64_t)1, reinterpret_cast<float*>(flag));
    const int32_t k_pad = ceil_div(k, KT) * KT;
    hipLaunchKernelGGL(k_sources_internal, dim3(ceil_div(k_pad, 256)), dim3(256), 0, st, k, k_pad, sources,
                       g->d.iperm, n, src_int, flag);
    PP_LAUNCH_CHECK("ppr sources");
    PP_HIP(hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    if (bad) return set_error(PP_E_RANGE, "a source lies outside [0, n)");
    if (g->d.nnz > 0)
        hipLaunchKernelGGL(k_zero_f32, dim3(std::min<int64_t>(ceil_div(g->d.nnz, 256), 65536)), dim3(256), 0, st,
                           g->d.nnz, grad);
    for (int32_t col0 = 0; col0 < k; col0 += KT) {
        pp_status s = unrolled_tile<KT>(g, k, col0, T, f, src_int, dLdXT, base, L, lambda0, grad, st);
        if (s != PP_OK) return s;
    }
    return PP_OK;
}

struct PprCall {
    pp_graph g;
    bool adjoint;
    pp_dir dir;
    int32_t k, iters, kt;
    float tol, f;
    const int32_t* sources;  // forward
    const float* x_caller;   // adjoint: forward solution
    const float* g_caller;   // adjoint: dL/dX
    float* out;              // X (forward) or Lambda (adjoint), caller layout
    float* grad;             // adjoint: per CSR slot
    char* base;
    PprLayout L;
    hipStream_t st;
};

template <int KT>
static pp_status ppr_call(const PprCall& c, int32_t* iters_done) {
    const int32_t n = c.g->d.n;
    int32_t* src_int = reinterpret_cast<int32_t*>(c.base + c.L.srcs);
    int32_t* flag = reinterpret_cast<int32_t*>(c.base + c.L.scal) + 8;
    if (!c.adjoint) {
        int32_t bad = 0;
        hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, c.st, (int64_t)1, reinterpret_cast<float*>(flag));
        const int32_t k_pad = ceil_div(c.k, KT) * KT;
        hipLaunchKernelGGL(k_sources_internal, dim3(ceil_div(k_pad, 256)), dim3(256), 0, c.st, c.k, k_pad, c.sources,
                           c.g->d.iperm, n, src_int, flag);
        PP_LAUNCH_CHECK("ppr sources");
        PP_HIP(hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, c.st));
        PP_HIP(hipStreamSynchronize(c.st));
        if (bad) return set_error(PP_E_RANGE, "a source lies outside [0, n)");
    } else if (c.g->d.nnz > 0) {
        hipLaunchKernelGGL(k_zero_f32, dim3(ceil_div(c.g->d.nnz, 256)), dim3(256), 0, c.st, c.g->d.nnz, c.grad);
    }
    int32_t most = 0;
    for (int32_t col0 = 0; col0 < c.k; col0 += KT) {
        float* latest = nullptr;
        int32_t done = 0;
        pp_status s = run_tile<KT>(c.g, c.adjoint, c.dir, c.k, col0, c.iters, c.tol, c.f, src_int, c.g_caller, c.base,
                                   c.L, &latest, &done, c.st);
        if (s != PP_OK) return s;
        most = std::max(most, done);
        hipLaunchKernelGGL(k_tile_to_caller<KT>, dim3(ceil_div((int64_t)n * KT, 256)), dim3(256), 0, c.st, n, c.k,
                           col0, c.g->d.perm, (const float*)latest, c.out);
        PP_LAUNCH_CHECK("ppr tile copy-out");
        if (c.adjoint) {
            float* t0 = reinterpret_cast<float*>(c.base + c.L.t0);
            float* ptl = (latest == t0) ? reinterpret_cast<float*>(c.base + c.L.t1) : t0;
            s = adjoint_grad<KT>(c.g, c.k, col0, c.f, latest, ptl, reinterpret_cast<float*>(c.base + c.L.part),
                                 c.x_caller, c.grad, c.st);
            if (s != PP_OK) return s;
        }
    }
    if (iters_done) *iters_done = most;
    return PP_OK;
}

static pp_status ppr_dispatch(const PprCall& c, int32_t* iters_done) {
    switch (c.kt) {
        case 8: return ppr_call<8>(c, iters_done);
        case 16: return ppr_call<16>(c, iters_done);
        case 32: return ppr_call<32>(c, iters_done);
        default: return ppr_call<64>(c, iters_done);
    }
}

static pp_status check_ppr(pp_graph g, pp_dir dir, int32_t k, int32_t iters, float tol, float f, int32_t kt,
                           void* scratch, size_t bytes, size_t need) {
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (dir != PP_PUSH && dir != PP_PULL && dir != PP_SWITCH)
        return set_error(PP_E_RANGE, "dir must be PP_PUSH, PP_PULL or PP_SWITCH");
    if (k < 0) return set_error(PP_E_SIZE, "k must be >= 0");
    if (!valid_kt(kt)) return set_error(PP_E_RANGE, "k_tile must be 8, 16, 32 or 64");
    if (iters < 0) return set_error(PP_E_RANGE, "iters must be >= 0");
    if (!(tol >= 0.f)) return set_error(PP_E_RANGE, "tol must be >= 0");
    if (!(f >= 0.f && f < 1.f)) return set_error(PP_E_RANGE, "f must lie in [0, 1)");
    if (!scratch) return set_error(PP_E_NULL, "scratch is NULL");
    if (bytes < need) return set_error(PP_E_WORKSPACE, "PPR scratch too small");
    if (reinterpret_cast<uintptr_t>(scratch) % 256 != 0) return set_error(PP_E_RANGE, "scratch must be 256-byte aligned");
    return PP_OK;
}

// k_tile = 1: the columns one after another, each with the single-vector
// pull or push sweep (the "k sequential sweeps" a batched run is measured
// against).  Scratch: the sources' internal ids and a flag.
static size_t single_scratch_bytes(int32_t k) { return align_up((size_t)std::max(k, 1) * 4, 256) + 256; }

static pp_status ppr_single(pp_graph g, pp_dir dir, int32_t k, const int32_t* sources, int32_t iters, float tol,
                            float f, float* X, void* scratch, size_t scratch_bytes, int32_t* iters_done,
                            hipStream_t st) {
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (dir != PP_PUSH && dir != PP_PULL) return set_error(PP_E_RANGE, "k_tile 1 runs PP_PUSH or PP_PULL sweeps");
    if (k < 0) return set_error(PP_E_SIZE, "k must be >= 0");
    if (iters < 0) return set_error(PP_E_RANGE, "iters must be >= 0");
    if (tol != 0.f) return set_error(PP_E_RANGE, "k_tile 1 runs a fixed number of sweeps (tol must be 0)");
    if (!(f >= 0.f && f < 1.f)) return set_error(PP_E_RANGE, "f must lie in [0, 1)");
    if (!scratch) return set_error(PP_E_NULL, "scratch is NULL");
    if (scratch_bytes < single_scratch_bytes(k)) return set_error(PP_E_WORKSPACE, "PPR scratch too small");
    if (reinterpret_cast<uintptr_t>(scratch) % 256 != 0) return set_error(PP_E_RANGE, "scratch must be 256-byte aligned");
    if (k > 0 && (!sources || !X)) return set_error(PP_E_NULL, "sources and X are required");
    if (iters_done) *iters_done = 0;
    if (k == 0) return PP_OK;
    int32_t* src_int = static_cast<int32_t*>(scratch);
    int32_t* flag = reinterpret_cast<int32_t*>(static_cast<char*>(scratch) + align_up((size_t)k * 4, 256));
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, st, (int64_t)1, reinterpret_cast<float*>(flag));
    hipLaunchKernelGGL(k_sources_internal, dim3(ceil_div(k, 256)), dim3(256), 0, st, k, k, sources, g->d.iperm,
                       g->d.n, src_int, flag);
    PP_LAUNCH_CHECK("ppr sources");
    std::vector<int32_t> s_int(k);
    int32_t bad = 0;
    PP_HIP(hipMemcpyAsync(s_int.data(), src_int, (size_t)k * 4, hipMemcpyDeviceToHost, st));
    PP_HIP(hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    if (bad) return set_error(PP_E_RANGE, "a source lies outside [0, n)");
    for (int32_t j = 0; j < k; ++j) {
        pp_status s = run_single_ppr(g, dir, s_int[j], iters, f, X + j, k, st);
        if (s != PP_OK) return s;
    }
    if (iters_done) *iters_done = iters;
    return PP_OK;
}

}  // namespace pp

using namespace pp;

PP_EXPORT size_t pp_ppr_scratch_bytes(pp_graph g, int32_t k, int32_t k_tile) {
    if (!g || k < 0) return 0;
    if (k_tile == 1) return single_scratch_bytes(k);
    if (!valid_kt(k_tile)) return 0;
    return ppr_layout(g->d.n, g->d.nnz, g->split_cap, k, k_tile, max_units(g, k_tile)).total;
}

PP_EXPORT pp_status pp_ppr_run(pp_graph g, pp_dir dir, int32_t k, const int32_t* sources, int32_t iters, float tol,
                               float f, int32_t k_tile, float* X, void* scratch, size_t scratch_bytes,
                               int32_t* iters_done, void* stream) {
    clear_error();
    if (k_tile == 1)
        return ppr_single(g, dir, k, sources, iters, tol, f, X, scratch, scratch_bytes, iters_done,
                          static_cast<hipStream_t>(stream));
    const size_t need = pp_ppr_scratch_bytes(g, k, k_tile);
    pp_status s = check_ppr(g, dir, k, iters, tol, f, k_tile, scratch, scratch_bytes, need);
    if (s != PP_OK) return s;
    if (k > 0 && (!sources || !X)) return set_error(PP_E_NULL, "sources and X are required");
    if (iters_done) *iters_done = 0;
    if (k == 0) return PP_OK;
    PprCall c{};
    c.g = g;
    c.adjoint = false;
    c.dir = dir;
    c.k = k;
    c.iters = iters;
    c.kt = k_tile;
    c.tol = tol;
    c.f = f;
    c.sources = sources;
    c.out = X;
    c.base = static_cast<char*>(scratch);
    c.L = ppr_layout(g->d.n, g->d.nnz, g->split_cap, k, k_tile, max_units(g, k_tile));
    c.st = static_cast<hipStream_t>(stream);
    return ppr_dispatch(c, iters_done);
}

PP_EXPORT pp_status pp_ppr_adjoint(pp_graph g, pp_dir dir, int32_t k, const float* X, const float* dLdX,
                                   int32_t iters, float tol, float f, int32_t k_tile, float* Lambda, float* grad_w,
                                   void* scratch, size_t scratch_bytes, int32_t* iters_done, void* stream) {
    clear_error();
    const size_t need = pp_ppr_scratch_bytes(g, k, k_tile);
    pp_status s = check_ppr(g, dir, k, iters, tol, f, k_tile, scratch, scratch_bytes, need);
    if (s != PP_OK) return s;
    if (k > 0 && (!X || !dLdX || !Lambda)) return set_error(PP_E_NULL, "X, dLdX and Lambda are required");
    if (g->d.nnz > 0 && !grad_w) return set_error(PP_E_NULL, "grad_w is required");
    if (iters_done) *iters_done = 0;
    if (k == 0) return PP_OK;
    PprCall c{};
    c.g = g;
    c.adjoint = true;
    c.dir = dir;
    c.k = k;
    c.iters = iters;
    c.kt = k_tile;
    c.tol = tol;
    c.f = f;
    c.x_caller = X;
    c.g_caller = dLdX;
    c.out = Lambda;
    c.grad = grad_w;
    c.base = static_cast<char*>(scratch);
    c.L = ppr_layout(g->d.n, g->d.nnz, g->split_cap, k, k_tile, max_units(g, k_tile));
    c.st = static_cast<hipStream_t>(stream);
    return ppr_dispatch(c, iters_done);
}

PP_EXPORT size_t pp_ppr_unrolled_scratch_bytes(pp_graph g, int32_t k, int32_t k_tile, int32_t T) {
    if (!g || !valid_kt(k_tile) || k < 0 || T < 0) return 0;
    return ppr_layout(g->d.n, g->d.nnz, g->split_cap, k, k_tile, max_units(g, k_tile), T).total;
}

PP_EXPORT pp_status pp_ppr_adjoint_unrolled(pp_graph g, int32_t k, const int32_t* sources, int32_t T, float f,
                                            int32_t k_tile, const float* dLdXT, float* Lambda0, float* grad_w,
                                            void* scratch, size_t scratch_bytes, void* stream) {
    clear_error();
    if (T < 0) return set_error(PP_E_RANGE, "T must be >= 0");
    const size_t need = pp_ppr_unrolled_scratch_bytes(g, k, k_tile, T);
    pp_status s = check_ppr(g, PP_PULL, k, T, 0.f, f, k_tile, scratch, scratch_bytes, need);
    if (s != PP_OK) return s;
    if (k > 0 && (!sources || !dLdXT || !Lambda0)) return set_error(PP_E_NULL, "sources, dLdXT and Lambda0 are required");
    if (g->d.nnz > 0 && !grad_w) return set_error(PP_E_NULL, "grad_w is required");
    if (k == 0) return PP_OK;
    char* base = static_cast<char*>(scratch);
    const PprLayout L = ppr_layout(g->d.n, g->d.nnz, g->split_cap, k, k_tile, max_units(g, k_tile), T);
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (k_tile) {
        case 8: return unrolled_call<8>(g, k, sources, T, f, dLdXT, Lambda0, grad_w, base, L, st);
        case 16: return unrolled_call<16>(g, k, sources, T, f, dLdXT, Lambda0, grad_w, base, L, st);
        case 32: return unrolled_call<32>(g, k, sources, T, f, dLdXT, Lambda0, grad_w, base, L, st);
        default: return unrolled_call<64>(g, k, sources, T, f, dLdXT, Lambda0, grad_w, base, L, st);
    }
}
