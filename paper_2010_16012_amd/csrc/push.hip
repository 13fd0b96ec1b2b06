// PageRank power-iteration step in its pushing form (Sec. 3.1 equation;
// Sec. 4.1 listing, pushing lines): every row scatters its contribution
// c[v] = f * x[v] / s(v) to the accumulators of its out-neighbours.
//
// Updates to the first `hot` targets are privatised per workgroup in LDS and
// merged in fixed order (Sec. 5 Partition-Awareness, the workgroup being the
// owner); the others are either hardware FP32 atomics or, binned, appended
// to per-workgroup slices of 16384-id bins and summed in LDS by a second
// kernel (the remote updates buffered instead of applied one by one).
#include <hip/hip_runtime.h>

#include <vector>

#include "pp_common.h"
#include "sweep.h"

namespace pp {

// ------------------------------------------------------------------ push
struct PushArgs {
    SweepPlan sp;
    const int32_t* off;    // CSR offsets
    const int32_t* idx;    // CSR indices
    const float* wt;       // weights in CSR slot order (weighted only)
    const int32_t* list;   // vertices grouped by out-degree bin
    const int32_t* tab;
    int32_t tab_cap;
    int32_t units;         // work units (= blocks of the one-shot layout)
    int32_t hot;           // targets below this id go to LDS first
    float* hot_part;       // [gridDim.x][hot] per-workgroup partial sums
    const float* c;        // contributions
    float* y;              // accumulator (internal ids), pre-set to (1-f)/n
    // binned push: target u >= hot goes to bin (u - hot) >> kPushBinShift
    int32_t nbins;
    const int32_t* pb_base;  // [gridDim.x][nbins] first pair of each slice
    int32_t* pb_cnt;         // [gridDim.x][nbins] slice sizes (written by the counting walk)
    int32_t* pb_fill;        // [gridDim.x][nbins] pairs this sweep wrote
    int2* pb_pairs;          // (target - hot - bin start, value bits)
};

// What a push sweep does with an update to a target past the privatised ones.
enum PushMode {
    kPushAtomic = 0,  // global FP32 atomic add
    kPushBinned = 1,  // append to this workgroup's slice of the target's bin
    kPushCount = 2    // registration: count the slice sizes, touch nothing else
};

// LDS after the privatised targets (binned and counting modes): per bin the
// workgroup's append counter, its slice start and its slice size.
struct PushLds {
    float* hot;
    int32_t* bin;  // [3][nbins]
};

// Adds val to target u: LDS for privatised (hot) targets, else by MODE.
template <bool HOT, int MODE>
__device__ __forceinline__ void push_to(const PushArgs& a, const PushLds& s, int32_t u, float val) {
    if (HOT && u < a.hot) {
        if (MODE != kPushCount) atomicAdd(&s.hot[u], val);
        return;
    }
    if (MODE == kPushAtomic) {
        unsafeAtomicAdd(&a.y[u], val);  // global_atomic_add_f32, result unused
        return;
    }
    const int32_t r = u - a.hot;
    const int32_t b = r >> kPushBinShift;
    const int32_t k = atomicAdd(&s.bin[b], 1);
    if (MODE == kPushBinned && k < s.bin[2 * a.nbins + b])
        a.pb_pairs[s.bin[a.nbins + b] + k] = make_int2(r & (kPushBinW - 1), __float_as_int(val));
}

// U index loads issued back to back, then the U adds.
template <int G, bool W, bool HOT, int MODE>
__device__ __forceinline__ void scatter_row(const PushArgs& a, const PushLds& s, float cv, int32_t b, int32_t e,
                                            int lane) {
    constexpr int U = unroll_for<G>();
    for (int32_t j0 = b + lane; j0 < e; j0 += U * G) {
        int32_t jj[U], uu[U];
#pragma unroll
        for (int k = 0; k < U; ++k) jj[k] = min(j0 + k * G, e - 1);
#pragma unroll
        for (int k = 0; k < U; ++k) uu[k] = a.idx[jj[k]];
        float val[U];
#pragma unroll
        for (int k = 0; k < U; ++k) val[k] = (W && MODE != kPushCount) ? cv * a.wt[jj[k]] : cv;
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (j0 + k * G < e) push_to<HOT, MODE>(a, s, uu[k], val[k]);
    }
}

// The contribution of row v; the counting walk visits every row.
template <int MODE>
__device__ __forceinline__ float push_cv(const PushArgs& a, int32_t v) {
    return (MODE == kPushCount) ? 1.f : a.c[v];
}

// Unit local_blk of bin `bin` for one kBlock-thread slice (thread tid).
template <int G, bool W, bool HOT, int MODE>
__device__ __forceinline__ void push_group(const PushArgs& a, const PushLds& s, int bin, int32_t local_blk, int tid) {
    constexpr int per_block = kBlock / G;
    const int32_t i = local_blk * per_block + tid / G;
    const int lane = tid & (G - 1);
    const int32_t count = a.sp.list_off[bin + 1] - a.sp.list_off[bin];
    if (i < count) {
        const int32_t v = a.list[a.sp.list_off[bin] + i];
        const float cv = push_cv<MODE>(a, v);
        if (cv != 0.f) scatter_row<G, W, HOT, MODE>(a, s, cv, a.off[v], a.off[v + 1], lane);
    }
}

// Persistent: a workgroup is SUB slices of kBlock threads; slice q of
// workgroup b takes units b*SUB + q, then strides by gridDim.x*SUB (a static
// assignment, which the binned mode's slice sizes rely on).  With HOT, LDS
// holds the workgroup's sums for targets [0, hot) (SUB = 4 lets one
// workgroup per CU privatise up to the whole LDS), written out at the end.
template <int SUB, bool W, bool HOT, int MODE>
__global__ __launch_bounds__(SUB * kBlock) void k_pr_push(PushArgs a) {
    extern __shared__ float s_dyn[];
    const PushLds s{s_dyn, reinterpret_cast<int32_t*>(s_dyn + a.hot)};
    if (HOT && MODE != kPushCount)
        for (int32_t i = threadIdx.x; i < a.hot; i += SUB * kBlock) s.hot[i] = 0.f;
    if (MODE != kPushAtomic) {
        for (int32_t b = threadIdx.x; b < a.nbins; b += SUB * kBlock) {
            s.bin[b] = 0;
            if (MODE == kPushBinned) {
                s.bin[a.nbins + b] = a.pb_base[(size_t)blockIdx.x * a.nbins + b];
                s.bin[2 * a.nbins + b] = a.pb_cnt[(size_t)blockIdx.x * a.nbins + b];
            }
        }
    }
    if (HOT || MODE != kPushAtomic) __syncthreads();
    const int q = threadIdx.x / kBlock;
    const int tid = threadIdx.x % kBlock;
    for (int32_t unit = blockIdx.x * SUB + q; unit < a.units; unit += gridDim.x * SUB) {
        const int bin = unit_bin(a.sp, unit);
        const int32_t lb = unit - a.sp.block_off[bin];
        switch (bin) {
            case 5: {
                const int32_t v = a.tab[lb];
                const int32_t b = a.tab[a.tab_cap + lb], e = a.tab[2 * a.tab_cap + lb];
                const float cv = push_cv<MODE>(a, v);
                if (cv != 0.f) scatter_row<kBlock, W, HOT, MODE>(a, s, cv, b, e, tid);
                break;
            }
            case 4: {
                const int32_t v = a.list[a.sp.list_off[4] + lb];
                const float cv = push_cv<MODE>(a, v);
                if (cv != 0.f) scatter_row<kBlock, W, HOT, MODE>(a, s, cv, a.off[v], a.off[v + 1], tid);
                break;
            }
            case 3: push_group<64, W, HOT, MODE>(a, s, 3, lb, tid); break;
            case 2: push_group<16, W, HOT, MODE>(a, s, 2, lb, tid); break;
            case 1: push_group<4, W, HOT, MODE>(a, s, 1, lb, tid); break;
            default: push_group<1, W, HOT, MODE>(a, s, 0, lb, tid); break;
        }
    }
    if (HOT || MODE != kPushAtomic) __syncthreads();
    if (HOT && MODE != kPushCount) {
        float* dst = a.hot_part + (size_t)blockIdx.x * a.hot;
        for (int32_t i = threadIdx.x; i < a.hot; i += SUB * kBlock) dst[i] = s.hot[i];
    }
    if (MODE == kPushCount)
        for (int32_t b = threadIdx.x; b < a.nbins; b += SUB * kBlock) a.pb_cnt[(size_t)blockIdx.x * a.nbins + b] = s.bin[b];
    if (MODE == kPushBinned)
        for (int32_t b = threadIdx.x; b < a.nbins; b += SUB * kBlock)
            a.pb_fill[(size_t)blockIdx.x * a.nbins + b] = min(s.bin[b], s.bin[2 * a.nbins + b]);
}

// Pairs are read once: non-temporal loads keep them from evicting the lines
// that are read again (about 2% off the push step at R-MAT scale 22; the
// pushes store them normally, where the L2 merges the scattered 8-byte
// stores into lines).
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));  // non-temporal loads take a native vector

// Binned push, second kernel: unit k sums the pairs of bin units[3k] written
// by workgroups [units[3k+1], units[3k+2]) into an LDS accumulator of the
// bin's kPushBinW targets (LDS float atomics), then writes it out whole as
// the unit's partial.  Each wavefront sums whole slices (wavefront j takes
// slices w0 + j, w0 + j + 16, ...): a slice holds about a thousand pairs,
// so a workgroup working through one slice at a time left most lanes idle
// and waited a round trip per slice.  The slice bounds are read through
// scalar loads.
__global__ __launch_bounds__(1024) void k_pr_push_bins(int32_t nbins, const int32_t* __restrict__ units,
                                                       const int32_t* __restrict__ base,
                                                       const int32_t* __restrict__ fill,
                                                       const int2* __restrict__ pairs, float* __restrict__ part) {
    extern __shared__ float acc[];
    const int32_t k = blockIdx.x;
    const int32_t b = uniform_load(units, 3 * k), w0 = uniform_load(units, 3 * k + 1),
                  w1 = uniform_load(units, 3 * k + 2);
    const int32_t bd = blockDim.x;
    for (int32_t i = threadIdx.x; i < kPushBinW; i += bd) acc[i] = 0.f;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int32_t nwv = bd / kWave;
    constexpr int kR = 4;  // pair loads in flight per lane
    for (int32_t w = w0 + wv; w < w1; w += nwv) {
        const int32_t lo = uniform_load(base + (size_t)w * nbins, b), cnt = uniform_load(fill + (size_t)w * nbins, b);
        for (int32_t i = lane; i < cnt; i += kR * kWave) {
            int2 e[kR];
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const i32x2 q = __builtin_nontemporal_load(reinterpret_cast<const i32x2*>(pairs) +
                                                           (lo + min(i + r * kWave, cnt - 1)));
                e[r] = make_int2(q.x, q.y);
            }
#pragma unroll
            for (int r = 0; r < kR; ++r)
                if (i + r * kWave < cnt) atomicAdd(&acc[e[r].x & (kPushBinW - 1)], __int_as_float(e[r].y));
        }
    }
    __syncthreads();
    float* dst = part + (size_t)k * kPushBinW;
    for (int32_t i = threadIdx.x; i < kPushBinW; i += bd) dst[i] = acc[i];
}

// y[u] += the partials of u's bin, u in [hot, n).
__global__ __launch_bounds__(256) void k_pr_push_bin_combine(int32_t n, int32_t hot, const int32_t* __restrict__ ulo,
                                                             const float* __restrict__ part, float* __restrict__ y) {
    const int32_t u = hot + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (u >= n) return;
    const int32_t r = u - hot;
    const int32_t b = r >> kPushBinShift, ul = r & (kPushBinW - 1);
    const int32_t k0 = ulo[b], k1 = ulo[b + 1];
    const float y0 = y[u];
    // the unit partials in order, four loads in flight; a missing one adds
    // +0, which leaves the sum (never -0: it starts at +0) unchanged
    float acc = 0.f;
    for (int32_t k = k0; k < k1; k += 4) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (k + j < k1) ? part[(size_t)(k + j) * kPushBinW + ul] : 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc += v[j];
    }
    y[u] = y0 + acc;
}

// y[u] += sum over workgroups of their LDS partials, u < hot (one writer per
// u; fixed summation order).  Block: 64 targets x 4 partial-row groups.
__global__ __launch_bounds__(256) void k_pr_push_hot_reduce(int32_t hot, int32_t parts,
                                                            const float* __restrict__ hot_part,
                                                            float* __restrict__ y) {
    __shared__ float s[4][64];
    const int32_t u = blockIdx.x * 64 + (threadIdx.x & 63);
    const int r = threadIdx.x >> 6;
    float acc = 0.f;
    if (u < hot) {
        // partials b = r, r + 4, ... in that order, eight loads in flight
        int32_t b = r;
        for (; b + 28 < parts; b += 32) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = hot_part[(size_t)(b + 4 * k) * hot + u];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += v[k];
        }
        for (; b < parts; b += 4) acc += hot_part[(size_t)b * hot + u];
    }
    s[r][threadIdx.x & 63] = acc;
    __syncthreads();
    if (r == 0 && u < hot) y[u] += (s[0][threadIdx.x] + s[1][threadIdx.x]) + (s[2][threadIdx.x] + s[3][threadIdx.x]);
}

// Launch shape of the push sweep: privatised targets, workgroup width (SUB
// slices of kBlock threads), grid, bins and LDS bytes.  The binned mode keeps
// three ints per bin in LDS next to the privatised targets, so it may
// privatise slightly fewer of them.
struct PushShape {
    int32_t hot, sub, grid, nbins;
    size_t lds;
};

static PushShape push_shape(pp_graph g, bool binned) {
    PushShape sh{};
    const int32_t n = g->d.n;
    int32_t hot = std::min(g->tune.hot, n);
    if (binned) {
        const int64_t fit = ((int64_t)g->max_lds - 12 * (int64_t)push_bins_cap(n)) / 4;
        hot = (int32_t)std::min<int64_t>(hot, std::max<int64_t>(fit, 0) & ~(int64_t)3);
    }
    sh.hot = hot;
    sh.nbins = (binned && hot > 0 && n > hot) ? ceil_div((int64_t)n - hot, kPushBinW) : 0;
    sh.lds = (size_t)std::max(hot, 0) * sizeof(float) + (size_t)sh.nbins * 3 * sizeof(int32_t);
    // more than 64 KB of privatised targets: 1024-thread workgroups (one per
    // CU holds the LDS), otherwise 256-thread workgroups
    sh.sub = ((size_t)std::max(hot, 0) * sizeof(float) > 65536) ? 4 : 1;
    sh.grid = std::max(1, std::min(ceil_div(g->push_plan.total_blocks, sh.sub), g->tune.push_blocks));
    return sh;
}

static PushArgs push_args(pp_graph g, const float* c, float* y, const PushShape& sh) {
    PushArgs a;
    a.sp = sweep_plan(g->push_plan);
    a.off = g->d.csr_off;
    a.idx = g->d.csr_idx;
    a.wt = g->d.csr_w;
    a.list = g->d.push_list;
    a.tab_cap = g->split_cap;
    a.tab = g->d.split_tab + 4 * (size_t)a.tab_cap + 1;
    a.units = g->push_plan.total_blocks;
    a.hot = sh.hot;
    a.hot_part = g->d.hot_part;
    a.c = c;
    a.y = y;
    a.nbins = sh.nbins;
    a.pb_base = g->d.pb_base;
    a.pb_cnt = g->d.pb_cnt;
    a.pb_fill = g->d.pb_fill;
    a.pb_pairs = g->d.pb_pairs;
    return a;
}

template <int SUB, bool W, bool HOT, int MODE>
static void launch_push_kernel(const PushArgs& a, const PushShape& sh, hipStream_t st) {
    const size_t lds = (HOT || MODE != kPushAtomic) ? sh.lds : 0;
    if (lds > 0) allow_dynamic_lds(reinterpret_cast<const void*>(&k_pr_push<SUB, W, HOT, MODE>), lds);
    hipLaunchKernelGGL((k_pr_push<SUB, W, HOT, MODE>), dim3(sh.grid), dim3(SUB * kBlock), lds, st, a);
}

template <int MODE>
static void launch_push_mode(pp_graph g, const PushArgs& a, const PushShape& sh, hipStream_t st) {
    const bool hot = sh.hot > 0;
    if (sh.sub == 4) {
        if (g->weighted) launch_push_kernel<4, true, true, MODE>(a, sh, st);
        else launch_push_kernel<4, false, true, MODE>(a, sh, st);
    } else if (g->weighted) {
        if (hot) launch_push_kernel<1, true, true, MODE>(a, sh, st);
        else launch_push_kernel<1, true, false, MODE>(a, sh, st);
    } else {
        if (hot) launch_push_kernel<1, false, true, MODE>(a, sh, st);
        else launch_push_kernel<1, false, false, MODE>(a, sh, st);
    }
}

pp_status build_push_bins(pp_graph g, hipStream_t st) {
    g->pbins = PushBins{};
    const int32_t n = g->d.n;
    if (!g->d.pb_base || g->push_plan.total_blocks == 0) return PP_OK;
    const PushShape sh = push_shape(g, true);
    if (sh.hot <= 0 || sh.nbins <= 0 || sh.nbins > push_bins_cap(n) || sh.grid > g->tune.push_blocks) return PP_OK;
    // walk the sweep's static assignment once, counting each workgroup's
    // updates per bin
    const PushArgs a = push_args(g, nullptr, nullptr, sh);
    launch_push_mode<kPushCount>(g, a, sh, st);
    PP_LAUNCH_CHECK("push bin count");
    const size_t slices = (size_t)sh.grid * sh.nbins;
    std::vector<int32_t> cnt(slices), base(slices);
    PP_HIP(hipMemcpyAsync(cnt.data(), g->d.pb_cnt, slices * 4, hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    // slices bin-major, so a bin's pairs are contiguous
    int64_t at = 0;
    for (int32_t b = 0; b < sh.nbins; ++b)
        for (int32_t w = 0; w < sh.grid; ++w) {
            base[(size_t)w * sh.nbins + b] = (int32_t)at;
            at += cnt[(size_t)w * sh.nbins + b];
        }
    if (at > g->d.nnz) return set_error(PP_E_GRAPH, "binned push: more updates than edges");
    // units of the summing kernel: runs of consecutive workgroups of one bin
    // with about `chunk` pairs
    const int64_t chunk = std::max<int64_t>((at + kPushBinUnits - 1) / kPushBinUnits, kPushBinMinUnit);
    std::vector<int32_t> units, ulo((size_t)sh.nbins + 1);
    for (int32_t b = 0; b < sh.nbins; ++b) {
        ulo[b] = (int32_t)(units.size() / 3);
        int64_t acc = 0;
        int32_t w0 = 0;
        for (int32_t w = 0; w < sh.grid; ++w) {
            acc += cnt[(size_t)w * sh.nbins + b];
            if (acc >= chunk) {
                units.insert(units.end(), {b, w0, w + 1});
                w0 = w + 1;
                acc = 0;
            }
        }
        if (acc > 0) units.insert(units.end(), {b, w0, sh.grid});
    }
    const int32_t nunits = (int32_t)(units.size() / 3);
    ulo[sh.nbins] = nunits;
    if (nunits > push_units_cap(n, g->d.nnz)) return set_error(PP_E_WORKSPACE, "binned push: unit table overflow");
    PP_HIP(hipMemcpyAsync(g->d.pb_base, base.data(), slices * 4, hipMemcpyHostToDevice, st));
    if (nunits > 0) PP_HIP(hipMemcpyAsync(g->d.pb_units, units.data(), units.size() * 4, hipMemcpyHostToDevice, st));
    PP_HIP(hipMemcpyAsync(g->d.pb_ulo, ulo.data(), ulo.size() * 4, hipMemcpyHostToDevice, st));
    PP_HIP(hipStreamSynchronize(st));
    g->pbins = PushBins{sh.nbins, sh.hot, sh.sub, sh.grid, nunits};
    return PP_OK;
}

// Accumulates the push sweep of c into y (internal ids, pre-set to base).
pp_status launch_push(pp_graph g, const float* c, float* y, hipStream_t st) {
    if (g->push_plan.total_blocks == 0) return PP_OK;
    const bool binned = g->pbins.nbins > 0;
    const PushShape sh = push_shape(g, binned);
    if (binned && (sh.hot != g->pbins.hot || sh.nbins != g->pbins.nbins || sh.grid != g->pbins.groups ||
                   sh.sub != g->pbins.sub))
        return set_error(PP_E_GRAPH, "binned push: launch shape differs from the registered one");
    const PushArgs a = push_args(g, c, y, sh);
    if (binned) launch_push_mode<kPushBinned>(g, a, sh, st);
    else launch_push_mode<kPushAtomic>(g, a, sh, st);
    if (sh.hot > 0)
        hipLaunchKernelGGL(k_pr_push_hot_reduce, dim3(ceil_div(sh.hot, 64)), dim3(256), 0, st, sh.hot, sh.grid,
                           (const float*)a.hot_part, y);
    if (binned) {
        if (g->pbins.units > 0) {
            const size_t lds = (size_t)kPushBinW * sizeof(float);
            allow_dynamic_lds(reinterpret_cast<const void*>(&k_pr_push_bins), lds);
            hipLaunchKernelGGL(k_pr_push_bins, dim3(g->pbins.units), dim3(1024), lds, st, sh.nbins,
                               (const int32_t*)g->d.pb_units, (const int32_t*)g->d.pb_base,
                               (const int32_t*)g->d.pb_fill, (const int2*)g->d.pb_pairs, g->d.pb_part);
        }
        hipLaunchKernelGGL(k_pr_push_bin_combine, dim3(ceil_div((int64_t)g->d.n - sh.hot, 256)), dim3(256), 0, st,
                           g->d.n, sh.hot, (const int32_t*)g->d.pb_ulo, (const float*)g->d.pb_part, y);
    }
    PP_LAUNCH_CHECK("k_pr_push");
    return PP_OK;
}

}  // namespace pp
