// Brandes betweenness centrality on the BFS step (Sec. 3.5; Sec. 4.5
// listing), for a set of sources, in pushing and pulling forms.
//
// Per source s, level by level:
//  forward   sigma(w) = sum of sigma(v) over the edges v->w with
//            dist(w) = dist(v) + 1 (shortest-path counts);
//            push: frontier vertices claim unvisited targets (CAS on dist)
//            and add their sigma with FP64 atomics; pull: every unvisited
//            vertex sums sigma over its in-neighbours in the frontier and
//            writes only itself.
//  backward  delta(v) = sigma(v) * sum of (1 + delta(w)) / sigma(w) over the
//            edges v->w with dist(w) = dist(v) + 1, deepest level first;
//            push: each vertex of level l+1 adds to its predecessors with FP64
//            atomics; pull: each vertex of level l sums over its successors.
//  bc(v) += delta(v) for v != s.
// sigma, delta and bc are FP64 (path counts stay exact up to 2^53).  The
// vertices in BFS order (`order`) with the host's per-level offsets give the
// frontiers of both phases.
#include <hip/hip_runtime.h>

#include <vector>

#include "pp_common.h"

namespace pp {

constexpr int kBcWaves = kBlock / kWave;

struct BcArgs {
    int32_t n;
    const int32_t* out_off;  // caller's CSR (out-edges)
    const int32_t* out_idx;
    const int32_t* in_off;   // caller's CSC (in-edges)
    const int32_t* in_idx;
    int32_t* dist;
    double* sigma;
    double* delta;
    int32_t* order;  // vertices in BFS order
    int32_t* cnt;    // vertices in order so far
    double* bc;
};

__device__ __forceinline__ uint64_t bc_lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// Appends the lanes with `mine` to order[] (one counter atomic per wave).
__device__ __forceinline__ void bc_append(const BcArgs& a, bool mine, int32_t w, int lane) {
    const uint64_t m = __ballot(mine);
    if (!m) return;
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(a.cnt, (int32_t)__popcll(m));
    base = __shfl(base, 0);
    if (mine) a.order[base + __popcll(m & bc_lanes_below(lane))] = w;
}

// Calls fn(valid, v, u) wave-collectively for every edge v->u of the rows
// (off/idx) of verts[0, count): 64 vertices per wave unit, rows of 64 or more
// edges walked by the whole wave, shorter ones enumerated densely.
template <typename Fn>
__device__ __forceinline__ void for_each_edge(const int32_t* verts, int32_t count, const int32_t* off,
                                              const int32_t* idx, Fn&& fn) {
    __shared__ int32_t s_start[kBcWaves][kWave];
    __shared__ int32_t s_rb[kBcWaves][kWave];
    __shared__ int32_t s_v[kBcWaves][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int32_t gwave = blockIdx.x * kBcWaves + w;
    const int32_t nwaves = gridDim.x * kBcWaves;
    for (int32_t base = gwave * kWave; base < count; base += nwaves * kWave) {
        const int32_t i = base + lane;
        const int32_t v = i < count ? verts[i] : -1;
        const int32_t rb = v >= 0 ? off[v] : 0, re = v >= 0 ? off[v + 1] : 0;
        const int32_t len = re - rb;
        uint64_t big = __ballot(len >= kWave);
        while (big) {
            const int src = __ffsll((long long)big) - 1;
            big &= big - 1;
            const int32_t bv = __shfl(v, src), bb = __shfl(rb, src), be = __shfl(re, src);
            for (int32_t j = bb + lane; j - lane < be; j += kWave) fn(j < be, bv, j < be ? idx[j] : -1);
        }
        const int32_t mine = len < kWave ? len : 0;
        int32_t incl = mine;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int32_t y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        const int32_t total = __shfl(incl, kWave - 1);
        s_start[w][lane] = incl - mine;
        s_rb[w][lane] = rb;
        s_v[w][lane] = v;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int32_t k = 0; k < total; k += kWave) {
            const int32_t e = k + lane;
            int32_t pv = -1, u = -1;
            if (e < total) {
                int lo = 0, hi = kWave;  // last lane whose range starts at or before e
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_start[w][mid] <= e) lo = mid;
                    else hi = mid;
                }
                pv = s_v[w][lo];
                u = idx[s_rb[w][lo] + (e - s_start[w][lo])];
            }
            fn(e < total, pv, u);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Sum of val(u) over the row [rb, re) of each lane's vertex (lanes with
// `own`), in stored order per lane; rows of 32 or more entries are summed by
// the wave (lane-strided, then a fixed shuffle tree).  Wave-collective.
constexpr int kBcU = 8;  // independent index loads in flight per lane

template <typename Val>
__device__ __forceinline__ double row_sum(bool own, int32_t rb, int32_t re, const int32_t* idx, int lane,
                                          Val&& val) {
    double acc = 0.0;
    const bool coop = own && (re - rb) >= 32;
    uint64_t big = __ballot(coop);
    while (big) {
        const int src = __ffsll((long long)big) - 1;
        big &= big - 1;
        const int32_t bb = __shfl(rb, src), be = __shfl(re, src);
        double t = 0.0;
        for (int32_t j0 = bb + lane; j0 < be; j0 += kBcU * kWave) {
            int32_t ii[kBcU];
#pragma unroll
            for (int k = 0; k < kBcU; ++k) ii[k] = (j0 + k * kWave < be) ? idx[j0 + k * kWave] : -1;
#pragma unroll
            for (int k = 0; k < kBcU; ++k)
                if (ii[k] >= 0) t += val(ii[k]);
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) t += __shfl_xor(t, d);
        if (lane == src) acc = t;
    }
    if (own && !coop) {
        for (int32_t j0 = rb; j0 < re; j0 += kBcU) {
            int32_t ii[kBcU];
#pragma unroll
            for (int k = 0; k < kBcU; ++k) ii[k] = (j0 + k < re) ? idx[j0 + k] : -1;
#pragma unroll
            for (int k = 0; k < kBcU; ++k)
                if (ii[k] >= 0) acc += val(ii[k]);
        }
    }
    return acc;
}

__global__ void k_bc_init(BcArgs a, int32_t s) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        a.dist[v] = v == s ? 0 : -1;
        a.sigma[v] = v == s ? 1.0 : 0.0;
        a.delta[v] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.order[0] = s;
        *a.cnt = 1;
    }
}

__global__ void k_bc_zero(int32_t n, double* bc) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) bc[v] = 0.0;
}

// Forward, pushing: the frontier order[lo, hi) (level l) expands along out-edges.
__global__ __launch_bounds__(kBlock) void k_bc_fwd_push(BcArgs a, int32_t l, int32_t lo, int32_t hi) {
    const int lane = threadIdx.x & (kWave - 1);
    for_each_edge(a.order + lo, hi - lo, a.out_off, a.out_idx, [&](bool valid, int32_t v, int32_t u) {
        bool claimed = false;
        if (valid) {
            int32_t d = a.dist[u];
            if (d == -1) {
                d = atomicCAS(&a.dist[u], -1, l + 1);
                claimed = d == -1;
                if (claimed) d = l + 1;
            }
            if (d == l + 1) unsafeAtomicAdd(&a.sigma[u], a.sigma[v]);
        }
        bc_append(a, claimed, u, lane);
    });
}

// Forward, pulling: every unvisited vertex sums sigma over its in-neighbours
// of level l; found vertices take level l+1.
__global__ __launch_bounds__(kBlock) void k_bc_fwd_pull(BcArgs a, int32_t l) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t base = blockIdx.x * blockDim.x + threadIdx.x - lane; base < a.n; base += stride) {
        const int32_t w = base + lane;
        const bool own = w < a.n && a.dist[w] == -1;
        const int32_t rb = own ? a.in_off[w] : 0, re = own ? a.in_off[w + 1] : 0;
        const double acc = row_sum(own, rb, re, a.in_idx, lane,
                                   [&](int32_t v) { return a.dist[v] == l ? a.sigma[v] : 0.0; });
        const bool found = own && acc > 0.0;
        if (found) {
            a.dist[w] = l + 1;
            a.sigma[w] = acc;
        }
        bc_append(a, found, w, lane);
    }
}

// Backward, pushing: every vertex w of order[lo, hi) (level l+1) adds
// sigma(v) (1 + delta(w)) / sigma(w) to each predecessor v (level l).
__global__ __launch_bounds__(kBlock) void k_bc_bwd_push(BcArgs a, int32_t l, int32_t lo, int32_t hi) {
    for_each_edge(a.order + lo, hi - lo, a.in_off, a.in_idx, [&](bool valid, int32_t w, int32_t v) {
        if (valid && a.dist[v] == l)
            unsafeAtomicAdd(&a.delta[v], a.sigma[v] * ((1.0 + a.delta[w]) / a.sigma[w]));
    });
}

// Backward, pulling: every vertex v of order[lo, hi) (level l) sums over its
// successors (level l+1) and writes delta(v).
__global__ __launch_bounds__(kBlock) void k_bc_bwd_pull(BcArgs a, int32_t l, int32_t lo, int32_t hi) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t base = lo + blockIdx.x * blockDim.x + threadIdx.x - lane; base < hi; base += stride) {
        const int32_t i = base + lane;
        const bool own = i < hi;
        const int32_t v = own ? a.order[i] : 0;
        const int32_t rb = own ? a.out_off[v] : 0, re = own ? a.out_off[v + 1] : 0;
        const double acc = row_sum(own, rb, re, a.out_idx, lane, [&](int32_t w) {
            return a.dist[w] == l + 1 ? (1.0 + a.delta[w]) / a.sigma[w] : 0.0;
        });
        if (own) a.delta[v] = a.sigma[v] * acc;
    }
}

__global__ void k_bc_acc(BcArgs a, int32_t s, int32_t count) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const int32_t v = a.order[i];
        if (v != s) a.bc[v] += a.delta[v];
    }
}

struct BcLayout {
    size_t dist, sigma, delta, order, cnt, total;
};

static BcLayout bc_layout(int32_t n) {
    BcLayout L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p = align_up(p + bytes, 256);
        return at;
    };
    L.dist = take((size_t)n * 4);
    L.sigma = take((size_t)n * 8);
    L.delta = take((size_t)n * 8);
    L.order = take((size_t)n * 4);
    L.cnt = take(4);
    L.total = p;
    return L;
}

}  // namespace pp

using namespace pp;

PP_EXPORT size_t pp_bc_workspace_bytes(pp_graph g) { return g ? bc_layout(g->d.n).total : 0; }

PP_EXPORT pp_status pp_bc_run(pp_graph g, pp_dir fwd_dir, pp_dir bwd_dir, int32_t num_sources,
                              const int32_t* sources, double* bc, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (!bc || !ws || (num_sources > 0 && !sources)) return set_error(PP_E_NULL, "bc, ws and sources are required");
    if ((fwd_dir != PP_PUSH && fwd_dir != PP_PULL) || (bwd_dir != PP_PUSH && bwd_dir != PP_PULL))
        return set_error(PP_E_RANGE, "directions must be PP_PUSH or PP_PULL");
    if (num_sources < 0) return set_error(PP_E_RANGE, "num_sources must be >= 0");
    const int32_t n = g->d.n;
    for (int32_t k = 0; k < num_sources; ++k)
        if (sources[k] < 0 || sources[k] >= n) return set_error(PP_E_RANGE, "source out of range");
    const BcLayout L = bc_layout(n);
    if (ws_bytes < L.total) return set_error(PP_E_WORKSPACE, "BC workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return set_error(PP_E_RANGE, "ws must be 256-byte aligned");
    char* w = static_cast<char*>(ws);
    BcArgs a;
    a.n = n;
    a.out_off = g->d.user_csr_off;
    a.out_idx = g->d.user_csr_idx;
    a.in_off = g->d.user_csc_off;
    a.in_idx = g->d.user_csc_idx;
    a.dist = reinterpret_cast<int32_t*>(w + L.dist);
    a.sigma = reinterpret_cast<double*>(w + L.sigma);
    a.delta = reinterpret_cast<double*>(w + L.delta);
    a.order = reinterpret_cast<int32_t*>(w + L.order);
    a.cnt = reinterpret_cast<int32_t*>(w + L.cnt);
    a.bc = bc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t vb = std::max(1, std::min(ceil_div(n, kBlock), 4096));
    const int32_t eb = g->num_cu * 8;  // blocks of the frontier kernels (grid-stride)
    hipLaunchKernelGGL(k_bc_zero, dim3(vb), dim3(kBlock), 0, st, n, bc);
    std::vector<int32_t> level_off;
    for (int32_t k = 0; k < num_sources; ++k) {
        const int32_t s = sources[k];
        hipLaunchKernelGGL(k_bc_init, dim3(vb), dim3(kBlock), 0, st, a, s);
        level_off.assign({0, 1});
        for (int32_t l = 0;; ++l) {
            const int32_t lo = level_off[l], hi = level_off[l + 1];
            if (fwd_dir == PP_PUSH)
                hipLaunchKernelGGL(k_bc_fwd_push, dim3(std::min(eb, ceil_div(hi - lo, kBlock) + 1)), dim3(kBlock), 0,
                                   st, a, l, lo, hi);
            else
                hipLaunchKernelGGL(k_bc_fwd_pull, dim3(vb), dim3(kBlock), 0, st, a, l);
            PP_LAUNCH_CHECK("k_bc_fwd");
            int32_t c = 0;
            PP_HIP(hipMemcpyAsync(&c, a.cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            PP_HIP(hipStreamSynchronize(st));
            if (c == hi) break;  // level l+1 is empty
            level_off.push_back(c);
        }
        // levels 0..D-1 are order[level_off[l], level_off[l+1])
        const int32_t D = (int32_t)level_off.size() - 1;
        for (int32_t l = D - 2; l >= 0; --l) {
            if (bwd_dir == PP_PUSH) {
                const int32_t lo = level_off[l + 1], hi = level_off[l + 2];
                hipLaunchKernelGGL(k_bc_bwd_push, dim3(std::min(eb, ceil_div(hi - lo, kBlock) + 1)), dim3(kBlock), 0,
                                   st, a, l, lo, hi);
            } else {
                const int32_t lo = level_off[l], hi = level_off[l + 1];
                hipLaunchKernelGGL(k_bc_bwd_pull, dim3(std::min(eb, ceil_div(hi - lo, kBlock) + 1)), dim3(kBlock), 0,
                                   st, a, l, lo, hi);
            }
        }
        hipLaunchKernelGGL(k_bc_acc, dim3(std::min(vb, ceil_div(level_off[D], kBlock) + 1)), dim3(kBlock), 0, st, a,
                           s, level_off[D]);
        PP_LAUNCH_CHECK("k_bc_bwd");
    }
    return PP_OK;
}
