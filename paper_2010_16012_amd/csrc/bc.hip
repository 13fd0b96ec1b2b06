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
// vertices in BFS order (`order`) with per-level offsets give the frontiers
// of both phases.
//
// The kernels walk the internal (degree-ordered) adjacency, so the vertices
// every frontier reaches -- the hubs -- have the lowest ids.  The pushing
// kernels add contributions to the first kBcHot ids into per-workgroup LDS
// accumulators and hand each total to memory once per workgroup: without
// this, a hub's claim and its FP64 additions arrive from every one of its
// frontier neighbours and serialise on one address.
//
// The forward pass keeps its level bookkeeping on the device: the last
// workgroup of a level kernel to finish records where the next level ends in
// `order` and whether it is empty.  The host launches forward kernels in
// batches (kernels past the last level return at once) and reads the state
// once per batch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "pp_common.h"

namespace pp {

constexpr int kBcWaves = kBlock / kWave;
constexpr int32_t kBcHot = 4096;  // LDS-accumulated targets of the pushing kernels (32 KB of FP64)

// Forward-pass state, then the level offsets: level l is
// order[lvl_off[l], lvl_off[l + 1]).
struct BcState {
    int32_t l;         // level the next forward kernel expands
    int32_t done;      // set once a forward kernel found its next level empty
    int32_t depth;     // non-empty levels (valid once done)
    int32_t finished;  // workgroups of the running forward kernel that have finished
};

struct BcArgs {
    int32_t n;
    int32_t hot;             // min(n, kBcHot)
    const int32_t* out_off;  // internal CSR (out-edges)
    const int32_t* out_idx;
    const int32_t* in_off;   // internal CSC (in-edges)
    const int32_t* in_idx;
    const int32_t* perm;     // internal -> caller id (nullable)
    const int32_t* iperm;    // caller -> internal id (nullable)
    int32_t* dist;
    double* sigma;
    double* delta;
    int32_t* order;    // vertices in BFS order
    int32_t* cnt;      // vertices in order so far
    BcState* st;
    int32_t* lvl_off;  // n + 2 entries, right after st
    double* bc;        // caller ids
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

// Position of lane `lane` of wavefront `gwave` (of `nwaves`) in pass `base`
// over a list: the 64 lanes of a wavefront take positions nwaves apart, so
// neighbouring list entries -- consecutive hubs in degree order, or hubs
// claimed together -- go to different wavefronts.
__device__ __forceinline__ int32_t spread(int32_t base, int lane, int32_t gwave, int32_t nwaves) {
    return base + lane * nwaves + gwave;
}

// Calls fn(valid, v, u) wave-collectively for every edge v->u of the rows
// (off/idx) of verts[0, count): 64 vertices per wave unit (spread over the
// list), rows of 64 or more edges walked by the whole wave, shorter ones
// enumerated densely.
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
    for (int32_t base = 0; base < count; base += nwaves * kWave) {
        const int32_t i = spread(base, lane, gwave, nwaves);
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

__global__ void k_bc_init(BcArgs a, int32_t s_user) {
    const int32_t s = a.iperm ? a.iperm[s_user] : s_user;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        a.dist[v] = v == s ? 0 : -1;
        a.sigma[v] = v == s ? 1.0 : 0.0;
        a.delta[v] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.order[0] = s;
        *a.cnt = 1;
        *a.st = BcState{0, 0, 0, 0};
        a.lvl_off[0] = 0;
        a.lvl_off[1] = 1;
    }
}

__global__ void k_bc_zero(int32_t n, double* bc) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) bc[v] = 0.0;
}

// End of a forward level kernel: the last workgroup to finish (every other
// one has then read the state) records the end of level l + 1 and whether it
// is empty, and advances the level.  Workgroup-collective.
// No device-wide fence is needed (one would write back the whole L2 per
// workgroup): the appends are returning atomics on the counter, complete
// before the barrier, so the last workgroup's atomic read of the counter sees
// them all; what it writes is read by the next kernel only.
__device__ __forceinline__ void bc_level_end(const BcArgs& a, int32_t l) {
    __shared__ int32_t s_last;
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&a.st->finished, 1) == (int32_t)gridDim.x - 1;
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        const int32_t c = atomicAdd(a.cnt, 0);
        a.lvl_off[l + 2] = c;
        if (c == a.lvl_off[l + 1]) {
            a.st->done = 1;
            a.st->depth = l + 1;
        }
        a.st->l = l + 1;
        a.st->finished = 0;
    }
}

// Zeroes the workgroup's hot accumulators.  Workgroup-collective.
__device__ __forceinline__ void hot_zero(double* s_acc, int32_t hot) {
    for (int32_t i = threadIdx.x; i < hot; i += blockDim.x) s_acc[i] = 0.0;
    __syncthreads();
}

// Forward, pushing: the frontier (level l) expands along out-edges.
__global__ __launch_bounds__(kBlock) void k_bc_fwd_push(BcArgs a) {
    __shared__ double s_acc[kBcHot];
    const BcState st = *a.st;
    if (st.done) return;
    const int32_t l = st.l, lo = a.lvl_off[l], hi = a.lvl_off[l + 1];
    const int lane = threadIdx.x & (kWave - 1);
    hot_zero(s_acc, a.hot);
    for_each_edge(a.order + lo, hi - lo, a.out_off, a.out_idx, [&](bool valid, int32_t v, int32_t u) {
        bool claimed = false;
        if (valid) {
            if (u < a.hot) {
                unsafeAtomicAdd(&s_acc[u], a.sigma[v]);
            } else {
                int32_t d = a.dist[u];
                if (d == -1) {
                    d = atomicCAS(&a.dist[u], -1, l + 1);
                    claimed = d == -1;
                    if (claimed) d = l + 1;
                }
                if (d == l + 1) unsafeAtomicAdd(&a.sigma[u], a.sigma[v]);
            }
        }
        bc_append(a, claimed, u, lane);
    });
    __syncthreads();
    // hot targets this workgroup reached: a target with a contribution is on
    // level l + 1 exactly when it had no distance before this level
    for (int32_t base = threadIdx.x - lane; base < a.hot; base += blockDim.x) {
        const int32_t u = base + lane;
        const double sum = u < a.hot ? s_acc[u] : 0.0;
        bool claimed = false;
        if (sum != 0.0) {
            int32_t d = a.dist[u];
            if (d == -1) {
                d = atomicCAS(&a.dist[u], -1, l + 1);
                claimed = d == -1;
                if (claimed) d = l + 1;
            }
            if (d == l + 1) unsafeAtomicAdd(&a.sigma[u], sum);
        }
        bc_append(a, claimed, u, lane);
    }
    bc_level_end(a, l);
}

// Forward, pulling: every unvisited vertex sums sigma over its in-neighbours
// of level l; found vertices take level l+1.
__global__ __launch_bounds__(kBlock) void k_bc_fwd_pull(BcArgs a) {
    const BcState st = *a.st;
    if (st.done) return;
    const int32_t l = st.l;
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * kBcWaves + threadIdx.x / kWave, nwaves = gridDim.x * kBcWaves;
    for (int32_t base = 0; base < a.n; base += nwaves * kWave) {
        const int32_t w = spread(base, lane, gwave, nwaves);
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
    bc_level_end(a, l);
}

// Backward, pushing: every vertex w of order[lo, hi) (level l+1) adds
// sigma(v) (1 + delta(w)) / sigma(w) to each predecessor v (level l); hot
// predecessors collect the sum of (1 + delta(w)) / sigma(w) in LDS first.
__global__ __launch_bounds__(kBlock) void k_bc_bwd_push(BcArgs a, int32_t l, int32_t lo, int32_t hi) {
    __shared__ double s_acc[kBcHot];
    const int lane = threadIdx.x & (kWave - 1);
    hot_zero(s_acc, a.hot);
    for_each_edge(a.order + lo, hi - lo, a.in_off, a.in_idx, [&](bool valid, int32_t w, int32_t v) {
        if (valid && a.dist[v] == l) {
            const double c = (1.0 + a.delta[w]) / a.sigma[w];
            if (v < a.hot) unsafeAtomicAdd(&s_acc[v], c);
            else unsafeAtomicAdd(&a.delta[v], a.sigma[v] * c);
        }
    });
    __syncthreads();
    for (int32_t base = threadIdx.x - lane; base < a.hot; base += blockDim.x) {
        const int32_t v = base + lane;
        const double sum = v < a.hot ? s_acc[v] : 0.0;
        if (sum != 0.0) unsafeAtomicAdd(&a.delta[v], a.sigma[v] * sum);
    }
}

// Backward, pulling: every vertex v of order[lo, hi) (level l) sums over its
// successors (level l+1) and writes delta(v).
__global__ __launch_bounds__(kBlock) void k_bc_bwd_pull(BcArgs a, int32_t l, int32_t lo, int32_t hi) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * kBcWaves + threadIdx.x / kWave, nwaves = gridDim.x * kBcWaves;
    for (int32_t base = lo; base < hi; base += nwaves * kWave) {
        const int32_t i = spread(base, lane, gwave, nwaves);
        const bool own = i < hi;
        const int32_t v = own ? a.order[i] : 0;
        const int32_t rb = own ? a.out_off[v] : 0, re = own ? a.out_off[v + 1] : 0;
        const double acc = row_sum(own, rb, re, a.out_idx, lane, [&](int32_t w) {
            return a.dist[w] == l + 1 ? (1.0 + a.delta[w]) / a.sigma[w] : 0.0;
        });
        if (own) a.delta[v] = a.sigma[v] * acc;
    }
}

// bc(v) += delta(v) for every vertex reached but the source (order[0]).
__global__ void k_bc_acc(BcArgs a, int32_t count) {
    for (int32_t i = 1 + blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const int32_t v = a.order[i];
        a.bc[a.perm ? a.perm[v] : v] += a.delta[v];
    }
}

struct BcLayout {
    size_t dist, sigma, delta, order, cnt, meta, total;
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
    L.meta = take(sizeof(BcState) + ((size_t)n + 2) * 4);  // state, then the level offsets
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
    a.hot = std::min(n, kBcHot);
    a.out_off = g->d.csr_off;
    a.out_idx = g->d.csr_idx;
    a.in_off = g->d.csc_off;
    a.in_idx = g->d.csc_idx;
    a.perm = g->d.perm;
    a.iperm = g->d.iperm;
    a.dist = reinterpret_cast<int32_t*>(w + L.dist);
    a.sigma = reinterpret_cast<double*>(w + L.sigma);
    a.delta = reinterpret_cast<double*>(w + L.delta);
    a.order = reinterpret_cast<int32_t*>(w + L.order);
    a.cnt = reinterpret_cast<int32_t*>(w + L.cnt);
    a.st = reinterpret_cast<BcState*>(w + L.meta);
    a.lvl_off = reinterpret_cast<int32_t*>(w + L.meta + sizeof(BcState));
    a.bc = bc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t vb = std::max(1, std::min(ceil_div(n, kBlock), 4096));
    const int32_t eb = g->num_cu * 8;  // blocks of the backward frontier kernels (grid-stride)
    // the pushing forward kernel: every workgroup zeroes and flushes its hot
    // accumulators, so a few per compute unit
    const int32_t pb = std::max(1, std::min(ceil_div(n, kBlock), 2 * g->num_cu));
    hipLaunchKernelGGL(k_bc_zero, dim3(vb), dim3(kBlock), 0, st, n, bc);
    PP_LAUNCH_CHECK("k_bc_zero");
    // host copy of the state and level offsets
    std::vector<int32_t> meta(sizeof(BcState) / 4 + (size_t)n + 2);
    int32_t batch = 4;
    for (int32_t k = 0; k < num_sources; ++k) {
        hipLaunchKernelGGL(k_bc_init, dim3(vb), dim3(kBlock), 0, st, a, sources[k]);
        // forward levels in batches; kernels past the last level return at once
        int32_t launched = 0;
        BcState hs{};
        for (;;) {
            for (int32_t i = 0; i < batch; ++i) {
                if (fwd_dir == PP_PUSH) hipLaunchKernelGGL(k_bc_fwd_push, dim3(pb), dim3(kBlock), 0, st, a);
                else hipLaunchKernelGGL(k_bc_fwd_pull, dim3(vb), dim3(kBlock), 0, st, a);
            }
            PP_LAUNCH_CHECK("k_bc_fwd");
            launched += batch;
            const size_t words = sizeof(BcState) / 4 + (size_t)std::min<int64_t>((int64_t)launched + 2, (int64_t)n + 2);
            PP_HIP(hipMemcpyAsync(meta.data(), a.st, words * 4, hipMemcpyDeviceToHost, st));
            PP_HIP(hipStreamSynchronize(st));
            std::memcpy(&hs, meta.data(), sizeof(BcState));
            if (hs.done) break;
            batch = std::min(batch * 2, 64);
        }
        // levels 0..D-1 are order[lvl_off[l], lvl_off[l+1]); the next source
        // starts with a batch one longer than this one's depth
        const int32_t D = hs.depth;
        const int32_t* off = meta.data() + sizeof(BcState) / 4;
        batch = std::max(2, D + 1);
        for (int32_t l = D - 2; l >= 0; --l) {
            if (bwd_dir == PP_PUSH) {
                const int32_t lo = off[l + 1], hi = off[l + 2];
                hipLaunchKernelGGL(k_bc_bwd_push, dim3(std::min(pb, ceil_div(hi - lo, kBlock) + 1)), dim3(kBlock), 0,
                                   st, a, l, lo, hi);
            } else {
                const int32_t lo = off[l], hi = off[l + 1];
                hipLaunchKernelGGL(k_bc_bwd_pull, dim3(std::min(eb, ceil_div(hi - lo, kBlock) + 1)), dim3(kBlock), 0,
                                   st, a, l, lo, hi);
            }
        }
        hipLaunchKernelGGL(k_bc_acc, dim3(std::min(vb, ceil_div(off[D], kBlock) + 1)), dim3(kBlock), 0, st, a, off[D]);
        PP_LAUNCH_CHECK("k_bc_bwd");
    }
    return PP_OK;
}
