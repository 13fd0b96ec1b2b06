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
// Sources run in batches of up to kBcBatch at once (the sources are
// independent, Sec. 4.5): every kernel has a grid row (blockIdx.y) per source
// of the batch, and each source owns a slab of the workspace (distances, path
// counts, dependencies, BFS order, level offsets).  The level bookkeeping of
// both passes is on the device: the last workgroup of a source's row to
// finish a level kernel records where its next level ends, whether it is
// empty, and (backward) which level comes next.  The host launches level
// kernels in batches (a source past its last level returns at once) and
// reads the states once per batch of forward levels; the backward levels
// follow without a read, and the dependencies are summed into bc in source
// order, without atomics.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "pp_common.h"

namespace pp {

constexpr int kBcWaves = kBlock / kWave;
constexpr int32_t kBcHot = 4096;  // LDS-accumulated targets of the pushing kernels (32 KB of FP64)

constexpr int32_t kBcBatch = 32;  // sources processed together

// Level state of one source (level l is order[lvl_off[l], lvl_off[l + 1])).
struct BcState {
    int32_t l;         // level the next forward kernel expands
    int32_t done;      // set once a forward kernel found its next level empty
    int32_t depth;     // non-empty levels (valid once done)
    int32_t finished;  // workgroups of the running forward kernel that have finished
    int32_t bl;        // level the next backward kernel completes (-1: none left)
    int32_t bfinished; // workgroups of the running backward kernel that have finished
    int32_t pad[2];
};

// Pointers of source 0 of a batch; source s is `stride` bytes further on
// (see slab()).  st is an array over the batch.
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
    int32_t* lvl_off;  // n + 2 entries
    BcState* st;
    size_t stride;     // bytes between the slabs of consecutive sources
    double* bc;        // caller ids
};

// The sources of a batch (caller ids), passed by value.
struct BcSources {
    int32_t s[kBcBatch];
};

template <typename T>
__device__ __forceinline__ T* shift(T* p, size_t bytes) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + bytes);
}

// The arguments of source `s` of the batch.
__device__ __forceinline__ BcArgs slab(const BcArgs& a0, int32_t s) {
    BcArgs a = a0;
    const size_t b = (size_t)s * a0.stride;
    a.dist = shift(a0.dist, b);
    a.sigma = shift(a0.sigma, b);
    a.delta = shift(a0.delta, b);
    a.order = shift(a0.order, b);
    a.cnt = shift(a0.cnt, b);
    a.lvl_off = shift(a0.lvl_off, b);
    a.st = a0.st + s;
    return a;
}

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

__global__ void k_bc_init(BcArgs a0, BcSources src) {
    const BcArgs a = slab(a0, blockIdx.y);
    const int32_t s_user = src.s[blockIdx.y];
    const int32_t s = a.iperm ? a.iperm[s_user] : s_user;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        a.dist[v] = v == s ? 0 : -1;
        a.sigma[v] = v == s ? 1.0 : 0.0;
        a.delta[v] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.order[0] = s;
        *a.cnt = 1;
        *a.st = BcState{0, 0, 0, 0, -1, 0, {0, 0}};
        a.lvl_off[0] = 0;
        a.lvl_off[1] = 1;
    }
}

__global__ void k_bc_zero(int32_t n, double* bc) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) bc[v] = 0.0;
}

// Is this workgroup the last of its source's row to finish the kernel?
// (Every other one has then read the state.)  Workgroup-collective.
// No device-wide fence is needed (one would write back the whole L2 per
// workgroup): the appends are returning atomics on the counter, complete
// before the barrier, so the last workgroup's atomic read of the counter sees
// them all; what it writes is read by later kernels only.
__device__ __forceinline__ bool bc_last_group(int32_t* finished) {
    __shared__ int32_t s_last;
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(finished, 1) == (int32_t)gridDim.x - 1;
    __syncthreads();
    return s_last != 0;
}

// End of a forward level kernel: the last workgroup records the end of level
// l + 1 and whether it is empty (then the backward pass starts at the second
// deepest level), and advances the level.  Workgroup-collective.
__device__ __forceinline__ void bc_level_end(const BcArgs& a, int32_t l) {
    if (bc_last_group(&a.st->finished) && threadIdx.x == 0) {
        const int32_t c = atomicAdd(a.cnt, 0);
        a.lvl_off[l + 2] = c;
        if (c == a.lvl_off[l + 1]) {
            a.st->done = 1;
            a.st->depth = l + 1;
            a.st->bl = l - 1;
        }
        a.st->l = l + 1;
        a.st->finished = 0;
    }
}

// End of a backward level kernel: the last workgroup moves to the level above.
__device__ __forceinline__ void bc_back_end(const BcArgs& a, int32_t l) {
    if (bc_last_group(&a.st->bfinished) && threadIdx.x == 0) {
        a.st->bl = l - 1;
        a.st->bfinished = 0;
    }
}

// Zeroes the workgroup's hot accumulators.  Workgroup-collective.
__device__ __forceinline__ void hot_zero(double* s_acc, int32_t hot) {
    for (int32_t i = threadIdx.x; i < hot; i += blockDim.x) s_acc[i] = 0.0;
    __syncthreads();
}

// Forward, pushing: the frontier (level l) expands along out-edges.
__global__ __launch_bounds__(kBlock) void k_bc_fwd_push(BcArgs a0) {
    __shared__ double s_acc[kBcHot];
    const BcArgs a = slab(a0, blockIdx.y);
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
__global__ __launch_bounds__(kBlock) void k_bc_fwd_pull(BcArgs a0) {
    const BcArgs a = slab(a0, blockIdx.y);
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

// Backward, pushing: every vertex w of level l+1 adds sigma(v) (1 + delta(w))
// / sigma(w) to each predecessor v (level l); hot predecessors collect the sum
// of (1 + delta(w)) / sigma(w) in LDS first.
__global__ __launch_bounds__(kBlock) void k_bc_bwd_push(BcArgs a0) {
    __shared__ double s_acc[kBcHot];
    const BcArgs a = slab(a0, blockIdx.y);
    const int32_t l = a.st->bl;
    if (l < 0) return;
    const int32_t lo = a.lvl_off[l + 1], hi = a.lvl_off[l + 2];
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
    bc_back_end(a, l);
}

// Backward, pulling: every vertex v of level l sums over its successors
// (level l+1) and writes delta(v).
__global__ __launch_bounds__(kBlock) void k_bc_bwd_pull(BcArgs a0) {
    const BcArgs a = slab(a0, blockIdx.y);
    const int32_t l = a.st->bl;
    if (l < 0) return;
    const int32_t lo = a.lvl_off[l], hi = a.lvl_off[l + 1];
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
    bc_back_end(a, l);
}

// bc(v) += delta_s(v) over the batch's sources s != v, in source order.
__global__ void k_bc_acc(BcArgs a0, BcSources src, int32_t count) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < a0.n; v += gridDim.x * blockDim.x) {
        const int32_t vu = a0.perm ? a0.perm[v] : v;
        double acc = 0.0;
        for (int32_t s = 0; s < count; ++s)
            if (src.s[s] != vu) acc += shift(a0.delta, (size_t)s * a0.stride)[v];
        a0.bc[vu] += acc;
    }
}

// One source's slab; the workspace holds the batch's states, then up to
// kBcBatch slabs.
struct BcLayout {
    size_t dist, sigma, delta, order, cnt, lvl_off, slab;
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
    L.lvl_off = take(((size_t)n + 2) * 4);
    L.slab = p;
    return L;
}

constexpr size_t kBcStates = (sizeof(BcState) * kBcBatch + 255) / 256 * 256;

}  // namespace pp

using namespace pp;

PP_EXPORT size_t pp_bc_workspace_bytes(pp_graph g) { return g ? kBcStates + kBcBatch * bc_layout(g->d.n).slab : 0; }

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
    if (ws_bytes < kBcStates + L.slab) return set_error(PP_E_WORKSPACE, "BC workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return set_error(PP_E_RANGE, "ws must be 256-byte aligned");
    // as many sources at once as the workspace holds, at most kBcBatch
    const int32_t per_batch = (int32_t)std::min<size_t>(kBcBatch, (ws_bytes - kBcStates) / L.slab);
    char* w = static_cast<char*>(ws);
    char* slab0 = w + kBcStates;
    BcArgs a;
    a.n = n;
    a.hot = std::min(n, kBcHot);
    a.out_off = g->d.csr_off;
    a.out_idx = g->d.csr_idx;
    a.in_off = g->d.csc_off;
    a.in_idx = g->d.csc_idx;
    a.perm = g->d.perm;
    a.iperm = g->d.iperm;
    a.dist = reinterpret_cast<int32_t*>(slab0 + L.dist);
    a.sigma = reinterpret_cast<double*>(slab0 + L.sigma);
    a.delta = reinterpret_cast<double*>(slab0 + L.delta);
    a.order = reinterpret_cast<int32_t*>(slab0 + L.order);
    a.cnt = reinterpret_cast<int32_t*>(slab0 + L.cnt);
    a.lvl_off = reinterpret_cast<int32_t*>(slab0 + L.lvl_off);
    a.st = reinterpret_cast<BcState*>(w);
    a.stride = L.slab;
    a.bc = bc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t vb = std::max(1, std::min(ceil_div(n, kBlock), 4096));
    // per source: every pushing workgroup zeroes and flushes its hot
    // accumulators, so a few per compute unit; the pulling kernels sweep
    // vertex or level lists grid-stride
    const int32_t pb = std::max(1, std::min(ceil_div(n, kBlock), 2 * g->num_cu));
    const int32_t fx = (fwd_dir == PP_PUSH) ? pb : vb;
    const int32_t bx = (bwd_dir == PP_PUSH) ? pb : std::min(vb, 2 * g->num_cu);
    hipLaunchKernelGGL(k_bc_zero, dim3(vb), dim3(kBlock), 0, st, n, bc);
    PP_LAUNCH_CHECK("k_bc_zero");
    std::vector<BcState> hs(per_batch);
    int32_t batch = 4;  // forward kernels per launch batch: one more than the last depth seen
    for (int32_t k0 = 0; k0 < num_sources; k0 += per_batch) {
        const int32_t cnt = std::min(per_batch, num_sources - k0);
        BcSources src{};
        for (int32_t i = 0; i < cnt; ++i) src.s[i] = sources[k0 + i];
        hipLaunchKernelGGL(k_bc_init, dim3(vb, cnt), dim3(kBlock), 0, st, a, src);
        // forward levels in batches; a source past its last level returns at once
        int32_t launched = 0, depth = 0;
        for (;;) {
            for (int32_t i = 0; i < batch; ++i) {
                if (fwd_dir == PP_PUSH) hipLaunchKernelGGL(k_bc_fwd_push, dim3(fx, cnt), dim3(kBlock), 0, st, a);
                else hipLaunchKernelGGL(k_bc_fwd_pull, dim3(fx, cnt), dim3(kBlock), 0, st, a);
            }
            PP_LAUNCH_CHECK("k_bc_fwd");
            launched += batch;
            PP_HIP(hipMemcpyAsync(hs.data(), a.st, sizeof(BcState) * cnt, hipMemcpyDeviceToHost, st));
            PP_HIP(hipStreamSynchronize(st));
            bool all = true;
            depth = 0;
            for (int32_t i = 0; i < cnt; ++i) {
                all = all && hs[i].done;
                depth = std::max(depth, hs[i].depth);
            }
            if (all || launched > n) break;
            batch = std::min(batch * 2, 64);
        }
        batch = std::max(2, depth + 1);
        // backward levels D-2 .. 0 of each source, its state counting down
        for (int32_t l = depth - 2; l >= 0; --l) {
            if (bwd_dir == PP_PUSH) hipLaunchKernelGGL(k_bc_bwd_push, dim3(bx, cnt), dim3(kBlock), 0, st, a);
            else hipLaunchKernelGGL(k_bc_bwd_pull, dim3(bx, cnt), dim3(kBlock), 0, st, a);
        }
        hipLaunchKernelGGL(k_bc_acc, dim3(vb), dim3(kBlock), 0, st, a, src, cnt);
        PP_LAUNCH_CHECK("k_bc_bwd");
    }
    return PP_OK;
}
