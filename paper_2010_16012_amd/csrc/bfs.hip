// BFS frontier step in its pushing (top-down) and pulling (bottom-up) forms
// (Sec. 3.3; Sec. 4.3 listing with every ready counter equal to one), and
// the per-level direction switch (Sec. 5 Generic-Switch, applied to BFS as in
// the direction-optimising BFS the paper cites in Sec. 1).
//
// One kernel expands one level.  Both forms leave the new frontier as a
// queue AND as a bitmap, so any sequence of directions works without
// conversion kernels.  Per-level statistics (|F|, out-edges of F, out-edges
// of unvisited vertices) live in three rotating device slots, so the switch
// is decided on the device and the host only polls for termination.
#include <hip/hip_runtime.h>

#include "pp_common.h"

namespace pp {

struct BfsSlot {
    int32_t n;         // frontier size (accumulated by the level that builds it)
    int32_t dir_prev;  // direction used to build this frontier
    int32_t n_prev;    // size of the frontier it was built from
    int32_t pad;
    int64_t m;         // out-edges of the frontier (accumulated)
    int64_t mu_base;   // out-edges of vertices unvisited before this frontier
};

struct BfsHdr {
    BfsSlot slot[3];
    int32_t levels;    // number of non-empty frontiers expanded so far
    int32_t last;      // index of the newest frontier
    int32_t root;
    int32_t pad;
    int64_t reached;
    int64_t edges;
    int8_t log_dir[PP_BFS_MAX_LOG];
    int32_t log_n[PP_BFS_MAX_LOG];
};

struct BfsLayout {
    size_t hdr, queue0, queue1, fb0, fb1, fb2, visited, total;
    int32_t words;
};

static BfsLayout bfs_layout(int32_t n) {
    BfsLayout L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p = align_up(p + bytes, 256);
        return at;
    };
    L.words = ceil_div(n, 64);
    L.hdr = take(sizeof(BfsHdr));
    L.queue0 = take((size_t)n * 4);
    L.queue1 = take((size_t)n * 4);
    L.fb0 = take((size_t)L.words * 8);
    L.fb1 = take((size_t)L.words * 8);
    L.fb2 = take((size_t)L.words * 8);
    L.visited = take((size_t)L.words * 8);
    L.total = p;
    return L;
}

struct BfsArgs {
    int32_t n;
    int32_t words;
    const int32_t* csr_off;
    const int32_t* csr_idx;
    const int32_t* csc_off;
    const int32_t* csc_idx;
    const int32_t* out_deg;
    int32_t* level;
    int32_t* parent;
    BfsHdr* hdr;
    int32_t* queue[2];
    uint64_t* fb[3];
    uint64_t* visited;
};

static BfsArgs bfs_args(pp_graph g, void* state, int32_t* level, int32_t* parent) {
    const BfsLayout L = bfs_layout(g->d.n);
    char* s = static_cast<char*>(state);
    BfsArgs a;
    a.n = g->d.n;
    a.words = L.words;
    a.csr_off = g->d.csr_off;
    a.csr_idx = g->d.csr_idx;
    a.csc_off = g->d.csc_off;
    a.csc_idx = g->d.csc_idx;
    a.out_deg = g->d.out_deg;
    a.level = level;
    a.parent = parent;
    a.hdr = reinterpret_cast<BfsHdr*>(s + L.hdr);
    a.queue[0] = reinterpret_cast<int32_t*>(s + L.queue0);
    a.queue[1] = reinterpret_cast<int32_t*>(s + L.queue1);
    a.fb[0] = reinterpret_cast<uint64_t*>(s + L.fb0);
    a.fb[1] = reinterpret_cast<uint64_t*>(s + L.fb1);
    a.fb[2] = reinterpret_cast<uint64_t*>(s + L.fb2);
    a.visited = reinterpret_cast<uint64_t*>(s + L.visited);
    return a;
}

constexpr int kBfsBlocks = 1024;  // fixed grid; every kernel loops over its work

__device__ __forceinline__ uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// Orders this wavefront's LDS traffic (the per-wave arrays below are never
// touched by other wavefronts, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
    return v;
}

// ------------------------------------------------------------------ init
__global__ void k_bfs_init(BfsArgs a, int32_t root, int64_t nnz) {
    const int32_t stride = gridDim.x * blockDim.x;
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int32_t v = t; v < a.n; v += stride) {
        a.level[v] = (v == root) ? 0 : -1;
        a.parent[v] = (v == root) ? root : -1;
    }
    const uint64_t rbit = 1ull << (root & 63);
    for (int32_t w = t; w < a.words; w += stride) {
        const uint64_t m = (w == (root >> 6)) ? rbit : 0ull;
        a.visited[w] = m;
        a.fb[0][w] = m;
        a.fb[1][w] = 0ull;
        a.fb[2][w] = 0ull;
    }
    if (t == 0) {
        a.queue[0][0] = root;
        BfsHdr* h = a.hdr;
        for (int i = 0; i < 3; ++i) h->slot[i] = BfsSlot{0, 0, 0, 0, 0, 0};
        const int32_t d = a.out_deg[root];
        h->slot[0] = BfsSlot{1, (int32_t)PP_PUSH, 0, 0, (int64_t)d, nnz};
        h->levels = 0;
        h->last = 0;
        h->root = root;
        h->reached = 0;
        h->edges = 0;
    }
}

// ------------------------------------------------------------------ level
// Claims u for parent v (top-down).  Wave-collective: every lane calls it.
__device__ __forceinline__ void td_claim(const BfsArgs& a, int32_t u, int32_t v, int32_t lvl, int32_t* q_next,
                                         uint64_t* fb_next, BfsSlot* nxt, int lane) {
    bool claimed = false;
    if (u >= 0) {
        const uint64_t bit = 1ull << (u & 63);
        if (!(a.visited[u >> 6] & bit)) {
            const uint64_t old = atomicOr(reinterpret_cast<unsigned long long*>(&a.visited[u >> 6]),
                                          (unsigned long long)bit);
            claimed = !(old & bit);
        }
        if (claimed) {
            a.level[u] = lvl + 1;
            a.parent[u] = v;
            atomicOr(reinterpret_cast<unsigned long long*>(&fb_next[u >> 6]), (unsigned long long)bit);
        }
    }
    const uint64_t mask = __ballot(claimed);
    if (mask == 0) return;
    const int64_t dsum = wave_sum64(claimed ? (int64_t)a.out_deg[u] : 0);
    int32_t base = 0;
    if (lane == 0) {
        base = atomicAdd(&nxt->n, (int32_t)__popcll(mask));
        atomicAdd(reinterpret_cast<unsigned long long*>(&nxt->m), (unsigned long long)dsum);
    }
    base = __shfl(base, 0);
    if (claimed) q_next[base + __popcll(mask & lanes_below(lane))] = u;
}

__device__ void level_top_down(const BfsArgs& a, int32_t lvl, int32_t nf, const int32_t* q_cur, int32_t* q_next,
                               uint64_t* fb_next, BfsSlot* nxt) {
    __shared__ int32_t s_start[kBlock / kWave][kWave];
    __shared__ int32_t s_rb[kBlock / kWave][kWave];
    __shared__ int32_t s_v[kBlock / kWave][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int32_t gwave = blockIdx.x * (kBlock / kWave) + w;
    const int32_t nwaves = gridDim.x * (kBlock / kWave);
    for (int32_t base = gwave * kWave; base < nf; base += nwaves * kWave) {
        const int32_t i = base + lane;
        const int32_t v = (i < nf) ? q_cur[i] : -1;
        const int32_t rb = (v >= 0) ? a.csr_off[v] : 0;
        const int32_t re = (v >= 0) ? a.csr_off[v + 1] : 0;
        const int32_t len = re - rb;
        // long rows: the whole wave walks one row at a time
        uint64_t big = __ballot(len >= kWave);
        while (big) {
            const int src = __ffsll((long long)big) - 1;
            big &= big - 1;
            const int32_t bv = __shfl(v, src), bb = __shfl(rb, src), be = __shfl(re, src);
            for (int32_t jb = bb; jb < be; jb += kWave) {
                const int32_t j = jb + lane;
                td_claim(a, (j < be) ? a.csr_idx[j] : -1, bv, lvl, q_next, fb_next, nxt, lane);
            }
        }
        // short rows: the wave's edges are enumerated densely through a scan
        const int32_t mine = (len < kWave) ? len : 0;
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
        wave_sync();
        for (int32_t k = 0; k < total; k += kWave) {
            const int32_t e = k + lane;
            int32_t u = -1, pv = -1;
            if (e < total) {
                int lo = 0, hi = kWave;  // last lane with start <= e
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_start[w][mid] <= e) lo = mid;
                    else hi = mid;
                }
                u = a.csr_idx[s_rb[w][lo] + (e - s_start[w][lo])];
                pv = s_v[w][lo];
            }
            td_claim(a, u, pv, lvl, q_next, fb_next, nxt, lane);
        }
        wave_sync();
    }
}

__device__ void level_bottom_up(const BfsArgs& a, int32_t lvl, const uint64_t* fb_cur, int32_t* q_next,
                                uint64_t* fb_next, BfsSlot* nxt) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int32_t nwaves = gridDim.x * (kBlock / kWave);
    for (int32_t w = gwave; w < a.words; w += nwaves) {
        const uint64_t vis = a.visited[w];
        const int32_t v = w * kWave + lane;
        const bool unvisited = (v < a.n) && !((vis >> lane) & 1ull);
        if (__ballot(unvisited) == 0) continue;
        const int32_t rb = unvisited ? a.csc_off[v] : 0;
        const int32_t re = unvisited ? a.csc_off[v + 1] : 0;
        bool found = false;
        int32_t par = -1;
        // long in-rows: the wave scans 64 in-neighbours at a time, stops at the first hit
        const bool coop = (re - rb) >= 32;
        uint64_t big = __ballot(coop);
        while (big) {
            const int src = __ffsll((long long)big) - 1;
            big &= big - 1;
            const int32_t bb = __shfl(rb, src), be = __shfl(re, src);
            for (int32_t jb = bb; jb < be; jb += kWave) {
                const int32_t j = jb + lane;
                const int32_t u = (j < be) ? a.csc_idx[j] : -1;
                const bool hit = (u >= 0) && ((fb_cur[u >> 6] >> (u & 63)) & 1ull);
                const uint64_t hm = __ballot(hit);
                if (hm) {
                    const int32_t p = __shfl(u, __ffsll((long long)hm) - 1);
                    if (lane == src) {
                        found = true;
                        par = p;
                    }
                    break;
                }
            }
        }
        // short in-rows: each lane scans its own, in stored order
        if (unvisited && !coop) {
            for (int32_t j = rb; j < re; ++j) {
                const int32_t u = a.csc_idx[j];
                if ((fb_cur[u >> 6] >> (u & 63)) & 1ull) {
                    found = true;
                    par = u;
                    break;
                }
            }
        }
        const uint64_t fm = __ballot(found);
        if (fm == 0) continue;
        if (found) {
            a.level[v] = lvl + 1;
            a.parent[v] = par;
        }
        const int64_t dsum = wave_sum64(found ? (int64_t)a.out_deg[v] : 0);
        int32_t base = 0;
        if (lane == 0) {
            fb_next[w] = fm;          // this wave owns word w: plain stores
            a.visited[w] = vis | fm;
            base = atomicAdd(&nxt->n, (int32_t)__popcll(fm));
            atomicAdd(reinterpret_cast<unsigned long long*>(&nxt->m), (unsigned long long)dsum);
        }
        base = __shfl(base, 0);
        if (found) q_next[base + __popcll(fm & lanes_below(lane))] = v;
    }
}

// Expands frontier `lvl` (slot lvl % 3) into lvl+1.  policy: PP_PUSH,
// PP_PULL or PP_SWITCH (decided here from the slot statistics).
__global__ __launch_bounds__(kBlock) void k_bfs_level(BfsArgs a, int32_t lvl, int32_t policy, float alpha,
                                                       float beta) {
    BfsHdr* h = a.hdr;
    const int sc = lvl % 3, sn = (lvl + 1) % 3, sz = (lvl + 2) % 3;
    const BfsSlot cur = h->slot[sc];
    const int32_t nf = cur.n;
    const bool lead = (blockIdx.x == 0 && threadIdx.x == 0);
    if (nf == 0) {
        if (lead) h->slot[sz] = BfsSlot{0, 0, 0, 0, 0, 0};
        return;
    }
    const int64_t mu = cur.mu_base - cur.m;  // out-edges of vertices not yet visited
    int32_t dir = policy;
    if (policy == PP_SWITCH) {
        if (lvl == 0 || cur.dir_prev == PP_PUSH) {
            dir = ((double)cur.m > (double)mu / (double)alpha) ? PP_PULL : PP_PUSH;
        } else {
            dir = ((double)nf < (double)a.n / (double)beta && nf < cur.n_prev) ? PP_PUSH : PP_PULL;
        }
    }
    if (lead) {
        h->slot[sz] = BfsSlot{0, 0, 0, 0, 0, 0};
        h->slot[sn].dir_prev = dir;
        h->slot[sn].n_prev = nf;
        h->slot[sn].mu_base = mu;
        if (lvl < PP_BFS_MAX_LOG) {
            h->log_dir[lvl] = (int8_t)dir;
            h->log_n[lvl] = nf;
        }
        h->levels = lvl + 1;
        h->last = lvl + 1;
        h->reached += nf;
        h->edges += cur.m;
    }
    // the bitmap two levels ahead is rewritten next level: clear it now
    uint64_t* fb_clear = a.fb[sz];
    for (int32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < a.words; w += gridDim.x * blockDim.x)
        fb_clear[w] = 0ull;
    if (dir == PP_PUSH)
        level_top_down(a, lvl, nf, a.queue[lvl & 1], a.queue[(lvl + 1) & 1], a.fb[sn], &h->slot[sn]);
    else
        level_bottom_up(a, lvl, a.fb[sc], a.queue[(lvl + 1) & 1], a.fb[sn], &h->slot[sn]);
}

static pp_status check_state(pp_graph g, void* state, size_t bytes) {
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (!state) return set_error(PP_E_NULL, "state is NULL");
    if (bytes < bfs_layout(g->d.n).total) return set_error(PP_E_WORKSPACE, "BFS state buffer too small");
    if (reinterpret_cast<uintptr_t>(state) % 256 != 0) return set_error(PP_E_RANGE, "state must be 256-byte aligned");
    return PP_OK;
}

static pp_status launch_level(pp_graph g, void* state, int32_t* level, int32_t* parent, int32_t lvl, int32_t policy,
                              float alpha, float beta, hipStream_t st) {
    BfsArgs a = bfs_args(g, state, level, parent);
    hipLaunchKernelGGL(k_bfs_level, dim3(kBfsBlocks), dim3(kBlock), 0, st, a, lvl, policy, alpha, beta);
    PP_LAUNCH_CHECK("k_bfs_level");
    return PP_OK;
}

}  // namespace pp

using namespace pp;

PP_EXPORT size_t pp_bfs_state_bytes(pp_graph g) { return g ? bfs_layout(g->d.n).total : 0; }

PP_EXPORT pp_status pp_bfs_init(pp_graph g, int32_t root, int32_t* level, int32_t* parent, void* state,
                                size_t state_bytes, void* stream) {
    clear_error();
    pp_status s = check_state(g, state, state_bytes);
    if (s != PP_OK) return s;
    if (!level || !parent) return set_error(PP_E_NULL, "level and parent are required");
    if (root < 0 || root >= g->d.n) return set_error(PP_E_RANGE, "root out of range");
    BfsArgs a = bfs_args(g, state, level, parent);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t blocks = std::min<int32_t>(ceil_div(g->d.n, 256), 4096);
    hipLaunchKernelGGL(k_bfs_init, dim3(blocks), dim3(256), 0, st, a, root, g->d.nnz);
    PP_LAUNCH_CHECK("k_bfs_init");
    return PP_OK;
}

static pp_status step(pp_graph g, void* state, int32_t* level, int32_t* parent, int32_t cur_level, int32_t dir,
                      void* stream) {
    clear_error();
    if (!g || !state || !level || !parent) return set_error(PP_E_NULL, "graph, state, level and parent are required");
    if (cur_level < 0 || cur_level >= g->d.n) return set_error(PP_E_RANGE, "cur_level out of range");
    return launch_level(g, state, level, parent, cur_level, dir, 14.f, 24.f, static_cast<hipStream_t>(stream));
}

PP_EXPORT pp_status pp_bfs_step_push(pp_graph g, void* state, int32_t* level, int32_t* parent, int32_t cur_level,
                                     void* stream) {
    return step(g, state, level, parent, cur_level, PP_PUSH, stream);
}

PP_EXPORT pp_status pp_bfs_step_pull(pp_graph g, void* state, int32_t* level, int32_t* parent, int32_t cur_level,
                                     void* stream) {
    return step(g, state, level, parent, cur_level, PP_PULL, stream);
}

static pp_status read_hdr(pp_graph g, void* state, BfsHdr* h, hipStream_t st) {
    const BfsLayout L = bfs_layout(g->d.n);
    PP_HIP(hipMemcpyAsync(h, static_cast<char*>(state) + L.hdr, sizeof(BfsHdr), hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    return PP_OK;
}

PP_EXPORT pp_status pp_bfs_frontier(pp_graph g, void* state, int32_t* size, void* stream) {
    clear_error();
    if (!g || !state || !size) return set_error(PP_E_NULL, "graph, state and size are required");
    BfsHdr h;
    pp_status s = read_hdr(g, state, &h, static_cast<hipStream_t>(stream));
    if (s != PP_OK) return s;
    *size = h.slot[h.last % 3].n;
    return PP_OK;
}

PP_EXPORT pp_status pp_bfs_run(pp_graph g, int32_t root, pp_dir policy, float alpha, float beta, int32_t* level,
                               int32_t* parent, void* state, size_t state_bytes, pp_bfs_stats* stats, void* stream) {
    clear_error();
    if (policy != PP_PUSH && policy != PP_PULL && policy != PP_SWITCH)
        return set_error(PP_E_RANGE, "policy must be PP_PUSH, PP_PULL or PP_SWITCH");
    if (!(alpha > 0.f)) alpha = 14.f;
    if (!(beta > 0.f)) beta = 24.f;
    pp_status s = pp_bfs_init(g, root, level, parent, state, state_bytes, stream);
    if (s != PP_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const BfsLayout L = bfs_layout(g->d.n);
    const BfsHdr* dh = reinterpret_cast<const BfsHdr*>(static_cast<char*>(state) + L.hdr);
    // Levels are launched in growing batches; kernels past the last level find
    // an empty frontier and return at once, so only termination needs a read.
    int32_t lvl = 0, batch = 2;
    const int32_t max_levels = g->d.n;  // a BFS has at most n non-empty frontiers
    for (;;) {
        for (int32_t i = 0; i < batch && lvl < max_levels; ++i, ++lvl) {
            s = launch_level(g, state, level, parent, lvl, policy, alpha, beta, st);
            if (s != PP_OK) return s;
        }
        int32_t nf = 0;
        PP_HIP(hipMemcpyAsync(&nf, &dh->slot[lvl % 3].n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        PP_HIP(hipStreamSynchronize(st));
        if (nf == 0 || lvl >= max_levels) break;
        batch = std::min<int32_t>(batch * 2, 64);
    }
    if (stats) {
        BfsHdr h;
        s = read_hdr(g, state, &h, st);
        if (s != PP_OK) return s;
        stats->levels = h.levels;
        stats->reached = (int32_t)h.reached;
        stats->edges_reached = h.edges;
        for (int i = 0; i < PP_BFS_MAX_LOG; ++i) {
            stats->dir[i] = (i < h.levels) ? h.log_dir[i] : (int8_t)-1;
            stats->frontier[i] = (i < h.levels) ? h.log_n[i] : 0;
        }
    }
    return PP_OK;
}
