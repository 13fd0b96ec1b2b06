// BFS frontier step in its pushing (top-down) and pulling (bottom-up) forms
// (Sec. 3.3; Sec. 4.3 listing with every ready counter equal to one), and
// the per-level direction switch (Sec. 5 Generic-Switch, applied to BFS as in
// the direction-optimising BFS the paper cites in Sec. 1).
//
// One kernel expands one level; top-down levels add a second kernel for the
// chunks of very long rows.  Both forms leave the new frontier as a queue AND
// a bitmap, so any sequence of directions works without conversions.
//
// Contention design: a device-scope atomic on one address serialises across
// the whole GPU, so no address is hit per edge or per wavefront step:
//  - the frontier queue is paged: each wavefront fills its own page of
//    kPage entries and takes a new page with one atomic when it is full;
//  - frontier statistics are summed per workgroup, one atomic each;
//  - top-down claims use one atomic OR on a 64-vertex visited word, tried
//    only after a plain read shows the vertex unvisited.
// Per-level statistics (|F|, out-edges of F, out-edges of unvisited
// vertices) live in three rotating slots so the direction is chosen on the
// device and the host only polls for termination.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pp_common.h"

namespace pp {

constexpr int32_t kPage = 256;      // queue entries per page
constexpr int32_t kBigRow = 1024;   // top-down rows longer than this are chunked
constexpr int32_t kBigInRow = 2048; // bottom-up in-rows longer than this are chunked
constexpr int kBfsMaxBlocks = 1024;

struct BfsSlot {
    int32_t n;         // frontier size (accumulated by the level that builds it)
    int32_t dir_prev;  // direction used to build this frontier
    int32_t n_prev;    // size of the frontier it was built from
    int32_t pages;     // queue pages used by this frontier
    int32_t big;       // chunk items queued while expanding this slot's level
    int32_t pad[3];
    int64_t m;         // out-edges of the frontier (accumulated)
    int64_t mu_base;   // out-edges of vertices unvisited before this frontier
    int64_t pad2[4];
};

struct BfsHdr {
    BfsSlot slot[3];
    int32_t levels;    // number of non-empty frontiers expanded so far
    int32_t last;      // index of the newest frontier
    int32_t root;
    int32_t overflow;  // set if a capacity bound was ever hit (never expected)
    int64_t reached;
    int64_t edges;
    int8_t log_dir[PP_BFS_MAX_LOG];
    int32_t log_n[PP_BFS_MAX_LOG];
};

struct BfsLayout {
    size_t hdr, queue0, queue1, fill0, fill1, fb0, fb1, fb2, visited, items, best, total;
    int32_t words, blocks, page_cap, item_cap;
};

static int32_t bfs_blocks(int32_t n) { return std::min(std::max(ceil_div(n, 2048), 4), kBfsMaxBlocks); }

static BfsLayout bfs_layout(int32_t n, int64_t nnz) {
    BfsLayout L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p = align_up(p + bytes, 256);
        return at;
    };
    L.words = ceil_div(n, 64);
    L.blocks = bfs_blocks(n);
    const int32_t waves = L.blocks * (kBlock / kWave);
    // full pages hold at most n entries; each wavefront of each of the two
    // kernels of a level leaves at most one partial page
    L.page_cap = ceil_div(n, kPage) + 2 * waves + 2;
    L.item_cap = (int32_t)std::min<int64_t>(2 * nnz / std::min(kBigRow, kBigInRow) + 64, INT32_MAX / 4);
    L.hdr = take(sizeof(BfsHdr));
    L.queue0 = take((size_t)L.page_cap * kPage * 4);
    L.queue1 = take((size_t)L.page_cap * kPage * 4);
    L.fill0 = take((size_t)L.page_cap * 4);
    L.fill1 = take((size_t)L.page_cap * 4);
    L.fb0 = take((size_t)L.words * 8);
    L.fb1 = take((size_t)L.words * 8);
    L.fb2 = take((size_t)L.words * 8);
    L.visited = take((size_t)L.words * 8);
    L.items = take((size_t)L.item_cap * 3 * 4);
    L.best = take((size_t)n * 4);
    L.total = p;
    return L;
}

struct BfsArgs {
    int32_t n;
    int32_t words;
    int32_t page_cap;
    int32_t item_cap;
    const int32_t* csr_off;
    const int32_t* csr_idx;
    const int32_t* csc_off;
    const int32_t* csc_idx;
    const int32_t* out_deg;
    const int32_t* perm;    // internal -> caller id (nullable)
    const int32_t* iperm;   // caller -> internal id (nullable)
    int32_t* level;         // caller ids
    int32_t* parent;        // caller ids
    BfsHdr* hdr;
    int32_t* queue[2];
    int32_t* fill[2];
    uint64_t* fb[3];
    uint64_t* visited;
    int32_t* items;         // (v, begin, end) chunk items of long rows
    int32_t* best;          // bottom-up: first hit position in a long in-row (INT32_MAX: none)
};

static BfsArgs bfs_args(pp_graph g, void* state, int32_t* level, int32_t* parent) {
    const BfsLayout L = bfs_layout(g->d.n, g->d.nnz);
    char* s = static_cast<char*>(state);
    BfsArgs a;
    a.n = g->d.n;
    a.words = L.words;
    a.page_cap = L.page_cap;
    a.item_cap = L.item_cap;
    a.csr_off = g->d.csr_off;
    a.csr_idx = g->d.csr_idx;
    a.csc_off = g->d.csc_off;
    a.csc_idx = g->d.csc_idx;
    a.out_deg = g->d.out_deg;
    a.perm = g->d.perm;
    a.iperm = g->d.iperm;
    a.level = level;
    a.parent = parent;
    a.hdr = reinterpret_cast<BfsHdr*>(s + L.hdr);
    a.queue[0] = reinterpret_cast<int32_t*>(s + L.queue0);
    a.queue[1] = reinterpret_cast<int32_t*>(s + L.queue1);
    a.fill[0] = reinterpret_cast<int32_t*>(s + L.fill0);
    a.fill[1] = reinterpret_cast<int32_t*>(s + L.fill1);
    a.fb[0] = reinterpret_cast<uint64_t*>(s + L.fb0);
    a.fb[1] = reinterpret_cast<uint64_t*>(s + L.fb1);
    a.fb[2] = reinterpret_cast<uint64_t*>(s + L.fb2);
    a.visited = reinterpret_cast<uint64_t*>(s + L.visited);
    a.items = reinterpret_cast<int32_t*>(s + L.items);
    a.best = reinterpret_cast<int32_t*>(s + L.best);
    return a;
}

__device__ __forceinline__ uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// Orders this wavefront's LDS traffic (the per-wave arrays are never touched
// by other wavefronts, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
    return v;
}

// ------------------------------------------------------------------ output
// A wavefront's open page of the next-frontier queue (wave-uniform values).
struct Pager {
    int32_t page;
    int32_t fill;
};

// Appends the values of the lanes with `mine` set (rank = their index among
// them, k = how many).  Wave-collective.
__device__ __forceinline__ void page_append(const BfsArgs& a, Pager& pg, bool mine, int32_t val, int32_t rank,
                                            int32_t k, int32_t* q, int32_t* fill, BfsSlot* nxt, int lane) {
    const int32_t room = (pg.page >= 0) ? kPage - pg.fill : 0;
    if (k <= room) {
        if (mine) q[pg.page * kPage + pg.fill + rank] = val;
        pg.fill += k;
        return;
    }
    // the first `room` items complete the open page, the rest start a new one
    int32_t np = 0;
    if (lane == 0) {
        if (pg.page >= 0) fill[pg.page] = kPage;
        np = atomicAdd(&nxt->pages, 1);
        if (np >= a.page_cap) atomicOr(&a.hdr->overflow, 1);
    }
    np = __shfl(np, 0);
    if (np >= a.page_cap) {  // cannot happen within the sizing bound; drop instead of writing out of range
        pg.page = -1;
        pg.fill = 0;
        return;
    }
    if (mine) {
        if (rank < room) q[pg.page * kPage + pg.fill + rank] = val;
        else q[np * kPage + (rank - room)] = val;
    }
    pg.page = np;
    pg.fill = k - room;
}

__device__ __forceinline__ void page_close(const Pager& pg, int32_t* fill, int lane) {
    if (lane == 0 && pg.page >= 0) fill[pg.page] = pg.fill;
}

// Per-workgroup sum of the new-frontier counters, then one atomic each.
__device__ __forceinline__ void flush_stats(int32_t cnt, int64_t deg, BfsSlot* nxt) {
    __shared__ int32_t s_cnt[kBlock / kWave];
    __shared__ int64_t s_deg[kBlock / kWave];
    cnt = wave_sum(cnt);
    deg = wave_sum(deg);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s_cnt[w] = cnt;
        s_deg[w] = deg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t c = 0;
        int64_t d = 0;
        for (int i = 0; i < kBlock / kWave; ++i) {
            c += s_cnt[i];
            d += s_deg[i];
        }
        if (c) {
            atomicAdd(&nxt->n, c);
            atomicAdd(reinterpret_cast<unsigned long long*>(&nxt->m), (unsigned long long)d);
        }
    }
}

// ------------------------------------------------------------------ init
__global__ void k_bfs_init(BfsArgs a, int32_t root_user, int64_t nnz) {
    const int32_t root = a.iperm ? a.iperm[root_user] : root_user;
    const int32_t stride = gridDim.x * blockDim.x;
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int32_t v = t; v < a.n; v += stride) {
        a.level[v] = (v == root_user) ? 0 : -1;
        a.parent[v] = (v == root_user) ? root_user : -1;
        a.best[v] = INT32_MAX;
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
        a.fill[0][0] = 1;
        BfsHdr* h = a.hdr;
        for (int i = 0; i < 3; ++i) h->slot[i] = BfsSlot{};
        h->slot[0].n = 1;
        h->slot[0].dir_prev = PP_PUSH;
        h->slot[0].pages = 1;
        h->slot[0].m = a.out_deg[root];
        h->slot[0].mu_base = nnz;
        h->levels = 0;
        h->last = 0;
        h->root = root;
        h->overflow = 0;
        h->reached = 0;
        h->edges = 0;
    }
}

// Queues (v, begin, end) chunk items of `chunk` edges for the lanes with
// `huge` set.  Wave-collective; one counter atomic per call.
__device__ __forceinline__ void queue_chunks(const BfsArgs& a, bool huge, int32_t v, int32_t rb, int32_t re,
                                             int32_t chunk, BfsSlot* nxt, int lane) {
    const int32_t nch = huge ? (re - rb + chunk - 1) / chunk : 0;
    int32_t incl = nch;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    const int32_t tot = __shfl(incl, kWave - 1);
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(&nxt->big, tot);
    base = __shfl(base, 0);
    for (int32_t k = 0; k < nch; ++k) {
        const int32_t it = base + incl - nch + k;
        if (it < a.item_cap) {
            a.items[3 * it] = v;
            a.items[3 * it + 1] = rb + k * chunk;
            a.items[3 * it + 2] = min(re, rb + (k + 1) * chunk);
        } else {
            atomicOr(&a.hdr->overflow, 2);
        }
    }
}

// ------------------------------------------------------------------ top-down
struct TdCtx {
    int32_t lvl;
    int32_t* q_next;
    int32_t* fill_next;
    uint64_t* fb_next;
    BfsSlot* nxt;
};

// Claims u for parent v.  Wave-collective: every lane calls it.
__device__ __forceinline__ void td_claim(const BfsArgs& a, const TdCtx& cx, Pager& pg, int32_t u, int32_t v,
                                         int32_t& cnt, int64_t& deg, int lane) {
    bool claimed = false;
    if (u >= 0) {
        const uint64_t bit = 1ull << (u & 63);
        if (!(a.visited[u >> 6] & bit)) {
            const uint64_t old =
                atomicOr(reinterpret_cast<unsigned long long*>(&a.visited[u >> 6]), (unsigned long long)bit);
            claimed = !(old & bit);
        }
        if (claimed) {
            const int32_t uu = user_id(a.perm, u);
            a.level[uu] = cx.lvl + 1;
            a.parent[uu] = user_id(a.perm, v);
            atomicOr(reinterpret_cast<unsigned long long*>(&cx.fb_next[u >> 6]), (unsigned long long)bit);
            cnt += 1;
            deg += a.out_deg[u];
        }
    }
    const uint64_t mask = __ballot(claimed);
    if (mask == 0) return;
    page_append(a, pg, claimed, u, __popcll(mask & lanes_below(lane)), __popcll(mask), cx.q_next, cx.fill_next,
                cx.nxt, lane);
}

__device__ void level_top_down(const BfsArgs& a, const TdCtx& cx, const int32_t* q_cur, const int32_t* fill_cur,
                               int32_t pages, int32_t& cnt, int64_t& deg, Pager& pg) {
    __shared__ int32_t s_start[kBlock / kWave][kWave];
    __shared__ int32_t s_rb[kBlock / kWave][kWave];
    __shared__ int32_t s_v[kBlock / kWave][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int32_t gwave = blockIdx.x * (kBlock / kWave) + w;
    const int32_t nwaves = gridDim.x * (kBlock / kWave);
    for (int32_t p = gwave; p < pages; p += nwaves) {
        const int32_t pfill = fill_cur[p];
        for (int32_t s = 0; s < pfill; s += kWave) {
            const int32_t i = s + lane;
            const int32_t v = (i < pfill) ? q_cur[p * kPage + i] : -1;
            const int32_t rb = (v >= 0) ? a.csr_off[v] : 0;
            const int32_t re = (v >= 0) ? a.csr_off[v + 1] : 0;
            int32_t len = re - rb;
            // very long rows: queue chunks for the second kernel
            const bool huge = len > kBigRow;
            if (__ballot(huge)) {
                queue_chunks(a, huge, v, rb, re, kBigRow, cx.nxt, lane);
                if (huge) len = 0;
            }
            // medium rows: the whole wave walks one row at a time
            uint64_t big = __ballot(len >= kWave);
            while (big) {
                const int src = __ffsll((long long)big) - 1;
                big &= big - 1;
                const int32_t bv = __shfl(v, src), bb = __shfl(rb, src), be = __shfl(re, src);
                for (int32_t jb = bb; jb < be; jb += kWave) {
                    const int32_t j = jb + lane;
                    td_claim(a, cx, pg, (j < be) ? a.csr_idx[j] : -1, bv, cnt, deg, lane);
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
                td_claim(a, cx, pg, u, pv, cnt, deg, lane);
            }
            wave_sync();
        }
    }
}

// ------------------------------------------------------------------ bottom-up
__device__ void level_bottom_up(const BfsArgs& a, int32_t lvl, const uint64_t* fb_cur, int32_t* q_next,
                                int32_t* fill_next, uint64_t* fb_next, BfsSlot* nxt, int32_t& cnt, int64_t& deg,
                                Pager& pg) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int32_t nwaves = gridDim.x * (kBlock / kWave);
    for (int32_t w = gwave; w < a.words; w += nwaves) {
        const uint64_t vis = a.visited[w];
        const int32_t v = w * kWave + lane;
        const bool unvisited = (v < a.n) && !((vis >> lane) & 1ull);
        if (__ballot(unvisited) == 0) continue;
        const int32_t rb = unvisited ? a.csc_off[v] : 0;
        int32_t re = unvisited ? a.csc_off[v + 1] : 0;
        bool found = false;
        int32_t par = -1;
        // very long in-rows: chunks scanned grid-wide by k_bfs_bu_big
        const bool huge = (re - rb) > kBigInRow;
        if (__ballot(huge)) {
            queue_chunks(a, huge, v, rb, re, kBigInRow, nxt, lane);
            if (huge) re = rb;
        }
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
            const int32_t vu = user_id(a.perm, v);
            a.level[vu] = lvl + 1;
            a.parent[vu] = user_id(a.perm, par);
            cnt += 1;
            deg += a.out_deg[v];
        }
        if (lane == 0) {
            fb_next[w] = fm;  // this wave owns word w: plain stores
            a.visited[w] = vis | fm;
        }
        page_append(a, pg, found, v, __popcll(fm & lanes_below(lane)), __popcll(fm), q_next, fill_next, nxt, lane);
    }
}

// Expands frontier `lvl` (slot lvl % 3) into lvl+1.  policy: PP_PUSH,
// PP_PULL or PP_SWITCH (decided here, identically in every workgroup, from
// the slot statistics).
__global__ __launch_bounds__(kBlock) void k_bfs_level(BfsArgs a, int32_t lvl, int32_t policy, float alpha,
                                                       float beta) {
    BfsHdr* h = a.hdr;
    const int sc = lvl % 3, sn = (lvl + 1) % 3, sz = (lvl + 2) % 3;
    const BfsSlot cur = h->slot[sc];
    const int32_t nf = cur.n;
    const bool lead = (blockIdx.x == 0 && threadIdx.x == 0);
    if (nf == 0) {
        if (lead) h->slot[sz] = BfsSlot{};
        return;
    }
    const int64_t mu = cur.mu_base - cur.m;  // out-edges of vertices not yet visited
    int32_t dir = policy;
    if (policy == PP_SWITCH) {
        if (lvl == 0 || cur.dir_prev == PP_PUSH)
            dir = ((double)cur.m > (double)mu / (double)alpha) ? PP_PULL : PP_PUSH;
        else
            dir = ((double)nf < (double)a.n / (double)beta && nf < cur.n_prev) ? PP_PUSH : PP_PULL;
    }
    if (lead) {
        h->slot[sz] = BfsSlot{};
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
    const int lane = threadIdx.x & (kWave - 1);
    int32_t cnt = 0;
    int64_t deg = 0;
    Pager pg{-1, 0};
    int32_t* q_next = a.queue[(lvl + 1) & 1];
    int32_t* fill_next = a.fill[(lvl + 1) & 1];
    if (dir == PP_PUSH) {
        TdCtx cx{lvl, q_next, fill_next, a.fb[sn], &h->slot[sn]};
        level_top_down(a, cx, a.queue[lvl & 1], a.fill[lvl & 1], min(cur.pages, a.page_cap), cnt, deg, pg);
    } else {
        level_bottom_up(a, lvl, a.fb[sc], q_next, fill_next, a.fb[sn], &h->slot[sn], cnt, deg, pg);
    }
    page_close(pg, fill_next, lane);
    flush_stats(cnt, deg, &h->slot[sn]);
}

// Second top-down pass: the chunk items queued for rows longer than kBigRow,
// one wavefront per chunk.
__global__ __launch_bounds__(kBlock) void k_bfs_td_big(BfsArgs a, int32_t lvl) {
    BfsHdr* h = a.hdr;
    const int sn = (lvl + 1) % 3;
    if (h->slot[sn].dir_prev != PP_PUSH) return;
    const int32_t items = min(h->slot[sn].big, a.item_cap);
    if (items == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int32_t nwaves = gridDim.x * (kBlock / kWave);
    int32_t cnt = 0;
    int64_t deg = 0;
    Pager pg{-1, 0};
    TdCtx cx{lvl, a.queue[(lvl + 1) & 1], a.fill[(lvl + 1) & 1], a.fb[sn], &h->slot[sn]};
    for (int32_t it = gwave; it < items; it += nwaves) {
        const int32_t v = a.items[3 * it], b = a.items[3 * it + 1], e = a.items[3 * it + 2];
        for (int32_t jb = b; jb < e; jb += kWave) {
            const int32_t j = jb + lane;
            td_claim(a, cx, pg, (j < e) ? a.csr_idx[j] : -1, v, cnt, deg, lane);
        }
    }
    page_close(pg, cx.fill_next, lane);
    flush_stats(cnt, deg, &h->slot[sn]);
}

// Bottom-up pass over the chunks of very long in-rows, one wavefront per
// chunk: the first frontier member in a chunk lowers best[v] to its slot.
// A chunk stops early once an earlier slot of the same row has a hit.
__global__ __launch_bounds__(kBlock) void k_bfs_bu_big(BfsArgs a, int32_t lvl) {
    BfsHdr* h = a.hdr;
    const int sc = lvl % 3, sn = (lvl + 1) % 3;
    if (h->slot[sn].dir_prev != PP_PULL) return;
    const int32_t items = min(h->slot[sn].big, a.item_cap);
    const uint64_t* fb_cur = a.fb[sc];
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int32_t nwaves = gridDim.x * (kBlock / kWave);
    for (int32_t it = gwave; it < items; it += nwaves) {
        const int32_t v = a.items[3 * it], b = a.items[3 * it + 1], e = a.items[3 * it + 2];
        for (int32_t jb = b; jb < e; jb += kWave) {
            if (__shfl(lane == 0 ? a.best[v] : 0, 0) < jb) break;  // an earlier slot already hit
            const int32_t j = jb + lane;
            const int32_t u = (j < e) ? a.csc_idx[j] : -1;
            const bool hit = (u >= 0) && ((fb_cur[u >> 6] >> (u & 63)) & 1ull);
            const uint64_t hm = __ballot(hit);
            if (hm) {
                if (lane == 0) atomicMin(&a.best[v], jb + __ffsll((long long)hm) - 1);
                break;
            }
        }
    }
}

// Finishes the long in-row vertices: one item per vertex (its first chunk)
// records the parent at best[v], sets the bitmaps and appends the vertex.
__global__ __launch_bounds__(kBlock) void k_bfs_bu_fin(BfsArgs a, int32_t lvl) {
    BfsHdr* h = a.hdr;
    const int sn = (lvl + 1) % 3;
    if (h->slot[sn].dir_prev != PP_PULL) return;
    const int32_t items = min(h->slot[sn].big, a.item_cap);
    if (items == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    int32_t cnt = 0;
    int64_t deg = 0;
    Pager pg{-1, 0};
    int32_t* q_next = a.queue[(lvl + 1) & 1];
    int32_t* fill_next = a.fill[(lvl + 1) & 1];
    const int32_t nthreads = gridDim.x * blockDim.x;
    const int32_t t0 = blockIdx.x * blockDim.x + threadIdx.x;
    // wave-uniform trip count so page_append stays wave-collective
    const int32_t trips = (items + nthreads - 1) / nthreads;
    for (int32_t r = 0; r < trips; ++r) {
        const int32_t it = t0 + r * nthreads;
        bool found = false;
        int32_t v = -1;
        if (it < items) {
            v = a.items[3 * it];
            if (a.items[3 * it + 1] == a.csc_off[v]) {  // first chunk of v
                const int32_t pos = a.best[v];
                if (pos != INT32_MAX) {
                    found = true;
                    const int32_t vu = user_id(a.perm, v);
                    a.level[vu] = lvl + 1;
                    a.parent[vu] = user_id(a.perm, a.csc_idx[pos]);
                    const uint64_t bit = 1ull << (v & 63);
                    atomicOr(reinterpret_cast<unsigned long long*>(&a.visited[v >> 6]), (unsigned long long)bit);
                    atomicOr(reinterpret_cast<unsigned long long*>(&a.fb[sn][v >> 6]), (unsigned long long)bit);
                    a.best[v] = INT32_MAX;
                    cnt += 1;
                    deg += a.out_deg[v];
                }
            }
        }
        const uint64_t fm = __ballot(found);
        if (fm) page_append(a, pg, found, v, __popcll(fm & lanes_below(lane)), __popcll(fm), q_next, fill_next,
                            &h->slot[sn], lane);
    }
    page_close(pg, fill_next, lane);
    flush_stats(cnt, deg, &h->slot[sn]);
}

static pp_status check_state(pp_graph g, void* state, size_t bytes) {
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (!state) return set_error(PP_E_NULL, "state is NULL");
    if (bytes < bfs_layout(g->d.n, g->d.nnz).total) return set_error(PP_E_WORKSPACE, "BFS state buffer too small");
    if (reinterpret_cast<uintptr_t>(state) % 256 != 0) return set_error(PP_E_RANGE, "state must be 256-byte aligned");
    return PP_OK;
}

static pp_status launch_level(pp_graph g, const BfsArgs& a, int32_t lvl, int32_t policy, float alpha, float beta,
                              hipStream_t st) {
    const int32_t blocks = bfs_blocks(g->d.n);
    hipLaunchKernelGGL(k_bfs_level, dim3(blocks), dim3(kBlock), 0, st, a, lvl, policy, alpha, beta);
    if (policy != PP_PULL && g->max_out_deg > kBigRow)
        hipLaunchKernelGGL(k_bfs_td_big, dim3(blocks), dim3(kBlock), 0, st, a, lvl);
    if (policy != PP_PUSH && g->max_in_deg > kBigInRow) {
        hipLaunchKernelGGL(k_bfs_bu_big, dim3(blocks), dim3(kBlock), 0, st, a, lvl);
        hipLaunchKernelGGL(k_bfs_bu_fin, dim3(blocks), dim3(kBlock), 0, st, a, lvl);
    }
    PP_LAUNCH_CHECK("k_bfs_level");
    return PP_OK;
}

static pp_status read_hdr(pp_graph g, void* state, BfsHdr* h, hipStream_t st) {
    const BfsLayout L = bfs_layout(g->d.n, g->d.nnz);
    PP_HIP(hipMemcpyAsync(h, static_cast<char*>(state) + L.hdr, sizeof(BfsHdr), hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    if (h->overflow) return set_error(PP_E_WORKSPACE, "BFS queue capacity exceeded");
    return PP_OK;
}

}  // namespace pp

using namespace pp;

PP_EXPORT size_t pp_bfs_state_bytes(pp_graph g) { return g ? bfs_layout(g->d.n, g->d.nnz).total : 0; }

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
    BfsArgs a = bfs_args(g, state, level, parent);
    return launch_level(g, a, cur_level, dir, 14.f, 24.f, static_cast<hipStream_t>(stream));
}

PP_EXPORT pp_status pp_bfs_step_push(pp_graph g, void* state, int32_t* level, int32_t* parent, int32_t cur_level,
                                     void* stream) {
    return step(g, state, level, parent, cur_level, PP_PUSH, stream);
}

PP_EXPORT pp_status pp_bfs_step_pull(pp_graph g, void* state, int32_t* level, int32_t* parent, int32_t cur_level,
                                     void* stream) {
    return step(g, state, level, parent, cur_level, PP_PULL, stream);
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
    const BfsLayout L = bfs_layout(g->d.n, g->d.nnz);
    const BfsHdr* dh = reinterpret_cast<const BfsHdr*>(static_cast<char*>(state) + L.hdr);
    BfsArgs a = bfs_args(g, state, level, parent);
    // Levels go out in growing batches; kernels past the last level find an
    // empty frontier and return at once, so only termination needs a read.
    int32_t lvl = 0, batch = 2;
    const int32_t max_levels = g->d.n;  // a BFS has at most n non-empty frontiers
    for (;;) {
        for (int32_t i = 0; i < batch && lvl < max_levels; ++i, ++lvl) {
            s = launch_level(g, a, lvl, policy, alpha, beta, st);
            if (s != PP_OK) return s;
        }
        int32_t nf = 0;
        PP_HIP(hipMemcpyAsync(&nf, &dh->slot[lvl % 3].n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        PP_HIP(hipStreamSynchronize(st));
        if (nf == 0 || lvl >= max_levels) break;
        batch = std::min<int32_t>(batch * 2, 64);
    }
    BfsHdr h;
    s = read_hdr(g, state, &h, st);
    if (s != PP_OK) return s;
    if (stats) {
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
