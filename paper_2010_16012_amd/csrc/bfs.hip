// BFS frontier step in its pushing (top-down) and pulling (bottom-up) forms
// (Sec. 3.3; Sec. 4.3 listing with every ready counter equal to one), and
// the per-level direction switch (Sec. 5 Generic-Switch, applied to BFS as in
// the direction-optimising BFS the paper cites in Sec. 1).
//
// One kernel expands one level; a second kernel takes the chunks of very long
// rows.  Both forms leave the new frontier as a queue AND a bitmap, so any
// sequence of directions works without conversions.  A bottom-up level with
// a sparse frontier streams the whole in-edge array instead of scanning row
// by row (see level_bottom_up_stream).
//
// Contention design: a device-scope atomic on one address serialises across
// the whole GPU, so no address is hit per edge or per wavefront step:
//  - the frontier queue is paged: each wavefront fills its own page of
//    kPage entries and takes a new page with one atomic when it is full.
//    The first `static_pages` pages (one per level-kernel wavefront) are
//    reserved: in a bottom-up level, which appends a lot, every wavefront
//    starts on its own reserved page and takes no atomic until it is full;
//    a top-down level leaves them unused, and its readers skip them;
//  - frontier statistics are summed per workgroup, one atomic each;
//  - top-down claims use one atomic OR on a 64-vertex visited word, tried,
//    on large levels, only after a plain read shows the vertex unvisited.
// Per-level statistics (|F|, out-edges of F, out-edges of unvisited
// vertices) live in three rotating slots so the direction is chosen on the
// device and the host only polls for termination.
//
// Bit tests against the hot prefix of a bitmap go to LDS: after degree
// relabelling the lowest vertex ids are the highest-degree vertices, which
// most edges point to.  On large levels every workgroup first copies the
// prefix of the bitmap it tests -- the frontier (bottom-up; read-only during
// the level) or the visited set (top-down; a snapshot that can only miss
// bits set later, so a clear bit still goes to global memory) -- into LDS.
// A sparse bottom-up frontier also gets an LDS summary with one bit per
// bitmap word, so tests against empty words need no global load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "pp_common.h"

namespace pp {

constexpr int32_t kPage = 256;      // queue entries per page
// Rows longer than one chunk are cut into chunk items that the whole grid
// shares, so no wavefront walks a long row alone while the others idle.
constexpr int32_t kBigRow = 256;    // top-down (out-rows)
// Top-down levels with fewer frontier out-edges than nnz >> kSmallLevelShift
// cut rows into chunks of kBigRowSmall: the few hub rows of such a level then
// spread over many more wavefronts of the chunk kernel.  At R-MAT scale 22
// (64 roots) push runs went from 1.482 to 1.41 ms per root and switch runs
// from 0.382 to 0.361; 16-, 64- and 128-edge chunks, and bounds of nnz/4,
// nnz/8 or nnz/128, were slower.
constexpr int32_t kBigRowSmall = 32;
constexpr int kSmallLevelShift = 5;
// the item buffer, sized for chunks of min(kBigRow, kBigInRow) edges, then also
// holds a small top-down level's kBigRowSmall-edge items
static_assert((1 << kSmallLevelShift) * kBigRowSmall >= kBigRow && kBigRowSmall <= kBigRow, "chunk item bound");
// bottom-up (in-rows): the level kernel scans the first kBigInRow entries of
// a longer in-row (the whole wavefront, as kCoopRow allows) and queues the
// rest as chunk items.  256 ran pull 3.5% and switch 10% slower at R-MAT
// scale 22; 64, 96 and 192 were slower too.  A row of up to 2 kBigInRow
// in-edges is scanned in stored order (prefix, then at most one chunk).
constexpr int32_t kBigInRow = 128;
constexpr int kBfsBlock = 1024;    // threads per workgroup of the level kernels
constexpr int kBfsWaves = kBfsBlock / kWave;
constexpr int32_t kStaticLds = 16384;  // LDS bytes kept for the kernels' own arrays
// Bottom-up levels with a sparse frontier keep, in LDS, one bit per frontier
// bitmap word (set if the word is nonzero): a test of a vertex whose word is
// empty then needs no global load.  At most kSumMax summary words (8 KB).
constexpr int32_t kSumMax = 1024;
// Visited words the chunk kernel's top-down items test in LDS (120 KB; one
// workgroup of it per compute unit).
constexpr int32_t kChunkStage = 15360;

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
    // Level index on the device, so that a run's launches carry no level
    // argument: a level kernel of parity p reads lv[p] and its lead thread
    // writes lv[p ^ 1] for the next one (no kernel writes what it reads);
    // c_lvl tells the chunk kernel which level it completes.
    int32_t lv[2];
    int32_t c_lvl;
    int32_t finished;  // an empty frontier was reached
    int32_t busy;      // level-kernel launches that found a non-empty frontier
    int32_t pad;
    int64_t reached;
    int64_t edges;
    int8_t log_dir[PP_BFS_MAX_LOG];
    int32_t log_n[PP_BFS_MAX_LOG];
};

struct BfsLayout {
    size_t hdr, queue0, queue1, fill0, fill1, fb0, fb1, fb2, visited, items, total;
    int32_t words, blocks, page_cap, item_cap, stage_words, sum_words;
};

// One workgroup per compute unit (the staged bitmap takes most of its LDS),
// fewer on small graphs.
static int32_t bfs_blocks(pp_graph g) { return std::max(1, std::min(ceil_div(g->d.n, 4096), g->num_cu)); }

static BfsLayout bfs_layout(pp_graph g) {
    const int32_t n = g->d.n;
    const int64_t nnz = g->d.nnz;
    BfsLayout L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p = align_up(p + bytes, 256);
        return at;
    };
    L.words = ceil_div(n, 64);
    L.blocks = bfs_blocks(g);
    const int32_t lds_words = std::max(0, (g->max_lds - kStaticLds) / 8);
    L.sum_words = (L.words > lds_words) ? std::min(ceil_div(L.words, 64), kSumMax) : 0;
    L.stage_words = std::max(0, std::min(L.words, lds_words - L.sum_words));
    const int32_t waves = L.blocks * kBfsWaves;
    // the reserved pages (one per level-kernel wavefront); full pages hold at
    // most n entries; each wavefront of the level kernel and of the chunk
    // kernel (at most twice as many wavefronts) leaves at most one partial page
    L.page_cap = waves + ceil_div(n, kPage) + 3 * waves + 2;
    // a row cut into chunks of c edges (longer than c) gives at most 2 len / c
    // items: a level queues at most 2 nnz / min(kBigRow, kBigInRow), and a
    // top-down level with m < nnz / 32 at most 2 m / 32 < nnz / 512 of
    // kBigRowSmall edges
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
    L.total = p;
    return L;
}

struct BfsArgs {
    int32_t n;
    int64_t nnz;
    int32_t words;
    // bitmap words that hold every vertex with an in-edge: only those can be
    // discovered, so bottom-up levels (and frontiers read from a bitmap,
    // which hold discovered vertices) stop there
    int32_t act_words;
    int32_t page_cap;
    int32_t item_cap;
    int32_t stage_words;    // bitmap words a workgroup may stage in LDS
    int32_t sum_words;      // LDS summary words (after the staged words; 0 = none)
    int32_t chunk_stage;    // visited words the chunk kernel may stage
    // chunk length of out-rows on small top-down levels: kBigRowSmall when
    // rows longer than kBigRow exist (the chunk kernel then follows every
    // level of a policy with top-down levels), else kBigRow (no items)
    int32_t td_small_row;
    int32_t static_pages;   // queue pages owned one per wavefront of the level kernel
    int64_t stage_min;      // stage only when the level examines at least this many edges
    const int32_t* csr_off;
    const int32_t* csr_idx;
    const int32_t* csc_off;
    const int32_t* csc_idx;
    const int32_t* csc_row;  // owner (row) of every CSC slot
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
    pp_bfs_level* log;      // per-level log (caller device memory; nullable)
    int32_t log_cap;        // entries of log
};

static BfsArgs bfs_args(pp_graph g, void* state, int32_t* level, int32_t* parent) {
    const BfsLayout L = bfs_layout(g);
    char* s = static_cast<char*>(state);
    BfsArgs a;
    a.n = g->d.n;
    a.nnz = g->d.nnz;
    a.words = L.words;
    a.act_words = ceil_div(g->in_active, 64);
    a.page_cap = L.page_cap;
    a.item_cap = L.item_cap;
    a.stage_words = L.stage_words;
    a.sum_words = L.sum_words;
    // never more than the level kernel stages: the LDS allowance covers both
    a.chunk_stage = std::min(std::min(L.words, kChunkStage), L.stage_words);
    a.td_small_row = (g->max_out_deg > kBigRow) ? kBigRowSmall : kBigRow;
    a.static_pages = L.blocks * kBfsWaves;
    // copying costs each workgroup stage_words loads; pay it only when the
    // level has at least two edges per staged word per workgroup
    a.stage_min = 2 * (int64_t)L.blocks * L.stage_words;
    a.csr_off = g->d.csr_off;
    a.csr_idx = g->d.csr_idx;
    a.csc_off = g->d.csc_off;
    a.csc_idx = g->d.csc_idx;
    a.csc_row = g->d.csc_row;
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
    a.log = nullptr;
    a.log_cap = 0;
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

// Copies bitmap words [0, sw) into LDS.  Workgroup-collective.
// 16-byte loads, four in flight per thread (src is 256-byte aligned).
__device__ __forceinline__ void stage_bits(uint64_t* s_bits, const uint64_t* src, int32_t sw) {
    const int32_t n2 = sw >> 1;
    const ulonglong2* s2 = reinterpret_cast<const ulonglong2*>(src);
    ulonglong2* d2 = reinterpret_cast<ulonglong2*>(s_bits);
    const int32_t bd = blockDim.x;
    for (int32_t i0 = threadIdx.x; i0 < n2; i0 += 4 * bd) {
        ulonglong2 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = s2[min(i0 + k * bd, n2 - 1)];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k * bd < n2) d2[i0 + k * bd] = v[k];
    }
    if ((sw & 1) && threadIdx.x == 0) s_bits[sw - 1] = src[sw - 1];
    __syncthreads();
}

// A frontier bitmap as a bottom-up level tests it: words [0, sw) staged in
// LDS, and for words below lim an LDS summary (bit w clear: word w is zero).
struct FbView {
    const uint64_t* s_bits;
    int32_t sw;
    const uint64_t* s_sum;
    int32_t lim;  // 0: no summary
    const uint64_t* g_bits;
};

// Bits are read from the 32-bit half of their 64-bit word (the same bit,
// little-endian): half the LDS bandwidth per test.
__device__ __forceinline__ bool fb_test(const FbView& f, int32_t u) {
    const int32_t w = u >> 6;
    if (w < f.sw) return (reinterpret_cast<const uint32_t*>(f.s_bits)[u >> 5] >> (u & 31)) & 1u;
    if (w < f.lim && !((reinterpret_cast<const uint32_t*>(f.s_sum)[w >> 5] >> (w & 31)) & 1u)) return false;
    return (reinterpret_cast<const uint32_t*>(f.g_bits)[u >> 5] >> (u & 31)) & 1u;
}

// Summary bits of bitmap words [from rounded down to 64, 64 * sum_words)
// (words past the bitmap read as zero).  Workgroup-collective; the caller
// ends it with a barrier.
__device__ __forceinline__ void build_summary(uint64_t* s_sum, const uint64_t* g_bits, int32_t words, int32_t from,
                                              int32_t sum_words) {
    // eight words per lane in flight before their ballots
    constexpr int kAhead = 8;
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t nw = blockDim.x / kWave;
    for (int32_t c0 = (from >> 6) + (int32_t)(threadIdx.x / kWave); c0 < sum_words; c0 += kAhead * nw) {
        uint64_t v[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            const int32_t c = c0 + k * nw, i = c * kWave + lane;
            v[k] = (c < sum_words && i < words) ? g_bits[i] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            const uint64_t m = __ballot(v[k] != 0ull);
            if (lane == 0 && c0 + k * nw < sum_words) s_sum[c0 + k * nw] = m;
        }
    }
}

// Summary only when the frontier is sparse enough for most words to be zero.
__device__ __forceinline__ bool use_summary(const BfsArgs& a, int32_t nf) {
    return a.sum_words > 0 && (int64_t)nf * 8 < a.words;
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
    __shared__ int32_t s_cnt[kBfsWaves];
    __shared__ int64_t s_deg[kBfsWaves];
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
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
            c += s_cnt[i];
            d += s_deg[i];
        }
        if (c) {
            atomicAdd(&nxt->n, c);
            atomicAdd(reinterpret_cast<unsigned long long*>(&nxt->m), (unsigned long long)d);
        }
    }
}

// The fields of a slot a level kernel reads at its start.
struct SlotView {
    int32_t n, dir_prev, n_prev, pages;
    int64_t m, mu_base;
};

__device__ __forceinline__ SlotView view(const BfsSlot& s) {
    return SlotView{s.n, s.dir_prev, s.n_prev, s.pages, s.m, s.mu_base};
}

// ------------------------------------------------------------------ init
__global__ void k_bfs_init(BfsArgs a, int32_t root_user, int64_t nnz) {
    const int32_t root = a.iperm ? a.iperm[root_user] : root_user;
    const int32_t stride = gridDim.x * blockDim.x;
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int32_t v = t; v < a.n; v += stride) {
        a.level[v] = (v == root_user) ? 0 : -1;
        a.parent[v] = (v == root_user) ? root_user : -1;
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
        // the root frontier looks built by a top-down level: first page after
        // the reserved ones
        a.queue[0][(size_t)a.static_pages * kPage] = root;
        a.fill[0][a.static_pages] = 1;
        BfsHdr* h = a.hdr;
        for (int i = 0; i < 3; ++i) {
            h->slot[i] = BfsSlot{};
            h->slot[i].pages = a.static_pages;
        }
        h->slot[0].n = 1;
        h->slot[0].dir_prev = PP_PUSH;
        h->slot[0].pages = a.static_pages + 1;
        h->slot[0].m = a.out_deg[root];
        h->slot[0].mu_base = nnz;
        h->levels = 0;
        h->last = 0;
        h->lv[0] = 0;
        h->lv[1] = 0;
        h->c_lvl = -1;
        h->finished = 0;
        h->busy = 0;
        h->root = root;
        h->overflow = 0;
        h->reached = 0;
        h->edges = 0;
    }
}

// Queues (v, begin, end) chunk items of `chunk` edges for the lanes with
// `huge` set; the whole wave writes each row's items.  Wave-collective; one
// counter atomic per call.
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
    uint64_t rows = __ballot(huge);
    while (rows) {
        const int src = __ffsll((long long)rows) - 1;
        rows &= rows - 1;
        const int32_t hv = __shfl(v, src), hb = __shfl(rb, src), he = __shfl(re, src);
        const int32_t first = base + __shfl(incl - nch, src), cnt = __shfl(nch, src);
        for (int32_t k = lane; k < cnt; k += kWave) {
            const int32_t it = first + k;
            if (it < a.item_cap) {
                a.items[3 * it] = hv;
                a.items[3 * it + 1] = hb + k * chunk;
                a.items[3 * it + 2] = min(he, hb + (k + 1) * chunk);
            } else {
                atomicOr(&a.hdr->overflow, 2);
            }
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
    const uint64_t* s_vis;  // LDS snapshot of visited words [0, sw)
    int32_t sw;
    // read the visited word before claiming: filters targets visited earlier,
    // which pays on large levels; small levels go straight to the atomic and
    // save a round trip
    bool probe;
    int32_t big_row;  // out-rows longer than this become chunk items
};

// Below this many frontier out-edges a level claims without probing first.
constexpr int64_t kProbeMin = 1 << 16;

// Claims the targets u[r] (parents pv[r]; -1 = no edge) of kTdU rounds of
// 64 edges.  The rounds are independent, so their loads and atomics are
// issued together and their latencies overlap.  Wave-collective.
constexpr int kTdU = 4;

// ONE_PARENT: every edge of the batch leaves one vertex, pv[0] (a row or a
// chunk of one), so its caller id is looked up once.
template <bool ONE_PARENT = false>
__device__ __forceinline__ void td_batch(const BfsArgs& a, const TdCtx& cx, Pager& pg, const int32_t (&u)[kTdU],
                                         const int32_t (&pv)[kTdU], int32_t& cnt, int64_t& deg, int lane) {
    // Bits are tested and claimed in the 32-bit half of their 64-bit word
    // (the same bit, little-endian), which halves the registers the loads
    // and claims in flight take.  An atomic on one half is as atomic as one
    // on the whole word for the other bits' owners.
    const uint32_t* s_vis32 = reinterpret_cast<const uint32_t*>(cx.s_vis);
    uint32_t* vis32 = reinterpret_cast<uint32_t*>(a.visited);
    bool cand[kTdU];
#pragma unroll
    for (int r = 0; r < kTdU; ++r) {
        // a set bit in the LDS snapshot is final; a clear one is checked in memory
        const int32_t w = u[r] >> 6;
        cand[r] = (u[r] >= 0) && (w >= cx.sw || !((s_vis32[u[r] >> 5] >> (u[r] & 31)) & 1u));
    }
    uint32_t word[kTdU];
#pragma unroll
    for (int r = 0; r < kTdU; ++r) word[r] = (cand[r] && cx.probe) ? vis32[u[r] >> 5] : (cand[r] ? 0u : ~0u);
    // the out-degree and the caller ids a claim needs are loaded in flight
    // with the claim itself
    bool need[kTdU];
    int32_t od[kTdU], uid[kTdU], pid[kTdU];
    const int32_t pid1 = (ONE_PARENT && a.perm && pv[0] >= 0) ? a.perm[pv[0]] : pv[0];
#pragma unroll
    for (int r = 0; r < kTdU; ++r) {
        need[r] = cand[r] && !((word[r] >> (u[r] & 31)) & 1u);
        od[r] = need[r] ? a.out_deg[u[r]] : 0;
        uid[r] = (need[r] && a.perm) ? a.perm[u[r]] : u[r];
        pid[r] = ONE_PARENT ? pid1 : ((need[r] && a.perm) ? a.perm[pv[r]] : pv[r]);
    }
    bool claimed[kTdU];
#pragma unroll
    for (int r = 0; r < kTdU; ++r) {
        claimed[r] = false;
        const uint32_t bit = 1u << (u[r] & 31);
        if (need[r]) {
            const uint32_t old = atomicOr(&vis32[u[r] >> 5], bit);
            claimed[r] = !(old & bit);
        }
    }
#pragma unroll
    for (int r = 0; r < kTdU; ++r) {
        if (claimed[r]) {
            a.level[uid[r]] = cx.lvl + 1;
            a.parent[uid[r]] = pid[r];
            atomicOr(reinterpret_cast<uint32_t*>(cx.fb_next) + (u[r] >> 5), 1u << (u[r] & 31));
            cnt += 1;
            deg += od[r];
        }
        const uint64_t mask = __ballot(claimed[r]);
        if (mask)
            page_append(a, pg, claimed[r], u[r], __popcll(mask & lanes_below(lane)), __popcll(mask), cx.q_next,
                        cx.fill_next, cx.nxt, lane);
    }
}

// Edges [b, e) of the row of v, 64 x kTdU at a time.  Wave-collective
// (b, e, v wave-uniform).
__device__ __forceinline__ void td_row(const BfsArgs& a, const TdCtx& cx, Pager& pg, int32_t v, int32_t b,
                                       int32_t e, int32_t& cnt, int64_t& deg, int lane) {
    for (int32_t jb = b; jb < e; jb += kTdU * kWave) {
        int32_t u[kTdU], pv[kTdU];
#pragma unroll
        for (int r = 0; r < kTdU; ++r) {
            const int32_t j = jb + r * kWave + lane;
            u[r] = (j < e) ? a.csr_idx[j] : -1;
            pv[r] = v;
        }
        td_batch<true>(a, cx, pg, u, pv, cnt, deg, lane);
    }
}

// Per-wavefront LDS arrays of the level kernel, shared by its paths: the
// top-down dense enumeration (each lane's first edge, row start and vertex)
// and the streamed bottom-up hit list (slot, source).
struct WaveLds {
    int32_t a[kBfsWaves][kWave];
    int32_t b[kBfsWaves][kWave];
    int32_t c[kBfsWaves][kWave];
};

// The 64 frontier vertices v of one unit (-1 = none) expand their out-rows.
// Wave-collective.
__device__ __forceinline__ void td_unit(const BfsArgs& a, const TdCtx& cx, WaveLds& sl, Pager& pg, int32_t v,
                                        int32_t& cnt, int64_t& deg) {
    auto& s_start = sl.a;
    auto& s_rb = sl.b;
    auto& s_v = sl.c;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int32_t rb = (v >= 0) ? a.csr_off[v] : 0;
    const int32_t re = (v >= 0) ? a.csr_off[v + 1] : 0;
    int32_t len = re - rb;
    // very long rows: queue chunks for the second kernel
    const bool huge = len > cx.big_row;
    if (__ballot(huge)) {
        queue_chunks(a, huge, v, rb, re, cx.big_row, cx.nxt, lane);
        if (huge) len = 0;
    }
    // medium rows: the whole wave walks one row at a time
    uint64_t big = __ballot(len >= kWave);
    while (big) {
        const int src = __ffsll((long long)big) - 1;
        big &= big - 1;
        td_row(a, cx, pg, __shfl(v, src), __shfl(rb, src), __shfl(re, src), cnt, deg, lane);
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
    if (total == 0) return;
    s_start[w][lane] = incl - mine;
    s_rb[w][lane] = rb;
    s_v[w][lane] = v;
    wave_sync();
    for (int32_t k = 0; k < total; k += kTdU * kWave) {
        int32_t u[kTdU], pv[kTdU];
#pragma unroll
        for (int r = 0; r < kTdU; ++r) {
            const int32_t e = k + r * kWave + lane;
            u[r] = -1;
            pv[r] = -1;
            if (e < total) {
                int lo = 0, hi = kWave;  // last lane with start <= e
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_start[w][mid] <= e) lo = mid;
                    else hi = mid;
                }
                u[r] = a.csr_idx[s_rb[w][lo] + (e - s_start[w][lo])];
                pv[r] = s_v[w][lo];
            }
        }
        td_batch(a, cx, pg, u, pv, cnt, deg, lane);
    }
    wave_sync();
}

// by_bitmap: the frontier is large, so it is read from its bitmap word by
// word (ascending ids: coalesced offsets, rows in memory order).  Otherwise
// it is read from the queue in units of 64 slots (a quarter page), one unit
// per wavefront at a time; a wavefront loads the page fills and entries of up
// to four of its units in one round trip (entries past a fill are stale but
// inside the queue).  A queue-driven level never reads the frontier bitmap,
// so its vertices clear their words there: the bitmap is clean when it is
// reused two levels on, without a full clear.
// Queue pages [first, pages) hold the frontier.
__device__ __forceinline__ void level_top_down(const BfsArgs& a, const TdCtx& cx, WaveLds& sl, const int32_t* q_cur,
                                               const int32_t* fill_cur, int32_t first, int32_t pages,
                                               uint64_t* fb_cur, bool by_bitmap, int32_t& cnt, int64_t& deg,
                                               Pager& pg) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * kBfsWaves + threadIdx.x / kWave;
    const int32_t nwaves = gridDim.x * kBfsWaves;
    if (by_bitmap) {
        for (int32_t unit = gwave; unit < a.act_words; unit += nwaves) {
            const uint64_t word = fb_cur[unit];
            if (word == 0) continue;
            td_unit(a, cx, sl, pg, ((word >> lane) & 1ull) ? unit * kWave + lane : -1, cnt, deg);
        }
        return;
    }
    constexpr int kUnitsPerPage = kPage / kWave;
    constexpr int kAhead = 4;
    const int32_t nunits = pages * kUnitsPerPage;
    for (int32_t u0 = first * kUnitsPerPage + gwave; u0 < nunits; u0 += kAhead * nwaves) {
        int32_t left[kAhead], qv[kAhead];  // entries of each unit (<= 0: none), lane's entry
#pragma unroll
        for (int j = 0; j < kAhead; ++j) {
            const int32_t unit = u0 + j * nwaves;
            left[j] = 0;
            qv[j] = -1;
            if (unit < nunits) {
                const int32_t p = unit / kUnitsPerPage, s = (unit % kUnitsPerPage) * kWave;
                left[j] = min(fill_cur[p], kPage) - s;
                qv[j] = q_cur[(size_t)p * kPage + s + lane];
            }
        }
#pragma unroll 1
        for (int j = 0; j < kAhead; ++j) {
            const int32_t n_here = left[0], q_here = qv[0];
#pragma unroll
            for (int t = 0; t + 1 < kAhead; ++t) {  // shift, so every index stays constant
                left[t] = left[t + 1];
                qv[t] = qv[t + 1];
            }
            if (n_here <= 0) continue;
            const int32_t v = (lane < n_here) ? q_here : -1;
            if (v >= 0) fb_cur[v >> 6] = 0ull;
            td_unit(a, cx, sl, pg, v, cnt, deg);
        }
    }
}

// ------------------------------------------------------------------ bottom-up
constexpr int kBuB = 4;  // in-edges one lane loads per step of a short row
constexpr int kBuU = 4;  // rounds of 64 in-edges a wave loads per step of a long row
constexpr int32_t kCoopRow = 128;  // in-rows at least this long are scanned by the whole wave

// Position of the first frontier member among csc_idx[b, e) (-1 if none),
// stopping at the first step that has one.  Wave-collective (b, e uniform).
__device__ __forceinline__ void bu_scan_row(const BfsArgs& a, const FbView& fv, int32_t b, int32_t e, int lane,
                                            int32_t& pos) {
    pos = -1;
    for (int32_t jb = b; jb < e; jb += kBuU * kWave) {
        int32_t u[kBuU];
#pragma unroll
        for (int r = 0; r < kBuU; ++r) {
            const int32_t j = jb + r * kWave + lane;
            u[r] = (j < e) ? a.csc_idx[j] : -1;
        }
        bool hit[kBuU];
#pragma unroll
        for (int r = 0; r < kBuU; ++r) hit[r] = (u[r] >= 0) && fb_test(fv, u[r]);
#pragma unroll
        for (int r = 0; r < kBuU; ++r) {
            const uint64_t hm = __ballot(hit[r]);
            if (hm) {
                pos = jb + r * kWave + __ffsll((long long)hm) - 1;
                return;
            }
        }
    }
}

__device__ __forceinline__ void level_bottom_up(const BfsArgs& a, int32_t lvl, const FbView& fv, int32_t* q_next, int32_t* fill_next,
                                uint64_t* fb_next, BfsSlot* nxt, int32_t& cnt, int64_t& deg, Pager& pg) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * kBfsWaves + threadIdx.x / kWave;
    const int32_t nwaves = gridDim.x * kBfsWaves;
    for (int32_t w = gwave; w < a.act_words; w += nwaves) {
        const uint64_t vis = a.visited[w];
        const int32_t v = w * kWave + lane;
        const bool unvisited = (v < a.n) && !((vis >> lane) & 1ull);
        if (__ballot(unvisited) == 0) continue;
        const int32_t rb = unvisited ? a.csc_off[v] : 0;
        int32_t re = unvisited ? a.csc_off[v + 1] : 0;
        bool found = false;
        int32_t par = -1;
        // in-rows of kCoopRow or more: the wave scans 64 x kBuU in-neighbours
        // at a time and stops at the first hit (one row after another, so the
        // threshold is high: shorter rows go per lane, all in parallel); of an
        // in-row longer than kBigInRow only the first kBigInRow entries are
        // scanned here (most hits come early) and, without a hit there, the
        // rest becomes chunk items for the grid
        const bool huge = (re - rb) > kBigInRow;
        const int32_t rest_b = rb + kBigInRow, rest_e = re;
        if (huge) re = rest_b;
        const bool coop = (re - rb) >= kCoopRow;
        uint64_t big = __ballot(coop);
        while (big) {
            const int src = __ffsll((long long)big) - 1;
            big &= big - 1;
            const int32_t bb = __shfl(rb, src), be = __shfl(re, src);
            int32_t p = -1;
            bu_scan_row(a, fv, bb, be, lane, p);
            if (lane == src && p >= 0) {
                found = true;
                par = a.csc_idx[p];
            }
        }
        const bool rest = huge && !found;
        if (__ballot(rest)) queue_chunks(a, rest, v, rest_b, rest_e, kBigInRow, nxt, lane);
        // short in-rows: each lane scans its own, in stored order, kBuB
        // independent loads at a time
        if (unvisited && !coop) {
            for (int32_t j = rb; j < re && !found; j += kBuB) {
                int32_t u[kBuB];
#pragma unroll
                for (int r = 0; r < kBuB; ++r) u[r] = (j + r < re) ? a.csc_idx[j + r] : -1;
                bool hit[kBuB];
#pragma unroll
                for (int r = 0; r < kBuB; ++r) hit[r] = (u[r] >= 0) && fb_test(fv, u[r]);
#pragma unroll
                for (int r = 0; r < kBuB; ++r)
                    if (hit[r] && !found) {
                        found = true;
                        par = u[r];
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

// Bottom-up level over the whole in-edge array, for a sparse frontier while
// most edges still belong to unvisited vertices.  Row by row, a wavefront
// walks its bitmap words one after another, and the hub words (64 rows of
// hundreds of edges each) serialise whole levels; streamed, every slot is
// read once in memory order with kStreamQ 16-byte loads (four slots each)
// in flight per lane: 8 KB per wavefront, which a CU needs to keep the
// stream near full bandwidth.  The slots whose source is in the frontier are
// collected per wavefront in LDS and resolved 64 at a time, one lane each:
// the vertex comes from csc_row and is claimed with an atomic OR, so its
// parent is some frontier in-neighbour (not necessarily the first in stored
// order).  An in-edge array that is not 16-byte aligned, and the slots past
// the last whole quad, take 4-byte loads.
constexpr int kStreamQ = 8;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // a native vector: non-temporal loads take it

// SINGLE: the frontier is one vertex, `single` (the root at level 0), so a
// test is one compare (no bitmap, staged or not).
template <bool SINGLE>
__device__ __forceinline__ void level_bottom_up_stream(const BfsArgs& a, int32_t lvl, const FbView& fv, int32_t single,
                                                       WaveLds& sl, int32_t* q_next, int32_t* fill_next,
                                                       uint64_t* fb_next, BfsSlot* nxt, int32_t& cnt, int64_t& deg,
                                                       Pager& pg) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int64_t gwave = blockIdx.x * kBfsWaves + w;
    const int64_t nwaves = (int64_t)gridDim.x * kBfsWaves;
    constexpr int kStreamU = 8;  // 4-byte loads per lane of the slot-by-slot loop
    constexpr int64_t kStep = kStreamU * kWave;
    int32_t nh = 0;  // hits held in sl.a / sl.b (wave-uniform)
    auto resolve = [&]() {
        wave_sync();
        bool claimed = false;
        int32_t v = -1;
        if (lane < nh) {
            const int32_t u = sl.b[w][lane];
            v = a.csc_row[sl.a[w][lane]];
            const uint64_t bit = 1ull << (v & 63);
            const uint64_t old =
                atomicOr(reinterpret_cast<unsigned long long*>(&a.visited[v >> 6]), (unsigned long long)bit);
            if (!(old & bit)) {
                claimed = true;
                const int32_t vu = user_id(a.perm, v);
                a.level[vu] = lvl + 1;
                a.parent[vu] = user_id(a.perm, u);
                atomicOr(reinterpret_cast<unsigned long long*>(&fb_next[v >> 6]), (unsigned long long)bit);
                cnt += 1;
                deg += a.out_deg[v];
            }
        }
        const uint64_t m = __ballot(claimed);
        if (m)
            page_append(a, pg, claimed, v, __popcll(m & lanes_below(lane)), __popcll(m), q_next, fill_next, nxt, lane);
        wave_sync();
        nh = 0;
    };
    // collects the hit slots of one round (slot index, source), resolving
    // the wavefront's list whenever the next hits would overflow it
    auto collect = [&](bool h, int64_t e, int32_t src) {
        const uint64_t m = __ballot(h);
        if (!m) return;
        const int32_t k = __popcll(m);
        if (nh + k > kWave) resolve();
        if (h) {
            const int32_t at = nh + __popcll(m & lanes_below(lane));
            sl.a[w][at] = (int32_t)e;
            sl.b[w][at] = src;
        }
        nh += k;
    };
    const bool quads = (reinterpret_cast<uintptr_t>(a.csc_idx) & 15) == 0;
    const int64_t nq = quads ? a.nnz / 4 : 0;  // whole quads streamed 16 bytes at a time
    constexpr int64_t kQStep = kStreamQ * kWave;
    const u32x4* q4 = reinterpret_cast<const u32x4*>(a.csc_idx);
    for (int64_t q0 = gwave * kQStep; q0 < nq; q0 += nwaves * kQStep) {
        u32x4 v[kStreamQ];
#pragma unroll
        for (int r = 0; r < kStreamQ; ++r) {
            const int64_t q = q0 + r * kWave + lane;
            v[r] = (q < nq) ? __builtin_nontemporal_load(q4 + q) : u32x4{~0u, ~0u, ~0u, ~0u};
        }
        bool hit[kStreamQ][4];
        bool any = false;
#pragma unroll
        for (int r = 0; r < kStreamQ; ++r) {
            const int32_t s4[4] = {(int32_t)v[r].x, (int32_t)v[r].y, (int32_t)v[r].z, (int32_t)v[r].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                hit[r][j] = (s4[j] >= 0) && (SINGLE ? s4[j] == single : fb_test(fv, s4[j]));
                any = any || hit[r][j];
            }
        }
        if (__ballot(any) == 0) continue;
#pragma unroll
        for (int r = 0; r < kStreamQ; ++r) {
            const int32_t s4[4] = {(int32_t)v[r].x, (int32_t)v[r].y, (int32_t)v[r].z, (int32_t)v[r].w};
            const int64_t e = 4 * (q0 + r * kWave + lane);
#pragma unroll
            for (int j = 0; j < 4; ++j) collect(hit[r][j], e + j, s4[j]);
        }
    }
    // the rest (everything when the array is not 16-byte aligned), slot by slot
    for (int64_t e0 = 4 * nq + gwave * kStep; e0 < a.nnz; e0 += nwaves * kStep) {
        int32_t u[kStreamU];
#pragma unroll
        for (int r = 0; r < kStreamU; ++r) {
            const int64_t e = e0 + r * kWave + lane;
            u[r] = (e < a.nnz) ? __builtin_nontemporal_load(a.csc_idx + e) : -1;
        }
        bool hit[kStreamU];
        bool any = false;
#pragma unroll
        for (int r = 0; r < kStreamU; ++r) {
            hit[r] = (u[r] >= 0) && (SINGLE ? u[r] == single : fb_test(fv, u[r]));
            any = any || hit[r];
        }
        if (__ballot(any) == 0) continue;
#pragma unroll
        for (int r = 0; r < kStreamU; ++r) collect(hit[r], e0 + r * kWave + lane, u[r]);
    }
    if (nh) resolve();
}

// Expands frontier `lvl` (slot lvl % 3) into lvl+1.  policy: PP_PUSH,
// PP_PULL or PP_SWITCH (decided here, identically in every workgroup, from
// the slot statistics).
// lvl_arg >= 0 names the level; -1 takes it from the header (lv[parity]).
__global__ __launch_bounds__(kBfsBlock) void k_bfs_level(BfsArgs a, int32_t lvl_arg, int32_t parity, int32_t policy,
                                                          float alpha, float beta) {
    extern __shared__ __align__(16) uint64_t s_bits[];  // staged with 16-byte stores
    __shared__ WaveLds s_wave;
    BfsHdr* h = a.hdr;
    // the three slots are read in the same round trip as the level index
    const SlotView v0 = view(h->slot[0]), v1 = view(h->slot[1]), v2 = view(h->slot[2]);
    const int32_t lvl = lvl_arg >= 0 ? lvl_arg : h->lv[parity];
    const int sc = lvl % 3, sn = (lvl + 1) % 3, sz = (lvl + 2) % 3;
    const SlotView cur = (sc == 0) ? v0 : ((sc == 1) ? v1 : v2);
    const int32_t nf = cur.n;
    const bool lead = (blockIdx.x == 0 && threadIdx.x == 0);
    if (nf == 0) {
        if (lead) {
            h->lv[parity ^ 1] = lvl;  // stays at the empty level
            h->c_lvl = -1;
            h->finished = 1;
        }
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
        BfsSlot fresh{};
        fresh.pages = a.static_pages;  // counting starts after the reserved pages
        h->slot[sz] = fresh;
        h->slot[sn].dir_prev = dir;
        h->slot[sn].n_prev = nf;
        h->slot[sn].mu_base = mu;
        if (lvl < PP_BFS_MAX_LOG) {
            h->log_dir[lvl] = (int8_t)dir;
            h->log_n[lvl] = nf;
        }
        if (lvl < a.log_cap) a.log[lvl] = pp_bfs_level{dir, nf, cur.m};
        h->levels = lvl + 1;
        h->last = lvl + 1;
        h->reached += nf;
        h->edges += cur.m;
        h->lv[parity ^ 1] = lvl + 1;
        h->c_lvl = lvl;
        h->busy += 1;
    }
    // the bitmap two levels ahead (frontier lvl - 1) is rewritten next level:
    // clear it now, unless level lvl - 1 was a queue-driven top-down level,
    // which cleared its words itself
    if (!(cur.dir_prev == PP_PUSH && cur.n_prev <= a.words)) {
        uint64_t* fb_clear = a.fb[sz];
        for (int32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < a.words; w += gridDim.x * blockDim.x)
            fb_clear[w] = 0ull;
    }
    const int lane = threadIdx.x & (kWave - 1);
    int32_t cnt = 0;
    int64_t deg = 0;
    // bottom-up: each wavefront starts on its reserved page
    Pager pg{(dir == PP_PULL) ? (int32_t)(blockIdx.x * kBfsWaves + threadIdx.x / kWave) : -1, 0};
    int32_t* q_next = a.queue[(lvl + 1) & 1];
    int32_t* fill_next = a.fill[(lvl + 1) & 1];
    // edges the level examines at most: the frontier's (top-down) or the
    // unvisited vertices' (bottom-up)
    const int32_t sw = ((dir == PP_PUSH ? cur.m : mu) >= a.stage_min) ? a.stage_words : 0;
    if (dir == PP_PUSH) {
        if (sw) stage_bits(s_bits, a.visited, sw);
        TdCtx cx{lvl, q_next, fill_next, a.fb[sn], &h->slot[sn], s_bits, sw, cur.m >= kProbeMin,
                 (cur.m < (a.nnz >> kSmallLevelShift)) ? a.td_small_row : kBigRow};
        // a frontier built top-down left the reserved pages unused
        level_top_down(a, cx, s_wave, a.queue[lvl & 1], a.fill[lvl & 1], (cur.dir_prev == PP_PULL) ? 0 : a.static_pages,
                       min(cur.pages, a.page_cap), a.fb[sc], nf > a.words, cnt, deg, pg);
    } else {
        // a sparse frontier while most in-edges still belong to unvisited
        // vertices: stream the in-edge array instead of scanning row by row
        // (its hits, the frontier's out-edges, must stay few)
        const bool stream = (int64_t)nf * 8 < a.words && 2 * mu >= a.nnz && 256 * cur.m <= a.nnz;
        // level 0: the frontier is the root alone, nothing to stage
        const int32_t single = (lvl == 0 && stream) ? h->root : -1;
        const int32_t sws = (single < 0) ? sw : 0;
        // the summary pays on large levels only (each workgroup builds it)
        const bool sum = sws && use_summary(a, nf);
        uint64_t* s_sum = s_bits + a.stage_words;
        if (sum) build_summary(s_sum, a.fb[sc], a.words, sws, a.sum_words);
        if (sws) stage_bits(s_bits, a.fb[sc], sws);
        const FbView fv{s_bits, sws, s_sum, sum ? min(a.words, a.sum_words * kWave) : 0, a.fb[sc]};
        if (single >= 0)
            level_bottom_up_stream<true>(a, lvl, fv, single, s_wave, q_next, fill_next, a.fb[sn], &h->slot[sn], cnt,
                                         deg, pg);
        else if (stream)
            level_bottom_up_stream<false>(a, lvl, fv, -1, s_wave, q_next, fill_next, a.fb[sn], &h->slot[sn], cnt,
                                          deg, pg);
        else
            level_bottom_up(a, lvl, fv, q_next, fill_next, a.fb[sn], &h->slot[sn], cnt, deg, pg);
    }
    page_close(pg, fill_next, lane);
    flush_stats(cnt, deg, &h->slot[sn]);
}

// Second pass of a level: the chunk items of the long rows, one wavefront
// per item.  Top-down chunks claim targets as the level kernel does.
// Bottom-up chunks of one in-row run independently: each scans its slice in
// stored order and the first chunk to find a frontier member claims the
// vertex with an atomic OR on its visited bit (so the parent is a frontier
// in-neighbour, not necessarily the first in stored order); a chunk whose
// vertex is already claimed is skipped.
// Two workgroups per compute unit: 32 wavefronts, 8 per SIMD, which caps the
// kernel at 64 VGPRs (the second bound is the minimum wavefronts per SIMD).
__global__ __launch_bounds__(kBfsBlock, 8) void k_bfs_chunks(BfsArgs a) {
    extern __shared__ __align__(16) uint64_t s_bits[];  // staged with 16-byte stores
    BfsHdr* h = a.hdr;
    // slot fields read in the same round trip as the level index
    int32_t bigs[3], dirs[3], ns[3];
    int64_t ms[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        bigs[i] = h->slot[i].big;
        dirs[i] = h->slot[i].dir_prev;
        ns[i] = h->slot[i].n;
        ms[i] = h->slot[i].m;
    }
    const int32_t lvl = h->c_lvl;
    if (lvl < 0) return;
    const int sc = lvl % 3, sn = (lvl + 1) % 3;
    const int32_t items = min((sn == 0) ? bigs[0] : ((sn == 1) ? bigs[1] : bigs[2]), a.item_cap);
    if (items == 0) return;
    const int32_t dir = (sn == 0) ? dirs[0] : ((sn == 1) ? dirs[1] : dirs[2]);
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t gwave = blockIdx.x * kBfsWaves + threadIdx.x / kWave;
    const int32_t nwaves = gridDim.x * kBfsWaves;
    int32_t cnt = 0;
    int64_t deg = 0;
    Pager pg{-1, 0};
    int32_t* q_next = a.queue[(lvl + 1) & 1];
    int32_t* fill_next = a.fill[(lvl + 1) & 1];
    if (dir == PP_PUSH) {
        // top-down items test the hottest visited words in LDS when the items
        // bring at least two edges per staged word (items of the chunk length
        // the level kernel used: the same rule on the frontier's out-edges)
        const int64_t m = (sc == 0) ? ms[0] : ((sc == 1) ? ms[1] : ms[2]);
        const int32_t clen = (m < (a.nnz >> kSmallLevelShift)) ? a.td_small_row : kBigRow;
        const int32_t sw = ((int64_t)items * clen >= 2 * (int64_t)gridDim.x * a.chunk_stage) ? a.chunk_stage : 0;
        if (sw) stage_bits(s_bits, a.visited, sw);
        TdCtx cx{lvl, q_next, fill_next, a.fb[sn], &h->slot[sn], s_bits, sw, true, kBigRow};
        for (int32_t it = gwave; it < items; it += nwaves)
            td_row(a, cx, pg, a.items[3 * it], a.items[3 * it + 1], a.items[3 * it + 2], cnt, deg, lane);
    } else {
        // Hits are collected per wavefront (vertex, slot) and claimed 64 at a
        // time, one lane each, so a claim's round trip is shared.
        __shared__ int32_t s_hv[kBfsWaves][kWave];
        __shared__ int32_t s_hp[kBfsWaves][kWave];
        const int w = threadIdx.x / kWave;
        int32_t nh = 0;  // wave-uniform
        auto claim_hits = [&]() {
            wave_sync();
            bool claimed = false;
            int32_t v = -1;
            if (lane < nh) {
                v = s_hv[w][lane];
                const uint64_t bit = 1ull << (v & 63);
                const uint64_t old =
                    atomicOr(reinterpret_cast<unsigned long long*>(&a.visited[v >> 6]), (unsigned long long)bit);
                if (!(old & bit)) {
                    claimed = true;
                    const int32_t vu = user_id(a.perm, v);
                    a.level[vu] = lvl + 1;
                    a.parent[vu] = user_id(a.perm, a.csc_idx[s_hp[w][lane]]);
                    atomicOr(reinterpret_cast<unsigned long long*>(&a.fb[sn][v >> 6]), (unsigned long long)bit);
                    cnt += 1;
                    deg += a.out_deg[v];
                }
            }
            const uint64_t m = __ballot(claimed);
            if (m)
                page_append(a, pg, claimed, v, __popcll(m & lanes_below(lane)), __popcll(m), q_next, fill_next,
                            &h->slot[sn], lane);
            wave_sync();
            nh = 0;
        };
        const uint64_t* fb_cur = a.fb[sc];
        // the summary (built by every workgroup) pays when the items bring at
        // least two edges per summarised word
        const bool sum = use_summary(a, (sc == 0) ? ns[0] : ((sc == 1) ? ns[1] : ns[2])) &&
                         (int64_t)items * kBigInRow >= 2 * (int64_t)gridDim.x * a.sum_words * kWave;
        if (sum) {
            build_summary(s_bits, fb_cur, a.words, 0, a.sum_words);
            __syncthreads();
        }
        const FbView fv{s_bits, 0, s_bits, sum ? min(a.words, a.sum_words * kWave) : 0, fb_cur};
        for (int32_t it = gwave; it < items; it += nwaves) {
            const int32_t v = a.items[3 * it], b = a.items[3 * it + 1], e = a.items[3 * it + 2];
            int32_t pos = -1;
            if (!((a.visited[v >> 6] >> (v & 63)) & 1ull)) bu_scan_row(a, fv, b, e, lane, pos);
            if (pos >= 0) {
                if (lane == 0) {
                    s_hv[w][nh] = v;
                    s_hp[w][nh] = pos;
                }
                if (++nh == kWave) claim_hits();
            }
        }
        if (nh) claim_hits();
    }
    page_close(pg, fill_next, lane);
    flush_stats(cnt, deg, &h->slot[sn]);
}

// ------------------------------------------------------------ deep graphs
// Top-down levels with small frontiers, many per launch, on ONE workgroup.
// A deep graph (a grid: thousands of levels of a few thousand vertices)
// spends its time on per-level launch latency, not on bytes.  This kernel
// keeps the frontier in LDS as (vertex, row begin, degree -> prefix) sets,
// claims targets with workgroup-scope atomics on the visited bitmap (only
// this workgroup runs, so they resolve in the local L2), and loads the row
// bounds of a vertex when it is claimed, so a level costs two dependent
// memory round trips (target ids, claims; the row bounds ride with the
// claims) and a few workgroup barriers.  It runs levels while the frontier
// has at most qcap vertices and ecap out-edges and the switch rule keeps
// top-down, then hands the state back exactly as a queue-driven top-down
// level kernel would have left it (queue pages, frontier bitmap, slots,
// level index, statistics), so the grid-wide kernels continue from there.
// It takes over only a compact top-down frontier (few queue pages, bitmap
// words of the previous frontier already clear) and otherwise returns at
// once without touching anything.
constexpr int32_t kMultiLevels = 32768;   // levels per launch (bounds its duration)
constexpr int32_t kMultiPages = 64;       // queue pages a taken-over frontier may span
constexpr int kMultiB = 8;                // edges a lane handles per round

struct MultiSet {
    int32_t* v;  // vertex
    int32_t* b;  // CSR row begin
    int32_t* p;  // degree, then exclusive prefix of the degrees ([nf] = total)
};

__device__ __forceinline__ MultiSet multi_set(int32_t* base, int32_t qcap, int which) {
    int32_t* s = base + (size_t)which * (3 * qcap + 1);
    return MultiSet{s, s + qcap, s + 2 * qcap};
}

// Would a level kernel expand frontier `lvl` (nf vertices, m out-edges,
// mu_base, built by dir_prev from n_prev vertices) top-down?
__device__ __forceinline__ bool multi_push(int32_t policy, float alpha, float beta, int32_t n, int32_t lvl,
                                           int32_t nf, int64_t m, int64_t mu_base, int32_t dir_prev, int32_t n_prev) {
    if (policy == PP_PUSH) return true;
    if (policy != PP_SWITCH) return false;
    const int64_t mu = mu_base - m;
    if (lvl == 0 || dir_prev == PP_PUSH) return !((double)m > (double)mu / (double)alpha);
    return (double)nf < (double)n / (double)beta && nf < n_prev;
}

// Exclusive prefix of p[0, cnt) in place (p[cnt] = total).  Workgroup-collective.
__device__ __forceinline__ void multi_scan(int32_t* p, int32_t cnt, int32_t* s_w) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int32_t per = (cnt + (int32_t)blockDim.x - 1) / (int32_t)blockDim.x;
    const int32_t i0 = min((int32_t)threadIdx.x * per, cnt), i1 = min(i0 + per, cnt);
    int32_t s = 0;
    for (int32_t i = i0; i < i1; ++i) s += p[i];
    int32_t incl = s;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == kWave - 1) s_w[w] = incl;
    __syncthreads();
    int32_t base = 0;
    for (int i = 0; i < w; ++i) base += s_w[i];
    int32_t at = base + incl - s;
    for (int32_t i = i0; i < i1; ++i) {
        const int32_t d = p[i];
        p[i] = at;
        at += d;
    }
    if (threadIdx.x == blockDim.x - 1) p[cnt] = base + incl;
    __syncthreads();
}

__global__ __launch_bounds__(kBfsBlock) void k_bfs_multi(BfsArgs a, int32_t policy, float alpha, float beta,
                                                         int32_t qcap, int32_t ecap) {
    extern __shared__ int32_t s_sets[];
    __shared__ int32_t s_start[kBfsBlock];  // first frontier entry of each thread's edge range
    __shared__ int32_t s_w[kBfsWaves];
    __shared__ int64_t s_m[kBfsWaves];
    __shared__ int32_t s_cnt;
    __shared__ int32_t s_hdr[8];
    __shared__ int64_t s_hdr64[2];
    BfsHdr* h = a.hdr;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    if (threadIdx.x == 0) {
        const int32_t lvl = h->lv[0];
        const SlotView cur = view(h->slot[lvl % 3]);
        const bool ok = !h->finished && cur.n > 0 && cur.n <= qcap && cur.m <= ecap && cur.dir_prev == PP_PUSH &&
                        cur.n_prev <= a.words && cur.pages - a.static_pages <= kMultiPages &&
                        multi_push(policy, alpha, beta, a.n, lvl, cur.n, cur.m, cur.mu_base, cur.dir_prev, cur.n_prev);
        s_hdr[0] = ok;
        s_hdr[1] = lvl;
        s_hdr[2] = cur.n;
        s_hdr[3] = cur.n_prev;
        s_hdr[4] = cur.pages;
        s_hdr64[0] = cur.m;
        s_hdr64[1] = cur.mu_base;
        s_cnt = 0;
    }
    __syncthreads();
    if (!s_hdr[0]) return;
    int32_t lvl = s_hdr[1], nf = s_hdr[2], n_prev = s_hdr[3];
    int64_t m = s_hdr64[0], mu_base = s_hdr64[1];
    // take over frontier lvl: its queue pages into set 0, its bitmap words
    // cleared (as a queue-driven level clears them), row bounds loaded
    int cur = 0;
    {
        const MultiSet A = multi_set(s_sets, qcap, 0);
        const int32_t* q = a.queue[lvl & 1];
        const int32_t* fill = a.fill[lvl & 1];
        const int32_t pages = min(s_hdr[4], a.page_cap);
        for (int32_t p = a.static_pages + w; p < pages; p += kBfsWaves) {
            const int32_t f = min(fill[p], kPage);
            int32_t base = 0;
            if (lane == 0 && f > 0) base = atomicAdd(&s_cnt, f);
            base = __shfl(base, 0);
            for (int32_t s = lane; s < f; s += kWave)
                if (base + s < qcap) A.v[base + s] = q[(size_t)p * kPage + s];
        }
        __syncthreads();
        // a frontier that does not match its slot (never expected) is left to
        // the level kernels, untouched
        if (s_cnt != nf) return;
        for (int32_t i = threadIdx.x; i < nf; i += blockDim.x) {
            const int32_t v = A.v[i];
            const int32_t rb = a.csr_off[v], re = a.csr_off[v + 1];
            A.b[i] = rb;
            A.p[i] = re - rb;
            a.fb[lvl % 3][v >> 6] = 0ull;
        }
        __syncthreads();
        multi_scan(A.p, nf, s_w);
    }
    int64_t reached = 0, edges = 0;
    for (int32_t run = 0;; ++run) {
        const MultiSet A = multi_set(s_sets, qcap, cur), B = multi_set(s_sets, qcap, cur ^ 1);
        // stop before a level that is empty, too large for the sets, past the
        // launch's budget, or one the switch rule would expand bottom-up
        if (nf == 0 || nf > qcap || m > ecap || run >= kMultiLevels ||
            !multi_push(policy, alpha, beta, a.n, lvl, nf, m, mu_base, PP_PUSH, n_prev))
            break;
        if (threadIdx.x == 0) {
            if (lvl < PP_BFS_MAX_LOG) {
                h->log_dir[lvl] = (int8_t)PP_PUSH;
                h->log_n[lvl] = nf;
            }
            if (lvl < a.log_cap) a.log[lvl] = pp_bfs_level{PP_PUSH, nf, m};
            s_cnt = 0;
        }
        reached += nf;
        edges += m;
        // thread t walks edges [t*c, t*c + c) of the frontier's out-edges;
        // s_start[t] is the entry holding edge t*c
        const int32_t mi = (int32_t)m;
        const int32_t c = max((mi + (int32_t)blockDim.x - 1) / (int32_t)blockDim.x, 1);
        for (int32_t i = threadIdx.x; i < nf; i += blockDim.x) {
            const int32_t lo = A.p[i], hi = A.p[i + 1];
            for (int32_t t = (lo + c - 1) / c; t * c < hi; ++t) s_start[t] = i;
        }
        __syncthreads();
        const int32_t k0 = (int32_t)threadIdx.x * c, k1 = min(k0 + c, mi);
        int32_t e = (k0 < mi) ? s_start[threadIdx.x] : 0;
        uint64_t* fb_next = a.fb[(lvl + 1) % 3];
        int32_t* q_next = a.queue[(lvl + 1) & 1];
        int64_t mloc = 0;
        for (int32_t kb = k0; kb - k0 < c; kb += kMultiB) {  // c is uniform: every lane takes every round
            int32_t u[kMultiB], pv[kMultiB];
#pragma unroll
            for (int r = 0; r < kMultiB; ++r) {
                const int32_t k = kb + r;
                u[r] = -1;
                pv[r] = -1;
                if (k < k1) {
                    while (A.p[e + 1] <= k) ++e;
                    pv[r] = A.v[e];
                    u[r] = a.csr_idx[A.b[e] + (k - A.p[e])];
                }
            }
            bool claimed[kMultiB];
#pragma unroll
            for (int r = 0; r < kMultiB; ++r) {
                claimed[r] = false;
                if (u[r] >= 0) {
                    const uint64_t bit = 1ull << (u[r] & 63);
                    const uint64_t old = __hip_atomic_fetch_or(reinterpret_cast<unsigned long long*>(&a.visited[u[r] >> 6]),
                                                               (unsigned long long)bit, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                    claimed[r] = !(old & bit);
                }
            }
            // one LDS counter atomic per wavefront and round
            int32_t rank[kMultiB], tot = 0;
#pragma unroll
            for (int r = 0; r < kMultiB; ++r) {
                const uint64_t bal = __ballot(claimed[r]);
                rank[r] = tot + __popcll(bal & lanes_below(lane));
                tot += __popcll(bal);
            }
            int32_t base = 0;
            if (lane == 0 && tot) base = atomicAdd(&s_cnt, tot);
            base = __shfl(base, 0);
#pragma unroll
            for (int r = 0; r < kMultiB; ++r) {
                if (!claimed[r]) continue;
                const int32_t x = u[r];
                const int32_t rb = a.csr_off[x], re = a.csr_off[x + 1];
                const int32_t uid = user_id(a.perm, x), pid = user_id(a.perm, pv[r]);
                a.level[uid] = lvl + 1;
                a.parent[uid] = pid;
                mloc += re - rb;
                const int32_t slot = base + rank[r];
                if (slot < qcap) {
                    B.v[slot] = x;
                    B.b[slot] = rb;
                    B.p[slot] = re - rb;
                } else {  // the next frontier outgrows the sets: it goes to the level kernels
                    q_next[(size_t)a.static_pages * kPage + slot] = x;
                    atomicOr(reinterpret_cast<unsigned long long*>(&fb_next[x >> 6]),
                             (unsigned long long)(1ull << (x & 63)));
                }
            }
        }
        mloc = wave_sum(mloc);
        if (lane == 0) s_m[w] = mloc;
        __syncthreads();
        int64_t mn = 0;
        for (int i = 0; i < kBfsWaves; ++i) mn += s_m[i];
        const int32_t nn = s_cnt;
        mu_base -= m;
        n_prev = nf;
        nf = nn;
        m = mn;
        ++lvl;
        cur ^= 1;
        if (nf <= qcap && m <= ecap) multi_scan(B.p, nf, s_w);
        else __syncthreads();  // everyone has read s_cnt and s_m
    }
    // hand frontier lvl back: queue pages, fills and bitmap bits, as a
    // queue-driven top-down level leaves them
    const MultiSet A = multi_set(s_sets, qcap, cur);
    int32_t* q = a.queue[lvl & 1];
    int32_t* fill = a.fill[lvl & 1];
    const int32_t inl = min(nf, qcap);
    for (int32_t i = threadIdx.x; i < inl; i += blockDim.x) {
        const int32_t v = A.v[i];
        q[(size_t)a.static_pages * kPage + i] = v;
        atomicOr(reinterpret_cast<unsigned long long*>(&a.fb[lvl % 3][v >> 6]), (unsigned long long)(1ull << (v & 63)));
    }
    const int32_t np = (nf + kPage - 1) / kPage;
    for (int32_t p = threadIdx.x; p < np; p += blockDim.x) fill[a.static_pages + p] = min(kPage, nf - p * kPage);
    if (threadIdx.x == 0) {
        BfsSlot fresh{};
        fresh.pages = a.static_pages;
        BfsSlot s = fresh;
        s.n = nf;
        s.dir_prev = PP_PUSH;
        s.n_prev = n_prev;
        s.pages = a.static_pages + np;
        s.m = m;
        s.mu_base = mu_base;
        h->slot[lvl % 3] = s;
        h->slot[(lvl + 1) % 3] = fresh;
        h->slot[(lvl + 2) % 3] = fresh;
        h->lv[0] = lvl;
        h->lv[1] = lvl;
        h->c_lvl = -1;
        h->levels = lvl;
        h->last = lvl;
        h->reached += reached;
        h->edges += edges;
        if (nf == 0) h->finished = 1;
    }
}

static pp_status check_state(pp_graph g, void* state, size_t bytes) {
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (!state) return set_error(PP_E_NULL, "state is NULL");
    if (bytes < bfs_layout(g).total) return set_error(PP_E_WORKSPACE, "BFS state buffer too small");
    if (reinterpret_cast<uintptr_t>(state) % 256 != 0) return set_error(PP_E_RANGE, "state must be 256-byte aligned");
    return PP_OK;
}

// Lets the staging kernels take LDS beyond the default 64 KiB.
static void allow_stage_lds(const BfsArgs& a) {
    const int bytes = (a.stage_words + a.sum_words) * 8;
    allow_dynamic_lds(reinterpret_cast<const void*>(&k_bfs_level), (size_t)bytes);
    allow_dynamic_lds(reinterpret_cast<const void*>(&k_bfs_chunks), (size_t)bytes);
}

// Dynamic LDS of the chunk kernel: the bottom-up summary or the top-down
// visited stage.
static size_t chunk_lds(const BfsArgs& a) { return (size_t)std::max(a.sum_words, a.chunk_stage) * 8; }

// Workgroups of the chunk kernel: one per compute unit.  Two per unit, each
// staging half as many visited words, ran top-down runs about 1.4% slower at
// R-MAT scale 22; half a workgroup per unit about 18% slower.
static int32_t chunk_blocks(pp_graph g) { return std::max(1, std::min(ceil_div(g->d.n, 4096), g->num_cu)); }

// Frontier sets of the one-workgroup launch: vertices per set (qcap) and
// out-edges per level (ecap) it takes on; 0 when it is off for this policy.
static void multi_caps(pp_graph g, int32_t policy, int32_t* qcap, int32_t* ecap) {
    constexpr int32_t kStatic = 8192;  // its static LDS (edge-range starts, reductions), rounded up
    const int32_t fit = std::max(0, (g->max_lds - kStatic) / 24 - 1);
    *qcap = (policy == PP_PULL) ? 0 : std::min(g->tune.bfs_multi_n, fit);
    *ecap = (*qcap > 0) ? g->tune.bfs_multi_m : 0;
    if (*ecap <= 0) *qcap = 0;
}

static size_t multi_lds(int32_t qcap) { return (size_t)(6 * qcap + 2) * 4; }

// Does a level of this policy on this graph ever queue chunk items?
static bool needs_chunks(pp_graph g, int32_t policy) {
    return (policy != PP_PULL && g->max_out_deg > kBigRow) || (policy != PP_PUSH && g->max_in_deg > kBigInRow);
}

// One level: the expansion kernel, then (when long rows can occur) the chunk
// kernel.  lvl >= 0 names the level; lvl = -1 takes it from the header, the
// level kernel reading lv[parity].
static pp_status launch_level(pp_graph g, const BfsArgs& a, int32_t lvl, int32_t parity, int32_t policy, float alpha,
                              float beta, hipStream_t st) {
    const int32_t blocks = bfs_blocks(g);
    const size_t lds = (size_t)(a.stage_words + a.sum_words) * 8;
    hipLaunchKernelGGL(k_bfs_level, dim3(blocks), dim3(kBfsBlock), lds, st, a, lvl, parity, policy, alpha, beta);
    if (needs_chunks(g, policy))
        hipLaunchKernelGGL(k_bfs_chunks, dim3(chunk_blocks(g)), dim3(kBfsBlock), chunk_lds(a), st, a);
    PP_LAUNCH_CHECK("k_bfs_level");
    return PP_OK;
}

// An instantiated HIP graph of `batch` levels (batch even; level kernels of
// parity 0, 1, 0, ...), built once per argument set and kept in the handle.
// Replaying it costs one launch instead of one or two per level.
static pp_status bfs_graph(pp_graph g, BfsArgs a, int32_t policy, float alpha, float beta, int32_t batch,
                           const void* state, hipGraphExec_t* out) {
    for (auto& e : g->bfs_graphs)
        if (e.state == state && e.level == a.level && e.parent == a.parent && e.policy == policy &&
            e.alpha == alpha && e.beta == beta && e.batch == batch && e.log == a.log && e.log_cap == a.log_cap) {
            *out = e.exec;
            return PP_OK;
        }
    constexpr size_t kMaxCached = 24;
    if (g->bfs_graphs.size() >= kMaxCached) {
        (void)hipGraphExecDestroy(g->bfs_graphs.front().exec);
        (void)hipGraphDestroy(g->bfs_graphs.front().graph);
        g->bfs_graphs.erase(g->bfs_graphs.begin());
    }
    const int32_t blocks = bfs_blocks(g);
    const unsigned lds = (unsigned)(a.stage_words + a.sum_words) * 8;
    const bool chunks = needs_chunks(g, policy);
    hipGraph_t graph = nullptr;
    PP_HIP(hipGraphCreate(&graph, 0));
    hipGraphNode_t prev = nullptr;
    auto add = [&](const void* fn, void** args, int32_t grid, unsigned shared) -> hipError_t {
        hipKernelNodeParams p{};
        p.func = const_cast<void*>(fn);
        p.gridDim = dim3(grid);
        p.blockDim = dim3(kBfsBlock);
        p.sharedMemBytes = shared;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node = nullptr;
        const hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p);
        if (e == hipSuccess) prev = node;
        return e;
    };
    hipError_t e = hipSuccess;
    // small top-down frontiers first go through the one-workgroup launch,
    // which returns at once when the frontier is not one it takes on
    int32_t qcap = 0, ecap = 0;
    multi_caps(g, policy, &qcap, &ecap);
    if (qcap > 0) {
        allow_dynamic_lds(reinterpret_cast<const void*>(&k_bfs_multi), multi_lds(qcap));
        void* margs[] = {&a, &policy, &alpha, &beta, &qcap, &ecap};
        e = add(reinterpret_cast<const void*>(&k_bfs_multi), margs, 1, (unsigned)multi_lds(qcap));
    }
    int32_t lvl = -1;
    for (int32_t i = 0; i < batch && e == hipSuccess; ++i) {
        int32_t parity = i & 1;
        void* largs[] = {&a, &lvl, &parity, &policy, &alpha, &beta};
        e = add(reinterpret_cast<const void*>(&k_bfs_level), largs, blocks, lds);
        if (e == hipSuccess && chunks) {
            void* cargs[] = {&a};
            e = add(reinterpret_cast<const void*>(&k_bfs_chunks), cargs, chunk_blocks(g), (unsigned)chunk_lds(a));
        }
    }
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_error(e, "BFS level graph");
    }
    g->bfs_graphs.push_back({state, a.level, a.parent, policy, alpha, beta, batch, a.log, a.log_cap, exec, graph});
    *out = exec;
    return PP_OK;
}

// Through the graph's pinned buffer: a direct copy, no staging.
static pp_status read_hdr(pp_graph g, void* state, BfsHdr* h, hipStream_t st) {
    static_assert(sizeof(BfsHdr) <= pp_graph_s::kBfsHdrHost, "pinned header buffer too small");
    const BfsLayout L = bfs_layout(g);
    PP_HIP(hipMemcpyAsync(g->bfs_hdr_host, static_cast<char*>(state) + L.hdr, sizeof(BfsHdr), hipMemcpyDeviceToHost,
                          st));
    PP_HIP(hipStreamSynchronize(st));
    std::memcpy(h, g->bfs_hdr_host, sizeof(BfsHdr));
    if (h->overflow) return set_error(PP_E_WORKSPACE, "BFS queue capacity exceeded");
    return PP_OK;
}

}  // namespace pp

using namespace pp;

PP_EXPORT size_t pp_bfs_state_bytes(pp_graph g) { return g ? bfs_layout(g).total : 0; }

PP_EXPORT pp_status pp_bfs_init(pp_graph g, int32_t root, int32_t* level, int32_t* parent, void* state,
                                size_t state_bytes, void* stream) {
    clear_error();
    pp_status s = check_state(g, state, state_bytes);
    if (s != PP_OK) return s;
    if (!level || !parent) return set_error(PP_E_NULL, "level and parent are required");
    if (root < 0 || root >= g->d.n) return set_error(PP_E_RANGE, "root out of range");
    BfsArgs a = bfs_args(g, state, level, parent);
    allow_stage_lds(a);
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
    allow_stage_lds(a);
    return launch_level(g, a, cur_level, 0, dir, 14.f, 24.f, static_cast<hipStream_t>(stream));
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
    return pp_bfs_run_log(g, root, policy, alpha, beta, level, parent, state, state_bytes, nullptr, 0, stats, stream);
}

// A run's batches of levels: the first covers the most level-kernel launches
// that found work in the recent runs with the policy on the graph (0: none
// yet); batches are even (level kernels of parity 0, 1, 0, ...).
constexpr int32_t kBfsMaxBatch = 256;  // deep graphs (grids) take long batches
static int32_t bfs_even(int32_t b) { return std::min(kBfsMaxBatch, std::max<int32_t>(2, (b + 1) & ~1)); }
static int32_t bfs_predicted(pp_graph g, int32_t policy) {
    int32_t p = 0;
    for (int i = 0; i < pp_graph_s::kBfsHist; ++i) p = std::max(p, g->bfs_hist[policy][i]);
    return p;
}
static void bfs_record(pp_graph g, int32_t policy, int32_t busy) {
    g->bfs_hist[policy][g->bfs_hist_pos[policy]] = busy;
    g->bfs_hist_pos[policy] = (g->bfs_hist_pos[policy] + 1) % pp_graph_s::kBfsHist;
}
// The run is over when the newest frontier is empty (or a level kernel found
// it so).
static bool bfs_done(const BfsHdr& h) { return h.finished || h.slot[h.last % 3].n == 0; }
static void bfs_fill_stats(const BfsHdr& h, pp_bfs_stats* stats) {
    stats->levels = h.levels;
    stats->reached = (int32_t)h.reached;
    stats->edges_reached = h.edges;
    for (int i = 0; i < PP_BFS_MAX_LOG; ++i) {
        stats->dir[i] = (i < h.levels) ? h.log_dir[i] : (int8_t)-1;
        stats->frontier[i] = (i < h.levels) ? h.log_n[i] : 0;
    }
}

PP_EXPORT pp_status pp_bfs_run_log(pp_graph g, int32_t root, pp_dir policy, float alpha, float beta, int32_t* level,
                                   int32_t* parent, void* state, size_t state_bytes, pp_bfs_level* log,
                                   int32_t log_cap, pp_bfs_stats* stats, void* stream) {
    clear_error();
    if (policy != PP_PUSH && policy != PP_PULL && policy != PP_SWITCH)
        return set_error(PP_E_RANGE, "policy must be PP_PUSH, PP_PULL or PP_SWITCH");
    if (log_cap < 0) return set_error(PP_E_RANGE, "log_cap must be >= 0");
    if (log_cap > 0 && !log) return set_error(PP_E_NULL, "log is required when log_cap > 0");
    if (!(alpha > 0.f)) alpha = 14.f;
    if (!(beta > 0.f)) beta = 24.f;
    pp_status s = pp_bfs_init(g, root, level, parent, state, state_bytes, stream);
    if (s != PP_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    BfsArgs a = bfs_args(g, state, level, parent);
    a.log = log;
    a.log_cap = log_cap;
    // Levels go out in batches with the level index kept on the device;
    // kernels past the last level find an empty frontier and return at once,
    // so only termination needs a read, which takes the whole header (the
    // statistics come with it).  The run is over when the newest frontier is
    // empty, so no launch is spent on finding that out.  The first batch
    // covers the most level-kernel launches that found work in the recent
    // runs with this policy on this graph, so a run of similar depth needs
    // one host read; a deeper run goes on in batches of 2, 4, 8, ...
    const int32_t predicted = bfs_predicted(g, policy);
    int32_t batch = predicted > 0 ? bfs_even(predicted) : 4;
    int32_t extra = 2;
    int32_t launched = 0;
    const int32_t max_levels = g->d.n + 1;  // at most n non-empty frontiers, then an empty one
    BfsHdr h;
    for (;;) {
        if (launched + batch <= max_levels) {  // a whole batch: replay its graph (launched stays even)
            hipGraphExec_t exec = nullptr;
            s = bfs_graph(g, a, policy, alpha, beta, batch, state, &exec);
            if (s != PP_OK) return s;
            PP_HIP(hipGraphLaunch(exec, st));
            launched += batch;
        } else {
            for (; launched < max_levels; ++launched) {
                s = launch_level(g, a, -1, launched & 1, policy, alpha, beta, st);
                if (s != PP_OK) return s;
            }
        }
        s = read_hdr(g, state, &h, st);
        if (s != PP_OK) return s;
        if (bfs_done(h) || launched >= max_levels) break;
        if (launched < predicted) {
            batch = bfs_even(predicted - launched);
        } else {
            batch = bfs_even(extra);
            extra = std::min(extra * 2, kBfsMaxBatch);
        }
    }
    bfs_record(g, policy, h.busy);
    if (stats) bfs_fill_stats(h, stats);
    return PP_OK;
}

// Many roots, one after another on the device: each root's init, one batch
// of levels sized from the history and a copy of its header go out back to
// back, and the host reads all the headers after one wait.  A root whose
// batch fell short is run again on its own.
PP_EXPORT pp_status pp_bfs_run_many(pp_graph g, int32_t k, const int32_t* roots, pp_dir policy, float alpha,
                                    float beta, int32_t* level, int32_t* parent, void* state, size_t state_bytes,
                                    pp_bfs_stats* stats, void* stream) {
    clear_error();
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (k < 0) return set_error(PP_E_RANGE, "k must be >= 0");
    if (policy != PP_PUSH && policy != PP_PULL && policy != PP_SWITCH)
        return set_error(PP_E_RANGE, "policy must be PP_PUSH, PP_PULL or PP_SWITCH");
    if (k == 0) return PP_OK;
    if (!roots || !stats) return set_error(PP_E_NULL, "roots and stats are required");
    for (int32_t i = 0; i < k; ++i)
        if (roots[i] < 0 || roots[i] >= g->d.n) return set_error(PP_E_RANGE, "root out of range");
    pp_status s = check_state(g, state, state_bytes);
    if (s != PP_OK) return s;
    if (!level || !parent) return set_error(PP_E_NULL, "level and parent are required");
    if (!(alpha > 0.f)) alpha = 14.f;
    if (!(beta > 0.f)) beta = 24.f;
    auto one = [&](int32_t i) {
        return pp_bfs_run_log(g, roots[i], policy, alpha, beta, level, parent, state, state_bytes, nullptr, 0,
                              &stats[i], stream);
    };
    int32_t i0 = 0;
    if (bfs_predicted(g, policy) == 0) {  // the first run with this policy sets the batch size
        s = one(0);
        if (s != PP_OK) return s;
        i0 = 1;
    }
    // two levels more than the deepest recent run: an empty level pair costs
    // a few microseconds, a root run again costs its whole run
    const int32_t predicted = bfs_predicted(g, policy);
    const int32_t batch = bfs_even(predicted + 2);
    if (batch > g->d.n + 1 || predicted >= kBfsMaxBatch) {  // tiny or deep graphs: root by root
        for (int32_t i = i0; i < k; ++i) {
            s = one(i);
            if (s != PP_OK) return s;
        }
        return PP_OK;
    }
    const size_t need = (size_t)(k - i0) * sizeof(BfsHdr);
    if (need > g->bfs_hdrs_cap) {
        if (g->bfs_hdrs_host) (void)hipHostFree(g->bfs_hdrs_host);
        g->bfs_hdrs_host = nullptr;
        g->bfs_hdrs_cap = 0;
        PP_HIP(hipHostMalloc(&g->bfs_hdrs_host, need, hipHostMallocDefault));
        g->bfs_hdrs_cap = need;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const BfsArgs a = bfs_args(g, state, level, parent);
    hipGraphExec_t exec = nullptr;
    s = bfs_graph(g, a, policy, alpha, beta, batch, state, &exec);
    if (s != PP_OK) return s;
    const char* hdr_dev = static_cast<const char*>(state) + bfs_layout(g).hdr;
    BfsHdr* hdrs = static_cast<BfsHdr*>(g->bfs_hdrs_host);
    for (int32_t i = i0; i < k; ++i) {
        s = pp_bfs_init(g, roots[i], level, parent, state, state_bytes, stream);
        if (s != PP_OK) return s;
        PP_HIP(hipGraphLaunch(exec, st));
        PP_HIP(hipMemcpyAsync(hdrs + (i - i0), hdr_dev, sizeof(BfsHdr), hipMemcpyDeviceToHost, st));
    }
    PP_HIP(hipStreamSynchronize(st));
    bool again = false, last_again = false;
    for (int32_t i = i0; i < k; ++i) {
        BfsHdr h;
        std::memcpy(&h, hdrs + (i - i0), sizeof(BfsHdr));
        if (h.overflow) return set_error(PP_E_WORKSPACE, "BFS queue capacity exceeded");
        if (bfs_done(h)) {
            bfs_record(g, policy, h.busy);
            bfs_fill_stats(h, &stats[i]);
        } else {
            s = one(i);
            if (s != PP_OK) return s;
            again = true;
            last_again = (i == k - 1);
        }
    }
    // level and parent hold the last root's run
    if (again && !last_again) return one(k - 1);
    return PP_OK;
}
