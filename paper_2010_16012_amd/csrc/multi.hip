// Many small graphs in one launch: PageRank (push or pull) and BFS for every
// graph of a concatenated arena, one workgroup per graph.
//
// Parallelism beyond one graph (the paper's sweeps are per graph; Sec. 4
// assumes up to one processor per vertex): a graph of at most kMultiMaxN
// vertices keeps its whole per-vertex state in the LDS of one compute unit,
// so the pull gathers and the push updates are LDS operations (ds_read /
// ds_add_f32) and the barrier between two sweeps is a workgroup barrier --
// no grid-wide synchronisation, no spin waits.  Workgroups take graphs
// largest first (longest-processing-time order) so the big graphs start
// first and small ones fill in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "pp_common.h"

namespace pp {

constexpr int kMultiBlock = 1024;
constexpr int kMultiGroup = 4;  // lanes per row
constexpr int kMultiU = 8;      // index loads in flight per lane
constexpr int kMultiPullU = 8;  // slots per lane and round of a pull row
constexpr int32_t kMultiMaxN = 16384;
// PageRank rows at least `big` long (tuned; 512 by default) get a whole
// wavefront each (up to kMultiBigCap of them per graph); a small group per
// row would leave the wavefront holding the hubs running long after the
// others.
constexpr int32_t kMultiBigCap = 512;
// Rows of `mid`..`big`-1 edges (64 by default) go to groups of ML lanes
// (tuned; 16 by default), up to kMultiMidCap of them per graph: in a small
// group such a row takes several rounds while the wavefront's other rows
// wait.  The short pull rows take PG lanes each (tuned; 2 by default; the
// push and BFS use kMultiGroup).
constexpr int32_t kMultiMidCap = 4096;

struct MultiEntry {
    int64_t vbase;  // first vertex of the graph in the vertex arenas (x, level, parent)
    int64_t obase;  // first entry of the graph's n+1 offsets in the offset arenas
    int64_t ebase;  // first slot of the graph in the index arenas
    int32_t n;
    int32_t nnz;
};

struct MultiArgs {
    const MultiEntry* table;  // LPT order
    int32_t count;
    const int32_t* off;       // per graph: n+1 local offsets, graphs back to back
    const uint16_t* idx;      // local vertex ids (below 16384, so 16 bits hold them)
    const int32_t* in_off;
    const uint16_t* in_idx;
    int32_t pr_dir;
    int32_t pr_iters;
    float f;
    float* x;                 // PageRank output, arena of vertices
    float* c_scratch;         // push: contributions, arena of vertices
    int32_t bfs_policy;       // -1: no BFS
    int32_t root;             // local root of every graph
    float alpha, beta;
    int32_t* level;
    int32_t* parent;
    const int32_t* err;       // set by k_multi_check when the arena is malformed
    int32_t big, mid;         // row-length thresholds of the wavefront and middle groups
};

__device__ __forceinline__ uint32_t bit_of(const uint32_t* bm, int32_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }

// U slots j0, j0 + STRIDE, ... of a row ending at re (j0 < re) added to an
// FP64 sum in slot order.  The index loads are clamped to the row's last
// slot and the LDS gathers issued together, so neither waits on the one
// before; slots past the row's end read the zero word s_zero.
template <int STRIDE, int U, typename I>
__device__ __forceinline__ void gather_row_slots(const I* __restrict__ ids, const float* s_c, const float* s_zero,
                                                 int32_t j0, int32_t re, double& acc) {
    const char* base = reinterpret_cast<const char*>(ids);
    const float* src[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int32_t j = j0 + k * STRIDE;
        const uint32_t boff = (uint32_t)min(j, re - 1) * (uint32_t)sizeof(I);
        const uint32_t id = *reinterpret_cast<const I*>(base + boff);
        src[k] = j < re ? s_c + id : s_zero;
    }
    float cv[U];
#pragma unroll
    for (int k = 0; k < U; ++k) cv[k] = *src[k];
#pragma unroll
    for (int k = 0; k < U; ++k) acc += (double)cv[k];
}

// Validates the arena before any sweep reads it, one workgroup per graph:
// the graph's n+1 offsets start at 0, never decrease and end at its nnz, and
// each of its nnz local ids lies below its n.  Both adjacencies are checked
// unless they alias.  Every read stays inside the graph's own offsets and
// slots, so a malformed arena is reported (PP_E_GRAPH), never walked.
constexpr int kCheckBlock = 256;

__device__ __forceinline__ bool offsets_ok(const int32_t* off, int32_t n, int32_t nnz) {
    bool ok = true;
    for (int32_t v = threadIdx.x; v < n; v += kCheckBlock) ok &= off[v] <= off[v + 1];
    if (threadIdx.x == 0) ok &= (off[0] == 0) && (off[n] == nnz);
    return ok;
}

__device__ __forceinline__ bool ids_ok(const uint16_t* idx, int32_t n, int32_t nnz) {
    uint32_t mx = 0;
    for (int32_t j = threadIdx.x; j < nnz; j += kCheckBlock) mx = max(mx, (uint32_t)idx[j]);
    return nnz == 0 || mx < (uint32_t)n;
}

__global__ __launch_bounds__(kCheckBlock) void k_multi_check(const MultiEntry* __restrict__ table,
                                                             const int32_t* __restrict__ off,
                                                             const uint16_t* __restrict__ idx,
                                                             const int32_t* __restrict__ in_off,
                                                             const uint16_t* __restrict__ in_idx, int32_t* err) {
    const MultiEntry e = table[blockIdx.x];
    bool ok = offsets_ok(off + e.obase, e.n, e.nnz) && ids_ok(idx + e.ebase, e.n, e.nnz);
    if (in_off != off || in_idx != idx)
        ok = ok && offsets_ok(in_off + e.obase, e.n, e.nnz) && ids_ok(in_idx + e.ebase, e.n, e.nnz);
    if (!ok) atomicOr(err, 1);
}

template <int PG, int ML>
__global__ __launch_bounds__(kMultiBlock) void k_multi(MultiArgs a) {
    extern __shared__ float lds[];
    __shared__ int32_t s_cnt[4];
    __shared__ int64_t s_m[2];
    const int32_t gi = blockIdx.x;
    if (gi >= a.count || *a.err) return;  // a malformed arena is never walked
    const int32_t big = a.big, mid = a.mid;
    const MultiEntry e = a.table[gi];
    const int32_t n = e.n;
    const int32_t* off = a.off + e.obase;
    const uint16_t* idx = a.idx + e.ebase;
    const int32_t* in_off = a.in_off + e.obase;
    const uint16_t* in_idx = a.in_idx + e.ebase;
    const int tid = threadIdx.x;
    const int lane = tid % kMultiGroup;
    const int grp = tid / kMultiGroup;
    constexpr int groups = kMultiBlock / kMultiGroup;
    constexpr int kWaves = kMultiBlock / kWave;
    const int wl = tid & (kWave - 1), wv = tid / kWave;
    // PageRank rows of the small groups: consecutive rows go to different
    // wavefronts (rows 16 q + w + k * groups for group q of wavefront w), so
    // neighbouring ids -- the hubs of an R-MAT graph -- are spread out
    const int32_t row0 = kWaves * ((tid % kWave) / kMultiGroup) + wv;

    // ---------------------------------------------------------------- PageRank
    __shared__ int32_t s_big[kMultiBigCap];
    __shared__ int32_t s_nbig;
    __shared__ int32_t s_mid[kMultiMidCap];
    __shared__ int32_t s_nmid;
    __shared__ float s_zero;
    if (a.pr_iters > 0) {
        const float base = (1.0f - a.f) / (float)n;
        // the long rows of the sweep's direction (in-rows pull, out-rows push)
        const int32_t* roff = (a.pr_dir == PP_PULL) ? in_off : off;
        if (tid == 0) {
            s_nbig = 0;
            s_nmid = 0;
            s_zero = 0.f;
        }
        __syncthreads();
        for (int32_t u = tid; u < n; u += kMultiBlock) {
            const int32_t d = roff[u + 1] - roff[u];
            if (d >= big) {
                const int32_t at = atomicAdd(&s_nbig, 1);
                if (at < kMultiBigCap) s_big[at] = u;
            } else if (d >= mid) {
                const int32_t at = atomicAdd(&s_nmid, 1);
                if (at < kMultiMidCap) s_mid[at] = u;
            }
        }
        __syncthreads();
        // more long (middle) rows than a list holds: those rows stay with the
        // small groups
        const int32_t nbig = (s_nbig <= kMultiBigCap) ? s_nbig : 0;
        const int32_t nmid = (s_nmid <= kMultiMidCap) ? s_nmid : 0;
        // does row length d belong to the small groups?
        auto grouped = [=](int32_t d) {
            return !((nbig > 0 && d >= big) || (nmid > 0 && d >= mid && d < big));
        };
        const int hl = wl & (ML - 1);  // lane within a middle-row group
        const int32_t mslot = (kWave / ML) * wv + wl / ML;  // its group
        constexpr int32_t mgroups = kMultiBlock / ML;
        if (a.pr_dir == PP_PULL) {
            float* s_c = lds;       // contributions of the current iterate
            float* s_y = lds + n;   // contributions of the next one
            for (int32_t u = tid; u < n; u += kMultiBlock) {
                const int32_t d = off[u + 1] - off[u];
                s_c[u] = d > 0 ? a.f * (1.0f / (float)n) / (float)d : 0.f;
            }
            __syncthreads();
            for (int32_t t = 0; t < a.pr_iters; ++t) {
                const bool last = (t == a.pr_iters - 1);
                // long in-rows: a whole wavefront each (FP64 sum per lane)
                for (int32_t i = wv; i < nbig; i += kWaves) {
                    const int32_t u = s_big[i];
                    double acc = 0.0;
                    const int32_t rb = in_off[u], re = in_off[u + 1];
                    for (int32_t j0 = rb + wl; j0 < re; j0 += kMultiU * kWave)
                        gather_row_slots<kWave, kMultiU>(in_idx, s_c, &s_zero, j0, re, acc);
#pragma unroll
                    for (int s = kWave / 2; s > 0; s >>= 1) acc += __shfl_xor(acc, s);
                    if (wl == 0) {
                        const float y = (float)((double)base + acc);
                        const int32_t d = off[u + 1] - off[u];
                        s_y[u] = d > 0 ? a.f * y / (float)d : 0.f;
                        if (last) a.x[e.vbase + u] = y;
                    }
                }
                // middle in-rows: 16 lanes each; the next row's offsets load
                // while this one is summed
                {
                    int32_t nu = 0, nrb = 0, nre = 0, nob = 0, noe = 0;
                    if (mslot < nmid) {
                        nu = s_mid[mslot];
                        nrb = in_off[nu];
                        nre = in_off[nu + 1];
                        nob = off[nu];
                        noe = off[nu + 1];
                    }
                    for (int32_t i = mslot; i < nmid; i += mgroups) {
                        const int32_t u = nu, rb = nrb, re = nre, ob = nob, oe = noe;
                        if (i + mgroups < nmid) {
                            nu = s_mid[i + mgroups];
                            nrb = in_off[nu];
                            nre = in_off[nu + 1];
                            nob = off[nu];
                            noe = off[nu + 1];
                        }
                        double acc = 0.0;
                        for (int32_t j0 = rb + hl; j0 < re; j0 += kMultiU * ML)
                            gather_row_slots<ML, kMultiU>(in_idx, s_c, &s_zero, j0, re, acc);
#pragma unroll
                        for (int s = ML / 2; s > 0; s >>= 1) acc += __shfl_xor(acc, s);
                        if (hl == 0) {
                            const float y = (float)((double)base + acc);
                            const int32_t d = oe - ob;
                            s_y[u] = d > 0 ? a.f * y / (float)d : 0.f;
                            if (last) a.x[e.vbase + u] = y;
                        }
                    }
                }
                // other rows: the group owning u gathers over its in-row (FP64
                // sum per lane, PG lanes per row, rows spread over
                // the wavefronts as above); the offsets and out-degree of the
                // group's next row load while this row is summed
                const int plane = tid % PG;
                const int32_t prow0 = kWaves * ((tid % kWave) / PG) + wv;
                constexpr int32_t pgroups = kMultiBlock / PG;
                int32_t nrb = 0, nre = 0, nob = 0, noe = 0;
                if (prow0 < n) {
                    nrb = in_off[prow0];
                    nre = in_off[prow0 + 1];
                    nob = off[prow0];
                    noe = off[prow0 + 1];
                }
                for (int32_t u = prow0; u < n; u += pgroups) {
                    double acc = 0.0;
                    const int32_t rb = nrb, re = nre, ob = nob, oe = noe;
                    if (u + pgroups < n) {
                        nrb = in_off[u + pgroups];
                        nre = in_off[u + pgroups + 1];
                        nob = off[u + pgroups];
                        noe = off[u + pgroups + 1];
                    }
                    if (!grouped(re - rb)) continue;  // group-uniform
                    for (int32_t j0 = rb + plane; j0 < re; j0 += kMultiPullU * PG)
                        gather_row_slots<PG, kMultiPullU>(in_idx, s_c, &s_zero, j0, re, acc);
#pragma unroll
                    for (int s = PG / 2; s > 0; s >>= 1) acc += __shfl_xor(acc, s);
                    if (plane == 0) {
                        const float y = (float)((double)base + acc);
                        const int32_t d = oe - ob;
                        s_y[u] = d > 0 ? a.f * y / (float)d : 0.f;
                        if (last) a.x[e.vbase + u] = y;
                    }
                }
                __syncthreads();
                float* tmp = s_c;
                s_c = s_y;
                s_y = tmp;
            }
        } else {
            // every out-edge adds the source's contribution to an FP64 LDS
            // accumulator (the order of the adds is arbitrary); contributions
            // live in the global scratch arena
            double* s_acc = reinterpret_cast<double*>(lds);
            float* c = a.c_scratch + e.vbase;
            for (int32_t u = tid; u < n; u += kMultiBlock) {
                const int32_t d = off[u + 1] - off[u];
                c[u] = d > 0 ? a.f * (1.0f / (float)n) / (float)d : 0.f;
                s_acc[u] = 0.0;
            }
            __syncthreads();
            for (int32_t t = 0; t < a.pr_iters; ++t) {
                const bool last = (t == a.pr_iters - 1);
                // long out-rows: a whole wavefront each
                for (int32_t i = wv; i < nbig; i += kWaves) {
                    const int32_t v = s_big[i];
                    const float cv = c[v];
                    if (cv == 0.f) continue;
                    const int32_t rb = off[v], re = off[v + 1];
                    for (int32_t j0 = rb + wl; j0 < re; j0 += kMultiU * kWave) {
                        int32_t ii[kMultiU];
#pragma unroll
                        for (int k = 0; k < kMultiU; ++k) {
                            const int32_t j = j0 + k * kWave;
                            ii[k] = j < re ? idx[j] : -1;
                        }
#pragma unroll
                        for (int k = 0; k < kMultiU; ++k)
                            if (ii[k] >= 0) atomicAdd(&s_acc[ii[k]], (double)cv);
                    }
                }
                // middle out-rows: 16 lanes each
                {
                    int32_t nv = 0, nb = 0, ne = 0;
                    float ncv = 0.f;
                    if (mslot < nmid) {
                        nv = s_mid[mslot];
                        ncv = c[nv];
                        nb = off[nv];
                        ne = off[nv + 1];
                    }
                    for (int32_t i = mslot; i < nmid; i += mgroups) {
                        const float cv = ncv;
                        const int32_t rb = nb, re = ne;
                        if (i + mgroups < nmid) {
                            nv = s_mid[i + mgroups];
                            ncv = c[nv];
                            nb = off[nv];
                            ne = off[nv + 1];
                        }
                        if (cv == 0.f) continue;
                        for (int32_t j0 = rb + hl; j0 < re; j0 += kMultiU * ML) {
                            int32_t ii[kMultiU];  // clamped to the row's last slot
#pragma unroll
                            for (int k = 0; k < kMultiU; ++k)
                                ii[k] = idx[(uint32_t)min(j0 + k * ML, re - 1)];
#pragma unroll
                            for (int k = 0; k < kMultiU; ++k)
                                if (j0 + k * ML < re) atomicAdd(&s_acc[ii[k]], (double)cv);
                        }
                    }
                }
                // two rows per group and round (v and v + groups), their index
                // loads issued together; the contributions and offsets of the
                // group's next two rows load while these are scattered
                float pc[2];
                int32_t pb[2], pe[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int32_t w = row0 + r * groups;
                    pc[r] = 0.f;
                    pb[r] = pe[r] = 0;
                    if (w < n) {
                        pc[r] = c[w];
                        pb[r] = off[w];
                        pe[r] = off[w + 1];
                    }
                }
                for (int32_t v = row0; v < n; v += 2 * groups) {
                    float cv[2];
                    int32_t rb[2], re[2];
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        cv[r] = pc[r];
                        rb[r] = pb[r];
                        re[r] = pe[r];
                        const int32_t w = v + (2 + r) * groups;
                        if (w < n) {
                            pc[r] = c[w];
                            pb[r] = off[w];
                            pe[r] = off[w + 1];
                        }
                        // nothing to scatter here: past the graph, a zero
                        // contribution, or a long row (done above)
                        if (v + r * groups >= n || cv[r] == 0.f || !grouped(re[r] - rb[r])) re[r] = rb[r];
                    }
                    const int32_t len = max(re[0] - rb[0], re[1] - rb[1]);
                    for (int32_t d = lane; d < len; d += kMultiU * kMultiGroup) {
                        // clamped into [0, re - 1]: a finished or empty row
                        // rereads a valid slot (the graph has edges, or len = 0)
                        int32_t ii[2][kMultiU];
#pragma unroll
                        for (int r = 0; r < 2; ++r)
#pragma unroll
                            for (int k = 0; k < kMultiU; ++k)
                                ii[r][k] = idx[(uint32_t)max(min(rb[r] + d + k * kMultiGroup, re[r] - 1), 0)];
#pragma unroll
                        for (int r = 0; r < 2; ++r)
#pragma unroll
                            for (int k = 0; k < kMultiU; ++k)
                                if (rb[r] + d + k * kMultiGroup < re[r]) atomicAdd(&s_acc[ii[r][k]], (double)cv[r]);
                    }
                }
                __syncthreads();
                for (int32_t u = tid; u < n; u += kMultiBlock) {
                    const float y = base + (float)s_acc[u];
                    const int32_t d = off[u + 1] - off[u];
                    c[u] = d > 0 ? a.f * y / (float)d : 0.f;
                    s_acc[u] = 0.0;
                    if (last) a.x[e.vbase + u] = y;
                }
                __syncthreads();
            }
        }
    }

    // ---------------------------------------------------------------- BFS
    if (a.bfs_policy < 0) return;
    const int32_t words = (n + 31) / 32;
    uint32_t* s_front = reinterpret_cast<uint32_t*>(lds);
    uint32_t* s_next = s_front + words;
    uint32_t* s_vis = s_next + words;
    const int32_t root = a.root;
    for (int32_t v = tid; v < n; v += kMultiBlock) {
        a.level[e.vbase + v] = (v == root) ? 0 : -1;
        a.parent[e.vbase + v] = (v == root) ? root : -1;
    }
    for (int32_t w = tid; w < words; w += kMultiBlock) {
        const uint32_t m = (w == (root >> 5)) ? (1u << (root & 31)) : 0u;
        s_front[w] = m;
        s_vis[w] = m;
        s_next[w] = 0u;
    }
    if (tid == 0) {
        s_cnt[0] = 1;                          // |F|
        s_m[0] = off[root + 1] - off[root];    // out-edges of F
        s_m[1] = (int64_t)(off[n] - off[root + 1] + off[root]);  // out-edges of unvisited vertices
        s_cnt[2] = PP_PUSH;                    // previous direction
        s_cnt[3] = 0;                          // previous |F|
    }
    __syncthreads();
    for (int32_t lvl = 0;; ++lvl) {
        const int32_t nf = s_cnt[0];
        if (nf == 0) break;
        const int64_t mf = s_m[0], mu = s_m[1];
        int32_t dir = a.bfs_policy;
        if (dir == PP_SWITCH) {
            if (lvl == 0 || s_cnt[2] == PP_PUSH) dir = ((double)mf > (double)mu / a.alpha) ? PP_PULL : PP_PUSH;
            else dir = ((double)nf < (double)n / a.beta && nf < s_cnt[3]) ? PP_PUSH : PP_PULL;
        }
        __syncthreads();
        if (tid == 0) {
            s_cnt[1] = 0;
            s_cnt[2] = dir;
            s_cnt[3] = nf;
        }
        if (tid < 2) s_m[tid] = 0;  // s_m[0] accumulates new out-edges; s_m[1] is recomputed below
        __syncthreads();
        int32_t my_new = 0;
        int64_t my_deg = 0;
        if (dir == PP_PUSH) {
            // frontier vertices claim unvisited out-neighbours (LDS atomic OR)
            for (int32_t v = grp; v < n; v += groups) {
                if (!bit_of(s_front, v)) continue;
                const int32_t rb = off[v], re = off[v + 1];
                for (int32_t j0 = rb + lane; j0 < re; j0 += kMultiU * kMultiGroup) {
                    // index loads clamped to the row's last slot, then every
                    // visited probe issued before the first claim (a probe only
                    // filters: the atomic OR decides)
                    int32_t ii[kMultiU];
#pragma unroll
                    for (int k = 0; k < kMultiU; ++k) ii[k] = idx[(uint32_t)min(j0 + k * kMultiGroup, re - 1)];
                    uint32_t seen[kMultiU];
#pragma unroll
                    for (int k = 0; k < kMultiU; ++k) seen[k] = s_vis[min(ii[k], n - 1) >> 5];
#pragma unroll
                    for (int k = 0; k < kMultiU; ++k) {
                        const int32_t u = ii[k];
                        if (j0 + k * kMultiGroup >= re || u >= n) continue;  // ids past the graph are ignored
                        const uint32_t b = 1u << (u & 31);
                        if (seen[k] & b) continue;
                        const uint32_t old = atomicOr(&s_vis[u >> 5], b);
                        if (!(old & b)) {
                            atomicOr(&s_next[u >> 5], b);
                            a.level[e.vbase + u] = lvl + 1;
                            a.parent[e.vbase + u] = v;
                            my_new += 1;
                            my_deg += off[u + 1] - off[u];
                        }
                    }
                }
            }
        } else {
            // unvisited vertices look for a frontier in-neighbour, first in stored order
            for (int32_t v = grp; v < n; v += groups) {
                if (bit_of(s_vis, v)) continue;
                const int32_t b0 = in_off[v], e0 = in_off[v + 1];
                int32_t hit = INT32_MAX;
                // kMultiU steps of kMultiGroup in-neighbours per round; the
                // first frontier member in stored order wins
                for (int32_t jb = b0; jb < e0 && hit == INT32_MAX; jb += kMultiU * kMultiGroup) {
                    // index loads clamped to the row's last slot, frontier words
                    // read together (ids past the graph read a valid word and
                    // are then ignored)
                    int32_t ii[kMultiU];
#pragma unroll
                    for (int k = 0; k < kMultiU; ++k)
                        ii[k] = in_idx[(uint32_t)min(jb + k * kMultiGroup + lane, e0 - 1)];
                    uint32_t fw[kMultiU];
#pragma unroll
                    for (int k = 0; k < kMultiU; ++k) fw[k] = s_front[min(ii[k], n - 1) >> 5];
                    int32_t pos = INT32_MAX;
#pragma unroll
                    for (int k = kMultiU - 1; k >= 0; --k) {
                        const int32_t j = jb + k * kMultiGroup + lane;
                        if (j < e0 && ii[k] < n && ((fw[k] >> (ii[k] & 31)) & 1u)) pos = j;
                    }
#pragma unroll
                    for (int s = kMultiGroup / 2; s > 0; s >>= 1) pos = min(pos, __shfl_xor(pos, s));
                    hit = pos;
                }
                if (hit != INT32_MAX && lane == 0) {
                    atomicOr(&s_next[v >> 5], 1u << (v & 31));  // words are shared by groups
                    a.level[e.vbase + v] = lvl + 1;
                    a.parent[e.vbase + v] = in_idx[hit];
                    my_new += 1;
                    my_deg += off[v + 1] - off[v];
                }
            }
        }
        if (my_new) {
            atomicAdd(&s_cnt[1], my_new);
            atomicAdd(reinterpret_cast<unsigned long long*>(&s_m[0]), (unsigned long long)my_deg);
        }
        __syncthreads();
        // next frontier; bottom-up discoveries become visited now
        for (int32_t w = tid; w < words; w += kMultiBlock) {
            const uint32_t nw = s_next[w];
            s_front[w] = nw;
            s_vis[w] |= nw;
            s_next[w] = 0u;
        }
        if (tid == 0) {
            s_cnt[0] = s_cnt[1];
            s_m[1] = mu - s_m[0];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side
template <int PG, int ML>
static void launch_multi_k(const MultiArgs& a, int32_t grid, size_t lds, hipStream_t st) {
    allow_dynamic_lds(reinterpret_cast<const void*>(&k_multi<PG, ML>), lds);
    hipLaunchKernelGGL((k_multi<PG, ML>), dim3(grid), dim3(kMultiBlock), lds, st, a);
}

// The instantiation for the tuned group widths (false: none).
static bool launch_multi(int32_t pg, int32_t ml, const MultiArgs& a, int32_t grid, size_t lds, hipStream_t st) {
    auto by_ml = [&](auto pg_tag) {
        constexpr int P = decltype(pg_tag)::value;
        switch (ml) {
            case 8: launch_multi_k<P, 8>(a, grid, lds, st); return true;
            case 16: launch_multi_k<P, 16>(a, grid, lds, st); return true;
            case 32: launch_multi_k<P, 32>(a, grid, lds, st); return true;
            default: return false;
        }
    };
    switch (pg) {
        case 1: return by_ml(std::integral_constant<int, 1>{});
        case 2: return by_ml(std::integral_constant<int, 2>{});
        case 4: return by_ml(std::integral_constant<int, 4>{});
        default: return false;
    }
}

// Workspace: the graph table (LPT order) and the validation error word, both
// written by one host copy, then the push contributions (one float per vertex).
struct MultiLayout {
    size_t table, err, cbuf, total;
};

static MultiLayout multi_layout(int32_t count, int64_t total_n) {
    MultiLayout L{};
    L.table = 0;
    L.err = (size_t)std::max(count, 1) * sizeof(MultiEntry);
    L.cbuf = align_up(L.err + sizeof(int32_t), 256);
    L.total = L.cbuf + align_up((size_t)std::max<int64_t>(total_n, 1) * 4, 256);
    return L;
}

// Scratch of pp_multi_run_static (for callers that cannot allocate device
// memory): the graph table, the validation word and the push contributions of
// one call live in this file-scope array, of which every device the library
// runs on holds one copy for the life of the process.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in symbol): the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kMultiStaticBytes = PP_MULTI_STATIC_BYTES;
static __device__ __align__(256) unsigned char scratch[kMultiStaticBytes];

constexpr int kMaxDevices = 64;

// Device address of this device's copy of `scratch` (looked up on the first
// call on each device, with that device current).
static pp_status static_scratch(void** out) {
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = 0;
    PP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(PP_E_UNSUPPORTED, "device ordinal beyond the static table");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(PP_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return PP_OK;
}

}  // namespace pp

using namespace pp;

PP_EXPORT size_t pp_multi_workspace_bytes(int32_t num_graphs, int64_t total_vertices) {
    if (num_graphs < 0 || total_vertices < 0) return 0;
    return multi_layout(num_graphs, total_vertices).total;
}

namespace pp {

// The call behind pp_multi_run and pp_multi_run_static: ws is the workspace
// (caller memory, or the static scratch of this file).
static pp_status multi_run(int32_t num_graphs, const int32_t* graph_n, const int64_t* graph_nnz, const int32_t* off,
                           const uint16_t* idx, const int32_t* in_off, const uint16_t* in_idx, pp_dir pr_dir,
                           int32_t pr_iters, float f, float* x, int32_t bfs_policy, int32_t bfs_root, float alpha,
                           float beta, int32_t* level, int32_t* parent, void* ws, size_t ws_bytes, bool static_ws,
                           void* stream) {
    clear_error();
    if (num_graphs < 0) return set_error(PP_E_SIZE, "num_graphs must be >= 0");
    if (num_graphs == 0) return PP_OK;
    if (!graph_n || !graph_nnz) return set_error(PP_E_NULL, "graph_n and graph_nnz (host arrays) are required");
    if (!off || !in_off || (!ws && !static_ws)) return set_error(PP_E_NULL, "off, in_off and ws are required");
    if (pr_dir != PP_PUSH && pr_dir != PP_PULL) return set_error(PP_E_RANGE, "pr_dir must be PP_PUSH or PP_PULL");
    if (pr_iters < 0) return set_error(PP_E_RANGE, "pr_iters must be >= 0");
    if (pr_iters > 0 && !x) return set_error(PP_E_NULL, "x is required when pr_iters > 0");
    if (!(f >= 0.f && f < 1.f)) return set_error(PP_E_RANGE, "f must lie in [0, 1)");
    if (bfs_policy != -1 && bfs_policy != PP_PUSH && bfs_policy != PP_PULL && bfs_policy != PP_SWITCH)
        return set_error(PP_E_RANGE, "bfs_policy must be -1, PP_PUSH, PP_PULL or PP_SWITCH");
    if (bfs_policy >= 0 && (!level || !parent)) return set_error(PP_E_NULL, "level and parent are required for BFS");
    if (!(alpha > 0.f)) alpha = 14.f;
    if (!(beta > 0.f)) beta = 24.f;
    std::vector<MultiEntry> ent(num_graphs);
    int64_t vb = 0, eb = 0, max_n = 1, total_nnz = 0;
    for (int32_t i = 0; i < num_graphs; ++i) {
        if (graph_n[i] < 1 || graph_n[i] > kMultiMaxN)
            return set_error(PP_E_SIZE, "every graph needs 1 <= n <= 16384 vertices");
        if (graph_nnz[i] < 0 || graph_nnz[i] > INT32_MAX) return set_error(PP_E_SIZE, "graph nnz out of range");
        if (bfs_policy >= 0 && (bfs_root < 0 || bfs_root >= graph_n[i]))
            return set_error(PP_E_RANGE, "bfs_root must be a vertex of every graph");
        ent[i] = MultiEntry{vb, vb + i, eb, graph_n[i], (int32_t)graph_nnz[i]};
        vb += graph_n[i];
        eb += graph_nnz[i];
        total_nnz += graph_nnz[i];
        max_n = std::max<int64_t>(max_n, graph_n[i]);
    }
    if (total_nnz > 0 && (!idx || !in_idx)) return set_error(PP_E_NULL, "idx and in_idx are required");
    const MultiLayout ML = multi_layout(num_graphs, vb);
    if (static_ws && ML.total > kMultiStaticBytes)
        return set_error(PP_E_WORKSPACE, "pp_multi_run_static: the graphs need " + std::to_string(ML.total) +
                                             " bytes of scratch, more than its " + std::to_string(kMultiStaticBytes) +
                                             " (use pp_multi_run with a caller workspace)");
    if (static_ws) {
        pp_status st_ptr = static_scratch(&ws);
        if (st_ptr != PP_OK) return st_ptr;
        ws_bytes = kMultiStaticBytes;
    }
    if (ws_bytes < ML.total) return set_error(PP_E_WORKSPACE, "workspace too small");
    // largest graphs first (workgroups are dispatched roughly in index order)
    std::vector<int32_t> order(num_graphs);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t p, int32_t q) {
        return (int64_t)ent[p].nnz + ent[p].n > (int64_t)ent[q].nnz + ent[q].n;
    });
    // the table in LPT order followed by a zero error word, copied together
    std::vector<char> head(ML.err + sizeof(int32_t), 0);
    MultiEntry* dev = reinterpret_cast<MultiEntry*>(head.data());
    for (int32_t i = 0; i < num_graphs; ++i) dev[i] = ent[order[i]];
    int dev_id = 0, lds_cu = 0;
    PP_HIP(hipGetDevice(&dev_id));
    PP_HIP(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id));
    const size_t lds = std::max<size_t>((size_t)max_n * 8, (size_t)3 * ((max_n + 31) / 32) * 4);
    if (lds > (size_t)lds_cu) return set_error(PP_E_UNSUPPORTED, "graphs too large for one workgroup's LDS");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MultiEntry* table = static_cast<MultiEntry*>(ws);
    int32_t* err = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + ML.err);
    PP_HIP(hipMemcpyAsync(table, head.data(), head.size(), hipMemcpyHostToDevice, st));
    const uint16_t* idx_chk = idx ? idx : in_idx;  // both NULL only when no graph has edges
    const uint16_t* in_idx_chk = in_idx ? in_idx : idx;
    hipLaunchKernelGGL(k_multi_check, dim3(num_graphs), dim3(kCheckBlock), 0, st, (const MultiEntry*)table, off,
                       idx_chk, in_off, in_idx_chk, err);
    PP_LAUNCH_CHECK("k_multi_check");
    MultiArgs a;
    a.table = table;
    a.count = num_graphs;
    a.off = off;
    a.idx = idx;
    a.in_off = in_off;
    a.in_idx = in_idx;
    a.pr_dir = pr_dir;
    a.pr_iters = pr_iters;
    a.f = f;
    a.x = x;
    a.c_scratch = reinterpret_cast<float*>(static_cast<char*>(ws) + ML.cbuf);
    a.bfs_policy = bfs_policy;
    a.root = bfs_root;
    a.alpha = alpha;
    a.beta = beta;
    a.level = level;
    a.parent = parent;
    a.err = err;
    const Tuning& t = tuning();
    a.big = t.multi_big;
    a.mid = t.multi_mid;
    if (!launch_multi(t.multi_pull_group, t.multi_mid_lanes, a, num_graphs, lds, st))
        return set_error(PP_E_RANGE, "many-graph tuning: unsupported group widths");
    PP_LAUNCH_CHECK("k_multi");
    int32_t herr = 0;
    PP_HIP(hipMemcpyAsync(&herr, err, sizeof(herr), hipMemcpyDeviceToHost, st));
    // the host table must outlive the asynchronous copy
    PP_HIP(hipStreamSynchronize(st));
    if (herr) return set_error(PP_E_GRAPH, "a graph of the arena has malformed offsets or an id past its n");
    return PP_OK;
}

}  // namespace pp

PP_EXPORT pp_status pp_multi_run(int32_t num_graphs, const int32_t* graph_n, const int64_t* graph_nnz,
                                 const int32_t* off, const uint16_t* idx, const int32_t* in_off,
                                 const uint16_t* in_idx, pp_dir pr_dir, int32_t pr_iters, float f, float* x,
                                 int32_t bfs_policy, int32_t bfs_root, float alpha, float beta, int32_t* level,
                                 int32_t* parent, void* ws, size_t ws_bytes, void* stream) {
    return multi_run(num_graphs, graph_n, graph_nnz, off, idx, in_off, in_idx, pr_dir, pr_iters, f, x, bfs_policy,
                     bfs_root, alpha, beta, level, parent, ws, ws_bytes, false, stream);
}

PP_EXPORT pp_status pp_multi_run_static(int32_t num_graphs, const int32_t* graph_n, const int64_t* graph_nnz,
                                        const int32_t* off, const uint16_t* idx, const int32_t* in_off,
                                        const uint16_t* in_idx, pp_dir pr_dir, int32_t pr_iters, float f, float* x,
                                        int32_t bfs_policy, int32_t bfs_root, float alpha, float beta,
                                        int32_t* level, int32_t* parent, void* stream) {
    return multi_run(num_graphs, graph_n, graph_nnz, off, idx, in_off, in_idx, pr_dir, pr_iters, f, x, bfs_policy,
                     bfs_root, alpha, beta, level, parent, nullptr, 0, true, stream);
}
