// PageRank power-iteration step in its pulling form (Sec. 3.1 equation;
// Sec. 4.1 listing, pulling lines), the push/pull hybrid, and the run loops
// of both forms (the push sweep itself is in push.hip).
//
// Work is described by degree-binned vertex lists: bin b owns a contiguous
// range of work units, heaviest bin first.  A vertex of bin b is owned by
// kBinLanes[b] lanes (1, 4, 16, a wavefront, a workgroup); bin 5 rows are
// cut into chunks of split_chunk edges.
//
// The contribution c[v] = f * x[v] / s(v) (s = out-degree or out-strength)
// is produced by the previous step's epilogue, so a gather reads ONE float
// per edge instead of the neighbour's rank and degree.
//
// Vectors the caller sees (x, y) are in caller ids; c, the push accumulator
// and everything per-edge are in internal ids (equal to caller ids unless the
// graph was relabelled): the first gather and the last write go through perm.
#include <hip/hip_runtime.h>

#include "pp_common.h"
#include "sweep.h"

namespace pp {

template <int G>
__device__ __forceinline__ float group_reduce(float v) {
#pragma unroll
    for (int s = G / 2; s > 0; s >>= 1) v += __shfl_xor(v, s);
    return v;
}

// Deterministic workgroup sum (fixed order: wavefront tree, then waves 0..3).
__device__ __forceinline__ float block_reduce(float v, float* red) {
    v = group_reduce<kWave>(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i) t += red[i];
    }
    __syncthreads();  // red[] may be reused right after
    return t;         // valid in thread 0
}

// Sum of c[idx[j]] (times the slot weight) over j = b + lane, b + lane + G, ...
// U index loads and then U gathers are issued back to back per lane (indices
// past the row end are clamped to its last slot and their values masked), so
// a row of up to U*G edges costs two dependent memory round trips.
// With HOT, entries below `hot` are read from the LDS copy s_c of c.
template <int G, int U, bool W, bool HOT = false>
__device__ __forceinline__ float gather_row(const int32_t* __restrict__ idx, const float* __restrict__ wt,
                                            const float* __restrict__ c, int32_t b, int32_t e, int lane,
                                            const float* s_c = nullptr, int32_t hot = 0) {
    float acc[U];
#pragma unroll
    for (int k = 0; k < U; ++k) acc[k] = 0.f;
    for (int32_t j0 = b + lane; j0 < e; j0 += U * G) {
        int32_t jj[U], ii[U];
#pragma unroll
        for (int k = 0; k < U; ++k) jj[k] = min(j0 + k * G, e - 1);
#pragma unroll
        for (int k = 0; k < U; ++k) ii[k] = idx[jj[k]];
        float v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (HOT) {
                // Two separate loads: an LDS read (index clamped into the
                // staged range) and a global load only on lanes that need
                // it.  A single conditional load would be merged into a flat
                // load, which occupies the vector-memory path even for LDS.
                const float lv = s_c[min(ii[k], hot - 1)];
                float gv = 0.f;
                if (ii[k] >= hot) gv = c[ii[k]];
                v[k] = (ii[k] < hot) ? lv : gv;
            } else {
                v[k] = c[ii[k]];
            }
        }
        if (W) {
#pragma unroll
            for (int k = 0; k < U; ++k) v[k] *= wt[jj[k]];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) acc[k] += (j0 + k * G < e) ? v[k] : 0.f;
    }
#pragma unroll
    for (int s = U / 2; s > 0; s >>= 1) {
#pragma unroll
        for (int k = 0; k < s; ++k) acc[k] += acc[k + s];
    }
    return acc[0];
}

// ------------------------------------------------------------------ pull
struct PullArgs {
    SweepPlan sp;          // used by the hybrid push part (out-degree bins)
    int32_t list_beg[PP_NUM_BINS];      // first entry of each bin's rows in `list`
    int32_t list_cnt[PP_NUM_BINS];      // rows of each bin this sweep covers
    int32_t wave_off[PP_NUM_BINS + 1];  // wavefront units per bin (persistent sweep)
    int32_t units;
    int32_t hot;           // contributions below this id are staged in LDS
    const int32_t* off;    // CSC offsets
    const int32_t* idx;    // CSC indices
    const float* wt;       // weights in CSC slot order (weighted only)
    const int32_t* list;   // vertices grouped by in-degree bin
    const int32_t* tab;    // bin-5 chunk table (v | begin | end | first)
    int32_t tab_cap;
    int32_t tab0;          // first chunk-table entry of this sweep's bin-5 units
    float* part;           // bin-5 partial sums (indexed like the chunk table)
    const float* c;        // contributions of the current iterate
    const float* inv_s;
    const int32_t* perm;   // internal -> caller id (nullable)
    float* c_next;         // contributions of the new iterate (nullable)
    float* y;              // new iterate, caller ids (nullable)
    int64_t y_stride;      // y[caller id * y_stride]: 1, or k for a column of an n x k matrix
    float base;            // teleport term of every row: (1-f)/n, or 0 when personalised
    int32_t tele_v;        // internal id of the personalised teleport row (-1: none)
    float tele;            // (1-f) added to row tele_v
    float f;
    int32_t skip_below;    // rows u < skip_below are left to the hybrid's push part (0: none)
    int32_t tail_beg;      // rows [tail_beg, tail_end) have no in-edges and no unit:
    int32_t tail_end;      // the tiled combine finishes them
};

// Teleport term of row u.
__device__ __forceinline__ float row_base(const PullArgs& a, int32_t u) {
    return a.base + ((u == a.tele_v) ? a.tele : 0.f);
}

// Owner of u writes y = teleport + acc and the next contribution.
__device__ __forceinline__ void pull_finish(const PullArgs& a, int32_t u, float acc) {
    const float yv = row_base(a, u) + acc;
    if (a.y) a.y[(int64_t)user_id(a.perm, u) * a.y_stride] = yv;
    if (a.c_next) a.c_next[u] = a.f * yv * a.inv_s[u];
}

// Which bin does wavefront unit `u` belong to?  Units run bin 5, 4, ..., 0.
__device__ __forceinline__ int wave_unit_bin(const int32_t* wo, int32_t u) {
    int b = PP_NUM_BINS - 1;
#pragma unroll
    for (int i = PP_NUM_BINS - 1; i > 0; --i)
        if (u >= wo[i - 1]) b = i - 1;
    return b;
}

// What a lane needs to run one wavefront unit of the pull sweep.  Bins 0-4:
// the row of the lane's group (-1 past the bin's end), its slot range and
// 1/s of the row (for the next contribution).  Bin 5: the chunk's row and
// slot range.
struct PullTask {
    int32_t bin;  // -1: no unit
    int32_t lu;   // unit within its bin
    int32_t row;
    int32_t b, e;
    float inv_s;
};

// First stage of a unit: its bin and the row from the bin's vertex list (or
// the chunk's row from the chunk table).
__device__ __forceinline__ PullTask pull_task(const PullArgs& a, int32_t unit, int lane) {
    PullTask t{-1, 0, -1, 0, 0, 0.f};
    if (unit >= a.units) return t;
    t.bin = wave_unit_bin(a.wave_off, unit);
    t.lu = unit - a.wave_off[t.bin];
    if (t.bin == PP_NUM_BINS - 1) {
        t.row = a.tab[a.tab0 + t.lu];
    } else {
        int g = kPullLanes[0];
#pragma unroll
        for (int b = 1; b < PP_NUM_BINS - 1; ++b)
            if (t.bin == b) g = kPullLanes[b];
        const int32_t i = t.lu * (kWave / g) + lane / g;
        t.row = (i < a.list_cnt[t.bin]) ? a.list[a.list_beg[t.bin] + i] : -1;
    }
    return t;
}

// Second stage: the slot range (and, bins 0-4, 1/s of the row).
__device__ __forceinline__ void pull_bounds(const PullArgs& a, PullTask& t) {
    if (t.bin == PP_NUM_BINS - 1) {
        t.b = a.tab[a.tab_cap + a.tab0 + t.lu];
        t.e = a.tab[2 * a.tab_cap + a.tab0 + t.lu];
    } else if (t.bin >= 0 && t.row >= 0) {
        t.b = a.off[t.row];
        t.e = a.off[t.row + 1];
        if (a.c_next) t.inv_s = a.inv_s[t.row];
    }
}

// Unit of bin BIN (0-4): kWave/G rows, G lanes each, U loads per lane.
template <int BIN, bool W, bool HOT>
__device__ __forceinline__ void pull_unit(const PullArgs& a, const PullTask& t, int lane, const float* s_c) {
    constexpr int G = kPullLanes[BIN];
    constexpr int U = kPullLoads[BIN];
    if (t.row < 0 || t.row < a.skip_below) return;  // whole groups leave together
    const int gl = lane & (G - 1);
    float acc = gather_row<G, U, W, HOT>(a.idx, a.wt, a.c, t.b, t.e, gl, s_c, a.hot);
    acc = group_reduce<G>(acc);
    if (gl == 0) {
        const float yv = row_base(a, t.row) + acc;
        if (a.y) a.y[(int64_t)user_id(a.perm, t.row) * a.y_stride] = yv;
        if (a.c_next) a.c_next[t.row] = a.f * yv * t.inv_s;
    }
}

// The wavefront units of a persistent pull sweep: this wavefront takes units
// first, first + nw, ...  The units are pipelined: while unit t gathers, the
// row bounds of unit t + nw and the list entry of unit t + 2 nw are already
// on their way, so a unit waits for two memory round trips (indices, then
// gathers) instead of four.  No atomics: every output has exactly one writer.
template <bool W, bool HOT>
__device__ __forceinline__ void pull_sweep(const PullArgs& a, const float* s_c, int32_t first, int32_t nw) {
    const int lane = threadIdx.x & (kWave - 1);
    PullTask next = pull_task(a, first, lane);
    pull_bounds(a, next);
    PullTask after = pull_task(a, first + nw, lane);
    for (int32_t unit = first; unit < a.units; unit += nw) {
        const PullTask t = next;
        next = after;
        pull_bounds(a, next);
        after = pull_task(a, unit + 2 * nw, lane);
        switch (t.bin) {
            case 5: {  // one chunk of a very long row -> partial sum, finished by k_pr_pull_fix
                if (t.row < a.skip_below) break;
                float acc =
                    gather_row<kPullLanes[5], kPullLoads[5], W, HOT>(a.idx, a.wt, a.c, t.b, t.e, lane, s_c, a.hot);
                acc = group_reduce<kWave>(acc);
                if (lane == 0) a.part[a.tab0 + t.lu] = acc;
                break;
            }
            case 4: pull_unit<4, W, HOT>(a, t, lane, s_c); break;
            case 3: pull_unit<3, W, HOT>(a, t, lane, s_c); break;
            case 2: pull_unit<2, W, HOT>(a, t, lane, s_c); break;
            case 1: pull_unit<1, W, HOT>(a, t, lane, s_c); break;
            default: pull_unit<0, W, HOT>(a, t, lane, s_c); break;
        }
    }
}

// Copies c[0, count) into LDS (float4 loads, four in flight per thread).
__device__ __forceinline__ void stage_lds(float* dst, const float* __restrict__ src, int32_t count) {
    const int32_t n4 = count >> 2;
    const float4* s4 = reinterpret_cast<const float4*>(src);
    float4* d4 = reinterpret_cast<float4*>(dst);
    const int32_t bd = blockDim.x;
    for (int32_t i0 = threadIdx.x; i0 < n4; i0 += 4 * bd) {
        float4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = s4[min(i0 + k * bd, n4 - 1)];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k * bd < n4) d4[i0 + k * bd] = v[k];
    }
    for (int32_t i = 4 * n4 + threadIdx.x; i < count; i += bd) dst[i] = src[i];
}

// Persistent pull sweep: every workgroup first copies c[0, hot) -- the
// contributions of the heaviest vertices, which most gathers hit -- into
// LDS, then its wavefronts take units w, w + W, ... (W = wavefronts in the
// grid).
template <bool W, bool HOT>
__global__ __launch_bounds__(1024) void k_pr_pull(PullArgs a) {
    extern __shared__ float s_c[];
    if (HOT) {
        if ((reinterpret_cast<uintptr_t>(a.c) & 15) == 0) stage_lds(s_c, a.c, a.hot);
        else for (int32_t i = threadIdx.x; i < a.hot; i += blockDim.x) s_c[i] = a.c[i];
        __syncthreads();
    }
    const int32_t nw = gridDim.x * (blockDim.x / kWave);
    // the unit number is wavefront-uniform: keep it (and the bin) in scalar registers
    const int32_t first = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    pull_sweep<W, HOT>(a, s_c, first, nw);
}

// Sums the chunk partials of split rows fix0, fix0 + 1, ... in chunk order
// (deterministic).
__global__ void k_pr_pull_fix(PullArgs a, int32_t nsplit, int32_t fix0) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x + fix0;
    if (i >= nsplit + fix0) return;
    const int32_t* first = a.tab + 3 * a.tab_cap;
    if (a.tab[first[i]] < a.skip_below) return;
    float acc = 0.f;
    for (int32_t e = first[i]; e < first[i + 1]; ++e) acc += a.part[e];
    pull_finish(a, a.tab[first[i]], acc);
}

// ------------------------------------------------------------ tiled pull
// The heaviest rows [0, R) pull their in-edges slice by slice (SlicePlan in
// pp_common.h): a workgroup stages the contributions of one source slice in
// LDS and each wavefront sums the segments of a unit -- at most 1,024
// consecutive 16-bit entries, lane l holding entries 16l .. 16l+15 (two
// 16-byte loads) -- so every gather is an LDS read.  A segment's partial is
// the in-lane sum of its entries plus, when it runs on, the sums of the next
// lanes up to the lane where the next segment starts (a segmented scan
// across the wavefront).  Each (slice, row) gets one partial (long segments
// one per chunk); k_pr_tiled_combine adds a row's partials in slice order,
// then its chunks in order.  The same sum as the plain pull in another fixed
// order: bit-reproducible.
struct TileArgs {
    const uint16_t* idx;      // units and chunks (bit 15: first entry of a segment)
    const int32_t* prow;      // row of every unit segment, in unit order
    const SliceUnit* units;
    const SliceSeg* segs;     // runs of one slice; workgroup b: runs [wg[b], wg[b+1])
    const int32_t* wg;
    float* part;              // partial sums [S*R], slice-major
    float* cpart;             // chunk partial sums
    const int32_t* cbeg;      // chunks of row u: [cbeg[u], cbeg[u+1])
    const float* c;           // contributions
    int32_t n, R, W, S, P;    // P: segments in prow
    int32_t idx_last;         // last 8-aligned start with 16 entries behind it
};

// What a lane loads for one unit ahead of running it: its 16 entries and the
// rows of segments lane, lane + 64, lane + 128, lane + 192 of the unit.
struct UnitData {
    SliceUnit d;
    uint4 q0, q1;
    uint32_t rows[4];
};

__device__ __forceinline__ SliceUnit no_unit() { return SliceUnit{0, 0, 0, 0}; }


// Every load is unconditional, at an address clamped into its array (what a
// lane should not use is masked when the unit runs): the compiler then knows
// how many loads are in flight and waits only for the older unit's.
// The entries are read once per sweep: non-temporal loads keep them from
// evicting the lines that are read again (about 3% off the sweep at R-MAT
// scale 22; the partials, written once and read once by the combine, are
// stored non-temporally for the same reason, about 2% more).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // non-temporal loads take a native vector
__device__ __forceinline__ UnitData unit_load(const TileArgs& t, const SliceUnit& d, int lane) {
    UnitData U;
    U.d = d;
    // d.a is 8-aligned: two aligned 16-byte loads
    const u32x4* q = reinterpret_cast<const u32x4*>(t.idx + min(d.a + 16 * lane, t.idx_last));
    const u32x4 a0 = __builtin_nontemporal_load(q), a1 = __builtin_nontemporal_load(q + 1);
    U.q0 = make_uint4(a0.x, a0.y, a0.z, a0.w);
    U.q1 = make_uint4(a1.x, a1.y, a1.z, a1.w);
#pragma unroll
    for (int i = 0; i < 4; ++i) U.rows[i] = (uint32_t)t.prow[min(max(d.p0 + lane + 64 * i, 0), t.P - 1)];
    return U;
}

// Entry j (0..15) of a lane's two loads.
__device__ __forceinline__ uint32_t unit_entry(const UnitData& U, int j) {
    const uint32_t w[8] = {U.q0.x, U.q0.y, U.q0.z, U.q0.w, U.q1.x, U.q1.y, U.q1.z, U.q1.w};
    return (w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
}

// Cross-lane moves through DPP: the data moves within the VALU, with no LDS
// round trip (the shuffles they replace were the tiled sweep's critical
// path).  A lane whose source lane lies outside its row, or whose row is
// masked off, gets 0.  Controls: row_shr:n = 0x110 + n; row_bcast:15 = 0x142
// (lane 15 of each row to the next row; rows 1 and 3 written); row_bcast:31
// = 0x143 (lane 31 to rows 2 and 3); wave_shr:1 = 0x138.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int dpp_take(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_takef(float x) {
    return __int_as_float(dpp_take<CTRL, ROWS>(__float_as_int(x)));
}

// Inclusive prefix sum over the wavefront (all lanes active).
__device__ __forceinline__ int wave_incl_sum(int x) {
    x += dpp_take<0x111>(x);
    x += dpp_take<0x112>(x);
    x += dpp_take<0x114>(x);
    x += dpp_take<0x118>(x);
    x += dpp_take<0x142, 0xa>(x);
    x += dpp_take<0x143, 0xc>(x);
    return x;
}

// One step of an inclusive segmented scan: a lane that has not started a
// segment since the source lane adds the source's sum in front of its own.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ void seg_step(float& x, int& fresh) {
    const float xs = dpp_takef<CTRL, ROWS>(x);
    const int fs = dpp_take<CTRL, ROWS>(fresh);
    if (!fresh) {
        x = xs + x;
        fresh = fs;
    }
}

// Runs one unit (sums: this wavefront's 256 LDS words).
__device__ __forceinline__ void unit_run(const TileArgs& t, const UnitData& U, int lane, const float* lds, float* sums) {
    const SliceUnit& d = U.d;
    if (d.b <= d.a) return;
    const int32_t nvalid = min(max(d.b - (d.a + 16 * lane), 0), 16);
    float v[16];
    uint32_t heads = 0;  // bit j: entry j starts a segment
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t e = unit_entry(U, j);
        const bool ok = j < nvalid;
        v[j] = lds[ok ? (e & (kSegHead - 1)) : (uint32_t)t.W];  // lds[W] is zero
        if (ok && (e & kSegHead)) heads |= 1u << j;
    }
    if (d.p0 < 0) {  // a chunk of one long segment: sum everything
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc += v[j];
        acc = group_reduce<kWave>(acc);
        if (lane == 0) t.cpart[-d.p0 - 1] = acc;
        return;
    }
    // segment ordinals: exclusive prefix count of heads over the lanes
    const int nh = __popc(heads);
    const int incl = wave_incl_sum(nh);
    const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
    const int pref = incl - nh;
    // in-lane sums: segments that end inside the lane go to sums[ordinal];
    // `lead` (entries before the lane's first head) closes a segment of an
    // earlier lane, `run` ends as the tail (entries from the last head on),
    // or the whole lane without a head
    float run = 0.f, lead = 0.f;
    int k = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (heads & (1u << j)) {
            if (k == 0) lead = run;
            else sums[pref + k - 1] = run;
            run = 0.f;
            ++k;
        }
        run += v[j];
    }
    // forward segmented scan: `open` is what the segment open at the end of
    // this lane holds so far (a lane with a head starts afresh from its
    // tail).  A lane with a head closes the segment open at its start with
    // its lead; the last lane closes the one still open (units hold whole
    // segments).  Fixed order, no cancellation: the sum stays reproducible.
    float open = run;
    int fresh = nh ? 1 : 0;
    seg_step<0x111>(open, fresh);
    seg_step<0x112>(open, fresh);
    seg_step<0x114>(open, fresh);
    seg_step<0x118>(open, fresh);
    seg_step<0x142, 0xa>(open, fresh);
    seg_step<0x143, 0xc>(open, fresh);
    const float before = dpp_takef<0x138>(open);  // the segment open at this lane's start
    if (nh && pref > 0) sums[pref - 1] = before + lead;
    if (lane == kWave - 1 && total > 0) sums[total - 1] = open;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float* part = t.part + (size_t)d.slice * t.R;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (lane + 64 * i < total) __builtin_nontemporal_store(sums[lane + 64 * i], &part[(size_t)U.rows[i]]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // sums[] is rewritten by the next unit
}

// Tiles first: for each run of this workgroup's units (one slice each) the
// slice is staged, then wavefront w runs units u0 + w, u0 + w + waves, ...,
// each unit's loads issued while the previous one is summed.  Then the plain
// pull of the rows >= R with c[0, hot) staged.
template <bool HOT>
__global__ __launch_bounds__(1024) void k_pr_tiled(TileArgs t, PullArgs a) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t waves = blockDim.x / kWave;
    const int32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    float* sums = lds + t.W + 4 + wv * (kTiledWaveLds / 4);
    int32_t cur = -1;
    const int32_t r_end = uniform_load(t.wg, (int32_t)blockIdx.x + 1);
    for (int32_t r = uniform_load(t.wg, (int32_t)blockIdx.x); r < r_end; ++r) {
        const SliceSeg run = uniform_load(t.segs, r);
        if (run.slice != cur) {
            __syncthreads();  // every wavefront is done with the staged slice
            const int32_t s0 = run.slice * t.W;
            stage_lds(lds, t.c + s0, min(t.W, t.n - s0));
            if (threadIdx.x == 0) lds[t.W] = 0.f;
            __syncthreads();
            cur = run.slice;
        }
        // two unit buffers used in turn (never copied: a copy of registers a
        // load is still filling would wait for every load in flight)
        int32_t k = run.u0 + wv;
        if (k >= run.u1) continue;
        UnitData ua = unit_load(t, uniform_load(t.units, k), lane), ub;
        SliceUnit dn = (k + waves < run.u1) ? uniform_load(t.units, k + waves) : no_unit();
        for (;;) {
            ub = unit_load(t, dn, lane);
            dn = (k + 2 * waves < run.u1) ? uniform_load(t.units, k + 2 * waves) : no_unit();
            unit_run(t, ua, lane, lds, sums);
            k += waves;
            if (k >= run.u1) break;
            ua = unit_load(t, dn, lane);
            dn = (k + 2 * waves < run.u1) ? uniform_load(t.units, k + 2 * waves) : no_unit();
            unit_run(t, ub, lane, lds, sums);
            k += waves;
            if (k >= run.u1) break;
        }
    }
    if (a.units == 0) return;
    if (HOT) {
        __syncthreads();
        stage_lds(lds, a.c, a.hot);
    }
    __syncthreads();
    const int32_t nw = gridDim.x * waves;
    const int32_t first = __builtin_amdgcn_readfirstlane(blockIdx.x * waves + wv);
    pull_sweep<false, HOT>(a, lds, first, nw);
}

// Rows [0, R): y = teleport + the S slice partials in slice order (eight
// loads in flight) + the row's chunk partials in order, then the next
// contribution.  Blocks past those of [0, R) take the rows without in-edges
// at the end of the id range: y = teleport term (an empty sum, as a unit of
// the plain pull would give them).
__global__ __launch_bounds__(256) void k_pr_tiled_combine(TileArgs t, PullArgs a) {
    const int32_t bd = blockDim.x;
    const int32_t rb = (t.R + bd - 1) / bd;
    if ((int32_t)blockIdx.x >= rb) {
        const int32_t v = a.tail_beg + ((int32_t)blockIdx.x - rb) * bd + (int32_t)threadIdx.x;
        if (v < a.tail_end) pull_finish(a, v, 0.f);
        return;
    }
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= t.R) return;
    const float* p = t.part + u;
    float acc = 0.f;
    int32_t s = 0;
    for (; s + 8 <= t.S; s += 8) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = p[(size_t)(s + k) * t.R];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += v[k];
    }
    for (; s < t.S; ++s) acc += p[(size_t)s * t.R];
    for (int32_t ch = t.cbeg[u]; ch < t.cbeg[u + 1]; ++ch) acc += t.cpart[ch];
    pull_finish(a, u, acc);
}

// Hybrid sweep, rows of the hot targets (u < hot): y = base + the sum of the
// workgroups' LDS partials in fixed order, then the next contribution (or,
// after the last step, x in caller ids).  Block: 64 targets x 4 row groups.
__global__ __launch_bounds__(256) void k_pr_hyb_hot(int32_t hot, int32_t parts, const float* __restrict__ hot_part,
                                                    float base, const float* __restrict__ inv_s, float f,
                                                    float* __restrict__ c_next, float* __restrict__ x_out,
                                                    const int32_t* __restrict__ perm) {
    __shared__ float s[4][64];
    const int32_t u = blockIdx.x * 64 + (threadIdx.x & 63);
    const int r = threadIdx.x >> 6;
    float acc = 0.f;
    if (u < hot)
        for (int32_t b = r; b < parts; b += 4) acc += hot_part[(size_t)b * hot + u];
    s[r][threadIdx.x & 63] = acc;
    __syncthreads();
    if (r == 0 && u < hot) {
        const float yv = base + ((s[0][threadIdx.x] + s[1][threadIdx.x]) + (s[2][threadIdx.x] + s[3][threadIdx.x]));
        if (c_next) c_next[u] = f * yv * inv_s[u];
        if (x_out) x_out[user_id(perm, u)] = yv;
    }
}

// c[u] = f * x[caller id of u] / s(u); optionally y[u] = base (push accumulator).
__global__ void k_pr_prologue(int32_t n, const float* __restrict__ x, const int32_t* __restrict__ perm,
                              const float* __restrict__ inv_s, float f, float* __restrict__ c,
                              float* __restrict__ y_init, float base) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    c[u] = f * x[user_id(perm, u)] * inv_s[u];
    if (y_init) y_init[u] = base;
}

// After a push sweep: c[u] = f * y[u] / s(u); reset the other accumulator to
// the teleport term (base, plus tele on row tele_v); copy the iterate out
// (caller ids, x_out[id * x_stride]) on the last step.
__global__ void k_pr_push_epilogue(int32_t n, const float* __restrict__ y, const float* __restrict__ inv_s, float f,
                                   float* __restrict__ c, float* __restrict__ y_reset, float base, int32_t tele_v,
                                   float tele, float* __restrict__ x_out, int64_t x_stride,
                                   const int32_t* __restrict__ perm) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const float yv = y[u];
    if (c) c[u] = f * yv * inv_s[u];
    if (y_reset) y_reset[u] = base + ((u == tele_v) ? tele : 0.f);
    if (x_out) x_out[(int64_t)user_id(perm, u) * x_stride] = yv;
}

// Start of a personalised run from x_0 = e_s (s internal): c = f x_0 / s(.),
// and, for the push form, the accumulator preset to the teleport (1-f) e_s.
// With x_out (iters = 0) x_0 itself is written out instead.
__global__ void k_ppr1_init(int32_t n, int32_t s, const float* __restrict__ inv_s, float f, float* __restrict__ c,
                            float* __restrict__ y_init, float* __restrict__ x_out, int64_t x_stride,
                            const int32_t* __restrict__ perm) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    c[u] = (u == s) ? f * inv_s[u] : 0.f;
    if (y_init) y_init[u] = (u == s) ? 1.f - f : 0.f;
    if (x_out) x_out[(int64_t)user_id(perm, u) * x_stride] = (u == s) ? 1.f : 0.f;
}

// ------------------------------------------------------------------ launchers
static float teleport(int32_t n, float f) { return (float)((1.0 - (double)f) / (double)n); }

Teleport uniform_teleport(int32_t n, float f) { return Teleport{teleport(n, f), -1, 0.f, 1}; }

// ------------------------------------------------------------------ hybrid
// The hybrid sweep's push part, laid out like the pull sweep (persistent
// wavefront units over the out-degree bins, G lanes per row, U loads in
// flight per lane): every row u adds c[u] to its targets below `hot` in this
// workgroup's LDS accumulator; other targets are skipped (the pull part
// computes their rows).  The accumulators are written to part[blockIdx][hot].
template <int G, int U, bool W>
__device__ __forceinline__ void scatter_hot(const int32_t* __restrict__ idx, const float* __restrict__ wt, float cv,
                                            int32_t b, int32_t e, int lane, float* s_y, int32_t hot) {
    for (int32_t j0 = b + lane; j0 < e; j0 += U * G) {
        int32_t jj[U], ii[U];
#pragma unroll
        for (int k = 0; k < U; ++k) jj[k] = min(j0 + k * G, e - 1);
#pragma unroll
        for (int k = 0; k < U; ++k) ii[k] = idx[jj[k]];
        float wv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) wv[k] = W ? wt[jj[k]] : 1.f;
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (j0 + k * G < e && ii[k] < hot) atomicAdd(&s_y[ii[k]], W ? cv * wv[k] : cv);
    }
}

template <int BIN, bool W>
__device__ __forceinline__ void hyb_push_unit(const PullArgs& a, int32_t lu, int lane, float* s_y) {
    constexpr int G = kPullLanes[BIN];
    constexpr int U = kPullLoads[BIN];
    const int32_t i = lu * (kWave / G) + lane / G;
    const int32_t count = a.sp.list_off[BIN + 1] - a.sp.list_off[BIN];
    if (i >= count) return;  // whole groups leave together
    const int32_t u = a.list[a.sp.list_off[BIN] + i];
    const float cv = a.c[u];
    if (cv == 0.f) return;
    scatter_hot<G, U, W>(a.idx, a.wt, cv, a.off[u], a.off[u + 1], lane & (G - 1), s_y, a.hot);
}

template <bool W>
__global__ __launch_bounds__(1024) void k_pr_hyb_push(PullArgs a) {
    extern __shared__ float s_y[];
    for (int32_t i = threadIdx.x; i < a.hot; i += blockDim.x) s_y[i] = 0.f;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t nw = gridDim.x * (blockDim.x / kWave);
    for (int32_t unit = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; unit < a.units; unit += nw) {
        const int bin = wave_unit_bin(a.wave_off, unit);
        const int32_t lu = unit - a.wave_off[bin];
        switch (bin) {
            case 5: {  // one chunk of a very long row
                const int32_t v = a.tab[lu];
                const float cv = a.c[v];
                if (cv != 0.f)
                    scatter_hot<kPullLanes[5], kPullLoads[5], W>(a.idx, a.wt, cv, a.tab[a.tab_cap + lu],
                                                                a.tab[2 * a.tab_cap + lu], lane, s_y, a.hot);
                break;
            }
            case 4: hyb_push_unit<4, W>(a, lu, lane, s_y); break;
            case 3: hyb_push_unit<3, W>(a, lu, lane, s_y); break;
            case 2: hyb_push_unit<2, W>(a, lu, lane, s_y); break;
            case 1: hyb_push_unit<1, W>(a, lu, lane, s_y); break;
            default: hyb_push_unit<0, W>(a, lu, lane, s_y); break;
        }
    }
    __syncthreads();
    float* dst = a.part + (size_t)blockIdx.x * a.hot;
    for (int32_t i = threadIdx.x; i < a.hot; i += blockDim.x) dst[i] = s_y[i];
}

// Launches the hybrid push part; *parts = its workgroups (rows of hot_part).
pp_status launch_hyb_push(pp_graph g, const float* c, int32_t hot, hipStream_t st, int32_t* parts) {
    PullArgs a{};
    a.sp = sweep_plan(g->push_plan);
    a.off = g->d.csr_off;
    a.idx = g->d.csr_idx;
    a.wt = g->d.csr_w;
    a.list = g->d.push_list;
    a.tab_cap = g->split_cap;
    a.tab = g->d.split_tab + 4 * (size_t)a.tab_cap + 1;
    a.part = g->d.hot_part;
    a.c = c;
    a.hot = hot;
    for (int b = 0; b <= PP_NUM_BINS; ++b) a.wave_off[b] = g->push_plan.wave_off[b];
    a.units = g->push_plan.total_wave_units;
    const int32_t tpb = 1024;
    const size_t lds = (size_t)hot * sizeof(float);
    int32_t per_cu = std::max(1, std::min<int32_t>(2, (int32_t)(g->lds_per_cu / std::max<size_t>(lds, 1))));
    const int32_t grid =
        std::max(1, std::min(std::min(g->num_cu * per_cu, ceil_div(a.units, tpb / kWave)), g->tune.push_blocks));
    *parts = grid;
    allow_dynamic_lds(reinterpret_cast<const void*>(g->weighted ? &k_pr_hyb_push<true> : &k_pr_hyb_push<false>), lds);
    if (g->weighted) hipLaunchKernelGGL((k_pr_hyb_push<true>), dim3(grid), dim3(tpb), lds, st, a);
    else hipLaunchKernelGGL((k_pr_hyb_push<false>), dim3(grid), dim3(tpb), lds, st, a);
    PP_LAUNCH_CHECK("k_pr_hyb_push");
    return PP_OK;
}

// Fields common to every pull launch.
static PullArgs pull_args(pp_graph g, const float* c, float* c_next, float* y, float f, int32_t skip_below,
                          const Teleport& tp) {
    PullArgs a{};
    a.skip_below = skip_below;
    a.sp = sweep_plan(g->pull_plan);
    a.off = g->d.csc_off;
    a.idx = g->d.csc_idx;
    a.wt = g->d.csc_w;
    a.list = g->d.pull_list;
    a.tab_cap = g->split_cap;
    a.tab = g->d.split_tab;
    a.tab0 = 0;
    a.part = g->d.split_part;
    a.c = c;
    a.inv_s = g->d.inv_s;
    a.perm = g->d.perm;
    a.c_next = c_next;
    a.y = y;
    a.y_stride = tp.y_stride;
    a.base = tp.base;
    a.tele_v = tp.vertex;
    a.tele = tp.extra;
    a.f = f;
    const int32_t lds_cap = std::max(g->max_lds, 0) / (int32_t)sizeof(float);
    a.hot = std::min(std::min(g->tune.pull_hot, g->d.n), lds_cap);
    return a;
}

pp_status launch_pull(pp_graph g, const float* c, float* c_next, float* y, float f, hipStream_t st,
                      int32_t skip_below, const Teleport* tpp) {
    const Teleport tp = tpp ? *tpp : uniform_teleport(g->d.n, f);
    PullArgs a = pull_args(g, c, c_next, y, f, skip_below, tp);
    const int32_t tpb = g->tune.pull_block;
    const SlicePlan& sl = g->slices;
    const BinPlan& pp_ = g->pull_plan;
    const bool hot = a.hot > 0;
    if (sl.rows > 0 && skip_below == 0 && !g->weighted) {
        // tiled rows [0, R), then the plain pull of the other rows in the same launch
        for (int b = 0; b < PP_NUM_BINS; ++b) {
            a.list_beg[b] = pp_.list_off[b] + sl.list_skip[b];
            a.list_cnt[b] = pp_.count[b] - sl.list_skip[b];
        }
        a.list_cnt[0] -= sl.tail;
        a.tail_beg = g->d.n - sl.tail;
        a.tail_end = g->d.n;
        for (int b = 0; b <= PP_NUM_BINS; ++b) a.wave_off[b] = sl.wave_off[b];
        a.units = sl.units;
        a.tab0 = sl.tab0;
        // named fields: a positional initializer silently shifts when a field is added
        TileArgs t{};
        t.idx = g->d.sl_idx;
        t.prow = g->d.sl_prow;
        t.units = g->d.sl_units;
        t.segs = g->d.sl_segs;
        t.wg = g->d.sl_wg;
        t.part = g->d.sl_part;
        t.cpart = g->d.sl_cpart;
        t.cbeg = g->d.sl_cbeg;
        t.c = c;
        t.n = g->d.n;
        t.R = sl.rows;
        t.W = sl.width;
        t.S = sl.slices;
        t.P = std::max(sl.pairs, 1);
        t.idx_last = sl.idx_size - 16;
        // the slice with its per-wavefront words, or the hot range of the rest
        const size_t lds = std::max(tiled_lds_bytes(sl.width, tpb / kWave), (size_t)a.hot * sizeof(float));
        if (hot) {
            allow_dynamic_lds(reinterpret_cast<const void*>(&k_pr_tiled<true>), lds);
            hipLaunchKernelGGL((k_pr_tiled<true>), dim3(sl.groups), dim3(tpb), lds, st, t, a);
        } else {
            allow_dynamic_lds(reinterpret_cast<const void*>(&k_pr_tiled<false>), lds);
            hipLaunchKernelGGL((k_pr_tiled<false>), dim3(sl.groups), dim3(tpb), lds, st, t, a);
        }
        hipLaunchKernelGGL(k_pr_tiled_combine, dim3(ceil_div(sl.rows, 256) + ceil_div(sl.tail, 256)), dim3(256), 0,
                           st, t, a);
        if (sl.nsplit > 0)
            hipLaunchKernelGGL(k_pr_pull_fix, dim3(ceil_div(sl.nsplit, 64)), dim3(64), 0, st, a, sl.nsplit, sl.fix0);
        PP_LAUNCH_CHECK("k_pr_tiled");
        return PP_OK;
    }
    for (int b = 0; b < PP_NUM_BINS; ++b) {
        a.list_beg[b] = pp_.list_off[b];
        a.list_cnt[b] = pp_.count[b];
    }
    for (int b = 0; b <= PP_NUM_BINS; ++b) a.wave_off[b] = pp_.wave_off[b];
    a.units = pp_.total_wave_units;
    if (a.units > 0) {
        // one workgroup per compute unit (more when they are small), never more than the work
        const size_t lds = hot ? (size_t)a.hot * sizeof(float) : 0;
        // as many workgroups per compute unit as 32 wavefronts and the LDS allow
        int32_t per_cu = std::max(2048 / tpb, 1);
        if (lds > 0) per_cu = std::max(1, std::min<int32_t>(per_cu, (int32_t)(g->lds_per_cu / lds)));
        const int32_t grid = std::max(1, std::min(g->num_cu * per_cu, ceil_div(a.units, tpb / kWave)));
        if (hot)
            allow_dynamic_lds(
                reinterpret_cast<const void*>(g->weighted ? &k_pr_pull<true, true> : &k_pr_pull<false, true>), lds);
        if (g->weighted) {
            if (hot) hipLaunchKernelGGL((k_pr_pull<true, true>), dim3(grid), dim3(tpb), lds, st, a);
            else hipLaunchKernelGGL((k_pr_pull<true, false>), dim3(grid), dim3(tpb), 0, st, a);
        } else {
            if (hot) hipLaunchKernelGGL((k_pr_pull<false, true>), dim3(grid), dim3(tpb), lds, st, a);
            else hipLaunchKernelGGL((k_pr_pull<false, false>), dim3(grid), dim3(tpb), 0, st, a);
        }
    }
    const int32_t nsplit = pp_.count[5];
    if (nsplit > 0) hipLaunchKernelGGL(k_pr_pull_fix, dim3(ceil_div(nsplit, 64)), dim3(64), 0, st, a, nsplit, 0);
    PP_LAUNCH_CHECK("k_pr_pull");
    return PP_OK;
}

// One personalised column with the single-vector sweeps: x_0 = e_s (s
// internal), iters steps of x <- (1-f) e_s + f P x in direction dir (PP_PULL
// or PP_PUSH), x_iters written to x_out[caller id * x_stride].  Uses the
// graph's iterate buffers, like pp_pr_run.
pp_status run_single_ppr(pp_graph g, pp_dir dir, int32_t s, int32_t iters, float f, float* x_out, int64_t x_stride,
                         hipStream_t st) {
    const int32_t n = g->d.n;
    const dim3 vb(ceil_div(n, 256)), vt(256);
    const float tele = 1.f - f;
    float* c = g->d.buf0;
    if (iters == 0) {
        hipLaunchKernelGGL(k_ppr1_init, vb, vt, 0, st, n, s, g->d.inv_s, f, c, (float*)nullptr, x_out, x_stride,
                           g->d.perm);
        PP_LAUNCH_CHECK("k_ppr1_init");
        return PP_OK;
    }
    if (dir == PP_PULL) {
        const Teleport tp{0.f, s, tele, x_stride};
        float* cn = g->d.buf1;
        hipLaunchKernelGGL(k_ppr1_init, vb, vt, 0, st, n, s, g->d.inv_s, f, c, (float*)nullptr, (float*)nullptr,
                           (int64_t)0, g->d.perm);
        PP_LAUNCH_CHECK("k_ppr1_init");
        for (int32_t t = 0; t < iters; ++t) {
            const bool last = (t == iters - 1);
            pp_status r = launch_pull(g, c, last ? nullptr : cn, last ? x_out : nullptr, f, st, 0, &tp);
            if (r != PP_OK) return r;
            std::swap(c, cn);
        }
        return PP_OK;
    }
    float* ya = g->d.buf1;
    float* yb = g->d.buf2;
    hipLaunchKernelGGL(k_ppr1_init, vb, vt, 0, st, n, s, g->d.inv_s, f, c, ya, (float*)nullptr, (int64_t)0,
                       g->d.perm);
    PP_LAUNCH_CHECK("k_ppr1_init");
    for (int32_t t = 0; t < iters; ++t) {
        const bool last = (t == iters - 1);
        pp_status r = launch_push(g, c, ya, st);
        if (r != PP_OK) return r;
        hipLaunchKernelGGL(k_pr_push_epilogue, vb, vt, 0, st, n, (const float*)ya, g->d.inv_s, f,
                           last ? nullptr : c, last ? nullptr : yb, 0.f, s, tele, last ? x_out : nullptr, x_stride,
                           g->d.perm);
        PP_LAUNCH_CHECK("k_pr_push_epilogue");
        std::swap(ya, yb);
    }
    return PP_OK;
}

static pp_status check_pr_args(pp_graph g, const void* x, const void* y, float f) {
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (!x || !y) return set_error(PP_E_NULL, "x and y are required");
    if (x == y) return set_error(PP_E_RANGE, "x and y must be distinct buffers");
    if (!(f >= 0.f && f < 1.f)) return set_error(PP_E_RANGE, "f must lie in [0, 1)");
    return PP_OK;
}

}  // namespace pp

using namespace pp;

PP_EXPORT pp_status pp_pr_pull(pp_graph g, const float* x, float* y, float f, void* stream) {
    clear_error();
    pp_status s = check_pr_args(g, x, y, f);
    if (s != PP_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t n = g->d.n;
    hipLaunchKernelGGL(k_pr_prologue, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, x, g->d.perm, g->d.inv_s, f,
                       g->d.buf0, (float*)nullptr, 0.f);
    PP_LAUNCH_CHECK("k_pr_prologue");
    return launch_pull(g, g->d.buf0, nullptr, y, f, st);
}

PP_EXPORT pp_status pp_pr_push(pp_graph g, const float* x, float* y, float f, void* stream) {
    clear_error();
    pp_status s = check_pr_args(g, x, y, f);
    if (s != PP_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t n = g->d.n;
    const dim3 vb(ceil_div(n, 256)), vt(256);
    hipLaunchKernelGGL(k_pr_prologue, vb, vt, 0, st, n, x, g->d.perm, g->d.inv_s, f, g->d.buf0, g->d.buf1,
                       teleport(n, f));
    PP_LAUNCH_CHECK("k_pr_prologue");
    s = launch_push(g, g->d.buf0, g->d.buf1, st);
    if (s != PP_OK) return s;
    hipLaunchKernelGGL(k_pr_push_epilogue, vb, vt, 0, st, n, (const float*)g->d.buf1, g->d.inv_s, f, (float*)nullptr,
                       (float*)nullptr, 0.f, -1, 0.f, y, (int64_t)1, g->d.perm);
    PP_LAUNCH_CHECK("k_pr_push_epilogue");
    return PP_OK;
}

PP_EXPORT pp_status pp_pr_run(pp_graph g, pp_dir dir, int32_t iters, float f, float* x_inout, void* stream) {
    clear_error();
    if (!g) return set_error(PP_E_NULL, "graph handle is NULL");
    if (!x_inout) return set_error(PP_E_NULL, "x_inout is required");
    if (!(f >= 0.f && f < 1.f)) return set_error(PP_E_RANGE, "f must lie in [0, 1)");
    if (iters < 0) return set_error(PP_E_RANGE, "iters must be >= 0");
    if (dir != PP_PUSH && dir != PP_PULL && dir != PP_SWITCH)
        return set_error(PP_E_RANGE, "dir must be PP_PUSH, PP_PULL or PP_SWITCH");
    if (iters == 0) return PP_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t n = g->d.n;
    const float base = teleport(n, f);
    const dim3 vb(ceil_div(n, 256)), vt(256);
    if (dir == PP_SWITCH) {
        // hybrid: edges into the first `hot` vertices are pushed into LDS
        // accumulators (no global atomics), all other rows pull
        const int32_t hot = std::min(g->tune.hot, n);
        float* c = g->d.buf0;
        float* cn = g->d.buf1;
        hipLaunchKernelGGL(k_pr_prologue, vb, vt, 0, st, n, (const float*)x_inout, g->d.perm, g->d.inv_s, f, c,
                           (float*)nullptr, 0.f);
        PP_LAUNCH_CHECK("k_pr_prologue");
        for (int32_t t = 0; t < iters; ++t) {
            const bool last = (t == iters - 1);
            if (hot > 0 && g->push_plan.total_wave_units > 0) {
                int32_t parts = 0;  // workgroups of the push part = rows of hot_part
                pp_status s = launch_hyb_push(g, c, hot, st, &parts);
                if (s != PP_OK) return s;
                hipLaunchKernelGGL(k_pr_hyb_hot, dim3(ceil_div(hot, 64)), dim3(256), 0, st, hot, parts,
                                   (const float*)g->d.hot_part, base, g->d.inv_s, f, last ? nullptr : cn,
                                   last ? x_inout : nullptr, g->d.perm);
            } else if (hot > 0) {  // no edges at all: the hot rows are the teleport alone
                hipLaunchKernelGGL(k_pr_hyb_hot, dim3(ceil_div(hot, 64)), dim3(256), 0, st, hot, 0,
                                   (const float*)g->d.hot_part, base, g->d.inv_s, f, last ? nullptr : cn,
                                   last ? x_inout : nullptr, g->d.perm);
            }
            pp_status s = launch_pull(g, c, last ? nullptr : cn, last ? x_inout : nullptr, f, st, hot);
            if (s != PP_OK) return s;
            PP_LAUNCH_CHECK("k_pr_hyb_hot");
            float* tmp = c;
            c = cn;
            cn = tmp;
        }
        return PP_OK;
    }
    if (dir == PP_PULL) {
        float* c = g->d.buf0;
        float* cn = g->d.buf1;
        hipLaunchKernelGGL(k_pr_prologue, vb, vt, 0, st, n, (const float*)x_inout, g->d.perm, g->d.inv_s, f, c,
                           (float*)nullptr, 0.f);
        PP_LAUNCH_CHECK("k_pr_prologue");
        for (int32_t t = 0; t < iters; ++t) {
            const bool last = (t == iters - 1);
            pp_status s = launch_pull(g, c, last ? nullptr : cn, last ? x_inout : nullptr, f, st);
            if (s != PP_OK) return s;
            float* tmp = c;
            c = cn;
            cn = tmp;
        }
        return PP_OK;
    }
    float* c = g->d.buf0;
    float* ya = g->d.buf1;
    float* yb = g->d.buf2;
    hipLaunchKernelGGL(k_pr_prologue, vb, vt, 0, st, n, (const float*)x_inout, g->d.perm, g->d.inv_s, f, c, ya, base);
    PP_LAUNCH_CHECK("k_pr_prologue");
    for (int32_t t = 0; t < iters; ++t) {
        const bool last = (t == iters - 1);
        pp_status s = launch_push(g, c, ya, st);
        if (s != PP_OK) return s;
        hipLaunchKernelGGL(k_pr_push_epilogue, vb, vt, 0, st, n, (const float*)ya, g->d.inv_s, f,
                           last ? nullptr : c, last ? nullptr : yb, base, -1, 0.f, last ? x_inout : nullptr,
                           (int64_t)1, g->d.perm);
        PP_LAUNCH_CHECK("k_pr_push_epilogue");
        float* tmp = ya;
        ya = yb;
        yb = tmp;
    }
    return PP_OK;
}
