/*
 * graphgen.c -- seeded synthetic graph inputs.
 *
 * This module only manufactures INPUTS: edge lists drawn from R-MAT,
 * Erdos-Renyi and 2D-grid models, their canonical adjacency-array form
 * (Sec. 2.2 of the paper: per-vertex neighbour arrays concatenated into
 * one array, plus per-vertex offsets), and seeded vectors (edge weights,
 * Gaussian loss coefficients, vertex picks).  It contains none of the
 * arithmetic of PageRank or BFS; both the product path and the oracle
 * consume what it produces.
 *
 * Random numbers come from one counter-based generator: the SplitMix64
 * output function (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) evaluated at state = key + (ctr+1)*G,
 * with key = mix(seed ^ mix(stream)) and G = 0x9E3779B97F4A7C15.  Any
 * element can therefore be regenerated independently of the others, and
 * OpenMP threads produce the same stream as a serial loop.
 *
 * All functions return 0 on success and a negative code on bad arguments.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t gg_key(uint64_t seed, uint64_t stream) {
    return gg_mix(seed ^ gg_mix(stream + GG_GAMMA));
}

static inline uint64_t gg_at(uint64_t key, uint64_t ctr) {
    return gg_mix(key + (ctr + 1) * GG_GAMMA);
}

/* Exposed so that tests can check the generator against its definition. */
uint64_t gg_rand(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return gg_at(gg_key(seed, stream), ctr);
}

/* Unbiased-enough bounded draw: high 64 bits of r * bound (Lemire's
 * multiply-shift reduction, without the rejection step; the bias is below
 * bound / 2^64 and irrelevant for graph sizes below 2^32). */
static inline uint64_t gg_bounded(uint64_t r, uint64_t bound) {
    return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

/* ------------------------------------------------------------------ */
/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each edge descends `scale`
 * levels of the adjacency matrix, choosing quadrant (0,0),(0,1),(1,0),(1,1)
 * with probabilities a, b, c, d = 1-a-b-c.  Level l fixes bit (scale-1-l)
 * of the source and of the destination.  Two 32-bit draws per 64-bit word.
 * No noise, no vertex permutation: vertex 0 is the heaviest vertex.      */
int gg_rmat_edges(int scale, int64_t num_edges, double a, double b, double c,
                  uint64_t seed, int32_t* src, int32_t* dst) {
    if (scale < 1 || scale > 30 || num_edges < 0 || !src || !dst) return -1;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -2;
    const uint64_t key = gg_key(seed, 1);
    const double two32 = 4294967296.0;
    const uint64_t tA = (uint64_t)(a * two32);
    const uint64_t tB = (uint64_t)((a + b) * two32);
    const uint64_t tC = (uint64_t)((a + b + c) * two32);
    const int words = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < num_edges; ++e) {
        uint32_t s = 0, t = 0;
        for (int w = 0; w < words; ++w) {
            uint64_t r = gg_at(key, (uint64_t)e * (uint64_t)words + (uint64_t)w);
            for (int h = 0; h < 2; ++h) {
                int l = 2 * w + h;
                if (l >= scale) break;
                uint64_t u = (h == 0) ? (r & 0xFFFFFFFFULL) : (r >> 32);
                uint32_t bs = 0, bt = 0;
                if (u < tA) { bs = 0; bt = 0; }
                else if (u < tB) { bs = 0; bt = 1; }
                else if (u < tC) { bs = 1; bt = 0; }
                else { bs = 1; bt = 1; }
                int bit = scale - 1 - l;
                s |= bs << bit;
                t |= bt << bit;
            }
        }
        src[e] = (int32_t)s;
        dst[e] = (int32_t)t;
    }
    return 0;
}

/* G(n, M)-style Erdos-Renyi draw: num_edges independent uniform pairs. */
int gg_er_edges(int64_t n, int64_t num_edges, uint64_t seed, int32_t* src, int32_t* dst) {
    if (n < 1 || n > 0x7fffffff || num_edges < 0 || !src || !dst) return -1;
    const uint64_t key = gg_key(seed, 2);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < num_edges; ++e) {
        src[e] = (int32_t)gg_bounded(gg_at(key, 2 * (uint64_t)e), (uint64_t)n);
        dst[e] = (int32_t)gg_bounded(gg_at(key, 2 * (uint64_t)e + 1), (uint64_t)n);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

static void sort_row(int32_t* p, int64_t len) {
    if (len < 24) {
        for (int64_t i = 1; i < len; ++i) {
            int32_t v = p[i];
            int64_t j = i - 1;
            while (j >= 0 && p[j] > v) { p[j + 1] = p[j]; --j; }
            p[j + 1] = v;
        }
    } else {
        qsort(p, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/*
 * Canonical adjacency array from an edge list: drop self-loops, optionally
 * add the reverse of every edge (symmetrise), sort each neighbour array
 * ascending and remove duplicates.  Output: off[n+1] (int64) and the first
 * off[n] entries of idx_work, which must hold `sym ? 2*E : E` int32s.
 * Returns the number of stored directed entries (nnz), or < 0 on error.
 */
int64_t gg_build_adjacency(int64_t n, int64_t num_edges, const int32_t* src, const int32_t* dst,
                           int sym, int64_t* off, int32_t* idx_work) {
    if (n < 1 || num_edges < 0 || !src || !dst || !off || !idx_work) return -1;
    int64_t* cur = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* len = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    if (!cur || !len) { free(cur); free(len); return -3; }
    for (int64_t e = 0; e < num_edges; ++e) {
        int32_t s = src[e], t = dst[e];
        if (s < 0 || s >= n || t < 0 || t >= n) { free(cur); free(len); return -2; }
        if (s == t) continue;
        cur[s + 1]++;
        if (sym) cur[t + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) cur[v + 1] += cur[v];
    int64_t* start = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!start) { free(cur); free(len); return -3; }
    memcpy(start, cur, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < num_edges; ++e) {
        int32_t s = src[e], t = dst[e];
        if (s == t) continue;
        idx_work[cur[s]++] = t;
        if (sym) idx_work[cur[t]++] = s;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n; ++v) {
        int32_t* p = idx_work + start[v];
        int64_t l = start[v + 1] - start[v];
        sort_row(p, l);
        int64_t k = 0;
        for (int64_t i = 0; i < l; ++i)
            if (k == 0 || p[i] != p[k - 1]) p[k++] = p[i];
        len[v] = k;
    }
    /* Compact left in vertex order; destinations never pass sources. */
    int64_t pos = 0;
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (pos != start[v]) memmove(idx_work + pos, idx_work + start[v], (size_t)len[v] * sizeof(int32_t));
        pos += len[v];
        off[v + 1] = pos;
    }
    free(start); free(cur); free(len);
    return pos;
}

/*
 * rows x cols 4-neighbour grid, row-major ids (vertex 0 is a corner), with
 * exactly `remove` of its 2*rows*cols-rows-cols undirected edges deleted.
 * The deleted set is the first `remove` positions of a seeded partial
 * Fisher-Yates shuffle of the edge ids (horizontal edges first, then
 * vertical).  Writes the symmetric adjacency array (rows sorted).
 * off has rows*cols+1 entries, idx capacity 4*rows*cols.  Returns nnz.
 */
int64_t gg_grid(int64_t rows, int64_t cols, int64_t remove, uint64_t seed, int64_t* off, int32_t* idx) {
    if (rows < 1 || cols < 1 || rows * cols > 0x7fffffff || !off || !idx) return -1;
    const int64_t nh = rows * (cols - 1), nv = (rows - 1) * cols, ne = nh + nv;
    if (remove < 0 || remove > ne) return -2;
    int32_t* perm = (int32_t*)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(int32_t));
    uint8_t* gone = (uint8_t*)calloc((size_t)(ne > 0 ? ne : 1), 1);
    if (!perm || !gone) { free(perm); free(gone); return -3; }
    for (int64_t i = 0; i < ne; ++i) perm[i] = (int32_t)i;
    const uint64_t key = gg_key(seed, 3);
    for (int64_t i = 0; i < remove; ++i) {
        int64_t j = i + (int64_t)gg_bounded(gg_at(key, (uint64_t)i), (uint64_t)(ne - i));
        int32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
        gone[perm[i]] = 1;
    }
    free(perm);
    const int64_t n = rows * cols;
    int64_t pos = 0;
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t r = v / cols, c = v % cols;
        /* neighbours in ascending id order: up, left, right, down */
        if (r > 0 && !gone[nh + (r - 1) * cols + c]) idx[pos++] = (int32_t)(v - cols);
        if (c > 0 && !gone[r * (cols - 1) + c - 1]) idx[pos++] = (int32_t)(v - 1);
        if (c < cols - 1 && !gone[r * (cols - 1) + c]) idx[pos++] = (int32_t)(v + 1);
        if (r < rows - 1 && !gone[nh + r * cols + c]) idx[pos++] = (int32_t)(v + cols);
        off[v + 1] = pos;
    }
    free(gone);
    return pos;
}

/* ------------------------------------------------------------------ */
/* out[i] = lo + (hi-lo)*u_i, u_i a 24-bit uniform in [0,1). */
int gg_uniform_f32(uint64_t seed, uint64_t stream, int64_t count, float lo, float hi, float* out) {
    if (count < 0 || !out) return -1;
    const uint64_t key = gg_key(seed, 100 + stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        double u = (double)(gg_at(key, (uint64_t)i) >> 40) * (1.0 / 16777216.0);
        out[i] = (float)(lo + (hi - lo) * u);
    }
    return 0;
}

/* Standard normals by the Box-Muller transform (one value per pair). */
int gg_normal_f32(uint64_t seed, uint64_t stream, int64_t count, float* out) {
    if (count < 0 || !out) return -1;
    const uint64_t key = gg_key(seed, 200 + stream);
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        double u1 = ((double)(gg_at(key, 2 * (uint64_t)i) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
        double u2 = (double)(gg_at(key, 2 * (uint64_t)i + 1) >> 11) * (1.0 / 9007199254740992.0);
        out[i] = (float)(sqrt(-2.0 * log(u1)) * cos(two_pi * u2));
    }
    return 0;
}

/* `count` distinct vertices with off[v+1] > off[v] (non-isolated when
 * min_deg >= 1), in draw order.  Returns -4 when not enough exist. */
int gg_pick_vertices(uint64_t seed, uint64_t stream, int64_t n, const int64_t* off, int64_t min_deg,
                     int64_t count, int32_t* out) {
    if (n < 1 || count < 0 || !off || (count > 0 && !out)) return -1;
    int64_t eligible = 0;
    for (int64_t v = 0; v < n; ++v) eligible += (off[v + 1] - off[v] >= min_deg);
    if (eligible < count) return -4;
    uint8_t* taken = (uint8_t*)calloc((size_t)n, 1);
    if (!taken) return -3;
    const uint64_t key = gg_key(seed, 300 + stream);
    int64_t got = 0;
    for (uint64_t ctr = 0; got < count; ++ctr) {
        int64_t v = (int64_t)gg_bounded(gg_at(key, ctr), (uint64_t)n);
        if (taken[v] || off[v + 1] - off[v] < min_deg) continue;
        taken[v] = 1;
        out[got++] = (int32_t)v;
    }
    free(taken);
    return 0;
}

/* Integers uniform in [lo, hi] (inclusive). */
int gg_uniform_int(uint64_t seed, uint64_t stream, int64_t count, int64_t lo, int64_t hi, int64_t* out) {
    if (count < 0 || hi < lo || !out) return -1;
    const uint64_t key = gg_key(seed, 400 + stream);
    for (int64_t i = 0; i < count; ++i)
        out[i] = lo + (int64_t)gg_bounded(gg_at(key, (uint64_t)i), (uint64_t)(hi - lo + 1));
    return 0;
}
