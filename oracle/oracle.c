/*
 * oracle.c -- plain, slow, sequential FP64 reference for the push/pull sweeps.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; it derives everything it
 * needs (degrees, in-adjacency) from the out-adjacency array it is given.
 *
 * Graph input: the adjacency array of Sec. 2.2 -- off[n+1] (int64) and
 * idx[off[n]] (int32); row v lists the targets of the edges leaving v.
 * d(v) = off[v+1]-off[v] is the out-degree.
 *
 * Readings of the paper used here (the text is silent or loose on these):
 *  - PageRank (Sec. 3.1 equation): x_{t+1}(u) = (1-f)/n + f * sum over edges
 *    (v,u) of x_t(v)/d(v).  Jacobi: x_{t+1} depends only on x_t.  A vertex with
 *    d(v)=0 contributes nothing; its mass is not redistributed.
 *  - x_0 = 1/n unless given; "T iterations" = T applications of the update.
 *  - BFS (Sec. 3.3 and the generalised BFS of Sec. 4.3 with every ready
 *    counter equal to one): level = hop distance from the root, -1 when
 *    unreachable; parent[root] = root, parent = -1 when unreachable.
 *  - Personalised PageRank (not defined in the paper): teleport (1-f)*e_s,
 *    x_0 = e_s; weighted transition P_uv = w(v->u)/s(v), s(v) = sum of the
 *    weights leaving v (unweighted: w = 1, s = d).
 *  - Adjoint (not in the paper): for the fixed point x = (1-f)e_s + f P x and
 *    L(X), Lambda solves (I - f P^T) Lambda = dL/dX and
 *    dL/dw(v->u) = (f/s(v)) * sum_j X[v,j] * (Lambda[u,j] - (P^T Lambda)[v,j]).
 *
 * All functions return 0 on success, < 0 on bad input or allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

/* In-adjacency (transpose) by a counting sort over destinations, scanning
 * sources in ascending order so each in-row lists sources ascending.
 * in_slot[j] = position in idx of the same directed edge. */
static int transpose(int64_t n, const int64_t* off, const int32_t* idx,
                     int64_t** in_off_p, int32_t** in_idx_p, int64_t** in_slot_p) {
    int64_t nnz = off[n];
    int64_t* in_off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* cur = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t* in_idx = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int64_t* in_slot = in_slot_p ? (int64_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t)) : NULL;
    if (!in_off || !cur || !in_idx || (in_slot_p && !in_slot)) {
        free(in_off); free(cur); free(in_idx); free(in_slot);
        return -3;
    }
    for (int64_t e = 0; e < nnz; ++e) {
        if (idx[e] < 0 || idx[e] >= n) { free(in_off); free(cur); free(in_idx); free(in_slot); return -2; }
        in_off[idx[e] + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) in_off[v + 1] += in_off[v];
    memcpy(cur, in_off, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int64_t p = cur[idx[e]]++;
            in_idx[p] = (int32_t)v;
            if (in_slot) in_slot[p] = e;
        }
    free(cur);
    *in_off_p = in_off;
    *in_idx_p = in_idx;
    if (in_slot_p) *in_slot_p = in_slot;
    return 0;
}

static int check_graph(int64_t n, const int64_t* off, const int32_t* idx) {
    if (n < 1 || !off || (off[n] > 0 && !idx)) return -1;
    if (off[0] != 0) return -2;
    for (int64_t v = 0; v < n; ++v)
        if (off[v + 1] < off[v]) return -2;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* PageRank, pulling form (Sec. 3.1 equation; Sec. 4.1 pulling update):
 * every vertex u sums x_t(v)/d(v) over its in-neighbours v. */
int orc_pagerank(int64_t n, const int64_t* off, const int32_t* idx, double f, int T,
                 const double* x0, double* x_out) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (T < 0 || !x_out) return -1;
    int64_t* in_off;
    int32_t* in_idx;
    if ((rc = transpose(n, off, idx, &in_off, &in_idx, NULL))) return rc;
    double* x = (double*)malloc((size_t)n * sizeof(double));
    double* y = (double*)malloc((size_t)n * sizeof(double));
    if (!x || !y) { free(x); free(y); free(in_off); free(in_idx); return -3; }
    for (int64_t v = 0; v < n; ++v) x[v] = x0 ? x0[v] : 1.0 / (double)n;
    const double base = (1.0 - f) / (double)n;
    for (int t = 0; t < T; ++t) {
        for (int64_t u = 0; u < n; ++u) {
            double acc = 0.0;
            for (int64_t j = in_off[u]; j < in_off[u + 1]; ++j) {
                int32_t v = in_idx[j];
                acc += x[v] / (double)(off[v + 1] - off[v]);
            }
            y[u] = base + f * acc;
        }
        double* tmp = x; x = y; y = tmp;
    }
    memcpy(x_out, x, (size_t)n * sizeof(double));
    free(x); free(y); free(in_off); free(in_idx);
    return 0;
}

/* The pulling form above with its row loop split over threads (OpenMP).
 * Every row is still summed by one thread in in-row order, so the result is
 * bit-identical to orc_pagerank; only the wall time differs.  Used to time the
 * oracle on all host cores (the pulling form has no write conflicts, Sec. 4.1).
 * *threads_out (nullable) receives the number of threads of the team. */
int orc_pagerank_threads(int64_t n, const int64_t* off, const int32_t* idx, double f, int T,
                         const double* x0, double* x_out, int* threads_out) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (T < 0 || !x_out) return -1;
    int64_t* in_off;
    int32_t* in_idx;
    if ((rc = transpose(n, off, idx, &in_off, &in_idx, NULL))) return rc;
    double* x = (double*)malloc((size_t)n * sizeof(double));
    double* y = (double*)malloc((size_t)n * sizeof(double));
    if (!x || !y) { free(x); free(y); free(in_off); free(in_idx); return -3; }
    for (int64_t v = 0; v < n; ++v) x[v] = x0 ? x0[v] : 1.0 / (double)n;
    const double base = (1.0 - f) / (double)n;
    int team = 1;
    for (int t = 0; t < T; ++t) {
#pragma omp parallel
        {
#pragma omp single
            team = omp_get_num_threads();
#pragma omp for schedule(dynamic, 4096)
            for (int64_t u = 0; u < n; ++u) {
                double acc = 0.0;
                for (int64_t j = in_off[u]; j < in_off[u + 1]; ++j) {
                    int32_t v = in_idx[j];
                    acc += x[v] / (double)(off[v + 1] - off[v]);
                }
                y[u] = base + f * acc;
            }
        }
        double* tmp = x; x = y; y = tmp;
    }
    if (threads_out) *threads_out = (T > 0) ? team : omp_get_max_threads();
    memcpy(x_out, x, (size_t)n * sizeof(double));
    free(x); free(y); free(in_off); free(in_idx);
    return 0;
}

/* PageRank, pushing form (Sec. 4.1 pushing update): every vertex v adds
 * x_t(v)/d(v) to each out-neighbour.  Same iterate as the pulling form up to
 * summation order; used as a self-check of the oracle. */
int orc_pagerank_push(int64_t n, const int64_t* off, const int32_t* idx, double f, int T,
                      const double* x0, double* x_out) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (T < 0 || !x_out) return -1;
    double* x = (double*)malloc((size_t)n * sizeof(double));
    double* y = (double*)malloc((size_t)n * sizeof(double));
    if (!x || !y) { free(x); free(y); return -3; }
    for (int64_t v = 0; v < n; ++v) x[v] = x0 ? x0[v] : 1.0 / (double)n;
    const double base = (1.0 - f) / (double)n;
    for (int t = 0; t < T; ++t) {
        for (int64_t u = 0; u < n; ++u) y[u] = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            int64_t d = off[v + 1] - off[v];
            if (d == 0) continue;
            double share = x[v] / (double)d;
            for (int64_t e = off[v]; e < off[v + 1]; ++e) y[idx[e]] += share;
        }
        for (int64_t u = 0; u < n; ++u) y[u] = base + f * y[u];
        double* tmp = x; x = y; y = tmp;
    }
    memcpy(x_out, x, (size_t)n * sizeof(double));
    free(x); free(y);
    return 0;
}

/* One PageRank update evaluated only at the m vertices `verts`, from a given
 * FP32 iterate x (the previous iterate of the run being checked). */
int orc_pagerank_step_at(int64_t n, const int64_t* off, const int32_t* idx, double f,
                         const float* x, int64_t m, const int32_t* verts, double* y_out) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (!x || m < 0 || (m > 0 && (!verts || !y_out))) return -1;
    int64_t* slot = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    double* acc = (double*)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    if (!slot || !acc) { free(slot); free(acc); return -3; }
    for (int64_t v = 0; v < n; ++v) slot[v] = -1;
    for (int64_t i = 0; i < m; ++i) {
        if (verts[i] < 0 || verts[i] >= n) { free(slot); free(acc); return -2; }
        slot[verts[i]] = i; /* a repeated vertex keeps one accumulator */
    }
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = off[v + 1] - off[v];
        if (d == 0) continue;
        double share = (double)x[v] / (double)d;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int64_t s = slot[idx[e]];
            if (s >= 0) acc[s] += share;
        }
    }
    const double base = (1.0 - f) / (double)n;
    for (int64_t i = 0; i < m; ++i) y_out[i] = base + f * acc[slot[verts[i]]];
    free(slot); free(acc);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Out-strength s(v): sum of weights leaving v (out-degree when w == NULL). */
static void out_strength(int64_t n, const int64_t* off, const float* w, double* s) {
    for (int64_t v = 0; v < n; ++v) {
        double acc = 0.0;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) acc += w ? (double)w[e] : 1.0;
        s[v] = acc;
    }
}

/* Personalised PageRank, one column per source: x_0 = e_s and
 * x_{t+1}(u) = (1-f)[u == s] + f * sum over edges (v,u) of w(v->u)/s(v) * x_t(v).
 * X is n*k row-major.  Stops after T updates, or earlier once the L1 change
 * of a column falls below tol (tol <= 0: exactly T).  iters_out[j] receives
 * the updates applied to column j (nullable). */
int orc_ppr(int64_t n, const int64_t* off, const int32_t* idx, const float* w,
            int64_t k, const int32_t* sources, double f, int T, double tol,
            double* X, int32_t* iters_out) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (k < 0 || T < 0 || !X || (k > 0 && !sources)) return -1;
    for (int64_t j = 0; j < k; ++j)
        if (sources[j] < 0 || sources[j] >= n) return -2;
    int64_t *in_off, *in_slot;
    int32_t* in_idx;
    if ((rc = transpose(n, off, idx, &in_off, &in_idx, &in_slot))) return rc;
    double* s = (double*)malloc((size_t)n * sizeof(double));
    double* x = (double*)malloc((size_t)n * sizeof(double));
    double* y = (double*)malloc((size_t)n * sizeof(double));
    if (!s || !x || !y) { free(s); free(x); free(y); free(in_off); free(in_idx); free(in_slot); return -3; }
    out_strength(n, off, w, s);
    for (int64_t j = 0; j < k; ++j) {
        const int32_t src = sources[j];
        for (int64_t v = 0; v < n; ++v) x[v] = 0.0;
        x[src] = 1.0;
        int t = 0;
        for (; t < T; ++t) {
            double change = 0.0;
            for (int64_t u = 0; u < n; ++u) {
                double acc = 0.0;
                for (int64_t q = in_off[u]; q < in_off[u + 1]; ++q) {
                    int32_t v = in_idx[q];
                    double wv = w ? (double)w[in_slot[q]] : 1.0;
                    acc += wv / s[v] * x[v];
                }
                y[u] = (u == src ? 1.0 - f : 0.0) + f * acc;
                change += fabs(y[u] - x[u]);
            }
            double* tmp = x; x = y; y = tmp;
            if (tol > 0.0 && change < tol) { ++t; break; }
        }
        for (int64_t v = 0; v < n; ++v) X[v * k + j] = x[v];
        if (iters_out) iters_out[j] = t;
    }
    free(s); free(x); free(y); free(in_off); free(in_idx); free(in_slot);
    return 0;
}

/* (P^T z)(v) = sum over out-edges (v,u) of w(v->u)/s(v) * z(u), for one column
 * stride k at column j. */
static double pt_apply(const int64_t* off, const int32_t* idx, const float* w, const double* s,
                       int64_t v, const double* Z, int64_t k, int64_t j) {
    if (s[v] == 0.0) return 0.0;
    double acc = 0.0;
    for (int64_t e = off[v]; e < off[v + 1]; ++e) acc += (w ? (double)w[e] : 1.0) * Z[(int64_t)idx[e] * k + j];
    return acc / s[v];
}

/* Adjoint of personalised PageRank with respect to the edge weights, at the
 * fixed point X (n*k).  G = dL/dX (n*k).  Lambda (n*k out) solves
 * Lambda = G + f P^T Lambda by the same Jacobi iteration (T updates or until
 * the L1 change < tol); grad (nnz out, CSR slot order) receives
 * dL/dw(v->u) = (f/s(v)) sum_j X[v,j] (Lambda[u,j] - (P^T Lambda)[v,j]). */
int orc_ppr_adjoint(int64_t n, const int64_t* off, const int32_t* idx, const float* w,
                    int64_t k, const double* X, const double* G, double f, int T, double tol,
                    double* Lambda, double* grad, int32_t* iters_out) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (k < 1 || T < 0 || !X || !G || !Lambda || !grad) return -1;
    double* s = (double*)malloc((size_t)n * sizeof(double));
    double* nxt = (double*)malloc((size_t)(n * k) * sizeof(double));
    if (!s || !nxt) { free(s); free(nxt); return -3; }
    out_strength(n, off, w, s);
    memcpy(Lambda, G, (size_t)(n * k) * sizeof(double));
    int t = 0;
    for (; t < T; ++t) {
        double change = 0.0;
        for (int64_t v = 0; v < n; ++v)
            for (int64_t j = 0; j < k; ++j) {
                double val = G[v * k + j] + f * pt_apply(off, idx, w, s, v, Lambda, k, j);
                change += fabs(val - Lambda[v * k + j]);
                nxt[v * k + j] = val;
            }
        memcpy(Lambda, nxt, (size_t)(n * k) * sizeof(double));
        if (tol > 0.0 && change < tol) { ++t; break; }
    }
    if (iters_out) *iters_out = t;
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t e = off[v]; e < off[v + 1]; ++e) grad[e] = 0.0;
        if (s[v] == 0.0) continue;
        for (int64_t j = 0; j < k; ++j) {
            double ptl = pt_apply(off, idx, w, s, v, Lambda, k, j);
            double xv = X[v * k + j];
            for (int64_t e = off[v]; e < off[v + 1]; ++e)
                grad[e] += xv * (Lambda[(int64_t)idx[e] * k + j] - ptl);
        }
        for (int64_t e = off[v]; e < off[v + 1]; ++e) grad[e] *= f / s[v];
    }
    free(s); free(nxt);
    return 0;
}

/* Unrolled adjoint: the exact gradient of L(X_T) for the T-step map
 * X_0 = e_s (per column), X_{t+1} = (1-f) E + f P X_t.  G = dL/dX_T (n*k).
 * The iterates X_0..X_{T-1} are recomputed and kept; then, for t = T-1 down
 * to 0 with Lambda = dL/dX_{t+1}:
 *   grad[v->u] += (f/s(v)) sum_j X_t[v,j] (Lambda[u,j] - (P^T Lambda)[v,j]),
 *   Lambda <- f P^T Lambda  (= dL/dX_t).
 * Lambda0 (n*k out) receives dL/dX_0; grad (nnz out, CSR slot order). */
int orc_ppr_adjoint_unrolled(int64_t n, const int64_t* off, const int32_t* idx, const float* w, int64_t k,
                             const int32_t* sources, double f, int T, const double* G, double* Lambda0,
                             double* grad) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (k < 1 || T < 0 || !sources || !G || !Lambda0 || !grad) return -1;
    for (int64_t j = 0; j < k; ++j)
        if (sources[j] < 0 || sources[j] >= n) return -2;
    const size_t cells = (size_t)(n * k);
    double* s = (double*)malloc((size_t)n * sizeof(double));
    double* hist = (double*)malloc(cells * (size_t)(T > 0 ? T : 1) * sizeof(double));
    double* lam = (double*)malloc(cells * sizeof(double));
    double* ptl = (double*)malloc(cells * sizeof(double));
    if (!s || !hist || !lam || !ptl) { free(s); free(hist); free(lam); free(ptl); return -3; }
    out_strength(n, off, w, s);
    /* forward, scattering along out-edges: X_{t+1}(u) += f w(v->u)/s(v) X_t(v) */
    if (T > 0) {
        for (size_t i = 0; i < cells; ++i) hist[i] = 0.0;
        for (int64_t j = 0; j < k; ++j) hist[(size_t)sources[j] * k + j] = 1.0;
    }
    for (int t = 0; t + 1 < T; ++t) {
        const double* x = hist + (size_t)t * cells;
        double* y = hist + (size_t)(t + 1) * cells;
        for (size_t i = 0; i < cells; ++i) y[i] = 0.0;
        for (int64_t j = 0; j < k; ++j) y[(size_t)sources[j] * k + j] = 1.0 - f;
        for (int64_t v = 0; v < n; ++v) {
            if (s[v] == 0.0) continue;
            for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                const double p = f * (w ? (double)w[e] : 1.0) / s[v];
                for (int64_t j = 0; j < k; ++j) y[(int64_t)idx[e] * k + j] += p * x[v * k + j];
            }
        }
    }
    for (int64_t e = 0; e < off[n]; ++e) grad[e] = 0.0;
    memcpy(lam, G, cells * sizeof(double));
    for (int t = T - 1; t >= 0; --t) {
        const double* x = hist + (size_t)t * cells;
        for (int64_t v = 0; v < n; ++v)
            for (int64_t j = 0; j < k; ++j) ptl[v * k + j] = pt_apply(off, idx, w, s, v, lam, k, j);
        for (int64_t v = 0; v < n; ++v) {
            if (s[v] == 0.0) continue;
            for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                double acc = 0.0;
                for (int64_t j = 0; j < k; ++j) acc += x[v * k + j] * (lam[(int64_t)idx[e] * k + j] - ptl[v * k + j]);
                grad[e] += f / s[v] * acc;
            }
        }
        for (size_t i = 0; i < cells; ++i) lam[i] = f * ptl[i];
    }
    memcpy(Lambda0, lam, cells * sizeof(double));
    free(s); free(hist); free(lam); free(ptl);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* BFS from `root` with a FIFO queue over out-edges (Sec. 3.3; the
 * generalised BFS of Sec. 4.3 with all ready counters equal to one and the
 * accumulation operator "record the discovering parent").  Returns the
 * number of levels (the eccentricity of the root plus one). */
int orc_bfs(int64_t n, const int64_t* off, const int32_t* idx, int64_t root,
            int32_t* level, int32_t* parent) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (root < 0 || root >= n || !level || !parent) return -1;
    int32_t* queue = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return -3;
    for (int64_t v = 0; v < n; ++v) { level[v] = -1; parent[v] = -1; }
    int64_t head = 0, tail = 0;
    level[root] = 0;
    parent[root] = (int32_t)root;
    queue[tail++] = (int32_t)root;
    int32_t maxlev = 0;
    while (head < tail) {
        int32_t v = queue[head++];
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t u = idx[e];
            if (u < 0 || u >= n) { free(queue); return -2; }
            if (level[u] == -1) {
                level[u] = level[v] + 1;
                parent[u] = v;
                if (level[u] > maxlev) maxlev = level[u];
                queue[tail++] = u;
            }
        }
    }
    free(queue);
    return maxlev + 1;
}

/* Replays a direction schedule level by level and counts what each step
 * examines (Sec. 4.3 cost terms).  dirs[l] = 0: top-down -- every out-edge of
 * every frontier vertex is examined.  dirs[l] = 1: bottom-up -- every
 * unvisited vertex scans its in-neighbours in stored order up to and
 * including the first one in the frontier.  For each step l < nsteps writes
 * frontier[l] (|F| before the step), examined[l] and discovered[l].
 * Returns the number of steps taken (stops early when F becomes empty). */
int orc_bfs_replay(int64_t n, const int64_t* off, const int32_t* idx, int64_t root,
                   int nsteps, const int8_t* dirs, int64_t* frontier, int64_t* examined,
                   int64_t* discovered) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (root < 0 || root >= n || nsteps < 0 || (nsteps > 0 && (!dirs || !frontier || !examined || !discovered)))
        return -1;
    int64_t *in_off;
    int32_t* in_idx;
    if ((rc = transpose(n, off, idx, &in_off, &in_idx, NULL))) return rc;
    int32_t* level = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!level) { free(in_off); free(in_idx); return -3; }
    for (int64_t v = 0; v < n; ++v) level[v] = -1;
    level[root] = 0;
    int64_t fsize = 1;
    int step = 0;
    for (; step < nsteps && fsize > 0; ++step) {
        int64_t exam = 0, found = 0;
        frontier[step] = fsize;
        if (dirs[step] == 0) {
            for (int64_t v = 0; v < n; ++v) {
                if (level[v] != step) continue;
                for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                    ++exam;
                    int32_t u = idx[e];
                    if (level[u] == -1) { level[u] = step + 1; ++found; }
                }
            }
        } else {
            for (int64_t v = 0; v < n; ++v) {
                if (level[v] != -1) continue;
                for (int64_t q = in_off[v]; q < in_off[v + 1]; ++q) {
                    ++exam;
                    if (level[in_idx[q]] == step) { level[v] = step + 1; ++found; break; }
                }
            }
        }
        examined[step] = exam;
        discovered[step] = found;
        fsize = found;
    }
    free(level); free(in_off); free(in_idx);
    return step;
}

/* ---------------------------------------------------------------------- */
/* Triangle counting (Sec. 3.2): tc(v) = number of triangles containing v,
 * for a symmetric graph with sorted rows; counted per vertex by intersecting
 * N(v) with N(u) for every neighbour u and halving. */
int orc_triangles(int64_t n, const int64_t* off, const int32_t* idx, int64_t* tc) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (!tc) return -1;
    for (int64_t v = 0; v < n; ++v) {
        int64_t cnt = 0;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t u = idx[e];
            int64_t a = off[v], b = off[u];
            while (a < off[v + 1] && b < off[u + 1]) {
                if (idx[a] < idx[b]) ++a;
                else if (idx[a] > idx[b]) ++b;
                else { if (idx[a] != v && idx[a] != u) ++cnt; ++a; ++b; }
            }
        }
        tc[v] = cnt / 2;
    }
    return 0;
}

/* Betweenness centrality restricted to a set of sources (Sec. 3.5; Brandes'
 * scheme as in the Sec. 4.5 listing): for every source s, a FIFO BFS over
 * out-edges counts shortest paths sigma(s, v); then, in reverse BFS order,
 * delta(s, v) = sum over successors w (edge v->w, dist w = dist v + 1) of
 * sigma(s,v)/sigma(s,w) * (1 + delta(s,w)).  bc[v] = sum over the sources
 * s != v of delta(s, v): pairs (s, t) are ordered, so on an undirected graph
 * every unordered pair counts twice, as in the paper's definition. */
int orc_bc(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* sources, int64_t ns, double* bc) {
    int rc = check_graph(n, off, idx);
    if (rc) return rc;
    if (!bc || (ns > 0 && !sources)) return -1;
    int32_t* dist = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* order = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    double* sigma = (double*)malloc((size_t)n * sizeof(double));
    double* delta = (double*)malloc((size_t)n * sizeof(double));
    if (!dist || !order || !sigma || !delta) { free(dist); free(order); free(sigma); free(delta); return -3; }
    for (int64_t v = 0; v < n; ++v) bc[v] = 0.0;
    for (int64_t k = 0; k < ns; ++k) {
        const int32_t s = sources[k];
        if (s < 0 || s >= n) { free(dist); free(order); free(sigma); free(delta); return -1; }
        for (int64_t v = 0; v < n; ++v) { dist[v] = -1; sigma[v] = 0.0; delta[v] = 0.0; }
        int64_t head = 0, tail = 0;
        dist[s] = 0;
        sigma[s] = 1.0;
        order[tail++] = s;
        while (head < tail) {
            const int32_t v = order[head++];
            for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                const int32_t w = idx[e];
                if (dist[w] < 0) { dist[w] = dist[v] + 1; order[tail++] = w; }
                if (dist[w] == dist[v] + 1) sigma[w] += sigma[v];
            }
        }
        for (int64_t i = tail - 1; i >= 0; --i) {
            const int32_t v = order[i];
            double acc = 0.0;
            for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                const int32_t w = idx[e];
                if (dist[w] == dist[v] + 1) acc += (1.0 + delta[w]) / sigma[w];
            }
            delta[v] = sigma[v] * acc;
            if (v != s) bc[v] += delta[v];
        }
    }
    free(dist); free(order); free(sigma); free(delta);
    return 0;
}
