/*
 * pp.h -- C ABI of libpp, the push/pull graph-sweep library for MI355X (gfx950).
 *
 * The library implements the per-iteration edge sweep of Besta et al., "To Push
 * or To Pull: On Reducing Communication and Synchronization in Graph
 * Computations" (HPDC'17), in its two forms:
 *   - push: a vertex scatters updates to its out-neighbours' shared state
 *     (write conflicts resolved with atomics; Sec. 3.8, Sec. 4.1 pushing line);
 *   - pull: a vertex gathers from its in-neighbours into state only it writes
 *     (no atomics; Sec. 3.8, Sec. 4.1 pulling line).
 * The sweeps are instantiated as the PageRank power-iteration step (FP32,
 * Sec. 3.1 equation, Sec. 4.1 listing) and the BFS frontier step (int32,
 * Sec. 3.3, Sec. 4.3 listing: top-down = push, bottom-up = pull), plus the
 * direction switch (Sec. 5 Generic-Switch; direction-optimising BFS cited in
 * Sec. 1).  Batched personalised PageRank, its adjoint with respect to edge
 * weights, and a many-graph launch sit on the same sweeps.
 *
 * Conventions shared by every entry point
 *  - Graph representation: the adjacency array of Sec. 2.2.  CSR = out-
 *    adjacency (row v lists targets of edges leaving v; used by push), CSC =
 *    in-adjacency (row u lists sources of edges entering u; used by pull).  A
 *    symmetric graph may pass the same arrays for both.  int32 offsets and
 *    indices; nnz must fit in int32.
 *  - Memory: every array argument is DEVICE memory owned by the caller unless
 *    stated otherwise.  The library never allocates or frees device memory;
 *    derived data lives in caller-provided workspaces whose size is queried
 *    first.  A graph handle keeps the caller's pointers: they must outlive it.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *    stream).  Compute calls enqueue work and return; results are valid once
 *    the stream is synchronised.  Calls marked SYNC wait on the stream.
 *  - Concurrency: calls that share a graph handle, a BFS state or a workspace
 *    must be ordered on one stream; overlapping them races.
 *  - Errors: every call returns a pp_status.  Arguments are validated on the
 *    host before anything is launched; on error nothing is enqueued and
 *    pp_last_error() (thread-local) describes the failure.  A HIP runtime error
 *    maps to PP_E_HIP with the runtime's message.
 */
#ifndef PP_H
#define PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PP_ABI_VERSION 1

typedef enum {
    PP_OK = 0,
    PP_E_NULL = -1,        /* a required pointer is NULL */
    PP_E_SIZE = -2,        /* n, nnz, k or another size is out of range */
    PP_E_RANGE = -3,       /* a scalar argument (f, root, iters, ...) is out of range */
    PP_E_GRAPH = -4,       /* the graph arrays are malformed (pp_graph_check) */
    PP_E_WORKSPACE = -5,   /* a workspace or state buffer is too small */
    PP_E_HIP = -6,         /* the HIP runtime reported an error */
    PP_E_UNSUPPORTED = -7  /* the combination of arguments is not supported */
} pp_status;

typedef enum { PP_PUSH = 0, PP_PULL = 1, PP_SWITCH = 2 } pp_dir;

/* Graph flags. */
#define PP_GRAPH_WEIGHTED 0x1u /* csr_w (and csc_to_csr) are given */
#define PP_GRAPH_RELABEL 0x2u  /* renumber vertices by decreasing degree inside the
                                  library (caller ids are kept at the ABI) */

typedef struct pp_graph_s* pp_graph;

int pp_abi_version(void);
const char* pp_last_error(void);

/* ------------------------------------------------------------------ graph */
/* Workspace bytes pp_graph_create needs for a graph of n vertices and nnz
 * stored directed edges (0 when n or nnz is out of range). */
size_t pp_graph_workspace_bytes(int32_t n, int64_t nnz, uint32_t flags);

/* Registers a graph (Sec. 2.2 adjacency arrays) and derives, on the device,
 * the out-degree d(v) (or out-strength s(v) = sum of weights when weighted),
 * its reciprocal (0 when d(v) = 0), and the vertex lists binned by degree
 * that the sweeps use to map rows of very different lengths onto lanes,
 * wavefronts and workgroups.  csr_off/csc_off: int32[n+1]; csr_idx/csc_idx:
 * int32[nnz]; csc may alias csr for symmetric graphs.  Weighted graphs
 * (PP_GRAPH_WEIGHTED) pass csr_w (float[nnz], one weight per CSR slot, > 0)
 * and csc_to_csr (int32[nnz], the CSR slot of each CSC slot).  ws: device
 * workspace of at least pp_graph_workspace_bytes(n, nnz, flags) bytes, kept
 * by the handle until pp_graph_destroy; it also holds the owner (row) of
 * every in-adjacency slot, which streamed bottom-up BFS levels use.  SYNC
 * (reads back bin sizes). */
pp_status pp_graph_create(int32_t n, int64_t nnz,
                          const int32_t* csr_off, const int32_t* csr_idx,
                          const int32_t* csc_off, const int32_t* csc_idx,
                          const float* csr_w, const int32_t* csc_to_csr,
                          uint32_t flags, void* ws, size_t ws_bytes, void* stream, pp_graph* out);

/* With PP_GRAPH_RELABEL the library keeps a renumbered copy of the adjacency
 * arrays in the workspace: vertices sorted by floor(log2(d_out + d_in + 1)),
 * heaviest first, ties in caller order.  Heavy rows then sit in one
 * contiguous id range, which the push sweep privatises in LDS and which keeps
 * the most-gathered entries in a compact, cache-resident prefix.  Every entry
 * point still takes and returns vectors in caller ids.  perm: int32[n] device
 * output, perm[i] = caller id of internal vertex i. */
pp_status pp_graph_relabel_map(pp_graph g, int32_t* perm, void* stream);

/* New edge weights for a graph registered with PP_GRAPH_WEIGHTED, in place:
 * csr_w (DEVICE float[nnz], caller CSR slot order, > 0, same structure) is
 * re-derived into the relabelled and CSC slot orders and the out-strengths
 * s(v) of the Sec. 3.1 transition P_uv = w(v->u)/s(v), as at registration,
 * without re-registering the graph.  Without PP_GRAPH_RELABEL the handle
 * keeps using csr_w itself, so it must stay valid and unchanged while the
 * graph is used; the csc_to_csr map given at registration must still be
 * valid.  PP_E_UNSUPPORTED for unweighted graphs.  ASYNC on `stream`. */
pp_status pp_graph_set_weights(pp_graph g, const float* csr_w, void* stream);

/* Frees the host handle (device memory stays with the caller). */
pp_status pp_graph_destroy(pp_graph g);

/* Device-side validation: offsets start at 0, are monotone and end at nnz;
 * every index lies in [0, n).  Returns PP_OK or PP_E_GRAPH.  SYNC. */
pp_status pp_graph_check(pp_graph g, void* stream);

/* Host copies of the degree-bin boundaries (for tests and tuning):
 * counts[0..PP_NUM_BINS) of vertices per bin, for the pull (in-degree) or
 * push (out-degree) lists. */
#define PP_NUM_BINS 6
pp_status pp_graph_bins(pp_graph g, pp_dir dir, int32_t* counts);

/* Degree thresholds of the bins (upper bounds of bins 0..4; bin 5 is the
 * rest) and the split chunk for the longest rows.  Defaults: 4, 16, 64, 1024,
 * 4096; chunk 4096.  Takes effect at the next pp_graph_create. */
pp_status pp_set_bin_thresholds(const int32_t* upper5, int32_t split_chunk);

/* Push-sweep tuning: the first `hot` vertices (internal ids) are accumulated
 * per workgroup in LDS and merged once per sweep (the Partition-Awareness
 * strategy of Sec. 5 with a workgroup as the owner); the sweep runs on
 * `push_blocks` persistent workgroups (of 256 threads, or of 1024 threads
 * when more than 16384 targets are privatised).  Defaults 8192 and 1024; hot
 * in [0, 40960] (0 disables), push_blocks in [1, 65536].  Takes effect at the
 * next pp_graph_create. */
pp_status pp_set_push_tuning(int32_t hot, int32_t push_blocks);

/* Binned push (on = 1, the default) or global atomics (on = 0) for the
 * updates a push sweep sends to targets past the `hot` privatised ones.
 * Binned: the sweep appends each such update as a (target, value) pair to its
 * workgroup's slice of the target's bin (16384 consecutive ids) with a plain
 * store, and a second kernel sums every bin in LDS; the slice sizes come from
 * one counting walk of the sweep's static work assignment at registration.
 * No global atomics remain (the remote updates of Sec. 5's
 * Partition-Awareness, buffered instead of applied one by one).  Needs hot >
 * 0; its workspace (8 bytes per edge plus tables) is part of
 * pp_graph_workspace_bytes.  Takes effect at the next pp_graph_create. */
pp_status pp_set_push_bins(int32_t on);

/* The binned-push layout of g: info[0..4) = bins (0: global atomics),
 * first binned target, workgroups of the sweep, units of the summing kernel. */
pp_status pp_graph_push_bins(pp_graph g, int32_t* info);

/* Pull-sweep tuning: each workgroup of the persistent pull sweep stages the
 * contributions of the first `pull_hot` vertices (internal ids; with
 * PP_GRAPH_RELABEL the heaviest ones, which most gathers hit) in LDS, capped
 * by the LDS one workgroup may use; pull_block threads per workgroup (256,
 * 512 or 1024).  Defaults 32768 and 1024.  Takes effect at the next
 * pp_graph_create. */
pp_status pp_set_pull_tuning(int32_t pull_hot, int32_t pull_block);

/* Tiled pull (relabelled unweighted graphs): the in-edges of the heaviest
 * rows -- a prefix [0, R) of the degree-ordered ids, R at most `rows`, every
 * such row with at least max(16, S/2) in-edges -- are regrouped at
 * registration by source slice of `width` ids (S slices).  A pull sweep then
 * stages one slice of contributions in LDS per tile of rows, so those rows
 * gather only from LDS through 16-bit offsets, writes one partial sum per
 * (slice, row) and adds each row's partials in slice order; the other rows
 * are pulled as usual in the same launch.  Same sum in a different fixed
 * order: still bit-reproducible.  rows = 0 turns it off (default 0); width a
 * multiple of 64 in [64, 32768] (default 32768: offsets within a slice take
 * 15 bits of a 16-bit entry).  Takes effect at the next
 * pp_graph_create; the workspace query accounts for it. */
pp_status pp_set_pull_slices(int32_t rows, int32_t width);

/* Deep-graph BFS (pp_bfs_run / pp_bfs_run_log with PP_PUSH or PP_SWITCH):
 * while a top-down frontier has at most max_frontier vertices and
 * max_edges out-edges, and the switch rule keeps top-down, whole levels run
 * inside one launch on one workgroup (frontier in LDS, no launch per level;
 * the per-level cost of Sec. 4.3 that grows with the diameter D).  Larger
 * frontiers go back to the grid-wide level kernels.  Levels and statistics
 * do not depend on it.  One compute unit sustains only so many misses in
 * flight, so this pays for narrow frontiers (a path: 3.4 against 6.7 us per
 * level) and not for frontiers of thousands of vertices.  Defaults 256 and
 * 1024; max_frontier is capped by the LDS of a workgroup (6144 on gfx950);
 * 0 turns it off.  Takes effect at the next pp_graph_create. */
pp_status pp_set_bfs_multi(int32_t max_frontier, int32_t max_edges);

/* The tiled-pull plan of g: info[0..4) = R, width, S, tiles (R = 0: off). */
pp_status pp_graph_slices(pp_graph g, int32_t* info);

/* --------------------------------------------------------------- PageRank */
/* One Jacobi step of the PageRank equation (Sec. 3.1):
 *   y[u] = (1-f)/n + f * sum over edges (v,u) of P_uv * x[v],
 * P_uv = 1/d(v) (unweighted) or w(v->u)/s(v) (weighted); a vertex with
 * d(v) = 0 contributes nothing.  x, y: float[n], distinct.  pp_pr_push
 * scatters along CSR rows with FP32 atomics (nnz atomic adds per call; the
 * summation order, hence the last bits, may vary between runs); pp_pr_pull
 * gathers along CSC rows with no atomics (bit-reproducible).  f in [0, 1).
 * Uses the graph's scratch: calls on one graph must be ordered. */
pp_status pp_pr_push(pp_graph g, const float* x, float* y, float f, void* stream);
pp_status pp_pr_pull(pp_graph g, const float* x, float* y, float f, void* stream);

/* iters Jacobi steps in direction dir starting from x_inout (float[n], x_0
 * in, x_iters out), with the contribution c[v] = f * x[v] * P-normaliser
 * computed once per step in the fused epilogue of the previous step.
 * PP_PUSH and PP_PULL as above.  PP_SWITCH chooses the direction per edge
 * class (the Partition-Awareness and switching ideas of Sec. 5 combined):
 * edges into the first `hot` vertices (internal ids, pp_set_push_tuning) are
 * pushed into per-workgroup LDS accumulators, which are summed in a fixed
 * order (no global atomics), and the rows of all other vertices pull.
 * iters >= 0. */
pp_status pp_pr_run(pp_graph g, pp_dir dir, int32_t iters, float f, float* x_inout, void* stream);

/* -------------------------------------------------------------------- BFS */
/* BFS state: frontier queues, frontier and visited bitmaps and counters
 * (device memory, caller-owned).  Size in bytes for graph g. */
size_t pp_bfs_state_bytes(pp_graph g);

/* Statistics of one BFS run (host struct). */
#define PP_BFS_MAX_LOG 64
typedef struct {
    int32_t levels;                   /* number of non-empty frontiers */
    int32_t reached;                  /* vertices with level >= 0 */
    int64_t edges_reached;            /* sum of out-degrees of reached vertices */
    int8_t dir[PP_BFS_MAX_LOG];       /* direction used to expand frontier l */
    int32_t frontier[PP_BFS_MAX_LOG]; /* |F| at level l */
} pp_bfs_stats;

/* Initialises a BFS from `root` (Sec. 3.3; Sec. 4.3 with every ready
 * counter equal to one): level[] = parent[] = -1 (int32[n], caller-owned,
 * kept by the state), level[root] = 0, parent[root] = root, F = {root}. */
pp_status pp_bfs_init(pp_graph g, int32_t root, int32_t* level, int32_t* parent,
                      void* state, size_t state_bytes, void* stream);

/* Expands the frontier of level cur_level (the number of steps taken since
 * pp_bfs_init) into level cur_level+1.  push = top-down: every frontier
 * vertex claims its unvisited out-neighbours (one atomic OR on the visited
 * bitmap per claim, wave-aggregated queue appends).  pull = bottom-up: every
 * unvisited vertex scans its in-neighbours in stored order and stops at the
 * first frontier member, which becomes its parent (no atomics on vertex
 * state; one counter update per wavefront).  Out-rows longer than 256 edges
 * are cut into 256-edge chunks that the whole grid shares (into 32-edge
 * chunks, rows past 32 edges, on a level with fewer than nnz/32 frontier
 * out-edges, when the graph has rows past 256); an in-row longer than 128
 * edges is scanned over its first 128 and its rest is cut into 128-edge
 * chunks.  A bottom-up vertex whose in-row is chunked takes the first frontier
 * member of whichever chunk claims it first (one atomic OR): rows of up to
 * 256 in-edges still take the first in stored order.  A bottom-up level with a sparse frontier
 * (8 |F| < ceil(n/64), its out-edges at most nnz/256) while at least half the
 * edges leave unvisited vertices streams the whole in-edge array instead, and
 * a vertex takes whichever frontier in-neighbour claims it first.  Either step may follow the other.  level/parent must be the arrays given to pp_bfs_init.  Enqueue
 * only; the frontier size is read with pp_bfs_frontier.  A step on an empty
 * frontier does nothing. */
pp_status pp_bfs_step_push(pp_graph g, void* state, int32_t* level, int32_t* parent, int32_t cur_level,
                           void* stream);
pp_status pp_bfs_step_pull(pp_graph g, void* state, int32_t* level, int32_t* parent, int32_t cur_level,
                           void* stream);

/* Size of the frontier produced by the last step (SYNC). */
pp_status pp_bfs_frontier(pp_graph g, void* state, int32_t* size, void* stream);

/* Whole BFS from root.  policy PP_PUSH / PP_PULL forces one direction;
 * PP_SWITCH chooses per level on the device: top-down -> bottom-up when
 * m_f > m_u / alpha, bottom-up -> top-down when n_f < n / beta and the
 * frontier shrinks (m_f: out-edges of the frontier, m_u: out-edges of
 * unvisited vertices, n_f: frontier size).  alpha, beta > 0 (defaults 14, 24
 * when <= 0 is passed).  Levels do not depend on the policy; parents are
 * any valid BFS parents.  stats: host, nullable.  SYNC.  The graph keeps the
 * recent runs' level counts, the instantiated level batches and a pinned
 * header buffer: BFS calls on one graph must not overlap across host
 * threads. */
pp_status pp_bfs_run(pp_graph g, int32_t root, pp_dir policy, float alpha, float beta,
                     int32_t* level, int32_t* parent, void* state, size_t state_bytes,
                     pp_bfs_stats* stats, void* stream);

/* One entry of a BFS level log: how frontier l was expanded (Sec. 4.3; the
 * statistics are those the switch rule of pp_bfs_run reads). */
typedef struct {
    int32_t dir;            /* PP_PUSH (top-down) or PP_PULL (bottom-up) */
    int32_t frontier;       /* n_f = |F_l| */
    int64_t frontier_edges; /* m_f = out-edges of F_l: the edges a top-down
                               expansion of F_l examines */
} pp_bfs_level;

/* pp_bfs_run that also writes entry l of `log` (DEVICE array of log_cap
 * entries, caller-owned) for every expanded frontier l < log_cap; pass
 * log_cap >= n + 1 to log every level of any run (a graph of n vertices has
 * at most n non-empty frontiers).  Entries past the last level are left
 * untouched.  log may be NULL only when log_cap is 0.  SYNC. */
pp_status pp_bfs_run_log(pp_graph g, int32_t root, pp_dir policy, float alpha, float beta,
                         int32_t* level, int32_t* parent, void* state, size_t state_bytes,
                         pp_bfs_level* log, int32_t log_cap, pp_bfs_stats* stats, void* stream);

/* pp_bfs_run from each of the k roots (HOST array) in turn, without a host
 * wait between them: every root's run goes to the device back to back (its
 * level batch sized from the recent runs with the policy on this graph) and
 * the host reads all the run headers after one wait.  A root whose run was
 * deeper than its batch is run again on its own, so the results are those of
 * pp_bfs_run.  stats[i] (HOST, k entries) describes the run from roots[i];
 * level and parent (n each, caller ids) hold the run from roots[k-1] when
 * the call returns.  The first call with a policy on a graph runs its first
 * root on its own to size the batches; graphs of more than 256 levels go
 * root by root.  Every root is checked before anything is launched
 * (PP_E_RANGE).  k = 0 does nothing.  SYNC. */
pp_status pp_bfs_run_many(pp_graph g, int32_t k, const int32_t* roots, pp_dir policy, float alpha, float beta,
                          int32_t* level, int32_t* parent, void* state, size_t state_bytes,
                          pp_bfs_stats* stats, void* stream);

/* ------------------------------------------------------ personalised PR */
/* Scratch bytes for pp_ppr_run / pp_ppr_adjoint with k columns processed in
 * tiles of k_tile (pp_ppr_run also takes k_tile = 1; 0 when an argument is
 * invalid). */
size_t pp_ppr_scratch_bytes(pp_graph g, int32_t k, int32_t k_tile);

/* Personalised PageRank for k sources at once (the PageRank equation of
 * Sec. 3.1 with its teleport term put on one vertex; not defined in the
 * paper): for column j, x_0 = e_{s_j} and
 *   x_{t+1}(u) = (1-f)[u == s_j] + f * sum over edges (v,u) of P_uv x_t(v).
 * sources: device int32[k], caller ids.  X: device float[n*k], row-major,
 * caller ids (output).  Columns run in tiles of k_tile (8, 16, 32, 64; the
 * last tile may be partial); a tile's rows hold k_tile contiguous values so every edge
 * moves one coalesced k_tile-float row.  dir PP_PULL gathers along CSC (no
 * atomics, deterministic), PP_PUSH scatters along CSR with FP64 atomics into
 * an FP64 accumulator.  PP_SWITCH applies the Generic-Switch strategy of
 * Sec. 5: while the tile's support (the vertices within t hops of its
 * sources) has at most m/14 out-edges, a sweep pushes from the support only
 * (sparse matrix times sparse vector along CSR, Sec. 7.1, FP64 atomics);
 * afterwards the tile continues with pulling sweeps.  Runs `iters` sweeps per
 * tile, or stops a tile early once the L1 change of its iterate in one sweep
 * is at most tol times the iterate's L1 norm (tol = 0: exactly iters; each
 * check synchronises the stream; PP_SWITCH also synchronises after each
 * sparse sweep).  iters_done (host, nullable): most sweeps any tile ran.
 * k_tile = 1 runs the columns one after another with the single-vector
 * PageRank sweeps of pp_pr_run (PP_PUSH or PP_PULL, tol = 0 only; it uses
 * the graph's iterate buffers, so it must not overlap pp_pr_run on the same
 * graph): the k sequential solves that batching is measured against.
 * SYNC when tol > 0 or dir = PP_SWITCH (and once to validate the sources). */
pp_status pp_ppr_run(pp_graph g, pp_dir dir, int32_t k, const int32_t* sources, int32_t iters, float tol,
                     float f, int32_t k_tile, float* X, void* scratch, size_t scratch_bytes,
                     int32_t* iters_done, void* stream);

/* Adjoint of personalised PageRank with respect to the edge weights, at the
 * fixed point X of pp_ppr_run (float[n*k], caller layout).  dLdX: float[n*k]
 * (caller layout).  Lambda (output, float[n*k]) solves
 *   Lambda = dLdX + f P^T Lambda,  (P^T z)(v) = (1/s(v)) sum over out-edges
 * (v,u) of w(v->u) z(u),
 * which is the transposed sweep: PP_PULL gathers along the CSR rows (the rows
 * the forward push scatters along), PP_PUSH scatters along CSC.  PP_SWITCH
 * (Sec. 5 Generic-Switch): Lambda's support starts at the nonzero rows of
 * dLdX and grows along in-edges; while its in-edges number at most nnz/14
 * the sweeps push from the support only, then dense pulls (a dense dLdX
 * switches at once).  grad_w
 * (output, float[nnz], the caller's CSR slot order):
 *   dL/dw(v->u) = (f/s(v)) sum_j X[v,j] (Lambda[u,j] - (P^T Lambda)[v,j]).
 * Unweighted graphs differentiate with respect to implicit unit weights.
 * iters/tol as in pp_ppr_run. */
pp_status pp_ppr_adjoint(pp_graph g, pp_dir dir, int32_t k, const float* X, const float* dLdX, int32_t iters,
                         float tol, float f, int32_t k_tile, float* Lambda, float* grad_w, void* scratch,
                         size_t scratch_bytes, int32_t* iters_done, void* stream);

/* ------------------------------------------------------- many graphs */
/* Device workspace bytes for pp_multi_run over num_graphs graphs holding
 * total_vertices vertices together. */
size_t pp_multi_workspace_bytes(int32_t num_graphs, int64_t total_vertices);

/* PageRank and BFS for many small unweighted graphs in one launch (beyond
 * the paper, which sweeps one graph at a time).  Graph i has graph_n[i]
 * vertices (1..16384) and graph_nnz[i] stored edges (HOST arrays).  Arenas
 * (device): off/in_off hold each graph's n+1 local offsets back to back (CSR
 * = out-adjacency, CSC = in-adjacency; may alias for symmetric graphs);
 * idx/in_idx each graph's local neighbour ids back to back as uint16 (a
 * graph has at most 16384 vertices, so 16 bits hold every id; half the
 * bytes of int32 ids per sweep).  Before any sweep a device pass checks
 * every graph: its offsets start at 0, never decrease and end at
 * graph_nnz[i], and every id lies below its n (both adjacencies unless they
 * alias); on failure nothing is computed, the outputs are left as they were
 * and the call returns PP_E_GRAPH.  The arena arrays themselves must be as
 * long as graph_n and graph_nnz say.  x (float),
 * level and parent (int32) each graph's n entries back to back.  Runs
 * pr_iters Jacobi steps of the PageRank equation (Sec. 3.1; x_0 = 1/n) in
 * direction pr_dir, then, unless bfs_policy is -1, a BFS from local vertex
 * bfs_root of every graph with policy PP_PUSH / PP_PULL / PP_SWITCH
 * (alpha, beta as in pp_bfs_run).  One workgroup holds one graph's state in
 * LDS: pull gathers and push updates are LDS operations and the barrier
 * between sweeps is a workgroup barrier.  Pull sums every row in FP64 (per
 * lane in slot order, then a fixed lane reduction), so results are
 * bit-reproducible; push accumulates in FP64 LDS atomics.  Graphs are taken
 * largest first.  SYNC. */
pp_status pp_multi_run(int32_t num_graphs, const int32_t* graph_n, const int64_t* graph_nnz,
                       const int32_t* off, const uint16_t* idx, const int32_t* in_off, const uint16_t* in_idx,
                       pp_dir pr_dir, int32_t pr_iters, float f, float* x,
                       int32_t bfs_policy, int32_t bfs_root, float alpha, float beta,
                       int32_t* level, int32_t* parent, void* ws, size_t ws_bytes, void* stream);

/* Work mapping of pp_multi_run / pp_multi_run_static, chosen by the
 * autotuner: PageRank rows of at least `big` edges take a whole wavefront,
 * rows of mid..big-1 edges a group of mid_lanes lanes (8, 16 or 32), the
 * other pull rows pull_group lanes (1, 2 or 4).  Results do not depend on
 * it beyond FP64 summation order.  Defaults 512, 64, 2, 16.  Takes effect at
 * the next call. */
pp_status pp_set_multi_tuning(int32_t big, int32_t mid, int32_t pull_group, int32_t mid_lanes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as pp_multi_run, with its scratch (graph table, validation word,
 * push contributions) in a fixed array of PP_MULTI_STATIC_BYTES inside the
 * library instead of a caller workspace.  Each device the library runs on
 * holds one such array for the life of the process.  The call allocates
 * nothing; it fails with PP_E_WORKSPACE when
 * pp_multi_workspace_bytes(num_graphs, total vertices) exceeds
 * PP_MULTI_STATIC_BYTES (16 MiB: about 4 million vertices in all).  All calls
 * on one device share its array, so calls that overlap on one device (other
 * threads, other streams) race; order them.  Arguments, errors and results
 * as pp_multi_run.  SYNC. */
#define PP_MULTI_STATIC_BYTES ((size_t)16 << 20)
pp_status pp_multi_run_static(int32_t num_graphs, const int32_t* graph_n, const int64_t* graph_nnz,
                              const int32_t* off, const uint16_t* idx, const int32_t* in_off, const uint16_t* in_idx,
                              pp_dir pr_dir, int32_t pr_iters, float f, float* x,
                              int32_t bfs_policy, int32_t bfs_root, float alpha, float beta,
                              int32_t* level, int32_t* parent, void* stream);

/* Scratch bytes for pp_ppr_adjoint_unrolled (k columns, tiles of k_tile, T
 * steps: it keeps T iterates of one tile). */
size_t pp_ppr_unrolled_scratch_bytes(pp_graph g, int32_t k, int32_t k_tile, int32_t T);

/* Unrolled adjoint: the exact gradient of a loss on X_T, the iterate after T
 * steps of the personalised PageRank update from X_0 = e_s (the map
 * pp_ppr_run computes with iters = T and tol = 0).  Given G = dL/dX_T
 * (device float[n*k], caller layout), the call recomputes X_0..X_{T-1} with
 * pulling sweeps, then runs T reverse steps: with Lambda = dL/dX_{t+1},
 *   dL/dw(v->u) += f/s(v) * sum_j X_t[v,j] (Lambda[u,j] - (P^T Lambda)[v,j]),
 *   Lambda <- f P^T Lambda.
 * Lambda0: device float[n*k], receives dL/dX_0.  grad_w: device float[nnz],
 * caller CSR slot order, overwritten.  sources: device int32[k].  Not in the
 * paper; the derivative of the Sec. 3.1 update with per-slot weights.  SYNC
 * (once, to validate the sources). */
pp_status pp_ppr_adjoint_unrolled(pp_graph g, int32_t k, const int32_t* sources, int32_t T, float f,
                                  int32_t k_tile, const float* dLdXT, float* Lambda0, float* grad_w,
                                  void* scratch, size_t scratch_bytes, void* stream);

/* ------------------------------------------------------- triangle counting */
/* Workspace bytes of pp_tc_run for graph g (device, caller-owned, 256-byte
 * aligned). */
size_t pp_tc_workspace_bytes(pp_graph g);

/* Triangles per vertex (Sec. 3.2; the NodeIterator listing of Sec. 4.2):
 * tc[v] = 1/2 * #{(w1, w2) : w1, w2 in N(v), w2 in N(w1)}, N = the graph's
 * CSR rows (out-neighbours), which must be in strictly ascending order (the
 * call fails with PP_E_GRAPH otherwise; tc is then undefined).  The counts of
 * one edge (v, w1) are found by intersecting the two rows.  dir = PP_PULL
 * credits v (each counter written once, no atomics); PP_PUSH credits w1 with
 * a 64-bit integer fetch-and-add.  On a symmetric graph both give the number
 * of triangles containing each vertex.  tc: int64[n] device, caller ids.
 * SYNC (reads the row-order check). */
pp_status pp_tc_run(pp_graph g, pp_dir dir, int64_t* tc, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------ betweenness centrality */
/* Workspace bytes of pp_bc_run for graph g (device, caller-owned, 256-byte
 * aligned): per source of a batch of up to 32, its distances, path counts,
 * dependencies, BFS order and level offsets (about 28 n bytes each).  A
 * smaller workspace (at least one source's share) runs smaller batches. */
size_t pp_bc_workspace_bytes(pp_graph g);

/* Betweenness centrality over a set of sources (Sec. 3.5; Brandes' scheme as
 * in the Sec. 4.5 listing): bc[v] = sum over sources s != v of
 * delta_s(v) = sum over t of sigma_st(v) / sigma_st, with sigma the number of
 * shortest paths along out-edges (ordered pairs: on an undirected graph each
 * unordered pair counts twice).  Per source, a level-synchronous forward pass
 * counts paths and a backward pass accumulates dependencies, deepest level
 * first.  fwd_dir PP_PUSH: frontier vertices claim targets (CAS on the
 * distance) and add their path counts with FP64 atomics; PP_PULL: unvisited
 * vertices sum over their in-neighbours in the frontier (owner writes).
 * bwd_dir PP_PUSH: vertices add to their predecessors' dependency with FP64
 * atomics; PP_PULL: vertices sum over their successors (owner writes).
 * sources: HOST int32[num_sources] (caller ids); bc: double[n] device,
 * caller ids, overwritten.  Sources run up to 32 at a time (they are
 * independent), each level kernel covering all sources of the batch; the
 * level bookkeeping is on the device.  The call synchronises the stream once
 * per batch of forward levels (usually once per batch of sources) to read
 * the depths, then queues the backward levels. */
pp_status pp_bc_run(pp_graph g, pp_dir fwd_dir, pp_dir bwd_dir, int32_t num_sources, const int32_t* sources,
                    double* bc, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PP_H */
