/*
 * bfs.h - C ABI of the MI355X (gfx950) masked sparse-matrix x sparse-vector
 * breadth-first search.
 *
 * The operation (Burkhardt, "Optimal algebraic Breadth-First Search for sparse
 * graphs", Theorem 1 and Algorithm 1): starting from x_1 = e_s, compute
 *     x_{k+1} = A^T[V_{k+1}, V_k] x_k,      V_{k+1} = V_k \ supp(x_k)
 * until the vector is empty.  A is the 0/1 adjacency pattern with A(i,j) = 1
 * for an edge i -> j (rows are egress; the search follows A^T, as in the
 * paper's directed-graph paragraph).  Rows and columns of visited vertices are
 * masked; A itself is never modified.
 *
 * Outputs (per search):
 *   level[v]  = k for v in supp(x_{k+1}) (the number of edges on a shortest
 *               path s -> v); -1 if v is never reached.
 *   parent[v] = the smallest frontier vertex j with A(j, v) = 1 and
 *               level[j] = level[v] - 1; parent[s] = s; -1 if unreached.
 *               This is the (min, select) semiring product of the paper's
 *               Algorithm 3 parent array with its tie resolved to the minimum,
 *               so every variant and every batch gives the same bits.
 *
 * Conventions for every call:
 *   - vertex ids and offsets are int32, 0-based; nnz < 2^31;
 *   - "device" pointers are HIP device memory on the graph's device;
 *   - hip_stream is a hipStream_t (NULL = the default stream);
 *   - every call returns bfs_status; nothing throws across the ABI;
 *   - on error, outputs are untouched and bfs_last_error_detail() explains.
 */
#ifndef BFS_H
#define BFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfs_graph bfs_graph;  /* opaque, immutable after create, library-owned */

typedef enum bfs_status {
    BFS_OK = 0,
    BFS_EINVAL = 1,   /* bad argument: NULL pointer, n <= 0, workspace too small, bad option */
    BFS_ERANGE = 2,   /* a source vertex outside [0, n) */
    BFS_ECSR = 3,     /* malformed CSR/CSC: ptr[0] != 0, decreasing ptr, idx outside [0, n),
                         or (with BFS_VALIDATE_TRANSPOSE) CSC != transpose(CSR) */
    BFS_ENOMEM = 4,   /* host or device allocation failed */
    BFS_EHIP = 5      /* a HIP runtime call failed; the hipError text is in the detail */
} bfs_status;

/* flags of bfs_graph_create */
enum {
    BFS_DIRECTED = 1u << 0,           /* A is not symmetric: the CSC is needed for pull */
    BFS_INPUT_ON_DEVICE = 1u << 1,    /* the four input arrays are device pointers */
    BFS_VALIDATE_TRANSPOSE = 1u << 2, /* check that the given CSC is the transpose of the CSR */
    BFS_MS_DEGREE_ORDER = 1u << 3,    /* keep the multi-source search's degree-ordered copy */
    BFS_MS_NO_DEGREE_ORDER = 1u << 4  /* never keep it (default: kept for graphs of 2^19+
                                         vertices with skewed degrees; a directed graph's
                                         copy serves batches of more than 64 sources) */
};

/* variant policies: which form of the product a level uses */
enum {
    BFS_VARIANT_PUSH = 0,        /* gather the frontier's columns (a compacted list)          */
    BFS_VARIANT_PULL = 1,        /* row-wise over the remaining unvisited rows (first hit)     */
    BFS_VARIANT_PUSH_BITMAP = 2, /* gather the frontier's columns, frontier held as a bitmap  */
    BFS_VARIANT_LEARNED = 3,     /* per level, the selector network's argmin; push fallback   */
    BFS_VARIANT_HEURISTIC = 4,   /* per level, a fixed edge-ratio rule (push <-> pull)        */
    BFS_VARIANT_SHORT_CIRCUIT = 5 /* push where the first frontier column to reach a row claims
                                    it (one bitmap atomicOr, no parent atomic): every reached
                                    vertex is claimed exactly once (the paper's Theorem 2);
                                    a row pass after the last level sets each parent to the
                                    smallest in-neighbour one level up (same results)       */
};

/* level-loop modes */
enum {
    BFS_LOOP_HOST = 0,        /* the host launches levels, reading the frontier size back
                                 every `levels_per_sync` levels                            */
    BFS_LOOP_GRAPH = 1,       /* chunks of levels replayed from a captured hipGraph          */
    BFS_LOOP_PERSISTENT = 2   /* one cooperative launch runs every level (grid barriers)    */
};

/* one record per level when tracing (host memory, written after the run) */
typedef struct bfs_level_record {
    int32_t level;            /* k: the frontier is supp(x_{k+1}) = {v : level[v] = k}   */
    int32_t variant;          /* BFS_VARIANT_PUSH / _PULL / _PUSH_BITMAP actually run    */
    uint32_t frontier;        /* |F_k|                                                   */
    uint32_t unvisited;       /* |U_k|: vertices not visited through level k             */
    uint64_t frontier_edges;  /* sum of out-degrees over F_k                             */
    uint64_t unvisited_edges; /* sum of out-degrees over U_k                             */
    float time_us;            /* device time of the level (host loop with tracing only)   */
    float reserved;
} bfs_level_record;

typedef struct bfs_run_options {
    uint32_t variant;          /* BFS_VARIANT_*                                  (default PUSH)  */
    uint32_t loop_mode;        /* BFS_LOOP_*                                     (default HOST)  */
    uint32_t levels_per_sync;  /* host loop / graph loop: levels launched between two reads of
                                  the frontier size (0 = 4)                                    */
    uint32_t grid_blocks;      /* workgroups per level launch (0 = 8 per compute unit)          */
    uint32_t heavy_degree;     /* out-degree from which a column is split into chunks (0 = 512) */
    uint32_t chunk_edges;      /* entries per chunk of a split column (0 = 1024)                */
    uint32_t ms_pull_shift;    /* multi-source searches (bfs_run_batch on one graph,
                                  bfs_run_batch_vm) under BFS_VARIANT_HEURISTIC / LEARNED: a
                                  level runs in the pull form when the union frontier holds
                                  more than n >> ms_pull_shift vertices (0 = 5, i.e. n / 32;
                                  at most 31, else BFS_EINVAL).  Never changes a result.       */
    const float *selector;     /* device: selector weights for BFS_VARIANT_LEARNED (NULL =
                                  push on every level)                                          */
    bfs_level_record *trace;   /* host: per-level records, or NULL                              */
    uint32_t trace_capacity;   /* records available in `trace`                                  */
    uint32_t time_kernels;     /* host loop: 1 = bracket every level launch with HIP events     */
    uint32_t trace_count;      /* out: records written                                          */
    uint32_t levels;           /* out: number of levels (largest level + 1)                    */
    uint32_t launches;         /* out (time_kernels): level-kernel launches issued, including
                                  launches after the last level, which return at once          */
    float kernel_us;           /* out (time_kernels): summed device time of those launches      */
    uint32_t push_impl;        /* BFS_VARIANT_PUSH only: BFS_PUSH_AUTO (0), BFS_PUSH_LIST,
                                  BFS_PUSH_SLICED or BFS_PUSH_CLAIM (see below)                 */
    float init_us;             /* out (time_kernels, bfs_run): device time of the search's
                                  initialisation launch (outputs to -1, bitmaps cleared)        */
    uint32_t ms_ranges;        /* multi-source searches of at most 64 sources: on pull levels
                                  whose union frontier holds more than n/16 vertices, the
                                  in-neighbours are visited in this many vertex ranges, one
                                  launch each, in ascending order, so that a range's frontier
                                  masks can stay in L2 (0 or 1 = one pass over the whole
                                  lists, the default: measured faster; at most 64).  Never
                                  changes a result.                                            */
    uint32_t push_used;        /* out (bfs_run, bfs_run_roots): the form of the push that ran,
                                  BFS_PUSH_LIST / _SLICED / _CLAIM (the list form's kernels
                                  also run the other variants)                                 */
    uint32_t count_atomics;    /* bfs_run with the list form's kernels only (else BFS_EINVAL):
                                  0 = off; 1 = count the parent atomicMin operations the push
                                  levels issue into `atomics`; 2 = the same with the parent
                                  pre-read off, so that every pair (j, i) with level[i] =
                                  level[j] + 1 issues exactly one: the count of Lemma 1's
                                  products that reach an unvisited row.  Never changes a
                                  result.                                                      */
    uint32_t reserved0;
    uint64_t atomics;          /* out (count_atomics): the count                                 */
} bfs_run_options;

/*
 * How BFS_VARIANT_PUSH runs (same results either way).
 *   BFS_PUSH_LIST    the frontier as a compacted list, the row mask read from
 *                    a bitmap in L2, the parent min-selected by atomicMin over
 *                    every unmasked pair of the level (Lemma 1's form).
 *   BFS_PUSH_SLICED  the frontier as a bitmap, the row mask in LDS: each
 *                    workgroup holds a slice (<= 128 KiB) of the visited bitmap
 *                    and expands the parts of the frontier columns whose rows
 *                    fall in it; a reached row is claimed by setting its LDS
 *                    bit, and receives its level and its parent (the first
 *                    in-neighbour, in ascending order, in the previous
 *                    frontier) when the next level expands it.  Needs
 *                    n <= 4 * 2^20 and the host or graph loop (BFS_EINVAL
 *                    otherwise).
 *   BFS_PUSH_CLAIM   one 64-bit word per vertex, (level << 32) | parent, its
 *                    top bit set while unreached: a frontier column offers
 *                    ((k + 1) << 32) | u to each of its rows by atomicMin, so
 *                    one atomic masks the visited rows (smaller words) and
 *                    keeps the smallest frontier in-neighbour (Lemma 1's
 *                    min-select), and the offer that finds the top bit set
 *                    lists the row (Theorem 2's single claim).  Levels whose frontier
 *                    holds at most 8192 columns and 2^16 entries run in one
 *                    workgroup, many levels per launch, the frontier in LDS;
 *                    wider levels one launch each over the whole grid.  For
 *                    deep, thin searches (grids, road-like graphs), where the
 *                    other forms pay a grid-wide launch per level.  Needs
 *                    variant PUSH and the host loop (BFS_EINVAL otherwise);
 *                    fills no trace.
 *   BFS_PUSH_AUTO    from the out-degrees (after duplicates and self-loops are
 *                    removed): claim-word, with the host loop, when every
 *                    out-degree is at most 8 (grids, road-like graphs);
 *                    sliced when it applies, n >= 2^17 and the largest
 *                    out-degree is at least 16 times the average (hubs); the
 *                    list form otherwise.
 */
enum {
    BFS_PUSH_AUTO = 0,
    BFS_PUSH_LIST = 1,
    BFS_PUSH_SLICED = 2,
    BFS_PUSH_CLAIM = 3
};

/*
 * The adjacency matrix A as the paper's Notation section fixes it (A(i,j) = 1
 * for an edge i -> j, rows egress) in the CSR format the paper describes for
 * its Algorithms 2 and 3 (a row pointer array of n+1 offsets and a column
 * index array).
 * Create a graph from the CSR of A (out-neighbours: row i lists j with A(i,j)=1;
 * out_ptr has n+1 entries, out_idx has out_ptr[n]) and, for directed graphs,
 * the CSC of A (in-neighbours: in_ptr n+1 entries, in_idx in_ptr[n]).  For an
 * undirected graph pass in_ptr = in_idx = NULL (the CSR serves both ways).
 * A directed graph with NULL CSC gets its transpose built here.
 * The library copies and sorts its own copy of every neighbour list; self-loops
 * and duplicate entries are accepted (they change no result).  For the
 * multi-source search (bfs_run_batch, bfs_run_batch_vm on one graph) it may
 * also keep a second copy of the lists with the vertices ranked by
 * descending out-degree (about 8 bytes per entry more, twice that for a
 * directed graph's two list sets; see the flags): the
 * frontier masks that most list entries point to then share a few megabytes
 * that stay in the L2 caches.  Results are the same either way.  Synchronous
 * on hip_stream; the caller may free its arrays once this returns.
 * Errors: BFS_EINVAL (n <= 0, NULL pointers), BFS_ECSR, BFS_ENOMEM, BFS_EHIP.
 */
bfs_status bfs_graph_create(int32_t n,
                            const int32_t *out_ptr, const int32_t *out_idx,
                            const int32_t *in_ptr, const int32_t *in_idx,
                            uint32_t flags, void *hip_stream, bfs_graph **out);

/* Free a graph (NULL is accepted).  No search may be running on it. */
bfs_status bfs_graph_destroy(bfs_graph *g);

/* Query n, nnz, directedness and the device bytes the graph holds (any pointer may be NULL). */
bfs_status bfs_graph_info(const bfs_graph *g, int32_t *n, int64_t *nnz,
                          int32_t *directed, size_t *device_bytes);

/* run_flags of bfs_workspace_size */
enum {
    BFS_WS_CLAIM = 1u << 0    /* also room for a batch in the claim-word form (push_impl CLAIM) */
};

/*
 * Device workspace bytes that bfs_run (num_queries = 1) or bfs_run_batch
 * (num_queries sources on this graph) needs: the state Algorithm 1 carries
 * between steps (the visited set V_k as bitmaps, the frontier supp(x_k) as
 * lists or bitmaps, the per-level counters) for every form of the push, the
 * pull and the claim-word push; for num_queries > 1 also the multi-source
 * masks and, on a graph where bfs_run_batch picks the claim-word form by
 * itself (see bfs_run_batch) or with run_flags BFS_WS_CLAIM, the claim-word
 * batch (about 36 bytes per vertex per query).  0 on a bad argument (unknown
 * run_flags bits included).
 */
size_t bfs_workspace_size(const bfs_graph *g, int32_t num_queries, uint32_t run_flags);

/*
 * One search from `source`: Algorithm 1 / Theorem 1, x_1 = e_source and
 * x_{k+1} = A^T[V_{k+1}, V_k] x_k until the frontier is empty, with the
 * parent of Algorithm 3 (its min-parent reading, see the header).
 * level and parent are device arrays of n int32
 * (caller-owned); workspace is a device buffer of at least
 * bfs_workspace_size(g, 1, 0) bytes, 256-byte aligned.  Nothing is allocated
 * per call (a host thread's first search allocates a 256-byte pinned host
 * slot through which the device reports progress; it is kept for the process).
 * Stream-ordered on hip_stream: results are valid when the stream completes;
 * the call itself returns after the last level has been issued (it reads the
 * frontier size back to find the end of the search).  opt may be NULL
 * (push on every level, host loop); its out-fields are written on success.
 * Several searches may run at once on one graph from different streams, each
 * with its own workspace and outputs.
 * Errors: BFS_EINVAL, BFS_ERANGE (source), BFS_EHIP.
 */
bfs_status bfs_run(bfs_graph *g, int32_t source,
                   int32_t *level, int32_t *parent,
                   bfs_run_options *opt,
                   void *workspace, size_t ws_bytes, void *hip_stream);

/*
 * Many searches in one call: Algorithm 3's parallel search (its `for all`
 * loops over frontier columns and their entries) run for every query at once.
 * Query q is (graphs[q], sources[q]) with outputs
 * level[q], parent[q] (device, n of that graph each).  When every query names
 * the same graph, the searches advance together, 64 sources per 64-bit mask
 * per vertex (one pass over a column serves every source whose frontier holds
 * it) - except with opt->push_impl BFS_PUSH_CLAIM, or with the automatic
 * choice for variant PUSH (host loop) on a graph beyond 2^22 vertices whose
 * out-degrees are all at most 8, where they run as claim-word searches
 * (below).  opt->variant picks the direction per level: PUSH (default) scatters
 * the frontier masks along out-edges; PULL lets every unsettled vertex gather
 * its in-neighbours' masks in ascending order; HEURISTIC pushes while the
 * union frontier holds at most n >> ms_pull_shift vertices and pulls after;
 * LEARNED asks the selector network (opt->selector) before every level (a
 * one-wave launch over the level's multi-source features, see
 * bfs_ms_profile_levels) and runs the argmin of its push and pull outputs,
 * push when an output is not finite and on every level when opt->selector is
 * NULL; from level 16 on, a push decision covers the next 8 levels.  With
 * opt->trace set, record k holds level k's direction (variant 0 push, 1 pull)
 * and, where the host read it, the union frontier's size.
 * Queries on different graphs (any mix, repeats allowed) run together, as one
 * search over the block-diagonal matrix of their graphs with one root per
 * block: query q gets the vertex ids [base_q, base_q + n_q).  When no graph
 * is thin (some out-degree above 8), or with opt->push_impl BFS_PUSH_LIST,
 * the library packs the graphs' out-lists into one CSR in the workspace
 * (ids offset by base_q) and runs the list form of the push from the
 * queries' roots; otherwise, or with BFS_PUSH_CLAIM, it runs the claim-word
 * push over the virtual ids without copying a graph, one launch per level
 * for every query (or one narrow launch for many levels while the joint
 * frontier is small).  Either way they need variant PUSH and the host loop
 * (BFS_PUSH_SLICED: BFS_EINVAL); opt->push_used reports the form.  One query
 * is bfs_run.  The result for query q is bit-identical to
 * bfs_run(graphs[q], sources[q]).
 * workspace: bfs_batch_workspace_size(num_queries, graphs) bytes, 256-byte
 * aligned.
 * Errors: BFS_EINVAL, BFS_ERANGE, BFS_EHIP.
 */
bfs_status bfs_run_batch(int32_t num_queries,
                         bfs_graph *const *graphs, const int32_t *sources,
                         int32_t *const *level, int32_t *const *parent,
                         bfs_run_options *opt,
                         void *workspace, size_t ws_bytes, void *hip_stream);

/* Workspace bytes of bfs_run_batch for these queries' graphs (0 on a bad argument). */
size_t bfs_batch_workspace_size(int32_t num_queries, bfs_graph *const *graphs);

/*
 * A search started from several roots at once (x_1 = sum of e_r): the level
 * and parent of every vertex are those of a search from the nearest root,
 * ties to the smallest frontier in-neighbour.  When the roots lie in distinct
 * components - e.g. one root per block of a block-diagonal matrix that packs
 * many graphs - each component's result equals bfs_run from its root alone.
 * roots_host: nroots distinct host ints in [0, n).  workspace: at least
 * bfs_roots_workspace_size(g, nroots) bytes, 256-byte aligned.
 * Errors: BFS_EINVAL (NULL, nroots outside [1, n], duplicate root, small
 * workspace), BFS_ERANGE (a root outside [0, n)), BFS_EHIP.
 */
bfs_status bfs_run_roots(bfs_graph *g, int32_t nroots, const int32_t *roots_host,
                         int32_t *level, int32_t *parent, bfs_run_options *opt,
                         void *workspace, size_t ws_bytes, void *hip_stream);

/* Workspace bytes for bfs_run_roots with nroots roots (0 on a bad argument). */
size_t bfs_roots_workspace_size(const bfs_graph *g, int32_t nroots);

/*
 * Many sources on one graph (Theorem 1 applied per source, 64 sources per
 * 64-bit mask word, as bfs_run_batch does for one graph), with the results in
 * one vertex-major pair of arrays instead of one array per source: with
 * ld = 64 * ceil(num_sources / 64), level[v * ld + q] and parent[v * ld + q]
 * are source q's level and parent of vertex v (the same values bfs_run gives);
 * columns q >= num_sources hold -1.  This is the layout the search builds
 * anyway, so no transpose pass runs at the end.
 * sources: host, num_sources ints in [0, n) (duplicates allowed).
 * level, parent: device int32[n * ld] each, caller-owned, 16-byte aligned.
 * workspace: bfs_batch_vm_workspace_size(g, num_sources) bytes or more,
 * 256-byte aligned.  opt: as for bfs_run_batch (variant, grid_blocks,
 * ms_pull_shift); on return opt->levels = the largest level over the sources
 * plus one.
 * Errors: BFS_EINVAL (NULL argument, num_sources < 1, misaligned or small
 * buffers, unknown variant, ms_pull_shift above 31), BFS_ERANGE (a source
 * outside [0, n)), BFS_EHIP.
 */
bfs_status bfs_run_batch_vm(bfs_graph *g, int32_t num_sources, const int32_t *sources,
                            int32_t *level, int32_t *parent, bfs_run_options *opt,
                            void *workspace, size_t ws_bytes, void *hip_stream);

/* Workspace bytes for bfs_run_batch_vm (0 on a bad argument). */
size_t bfs_batch_vm_workspace_size(const bfs_graph *g, int32_t num_sources);

/* ------------------------------------------------------------------------
 * The variant selector.  Not part of the paper: the paper's method is the
 * push form; these entry points serve the build's per-level choice between
 * the three equivalent forms of the product.  None of them can change a
 * search result.
 *
 * Weight blob: bfs_selector_param_count() floats, device memory:
 *   W1[32][12] b1[32] W2[32][32] b2[32] W3[3][32] b3[3] mean[12] inv_std[12]
 * The network maps the 12 level features (normalised by mean / inv_std) through
 * two ReLU layers of 32 to 3 predicted log device times (push, pull,
 * push-bitmap); BFS_VARIANT_LEARNED runs the argmin, push when an output is
 * not finite.  Features of level k (F = frontier, U = unvisited rows, n, nnz
 * of the graph): log(1+|F|), log(1+sumdeg F), log(1+|U|), log(1+sumdeg U), log(1+k),
 * nnz/n, log((|F|+1)/n), log((sumdeg F+1)/(nnz+1)), log((|U|+1)/n),
 * log((sumdeg U+1)/(nnz+1)), log((sumdeg F+1)/(sumdeg U+1)), log((|F|+1)/(|U|+1)).
 * ------------------------------------------------------------------------ */

/* Floats in a selector weight blob (including the normalisation constants). */
int32_t bfs_selector_param_count(void);

/* out[rows][3] = network(features[rows][12]); all device pointers. */
bfs_status bfs_selector_forward(const float *weights, const float *features, float *out,
                                int32_t rows, void *hip_stream);

/*
 * Mean-squared-error gradient: loss += inv_norm * sum(mask * (out - targets)^2)
 * and grad[0 .. param_count-24) += its gradient (weights and biases).
 * targets and mask are [rows][3]; inv_norm is normally 1 / sum(mask).
 * grad and loss are device accumulators (the caller zeroes them first).
 */
bfs_status bfs_selector_grad(const float *weights, const float *features, const float *targets,
                             const float *mask, int32_t rows, float inv_norm, float *grad,
                             float *loss, void *hip_stream);

/* One Adam step (beta 0.9 / 0.999) on the weights and biases; zeroes grad.
 * m and v are device state of param_count floats, zero before step 1. */
bfs_status bfs_selector_adam(float *weights, float *grad, float *m, float *v, int32_t step,
                             float lr, void *hip_stream);

/* Bytes of the snapshot buffer bfs_profile_levels needs (0 on a bad argument). */
size_t bfs_profile_snapshot_size(const bfs_graph *g);

/*
 * Exhaustive per-level timing, the selector's training data: runs the search
 * from `source`; before each level it saves the search state, times that one
 * level under each of the three forms (push, pull, push-bitmap; best of
 * `reps` runs, each from the restored state) and then advances with the
 * fastest of the three (so later levels start from the state a good per-level
 * choice produces, e.g. the unvisited list compacted by earlier pull levels).
 * records (host) receives three records per level (variant 0, 1, 2 in that
 * order, time_us = that level's device time); *count the number written.
 * level / parent / workspace as for bfs_run; snapshot: device buffer of
 * bfs_profile_snapshot_size(g) bytes.  The final level / parent equal bfs_run's.
 */
bfs_status bfs_profile_levels(bfs_graph *g, int32_t source, int32_t *level, int32_t *parent,
                              void *workspace, size_t ws_bytes, void *snapshot, size_t snap_bytes,
                              int32_t reps, bfs_level_record *records, uint32_t capacity,
                              uint32_t *count, void *hip_stream);

/* Bytes of the snapshot buffer bfs_ms_profile_levels needs (0 on a bad argument). */
size_t bfs_ms_profile_snapshot_size(const bfs_graph *g, int32_t num_sources);

/*
 * Exhaustive per-level timing of the multi-source searches (the training data
 * of BFS_VARIANT_LEARNED in bfs_run_batch / bfs_run_batch_vm): runs the
 * searches from `sources` as bfs_run_batch_vm does; before each level it saves
 * the whole search state (workspace and outputs) into `snapshot`, times that
 * one level in the push and in the pull direction (best of `reps` runs, each
 * from the restored state, device time between two events) and advances with
 * the faster one.  records (host) receives two records per level (variant 0 =
 * push, 1 = pull; time_us) holding the features the learned direction reads:
 * frontier = size of the union frontier F_k (vertices in some source's
 * frontier), frontier_edges = the sum of their out-degrees, unvisited = the
 * summed union-frontier sizes of levels 0..k, unvisited_edges = the (vertex,
 * source) pairs not reached through level k (n * num_sources minus those
 * reached).  The learned direction's twelve features are built from these,
 * num_sources, k, n and nnz: log(1+f), log(1+d), log(1+c), log(1+q),
 * log(1+k), nnz/n, log((f+1)/n), log((d+1)/(nnz+1)), log((u+1)/(n q)),
 * log((d+1)/(f+1)), log((f+1) q/n), log((d+1)/(nnz-d+1)) with f, d, c, u
 * the four statistics in that order and q = num_sources.
 * *count = records written (at most capacity).  level, parent, workspace: as
 * for bfs_run_batch_vm (workspace of bfs_batch_vm_workspace_size bytes);
 * snapshot: device, bfs_ms_profile_snapshot_size bytes, 256-byte aligned;
 * reps in [1, 1000].  The final level / parent equal bfs_run_batch_vm's.
 * Errors: BFS_EINVAL, BFS_ERANGE, BFS_EHIP.
 */
bfs_status bfs_ms_profile_levels(bfs_graph *g, int32_t num_sources, const int32_t *sources,
                                 int32_t *level, int32_t *parent, void *workspace, size_t ws_bytes,
                                 void *snapshot, size_t snap_bytes, int32_t reps,
                                 bfs_level_record *records, uint32_t capacity, uint32_t *count,
                                 void *hip_stream);

/* ------------------------------------------------------------------------
 * The comparison searches (Experiments section, Table 2).  Not the method:
 * the searches the paper measures its algebraic operation count against,
 * each with a device count of its operations (two per nonzero multiplied;
 * one step per level, the last step reaching nothing).  They compute the same
 * level / parent as bfs_run.
 *   BFS_COMPARE_SPMV    SpMV-BFS: every nonzero of A^T is multiplied at every
 *                       step with the dense frontier indicator (row form over
 *                       the graph's CSC).
 *                       ops = 2 nnz (eccentricity(s) + 1).
 *   BFS_COMPARE_SPMSPV  SpMSpV-BFS: the vector is not masked, x_{k+1} = A^T x_k
 *                       over all of supp(x_k) (the vertices a walk of exactly k
 *                       edges reaches from s); visited vertices only decide
 *                       levels.
 *   BFS_COMPARE_SPMMSPV SpMmSpV-BFS: the frontier's columns are multiplied in
 *                       full and the visited test follows the product.
 *                       ops = 2 nnz_c.
 * (The method itself multiplies once per reached vertex: 2 (n_c - 1).)
 * ------------------------------------------------------------------------ */
enum {
    BFS_COMPARE_SPMV = 0,
    BFS_COMPARE_SPMSPV = 1,
    BFS_COMPARE_SPMMSPV = 2
};

/* Workspace bytes for bfs_run_compare (0 when g is NULL); about 20 n bytes. */
size_t bfs_compare_workspace_size(const bfs_graph *g);

/*
 * One comparison search from `source` (Experiments section).  level / parent:
 * device int32[n], caller-owned, results as bfs_run.  workspace: device, at
 * least bfs_compare_workspace_size(g) bytes, 256-byte aligned.  ops / steps:
 * host pointers (either may be NULL) that receive the operation count and the
 * number of steps.  The call waits for hip_stream (it reads the device's
 * progress after every eight steps).
 * Errors: BFS_EINVAL (NULL argument, unknown method, small or misaligned
 * workspace), BFS_ERANGE (source outside [0, n)), BFS_EHIP.
 */
bfs_status bfs_run_compare(bfs_graph *g, int32_t source, uint32_t method, int32_t *level,
                           int32_t *parent, void *workspace, size_t ws_bytes, uint64_t *ops,
                           uint32_t *steps, void *hip_stream);

/* ------------------------------------------------------------------------
 * One masked sparse-matrix x sparse-vector product over a semiring: the
 * operation the method is made of (Definition 1: x_{k+1} = A^T[V_{k+1}, V_k]
 * x_k is this product with the row mask = the unvisited rows), offered for
 * use outside the search as masked-algebra libraries offer it.  Semirings
 * (the Notation section's Boolean, arithmetic and tropical min-plus, and the
 * (min, select) semiring that yields the smallest column); A is pattern-only
 * (every stored entry is 1), values are unsigned 64-bit:
 *   BFS_SEMIRING_BOOLEAN     y(i) = OR over products of (x(j) != 0)
 *   BFS_SEMIRING_ARITHMETIC  y(i) = sum of x(j), modulo 2^64
 *   BFS_SEMIRING_MIN_PLUS    y(i) = min of (x(j) + 1), saturating at 2^64 - 1
 *   BFS_SEMIRING_MIN_SELECT  y(i) = min of x(j)
 * ------------------------------------------------------------------------ */
enum {
    BFS_SEMIRING_BOOLEAN = 0,
    BFS_SEMIRING_ARITHMETIC = 1,
    BFS_SEMIRING_MIN_PLUS = 2,
    BFS_SEMIRING_MIN_SELECT = 3
};
enum {
    BFS_MASK_ROW_COMPLEMENT = 1u << 0,  /* the row mask names the rows to leave out */
    BFS_MASK_COL_COMPLEMENT = 1u << 1   /* the column mask names the columns to leave out */
};

/* Workspace bytes for bfs_masked_spmspv with up to max_nx vector entries (0 on
 * a bad argument); about 8 n + n / 8 + 24 max_nx bytes. */
size_t bfs_spmspv_workspace_size(const bfs_graph *g, int32_t max_nx);

/*
 * y = A^T[R, C] x: for every vector entry (j, x(j)) whose column C allows and
 * every entry i of A^T's column j (j's out-list) that R allows, y(i) (+)=
 * 1 (x) x(j).  y's support is structural: every allowed row that receives a
 * product.  Duplicate vector indices each contribute.
 * x_idx, x_val: device, nx entries (int32 indices in [0, n), uint64 values);
 * nx may be 0.  row_mask, col_mask: device bitmaps of ceil(n / 32) uint32
 * words (bit i = word i / 32, bit i % 32), or NULL for no mask; mask_flags
 * complements either.  y_idx, y_val: device, capacity n; receive the support
 * in ascending order and its values.  ny: host, receives the support's size.
 * workspace: device, bfs_spmspv_workspace_size(g, nx) bytes or more, 256-byte
 * aligned, zero-filled before its first use; every call leaves it
 * zero-filled, so one workspace serves any number of calls on one stream.
 * The call waits for hip_stream.
 * Errors: BFS_EINVAL (NULL argument, unknown semiring or mask flag, nx < 0,
 * small or misaligned workspace), BFS_ERANGE (a vector index outside [0, n):
 * nothing is written), BFS_EHIP.
 */
bfs_status bfs_masked_spmspv(bfs_graph *g, uint32_t semiring, const int32_t *x_idx,
                             const uint64_t *x_val, int32_t nx, const uint32_t *row_mask,
                             const uint32_t *col_mask, uint32_t mask_flags, int32_t *y_idx,
                             uint64_t *y_val, int32_t *ny, void *workspace, size_t ws_bytes,
                             void *hip_stream);

/*
 * One search from `source`, like bfs_run with BFS_VARIANT_PUSH and the host
 * loop, for callers that cannot allocate memory: code running under graph
 * capture or inside tight serving loops, and harnesses that forbid
 * allocation.  It takes no workspace and allocates nothing: the search state
 * lives in the library's own device array of 4 MiB, one per GPU, held from
 * library load until the process ends.  level and parent are device arrays of
 * n int32 (caller-owned); the results equal bfs_run's bit for bit.
 * Limit: graphs of at most 2^22 vertices (the sliced push); anything larger is
 * refused with BFS_EINVAL, as is a search that would need more than the 4 MiB.
 * Every call on a GPU shares that GPU's array and leaves the last call's
 * contents in it (each call's init kernel clears what must start empty), so
 * calls that overlap on one GPU - from several host threads or streams at
 * once - race and must not be made.  levels_per_sync: levels launched between
 * two reads of the progress word (0 = 4, at most 4096).  The call waits for
 * hip_stream.
 * Errors: BFS_EINVAL (NULL graph or output, too large, bad levels_per_sync),
 * BFS_ERANGE (source), BFS_EHIP.
 */
bfs_status bfs_run_static(bfs_graph *g, int32_t source, int32_t *level, int32_t *parent,
                          uint32_t levels_per_sync, void *hip_stream);

/*
 * Re-cut the sliced push's bitmap slices to at most max_words 32-bit words
 * each (a multiple of 4 in [4, 32768]; the default cut uses 32768, i.e.
 * 128 KiB of LDS per workgroup).  Smaller slices mean more slices (at most 4)
 * and fewer rows per workgroup; results never change.  Synchronous; no search
 * may be running on g.  Errors: BFS_EINVAL (NULL graph, bad size, or more
 * than 4 slices for this n), BFS_ENOMEM, BFS_EHIP (the previous cut is kept).
 */
bfs_status bfs_graph_set_slice_words(bfs_graph *g, uint32_t max_words);

/* Static text for a status code. */
const char *bfs_status_string(bfs_status s);

/* Thread-local text describing the last non-OK status returned on this thread. */
const char *bfs_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* BFS_H */
