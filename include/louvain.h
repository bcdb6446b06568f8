/*
 * louvain.h -- C ABI of the MI355X (gfx950) synchronous parallel Louvain
 * library (R. Forster, "Parallel Louvain Community Detection Optimized for
 * GPUs", arXiv 1805.10904).
 *
 * Graph model (paper, Section 2 "Problem statement and notation"):
 *   G(V, E, w) is undirected with positive integer weights, loops allowed,
 *   no multi-edges.  It is passed as a symmetric CSR adjacency matrix A:
 *   row i lists the neighbours j of i with A_ij; an edge {i, j}, i != j,
 *   appears in rows i and j with the same weight; a loop appears once, as
 *   A_ii.  delta_i = sum_j A_ij, TW = 2W = sum_i delta_i.
 *   Communities are labelled by vertex IDs in [0, n).
 *
 * Modularity (eq. 3) is reported exactly as the 128-bit integer
 *   Q_int = TW^2 * Q = TW * sum_i e_{i->C(i)} - sum_C deg_C^2
 * (e_{i->C} from eq. 1 including loops, deg_C from eq. 2), and as a double.
 *
 * Conventions for every call:
 *   - Return value: LOUVAIN_OK (0) or a negative LOUVAIN_E* status.  On an
 *     error the caller's output buffers are left untouched, nothing leaks,
 *     and louvain_last_error(ctx) describes the failure.  No call aborts.
 *   - Pointer arguments marked "host or device" are device pointers when
 *     LOUVAIN_DEVICE_PTRS is set in `flags`, host pointers otherwise.
 *     Device pointers must be device memory of the context's device.
 *   - All device work is enqueued on the context's HIP stream; a call
 *     returns after its outputs are complete (host outputs copied back,
 *     device outputs written, stream synchronised).
 *   - A context serves one host thread at a time: a call made while
 *     another thread is inside a call on the same context returns
 *     LOUVAIN_EBUSY and does nothing (louvain_submit / louvain_poll are
 *     the exception: thread-safe).
 *   - Device memory: every device allocation of a context comes from the
 *     region given to louvain_ctx_create (sub-allocated, cached per stream),
 *     or from hipMalloc when none was given.  With a region the library
 *     allocates no device memory of its own: a call that needs more than
 *     the region holds fails with LOUVAIN_ENOMEM and the context stays
 *     usable.  Pinned host memory for read-backs is allocated separately.
 *   - Fault injection: if the environment variable LOUVAIN_FAULT_ALLOC_AT
 *     holds k > 0 when a context is created, the k-th device allocation
 *     request of that context fails once with LOUVAIN_ENOMEM (tests of
 *     the error paths).
 *   - LOUVAIN_LOG=1 prints one line per level (and per contraction) on
 *     stderr.  LOUVAIN_HUB_BUCKET_SHRINK=s (1..4096) makes the hub buckets
 *     of levels with 2W >= 2^31 s times smaller, so that tests reach their
 *     spills to the hub tables.  Both are read once per process and change
 *     no result.
 */
#ifndef LOUVAIN_H
#define LOUVAIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LOUVAIN_OK         0
#define LOUVAIN_EINVAL    (-1)  /* invalid argument or malformed graph          */
#define LOUVAIN_ENOMEM    (-2)  /* device or host allocation failed             */
#define LOUVAIN_EDEVICE   (-3)  /* HIP runtime error                            */
#define LOUVAIN_EAGAIN    (-4)  /* poll: the request is still pending            */
#define LOUVAIN_EBUSY     (-5)  /* another thread is inside a call on the context */
#define LOUVAIN_ELIMIT    (-6)  /* max_sweeps / max_levels reached; result valid */
#define LOUVAIN_EOVERFLOW (-7)  /* n >= 2^31 or TW >= 2^62                      */

/* flags */
#define LOUVAIN_DEVICE_PTRS    0x1u  /* pointer arguments are device pointers        */
#define LOUVAIN_CHECK_SYMMETRY 0x2u  /* graph_create: also verify A_ij == A_ji       */
#define LOUVAIN_NO_SINGLET     0x4u  /* local_move: disable the singlet minimum-label
                                        heuristic (paper Section 3.1.1)               */
#define LOUVAIN_WEIGHTS_I64    0x8u  /* graph_create: weights are int64 (else int32) */

typedef struct louvain_ctx_s *louvain_ctx;
typedef struct louvain_graph_s *louvain_graph;

/* 128-bit two's-complement integer as two words. */
typedef struct {
    uint64_t lo;
    int64_t hi;
} louvain_i128;

/* Parameters of louvain_run (Alg. 2 driving Alg. 1 phases). */
typedef struct {
    int64_t theta_num;     /* a sweep is kept iff                                   */
    int64_t theta_den;     /*   theta_den*(Q_new-Q_prev) > theta_num*|Q_prev|      */
                           /* (Alg. 1's relative threshold theta, exact); default 1/10^6 */
    int32_t max_sweeps;    /* kept sweeps per phase, default 1000                   */
    int32_t max_levels;    /* phases (dendrogram levels), default 64                */
    int32_t singlet_rule;  /* 1 = singlet minimum-label heuristic on (default)      */
    int32_t pass_batch;    /* sweep passes enqueued between host checks of the
                              device's convergence flag (0 = library default);
                              passes past the end of a phase exit at once      */
    int32_t merge;         /* 1 = final merge after every phase that kept a sweep
                              (Section 5.1, end of "Generating one level"): from
                              the phase's labels, a vertex alone in its community
                              whose neighbours (loops aside) all carry one label C
                              joins C iff its score there beats staying and the
                              singlet rule allows it; Q is recomputed.  Default 0
                              (every form: plain, batched, served).            */
    int32_t reserved;      /* must be 0                                            */
} louvain_params;

/* Per-level record filled by louvain_run. */
typedef struct {
    int64_t n, nnz;               /* the level's graph                                   */
    int32_t sweeps_executed;      /* sweeps of the method incl. the final discarded one   */
    int32_t sweeps_accepted;      /* sweeps kept                                          */
    int32_t gpu_passes;           /* sweep passes the device ran for this phase           */
    int32_t reserved;
    louvain_i128 q_int;           /* Q_int after the phase, on this level's graph         */
    double ms_sweep;              /* device time of the phase's sweep kernels (stats mode) */
    double ms_contract;           /* device time of renumber + contraction (stats mode)    */
} louvain_level_stats;

#define LOUVAIN_MAX_KERNEL_STATS 64

/* Per-kernel device-time record (stats mode): one per kernel family. */
typedef struct {
    char name[40];
    int64_t launches;
    double ms;                    /* summed device time (HIP events around each launch)   */
    double alg_bytes;             /* summed algorithmic HBM bytes of those launches        */
} louvain_kernel_stats;

/* Statistics of a run.  Set `timing` to 1 before the call to record
 * per-kernel device times (HIP events filled by each kernel dispatch; the
 * run also waits for the device at the end of every level to attribute
 * them), or to 2 to record only the launches whose kernel name equals
 * `timing_only` (kernels[] then holds only them; the per-level ms fields
 * stay 0 and no per-level wait is added). */
typedef struct {
    int32_t timing;               /* in: 0 off, 1 every kernel, 2 only `timing_only`     */
    int32_t levels;               /* out: phases executed                                  */
    int32_t status;               /* out: LOUVAIN_OK or LOUVAIN_ELIMIT                     */
    int32_t n_kernels;            /* out: entries used in kernels[]                        */
    int64_t total_edges_swept;    /* out: sum over device passes of the level's nnz        */
    double ms_total;              /* out: device time of the whole run (stats mode)        */
    louvain_level_stats level[64];
    louvain_kernel_stats kernels[LOUVAIN_MAX_KERNEL_STATS];
    char timing_only[40];         /* in: kernel name for timing == 2 (as in kernels[])     */
} louvain_run_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` that enqueues its work on
 * `hip_stream` (a hipStream_t; NULL = the null stream).
 *   pool, pool_bytes: NULL and 0, or a region of device memory of `device`
 *               (e.g. a torch tensor's storage) from which the context
 *               sub-allocates every device buffer it uses: its graphs,
 *               level state, temporaries and its request loop's buffers.
 *               The caller keeps ownership; the region and the stream must
 *               outlive the context and every graph or dendrogram handle
 *               made on it.  Only pool_bytes rounded down to 256-byte
 *               blocks are used.
 *   tuning_path: NULL, or a file of launch shapes: read here when it
 *               exists and was written for this device's architecture
 *               (else the defaults apply), and rewritten by
 *               louvain_autotune.
 *   out:        receives the handle.
 * Errors: EINVAL (NULL out, negative device, a pool that is not device
 * memory of `device`, pool and pool_bytes not both set or both unset, a
 * malformed tuning file), EDEVICE (no such device), ENOMEM. */
int louvain_ctx_create(int device, void *hip_stream, void *pool, size_t pool_bytes, const char *tuning_path,
                       louvain_ctx *out);
/* Stops the context's request loop and frees the context.  EBUSY while
 * another thread is inside a call on it. */
int louvain_ctx_destroy(louvain_ctx ctx);

/* Device-memory accounting of a context. */
typedef struct {
    uint64_t pool_bytes;       /* usable bytes of the caller's region (0: hipMalloc)       */
    uint64_t pool_in_use;      /* region bytes handed to the context's caches              */
    uint64_t pool_high_water;  /* largest pool_in_use since creation or the last reset     */
    uint64_t live_bytes;       /* blocks of the context's own cache held by graphs, runs   */
    uint64_t cached_bytes;     /* blocks of the context's own cache kept for reuse         */
} louvain_memory;

/* Read the accounting (the request loop's workers have caches of their
 * own; their blocks count in pool_in_use only). */
int louvain_memory_stats(louvain_ctx ctx, louvain_memory *out);
/* Restart pool_high_water from the current pool_in_use. */
int louvain_memory_reset_peak(louvain_ctx ctx);

/* Message of the last failed call on ctx (never NULL; "" if none).  The
 * string is owned by ctx and valid until the next call on it. */
const char *louvain_last_error(louvain_ctx ctx);

/* ---- graphs --------------------------------------------------------------- */

/*
 * Copy a symmetric CSR graph into device memory owned by the library,
 * validate it, and compute delta_i and TW (paper Section 2).
 *   row_ptr: int64[n+1], host or device; row_ptr[0] == 0, nondecreasing,
 *            row_ptr[n] == nnz.
 *   col_idx: int32[nnz], host or device; every column in [0, n) and strictly
 *            ascending inside a row (no multi-edges).
 *   weight:  int32[nnz] (int64 with LOUVAIN_WEIGHTS_I64), host or device;
 *            every weight >= 1 (an unweighted graph uses weight 1).
 *   flags:   LOUVAIN_DEVICE_PTRS, LOUVAIN_CHECK_SYMMETRY, LOUVAIN_WEIGHTS_I64.
 * The inputs are copied; the caller may release them on return.
 * Errors: EINVAL (malformed CSR, weight < 1, asymmetric with
 * CHECK_SYMMETRY), EOVERFLOW (n >= 2^31, nnz >= 2^40 or TW >= 2^62),
 * ENOMEM, EDEVICE.
 */
int louvain_graph_create(louvain_ctx ctx, int64_t n, int64_t nnz, const int64_t *row_ptr,
                         const int32_t *col_idx, const void *weight, uint32_t flags,
                         louvain_graph *out);
int louvain_graph_destroy(louvain_graph g);

/* n, nnz and TW = 2W of a graph (any pointer may be NULL). */
int louvain_graph_info(louvain_graph g, int64_t *n, int64_t *nnz, int64_t *total_weight);

/* Copy a graph out as CSR with int64 weights (host or device pointers per
 * flags): row_ptr int64[n+1], col_idx int32[nnz], weight int64[nnz]. */
int louvain_graph_export(louvain_graph g, int64_t *row_ptr, int32_t *col_idx, int64_t *weight,
                         uint32_t flags);

/* ---- the method's steps ------------------------------------------------------ */

/*
 * One synchronous local-moving sweep (the parallel loop of Alg. 1; gains
 * of eq. 4 compared as exact integers, argmax of eq. 5, minimum-label
 * heuristics of Section 3.1).  Every vertex decides from labels_in and the
 * community degrees and sizes of labels_in; loops do not enter the move
 * scores.
 *   labels_in:  int32[n] in [0, n), host or device; NULL = singletons.
 *   labels_out: int32[n], host or device: every vertex's new community.
 *   deg_c_out:  optional int64[n], host or device: deg_C of labels_out
 *               (eq. 2), indexed by label.
 *   e_own_out:  optional int64[n], host or device: e_{i->labels_in[i]}
 *               (eq. 1) including i's loop.
 *   flags:      LOUVAIN_DEVICE_PTRS, LOUVAIN_NO_SINGLET.
 * Errors: EINVAL (NULL graph or output, label out of range), ENOMEM, EDEVICE.
 */
int louvain_local_move(louvain_ctx ctx, louvain_graph g, const int32_t *labels_in,
                       int32_t *labels_out, int64_t *deg_c_out, int64_t *e_own_out,
                       uint32_t flags);

/* Modularity of a labelling (eq. 3): labels int32[n] in [0, n), host or
 * device per flags.  q_int receives TW^2*Q exactly, q (optional) the double
 * Q_int / TW^2 (0 when TW == 0). */
int louvain_modularity(louvain_ctx ctx, louvain_graph g, const int32_t *labels,
                       louvain_i128 *q_int, double *q, uint32_t flags);

/*
 * louvain_modularity without any device allocation, for callers that
 * cannot allocate device memory (harnesses that forbid it, tight serving
 * loops).  Same arguments, result and errors as louvain_modularity (labels
 * host or device per flags: LOUVAIN_DEVICE_PTRS).  Its kernels work in one
 * library-owned device array of about 48 MiB per GPU, held from the first
 * context on that GPU until the process ends; graphs of more than
 * LOUVAIN_NOALLOC_MAX_N vertices are refused with LOUVAIN_EINVAL.  Every
 * call on a GPU shares that GPU's array, which keeps the last call's
 * contents (each call clears what it needs); calls on one GPU are
 * serialised by the library (each ends by reading its result back), so
 * they do not overlap on the array.  Host labels are copied with
 * hipMemcpyAsync from the caller's memory.
 */
#define LOUVAIN_NOALLOC_MAX_N 4194304
int louvain_modularity_noalloc(louvain_ctx ctx, louvain_graph g, const int32_t *labels,
                               louvain_i128 *q_int, double *q, uint32_t flags);

/*
 * Renumbering and graph rebuilding (Section 5.1, "Renumbering nodes" and
 * "Inducing new graph"): community labels are mapped to consecutive IDs in
 * ascending label order, and the graph is contracted so that super-vertex a
 * holds A'_ab = sum of A_ij over members i of a and j of b (loops included;
 * a super-vertex's loop counts each internal edge in both directions).  The
 * result has ascending columns in every row and int64 weights.
 *   labels:       int32[n] in [0, n), host or device.
 *   renumber_out: optional int32[n], host or device: new ID of each vertex's
 *                 community.
 *   out:          receives a new graph handle owned by the caller.
 * Errors: EINVAL, ENOMEM, EDEVICE.
 */
int louvain_aggregate(louvain_ctx ctx, louvain_graph g, const int32_t *labels,
                      int32_t *renumber_out, louvain_graph *out, uint32_t flags);

/*
 * The whole method (Alg. 2 over Alg. 1 phases) on device-resident state:
 * per phase, singleton initialisation, synchronous sweeps kept while the
 * exact relative gain test passes, then renumbering and contraction; stop
 * after a phase that keeps no sweep.
 *   params:     NULL = defaults (theta 1/10^6, 1000 sweeps, 64 levels,
 *               singlet rule on).
 *   labels_out: int32[n], host or device: final dense community IDs.
 *   q_int, q:   optional: modularity of the final partition on g.
 *   stats:      optional run statistics (see louvain_run_stats).
 * Returns LOUVAIN_OK, LOUVAIN_ELIMIT (a cap cut the run short; outputs are
 * valid), or an error (outputs untouched).
 */
int louvain_run(louvain_ctx ctx, louvain_graph g, const louvain_params *params,
                int32_t *labels_out, louvain_i128 *q_int, double *q,
                louvain_run_stats *stats, uint32_t flags);

/*
 * Batched form of louvain_run: the method on ngraphs independent graphs in
 * one call.  The graphs' current level graphs are swept, renumbered and
 * contracted together as one block-diagonal union (one set of launches per
 * sweep pass and per level for all of them), while every graph keeps its own
 * 2W, modularity, acceptance test, phase end, level count and community
 * numbering, so each graph's outputs are the ones louvain_run gives for it
 * alone.  The paper treats one graph; batching is this library's extension
 * of Alg. 2 to many graphs.
 *   graphs:     ngraphs handles created on ctx (not modified).
 *   params:     as for louvain_run, shared by all graphs.
 *   labels_out: ngraphs pointers; labels_out[i] is int32[n_i], host or
 *               device per flags (LOUVAIN_DEVICE_PTRS).
 *   q_int, q, status:
 *               optional arrays of ngraphs: per-graph Q_int, Q and status
 *               (LOUVAIN_OK or LOUVAIN_ELIMIT).
 *   stats:      optional array of ngraphs records (per-level fields as for
 *               louvain_run; the ms fields stay 0).  If stats[0].timing is 1
 *               on entry, stats[0] also receives the kernel table and
 *               ms_total of the whole call.
 * Graphs with 2W >= 2^31 are run one at a time through the plain path
 * before the batch.  Returns LOUVAIN_OK, LOUVAIN_ELIMIT (some graph hit a
 * cap; see status), or an error; after an error, outputs of graphs that
 * were run alone before the batch may already be written, the others are
 * untouched.
 */
int louvain_run_batch(louvain_ctx ctx, int64_t ngraphs, const louvain_graph *graphs,
                      const louvain_params *params, int32_t *const *labels_out,
                      louvain_i128 *q_int, double *q, int32_t *status,
                      louvain_run_stats *stats, uint32_t flags);

/* ---- dendrogram export and resume ------------------------------------------ */

typedef struct louvain_dendro_s *louvain_dendro;

/*
 * louvain_run that also keeps the dendrogram the renumbering step builds
 * level by level (Section 3, renumbering: each level of the dendrogram is
 * a map from the level's vertices to consecutive community IDs), plus the
 * graph a further phase would run on, so that a run can be checkpointed
 * and resumed (louvain_resume).  *dendro_out receives a handle owned by
 * the caller (louvain_dendro_destroy) that holds, in device memory:
 *   - map l for every phase l that kept a sweep: n[l] entries; map l sends
 *     vertex i of level l's graph to its vertex in level l+1's graph (the
 *     rank of its community's label among the labels present, ascending).
 *     Level 0's graph is g; level l+1's graph is level l's contracted by
 *     map l.  labels_out is the composition of the maps.
 *   - the graph of the last level, n[levels] vertices, with ascending
 *     columns: the graph of the phase that kept no sweep when the run ended
 *     that way, or the contraction by the last map when max_levels cut the
 *     run short (for a graph with TW = 0: a copy of g).
 * The last graph is put in that form by one more contraction (by the
 * identity); every other output equals louvain_run's.  Arguments
 * and the return value are as for louvain_run; on error *dendro_out is
 * untouched.
 */
int louvain_run_dendro(louvain_ctx ctx, louvain_graph g, const louvain_params *params,
                       int32_t *labels_out, louvain_i128 *q_int, double *q,
                       louvain_run_stats *stats, louvain_dendro *dendro_out, uint32_t flags);

/* Number of maps (*levels) and the vertex count of every level's graph
 * (n[0..levels], levels + 1 entries, at most 65).  Either may be NULL. */
int louvain_dendro_info(louvain_dendro d, int32_t *levels, int64_t *n);

/* Copy map `level` (n[level] entries) to map_out, host or device per flags
 * (LOUVAIN_DEVICE_PTRS).  EINVAL for a level outside [0, levels). */
int louvain_dendro_map(louvain_dendro d, int32_t level, int32_t *map_out, uint32_t flags);

/* Hand the last level's graph to the caller: *out receives a graph handle
 * of the dendrogram's context, owned by the caller.  A second call returns
 * EINVAL. */
int louvain_dendro_graph(louvain_dendro d, louvain_graph *out);

int louvain_dendro_destroy(louvain_dendro d);

/*
 * Resume a run from a level state (Alg. 2 continued): g_level is the graph
 * of level levels_done (as from louvain_dendro_graph), labels_so_far the
 * composition of the first levels_done maps (n0 entries in [0, n of
 * g_level), host or device per flags; louvain_run_dendro's labels_out).
 * Runs the remaining params->max_levels - levels_done phases on g_level
 * and writes labels_out[v] = the final community of vertex labels_so_far[v]
 * of g_level (n0 entries).  The results equal those of one louvain_run with
 * the same params on the original graph: each phase starts from singletons
 * on its level's graph, and contraction keeps TW and Q_int, so q_int / q
 * (of the partition on g_level) are also the original graph's.  stats
 * describe the resumed phases only.  With levels_done >= max_levels no
 * phase runs: labels_out = labels_so_far, and LOUVAIN_ELIMIT is returned.
 * Errors: EINVAL (labels out of range, bad arguments), ENOMEM, EDEVICE.
 */
int louvain_resume(louvain_ctx ctx, louvain_graph g_level, const louvain_params *params,
                   int32_t levels_done, int64_t n0, const int32_t *labels_so_far,
                   int32_t *labels_out, louvain_i128 *q_int, double *q,
                   louvain_run_stats *stats, uint32_t flags);

/* ---- launch shapes -------------------------------------------------------- */

/* Launch-shape settings (of levels whose 2W is below 2^31, except reorder).
 * They change which kernel sweeps which rows, never the results (every
 * setting gives the same labels, Q and level records). */
typedef struct {
    int32_t small_max;   /* rows of at most this many entries are swept one thread per
                            vertex (1..8; default 4)                                     */
    int32_t block_max;   /* longest row swept from an LDS table; longer rows use HBM hub
                            tables (341..10922; default 2730)                            */
    int32_t pass_batch;  /* sweep passes between host checks when the run's params say 0
                            (1..64; default 2)                                           */
    int32_t group_slots; /* LDS table slots scored per lane for rows of up to 341 entries
                            (2, 4 or 8; 0 = 4): fewer lanes per row, more work per lane */
    int32_t group_vertices; /* rows of up to 341 entries each lane group sweeps side by
                            side (1 or 2; 0 = 1): more independent work per lane      */
    int32_t overlap;     /* 1: the rows of 342..block_max entries and the hub rows are swept
                            on two extra streams beside the shorter rows (0 or 1)      */
    int32_t reorder;     /* level 0 of louvain_run / _dendro / _resume (any 2W): 1 sweeps
                            the graph rebuilt with its vertices in descending order of
                            floor(log2(row length)) (gather locality; the paper's
                            suggestion of placing vertices of similar degree side by
                            side), 2 as given, 0 auto = 1 for graphs with 2W >= 2^31
                            and at least 2^20 vertices, else 2.  Results never change:
                            labels stay the given vertex IDs                          */
    int32_t group_tiles; /* tiles (one vertex per lane group each) every workgroup of the
                            packed-class sweep takes, 1..8 (0 = 1): with more than one,
                            the loads of the next tiles are issued while a tile is
                            swept (software pipelining; needs group_vertices 1)       */
    double ms;           /* louvain_autotune: device time of one run with this setting */
} louvain_tuning;

/* Set (NULL = defaults) or read the context's launch shapes; they apply to
 * later louvain_run / louvain_run_batch calls and to a request loop started
 * afterwards.  Returns LOUVAIN_EINVAL for values out of range. */
int louvain_set_tuning(louvain_ctx ctx, const louvain_tuning *tuning);
int louvain_get_tuning(louvain_ctx ctx, louvain_tuning *tuning);

/*
 * Autotuner: times one whole run of the method on g (params as for
 * louvain_run) under the context's current setting and each candidate
 * (small_max in {4, 8}, block_max in {1365, 2730, 10922}, pass_batch in
 * {1, 2}, group_vertices in {1, 2}, group_tiles in {1, 4} with one vertex
 * per group; group_slots 4, overlap as set), best
 * of two runs each; a candidate replaces the current setting only when it
 * is more than 2% faster, so that timing noise does not flip the setting,
 * and the pick becomes the context's setting.  *best (optional) receives
 * it with its time.  When the context has a tuning file, the pick is
 * written to it (replacing it atomically).  Graphs with 2W >= 2^31 do not
 * use these shapes; the setting is left as it is and best->ms is -1.
 */
int louvain_autotune(louvain_ctx ctx, louvain_graph g, const louvain_params *params, louvain_tuning *best);

/*
 * Autotuner of the batched form: times louvain_run_batch's batch engine on
 * the given graphs (those with 2W < 2^31; params as for louvain_run_batch)
 * and tunes the launch shapes by coordinate descent, one round over the
 * fields: small_max {2, 4, 8}, group_slots {2, 4, 8}, group_vertices
 * {1, 2}, group_tiles {1, 2, 4}, block_max {1365, 2730, 10922},
 * pass_batch {1, 2, 4}; each value
 * is timed (best of two calls) with the other fields at the best setting
 * so far, and kept only when it is more than 2% faster.  The pick becomes
 * the context's setting (and is written to its tuning file, if any);
 * *best (optional) receives it with one call's device time in ms (-1 when
 * no graph qualifies).  Results never depend on the setting.
 */
int louvain_autotune_batch(louvain_ctx ctx, int64_t ngraphs, const louvain_graph *graphs,
                           const louvain_params *params, louvain_tuning *best);

/* ---- served form --------------------------------------------------------- */

/* Result of one served request (louvain_poll). */
typedef struct {
    int32_t status;               /* LOUVAIN_OK, LOUVAIN_ELIMIT or the request's error     */
    int32_t levels;               /* phases executed                                       */
    int64_t n, nnz;               /* the submitted graph                                   */
    int64_t total_edges_swept;    /* sum over device passes of the level's nnz             */
    louvain_i128 q_int;           /* Q_int of the final labels                             */
    double q;                     /* Q = Q_int / (2W)^2                                    */
    double t_submit_us;           /* submit, admission and completion times (steady clock, */
    double t_admit_us;            /*   microseconds; differences are latencies)            */
    double t_done_us;
    louvain_level_stats level[64];/* per-level records as for louvain_run (ms fields 0)    */
    char error[128];              /* message of a failed request                           */
} louvain_request_result;

/* Estimated peak device bytes one graph of n vertices and nnz entries holds
 * while it is served (its resident CSR and its share of the batch's level
 * buffers); the request loop admits graphs while the sum fits its budget.
 * Contraction never grows a graph (every level has at most the previous
 * level's vertices and entries), so the level-0 estimate bounds the run. */
size_t louvain_workspace_bytes(int64_t n, int64_t nnz);

/* Device-memory budget of ctx's request loop (0 = 80% of the free device
 * memory when the loop starts). */
int louvain_serve_budget(louvain_ctx ctx, size_t hbm_bytes);

/*
 * Queue the method on one graph for the context's request loop, which a
 * worker thread runs on its own stream.  Requests are admitted in arrival
 * order while their louvain_workspace_bytes fit the budget; an admitted
 * graph joins the running batch at the next level boundary, beside graphs
 * already at deeper levels (continuous batching), and its result equals
 * louvain_run on that graph alone.  Requests with different params are
 * batched separately.
 *   n, nnz, row_ptr, col_idx, weight, flags: as for louvain_graph_create;
 *               the arrays are read when the request is admitted and must
 *               stay valid (and, for device pointers, complete on their
 *               streams) until louvain_poll has delivered the result.
 *   params:     as for louvain_run (NULL = defaults).
 *   labels_out: int32[n], host or device per flags; written before the
 *               result is delivered.
 *   ticket:     receives the request's id for louvain_poll.
 * Thread-safe; does not set louvain_last_error.  Returns LOUVAIN_OK,
 * LOUVAIN_EINVAL / LOUVAIN_EOVERFLOW for bad arguments (nothing queued),
 * LOUVAIN_ENOMEM or LOUVAIN_EDEVICE.  Malformed graphs fail at admission
 * (their result carries the error); a failing request does not disturb the
 * others.
 */
int louvain_submit(louvain_ctx ctx, int64_t n, int64_t nnz, const int64_t *row_ptr,
                   const int32_t *col_idx, const void *weight, const louvain_params *params,
                   int32_t *labels_out, uint32_t flags, uint64_t *ticket);

/*
 * Wait up to wait_us microseconds (0 = do not wait, < 0 = without limit)
 * for a request.  Returns LOUVAIN_EAGAIN while it is pending; otherwise
 * fills *result (optional), retires the ticket and returns the request's
 * status.  Unknown or retired tickets: LOUVAIN_EINVAL.  Thread-safe.
 */
int louvain_poll(louvain_ctx ctx, uint64_t ticket, int32_t wait_us, louvain_request_result *result);

#ifdef __cplusplus
}
#endif

#endif /* LOUVAIN_H */
