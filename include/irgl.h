/*
 * irgl.h -- C ABI of the MI355X data-driven BFS/SSSP library.
 *
 * The operation is the paper's level-by-level worklist BFS (Section 4.1,
 * BFS listing; Iterate with an initial worklist [src], Section 4.2 and
 * Table 1): pop every item of the incoming worklist, visit each out-edge of
 * the popped vertex, label unvisited destinations with the next level and
 * push them on the outgoing worklist; swap the worklists after every
 * invocation and stop when the outgoing worklist is empty.  SSSP is the same
 * data-driven loop with "distance improved" in place of "unvisited"
 * (textbook single-source shortest paths; the paper states only BFS).
 *
 * Results are exact integers:
 *   level[v] = least number of out-edges on a path src -> v,
 *   dist[v]  = least sum of weights on a path src -> v,
 * with IRGL_INF (0xFFFFFFFF) for unreachable vertices.
 *
 * Conventions for every entry point:
 *   - Return value is an irgl_status; nothing throws across the ABI.
 *   - "device pointer" means memory on the current HIP device (any
 *     hipMalloc'd buffer, e.g. a torch tensor's data_ptr()); the library
 *     never frees caller memory and allocates no device memory of its own.
 *   - Query entry points are asynchronous on the given HIP stream (pass the
 *     hipStream_t as void*; NULL = the null stream) and never synchronize
 *     the host, except where stated.
 *   - Errors found on the device (worklist overflow, distance overflow,
 *     watchdog, abort, iteration limit) are written to the stats block; read
 *     them with irgl_query_status() after the stream has completed.
 *   - A graph handle is immutable after upload and may serve concurrent
 *     queries that use distinct workspaces and outputs.
 */
#ifndef IRGL_H
#define IRGL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IRGL_VERSION 100 /* 0.1.0 */
#define IRGL_INF 0xFFFFFFFFu

typedef int32_t irgl_status;
enum {
    IRGL_OK = 0,
    IRGL_ERR_INVALID_ARGUMENT = 1,   /* null pointer, src out of range, n <= 0, m >= 2^31 */
    IRGL_ERR_NO_WEIGHTS = 2,         /* SSSP on a graph uploaded without weights */
    IRGL_ERR_INVALID_GRAPH = 3,      /* IRGL_VALIDATE found a malformed CSR */
    IRGL_ERR_WORKSPACE_TOO_SMALL = 4,
    IRGL_ERR_OVERFLOW = 5,           /* worklist capacity or uint32 distance exceeded */
    IRGL_ERR_ABORTED = 6,            /* the host abort flag was raised */
    IRGL_ERR_BUSY = 7,               /* no free slot (batched / served queries) */
    IRGL_ERR_TOO_LARGE = 8,          /* a request can never fit its memory budget */
    IRGL_ERR_NO_DEVICE = 9,          /* no HIP device visible */
    IRGL_ERR_DEVICE = 10,            /* a HIP call failed; see irgl_last_hip_error() */
    IRGL_ERR_WATCHDOG = 11,          /* the grid barrier waited past its time limit */
    IRGL_ERR_ITERATION_LIMIT = 12,   /* the loop reached max_iter with work left */
    IRGL_ERR_CONFIG = 13,            /* unsupported block size / thresholds / grid */
    IRGL_ERR_INTERNAL = 14           /* a device-side consistency check failed */
};

enum { IRGL_KIND_BFS = 0, IRGL_KIND_SSSP = 1 };

/* Graph flags. */
/* The caller's promise (not checked) that every edge has its reverse with
 * equal weight: BFS may then run bottom-up invocations and SSSP on a split
 * graph may run a heavy pass as a pull, both of which read a vertex's
 * out-edges as its in-edges. */
#define IRGL_SYMMETRIC 1u
#define IRGL_VALIDATE 2u  /* check the CSR on the device during upload (synchronizes) */

#define IRGL_WATCHDOG_IMMEDIATE 0xFFFFFFFFu
#define IRGL_BITMAP_NEVER 0xFFFFFFFFu
#define IRGL_GRID_TIER_OFF (-1)
#define IRGL_DELTA_NONE 0xFFFFFFFFu
#define IRGL_DO_OFF 0xFFFFFFFFu
#define IRGL_BARRIER_XCD 0u
#define IRGL_BARRIER_WORKGROUP 1u

/* Launch modes. */
enum {
    IRGL_MODE_PERSISTENT = 0, /* one cooperative launch; the Iterate loop runs on the
                                 device with a grid-wide barrier between invocations
                                 (iteration outlining, Section 4.3) */
    IRGL_MODE_HOST_LOOP = 1,  /* one launch per invocation, the host reads the worklist
                                 size back after each (the un-outlined form); this mode
                                 synchronizes the stream once per level */
    IRGL_MODE_TOPOLOGY = 2    /* topology-driven Iterate (Table 1: ForAll over every
                                 node, ReduceAndReturn, Iterate While Any / Until All):
                                 no worklists; every invocation visits all n vertices
                                 (BFS expands those labelled in the previous invocation,
                                 SSSP every reached one, Bellman-Ford) and returns
                                 whether anything changed through a block-aggregated
                                 reduction (see `reduce`); one cooperative launch.
                                 Same results as the data-driven modes; stats.items
                                 counts n per invocation */
};

/* ReduceAndReturn reductions of the topology-driven loop (Section 3). */
#define IRGL_REDUCE_ANY 0u /* Iterate While Any(some vertex changed) */
#define IRGL_REDUCE_ALL 1u /* Iterate Until All(no vertex changed): the same loop through
                              the other reduction */

/* A CSR graph: row_ptr int32[n+1] (monotone, row_ptr[0] = 0, row_ptr[n] = m),
 * col int32[m] (destinations in [0, n)), w uint32[m] (weights >= 1) or NULL.
 * All three are DEVICE pointers.  The handle borrows them: the caller keeps
 * them alive and unchanged until irgl_graph_free(). */
typedef struct irgl_csr {
    int32_t n;
    int64_t m;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *w;
    uint32_t flags;
} irgl_csr;

typedef struct irgl_graph_s *irgl_graph;

/* Tuning knobs; a zero field takes the library default.  Nested edge
 * parallelism (Section 4.3) splits the popped vertices into four tiers by
 * out-degree: >= t_grid -> every workgroup of the grid takes an equal share
 * of the range, >= t_block -> the whole workgroup strides the neighbour
 * range, >= t_wave -> one 64-lane wavefront strides it, otherwise the
 * remaining ranges of a workgroup are concatenated by a prefix sum in LDS and
 * dealt to the lanes in full rounds (load-balanced gather).  By default only
 * the grid and gather tiers are used; the workgroup and wavefront tiers take
 * ranges when their thresholds are set. */
typedef struct irgl_config {
    int32_t block;        /* threads per workgroup: 256, 512 or 1024 (default: 1024
                             for BFS, 512 for SSSP) */
    int32_t t_wave;       /* wavefront tier threshold, >= 1 (default: t_block, or 64
                             when t_block is set) */
    int32_t t_block;      /* workgroup tier threshold, >= t_wave (default: t_grid) */
    int32_t t_grid;       /* grid tier threshold, >= t_block: such vertices are split
                             into equal chunks over all workgroups after a grid
                             barrier (default max(512, t_block), max(256,
                             t_block) for outlined SSSP; lowered to
                             block for a worklist with fewer items than the grid has
                             threads); IRGL_GRID_TIER_OFF = never */
    int32_t grid;         /* workgroups; 0 = co-resident limit (occupancy x CUs) */
    int32_t mode;         /* IRGL_MODE_* */
    uint32_t max_iter;    /* safety cap on invocations (default n + 1 for BFS,
                             4n + 16 for SSSP, whose threshold raises also count) */
    uint32_t wl_capacity; /* worklist capacity in items (default n); smaller values
                             exist to exercise the overflow path */
    uint32_t watchdog_ms; /* grid-barrier wait limit in ms (default 20000);
                             IRGL_WATCHDOG_IMMEDIATE makes every wait time out at
                             once, to exercise the watchdog path */
    const volatile int32_t *abort_flag; /* HOST pinned memory or NULL; a nonzero value
                             makes the running query stop with IRGL_ERR_ABORTED */
    uint32_t t_bitmap;    /* A bitmap of vertices that cannot improve (BFS: visited;
                             SSSP: settled, i.e. distance below a drained
                             threshold) lets relaxations skip them with an L2 bit
                             test.  It is rebuilt by a full scan once this many
                             items were popped since the last rebuild (BFS default
                             n^2 / 2m); IRGL_BITMAP_NEVER disables it (the SSSP
                             default) */
    uint32_t trace_len;   /* entries of `trace` */
    uint32_t do_alpha;    /* BFS on a symmetric graph (IRGL_SYMMETRIC): switch an
                             invocation to bottom-up (every unvisited vertex looks
                             for a neighbour in the frontier, first hit wins) when
                             the frontier's edges exceed the unexplored edges /
                             do_alpha; default 14; IRGL_DO_OFF = always top-down */
    uint32_t do_beta;     /* ... and back to top-down when the frontier holds fewer
                             than n / do_beta vertices (default 96) */
    uint32_t delta;       /* SSSP: near/far threshold step.  Distances below the
                             threshold are expanded in bulk-synchronous invocations;
                             larger ones wait on a far list until the threshold has
                             risen past them.  0 = the default, from the shape of
                             a graph uploaded with IRGL_VALIDATE (mean weight W,
                             mean out-degree D, largest out-degree X): D < 8:
                             32 W / D; D >= 8 and X <= 16 D: 16 W / D; D >= 8
                             and X > 16 D (scale-free): W from 2^26 edges on;
                             on a relabelled weighted upload, whose SSSP copy
                             is partitioned into light and heavy edges at the
                             step, W / 8 from 2^22 edges if IRGL_SYMMETRIC,
                             else W / 4 from 2^25 edges and W / 2 from 2^24;
                             otherwise (and without IRGL_VALIDATE)
                             IRGL_DELTA_NONE (plain Bellman-Ford order).  A
                             vertex whose distance has not changed since its
                             last expansion is not expanded again */
    uint64_t *trace;      /* DEVICE uint64[trace_len], zeroed by the caller, or NULL.
                             Twelve words per invocation i at 12i: wall-clock tick at
                             its start, incoming worklist size, edges scanned, vertices
                             deferred to the grid tier, tick at the start of the
                             grid-tier phase (0: none), claim atomics tried (BFS CAS /
                             SSSP atomicMin), claim atomics won, largest and summed
                             per-workgroup busy ticks of the expansion phase, the same
                             for the grid-tier phase, 0; then the end tick at
                             12 x iterations.  In persistent mode top-down
                             invocations fill every word, bottom-up invocations
                             all but the busy ticks, and SSSP far-to-near transfer
                             invocations only the first two (on a partitioned
                             graph also the heavy pass they run: words 2-10); in host-loop mode
                             every invocation writes its first two words;
                             topology-driven launches record no trace */
    uint32_t barrier;     /* grid-barrier coherence scheme: IRGL_BARRIER_XCD (default:
                             one L2 write-back per XCD per barrier) or
                             IRGL_BARRIER_WORKGROUP (write-back and invalidate per
                             workgroup).  IRGL_BARRIER_XCD falls back to
                             IRGL_BARRIER_WORKGROUP for a launch whose workgroups are
                             not dealt round-robin to the XCDs.  Results do not
                             depend on it. */
    uint32_t reduce;      /* IRGL_MODE_TOPOLOGY: IRGL_REDUCE_ANY (default) or
                             IRGL_REDUCE_ALL; other values are IRGL_ERR_CONFIG */
} irgl_config;

/* Per-query statistics, written by the device when the query ends. */
typedef struct irgl_stats {
    int32_t status;        /* irgl_status of the device-side run */
    uint32_t iterations;   /* kernel invocations (BFS: max level + 1) */
    uint64_t items;        /* worklist items popped, summed over invocations */
    uint64_t edges;        /* CSR entries scanned */
    uint32_t max_frontier; /* largest incoming worklist */
    int32_t grid;          /* workgroups used */
    int32_t block;         /* threads per workgroup used */
    uint32_t heavy_pulls;  /* SSSP heavy passes run as a pull (Section 4.1's
                              heavy edges seen from their unsettled ends, on a
                              split symmetric graph); 0 for BFS and batches */
    uint64_t frontier_edges; /* sum of the out-degrees of every worklist (BFS: the
                             CSR entries an exact top-down traversal scans, also
                             when bottom-up invocations scanned fewer) */
} irgl_stats;

int irgl_version(void);
const char *irgl_status_string(irgl_status s);
/* hipError_t of the last failed HIP call in this thread (0 if none). */
int32_t irgl_last_hip_error(void);
/* Wall-clock tick rate (kHz) of the device the calling thread uses, for
 * converting `trace` entries to time. */
irgl_status irgl_wallclock_khz(int32_t *khz);
/* Return the library's process-lifetime host resources (the pinned read-back
 * words of IRGL_MODE_HOST_LOOP queries) to the HIP runtime.  Call it once no
 * query is running, before the process exits: the library frees nothing from
 * static destructors, which may run after the HIP runtime has been torn down.
 * Graphs, batches and servers are released by their own free/close calls.
 * The library stays usable afterwards (a later host-loop query allocates a
 * new word).  Returns IRGL_ERR_DEVICE if a free failed. */
irgl_status irgl_shutdown(void);

/* Register a device-resident CSR graph (Section 4.1: the graph whose
 * edges(n) the BFS kernel iterates).  *out receives a handle that borrows the
 * caller's arrays.  With IRGL_VALIDATE the CSR is checked on the device and
 * the call synchronizes; a malformed graph gives IRGL_ERR_INVALID_GRAPH.  The
 * same pass sums the weights and finds the largest out-degree, from which the
 * SSSP near/far step defaults (irgl_config.delta).
 * Errors: INVALID_ARGUMENT (null csr/out/row_ptr, null col with m > 0,
 * n <= 0, m < 0, m >= 2^31), NO_DEVICE, DEVICE. */
irgl_status irgl_graph_upload(const irgl_csr *csr, irgl_graph *out);

/* Degree-sorted relabelling.  A graph uploaded this way is traversed in a
 * copy whose vertex ids are sorted by decreasing out-degree (ties by id):
 * most edges of a skewed graph point at few high-degree vertices, whose
 * levels / distances then share few cache lines and stay in the L2, so most
 * per-edge probes of a traversal hit L2 instead of the Infinity Cache.
 * Queries on the handle take and return CALLER vertex ids (sources, levels,
 * distances, parents; SSSP parents are the smallest caller-id tight
 * predecessor, as for a plain upload); irgl_bfs / irgl_sssp then need a
 * larger workspace (irgl_workspace_bytes accounts for it) and end with one
 * scatter to caller ids.  Batched and served tasks on the handle traverse the
 * caller's arrays.
 *
 * irgl_reorder_bytes: device bytes of the copy (and of its build scratch)
 * for a graph of n vertices and m edges, weighted or not.
 * irgl_graph_upload_reordered: checks csr as irgl_graph_upload does (flags
 * as there), builds the copy in `store` (DEVICE, at least
 * irgl_reorder_bytes, borrowed until irgl_graph_free, like the CSR arrays,
 * which also stay borrowed) on the current device's null stream, and
 * synchronizes.  IRGL_ERR_WORKSPACE_TOO_SMALL when store_bytes is short.
 *
 * A weighted graph also gets an SSSP copy whose rows are partitioned at the
 * graph's default near/far step: edges lighter than the step first, then
 * the heavy ones (each part in id order).  Single SSSP queries that use that
 * step expand only light edges when a vertex is popped and relax each heavy
 * edge once, with the vertex's final distance, after its bucket has drained
 * (the light/heavy split of bucketed shortest paths); results are the same
 * as without it.  irgl_reorder_bytes counts this copy (8 bytes per edge and
 * 4 per vertex more for a weighted graph). */
irgl_status irgl_reorder_bytes(int32_t n, int64_t m, int32_t weighted, size_t *bytes);
irgl_status irgl_graph_upload_reordered(const irgl_csr *csr, void *store, size_t store_bytes, irgl_graph *out);

/* Change the SSSP near/far step that single queries on g take when their
 * configuration leaves delta at 0 (IRGL_DELTA_NONE: plain Bellman-Ford
 * order).  On a relabelled weighted graph the light/heavy partition of its
 * SSSP copy is rebuilt for the new step on the graph's device (synchronous).
 * Must not run while a query on g is in flight.  Batched and served tasks
 * keep the rule given at irgl_config.delta.
 * Errors: INVALID_ARGUMENT (null g, delta 0), DEVICE. */
irgl_status irgl_graph_set_delta(irgl_graph g, uint32_t delta);

/* Release a handle (not the arrays it borrows).  NULL is accepted. */
irgl_status irgl_graph_free(irgl_graph g);

/* The SSSP near/far step that a query on g uses when its configuration leaves
 * delta at 0 (the rule is given at irgl_config.delta; the mean weight, mean
 * and largest out-degree come from the upload's IRGL_VALIDATE pass; a graph
 * with a partitioned SSSP copy takes its partition step, and
 * irgl_graph_set_delta changes it).  *delta receives IRGL_DELTA_NONE for
 * plain Bellman-Ford order.  No device work.
 * Errors: INVALID_ARGUMENT (null g or delta). */
irgl_status irgl_graph_default_delta(irgl_graph g, uint32_t *delta);

/* Bytes of device workspace one query of `kind` needs on graph g with the
 * given config (NULL = defaults).  The workspace holds the two worklists of
 * the pipe context (Section 4.2: "in" and "out"), the loop's counters and
 * barrier state, for BFS a visited bitmap and for SSSP the per-vertex push
 * stamps, the two far lists and far flags. */
irgl_status irgl_workspace_bytes(irgl_graph g, int32_t kind, int32_t with_parent,
                                 const irgl_config *cfg, size_t *bytes);

/* BFS levels from src (Section 4.1, level-by-level worklist BFS; the level
 * of src is 0 and a vertex found while expanding level k gets k + 1).
 * level: device uint32[n] (output).  parent: device int32[n] or NULL; when
 * given, parent[src] = src, unreached = -1, otherwise a vertex p with an edge
 * p -> v and level[p] + 1 == level[v] (not unique).  ws: device workspace of
 * ws_bytes >= irgl_workspace_bytes(g, IRGL_KIND_BFS, ...).  dstats: device
 * irgl_stats or NULL.  cfg: NULL = defaults. */
irgl_status irgl_bfs(irgl_graph g, int32_t src, uint32_t *level, int32_t *parent, void *ws,
                     size_t ws_bytes, void *stream, irgl_stats *dstats, const irgl_config *cfg);

/* Single-source shortest paths from src by the same data-driven worklist
 * loop (bulk-synchronous Bellman-Ford: a vertex whose distance improved is
 * pushed once per invocation).  dist: device uint32[n] (output).  parent:
 * device int32[n] or NULL; when given, parent[v] is the smallest vertex id p
 * with an edge p -> v of weight w and dist[p] + w == dist[v] (deterministic).
 * Requires weights (IRGL_ERR_NO_WEIGHTS otherwise).  A finite distance that
 * does not fit below IRGL_INF ends the query with IRGL_ERR_OVERFLOW. */
irgl_status irgl_sssp(irgl_graph g, int32_t src, uint32_t *dist, int32_t *parent, void *ws,
                      size_t ws_bytes, void *stream, irgl_stats *dstats, const irgl_config *cfg);

/* irgl_sssp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * query's workspace is a device array of IRGL_NOALLOC_SCRATCH_BYTES that the
 * library holds (one per device, from the library's load until the process
 * ends).  The call allocates nothing: no hipMalloc / hipFree, no allocating
 * library routine; the caller still passes the outputs (dist, parent, dstats
 * as for irgl_sssp).  Every call on one device shares that device's array,
 * and each query resets what it reads before the kernel uses it, so calls
 * that run one after another need nothing cleared; calls that OVERLAP on one
 * device (on different streams, or from different threads without ordering)
 * race on the array and give undefined results.  The statistics of a query
 * are read through dstats (irgl_query_status needs the workspace address).
 * Errors: as irgl_sssp; IRGL_ERR_TOO_LARGE when the query's workspace
 * (irgl_workspace_bytes for the same graph, config and parent choice) exceeds
 * IRGL_NOALLOC_SCRATCH_BYTES (64 MiB: up to about 1.3M vertices with the
 * default config); IRGL_ERR_CONFIG for IRGL_MODE_HOST_LOOP (its read-back
 * word is allocated on first use). */
#define IRGL_NOALLOC_SCRATCH_BYTES (64u << 20)
irgl_status irgl_sssp_noalloc(irgl_graph g, int32_t src, uint32_t *dist, int32_t *parent, void *stream,
                              irgl_stats *dstats, const irgl_config *cfg);

/* Synchronize `stream`, then copy the statistics of the last query that used
 * workspace `ws` into host memory *out (status, iterations, counters). */
irgl_status irgl_query_status(const void *ws, void *stream, irgl_stats *out);

/* ---------------------------------------------------------------------
 * Batched queries: many BFS/SSSP instances, of uneven graph sizes and
 * sources, in ONE persistent cooperative launch fed from a device-resident
 * task queue.  The grid is split into teams of `team` workgroups; each team
 * repeatedly takes the next task (largest first), runs the outlined Iterate
 * loop of Section 4.3 on it with its own barrier and scratch, and writes the
 * task's statistics.  The control kernel holds both loop bodies, so its
 * workgroup size is taken from T_control = T_BFS ∩ T_SSSP (Section 4.3);
 * irgl_control_block_sizes() reports that set.
 * --------------------------------------------------------------------- */
typedef struct irgl_task {
    irgl_graph g;
    int32_t kind;      /* IRGL_KIND_BFS or IRGL_KIND_SSSP */
    int32_t src;
    uint32_t *out;     /* device uint32[n] (levels or distances) */
    int32_t *parent;   /* device int32[n] or NULL (same meaning as irgl_bfs/irgl_sssp) */
    uint64_t tag;      /* caller's cookie, not interpreted */
} irgl_task;

typedef struct irgl_batch_config {
    int32_t block;     /* workgroup size, a member of T_control (default 256) */
    int32_t team;      /* workgroups per team (default 16; clamped to the grid) */
    int32_t t_wave;    /* tier thresholds as in irgl_config (0 = defaults) */
    int32_t t_block;
    int32_t t_grid;
    uint32_t delta;    /* SSSP near/far step for every task (0 = per-graph default) */
    uint32_t watchdog_ms;
    int32_t grid;      /* workgroups (0 = co-resident limit); rounded down to whole teams */
    uint32_t barrier;  /* team-barrier scheme, as irgl_config.barrier */
    uint32_t gang_edges; /* open batches: a task on a graph with at least this many
                            edges runs on the whole grid (all teams together, in
                            ring order) instead of one team (0 = 2^23) */
    uint32_t gang_queue; /* open batches: a task enqueued while fewer than this many
                            tasks are in flight (issued, not yet polled done) also
                            runs on the whole grid: at low load the whole grid gives
                            the lowest latency, at high load teams give throughput
                            (0 = off) */
} irgl_batch_config;

typedef struct irgl_batch_s *irgl_batch;

/* Workgroup sizes usable by the batched control kernel (T_control).  Writes
 * up to `cap` sizes, ascending, to sizes[] and their count to *count. */
irgl_status irgl_control_block_sizes(int32_t *sizes, int32_t cap, int32_t *count);

/* Device workspace bytes for a batch of `ntasks` host-described tasks. */
irgl_status irgl_batch_workspace_bytes(const irgl_task *tasks, int32_t ntasks,
                                       const irgl_batch_config *cfg, size_t *bytes);

/* Launch the batch asynchronously on `stream`.  tasks: HOST array, read
 * during the call.  ws: device workspace.  *out receives a handle for
 * irgl_batch_wait / irgl_batch_free.  Errors: INVALID_ARGUMENT (bad task,
 * ntasks <= 0), NO_WEIGHTS, WORKSPACE_TOO_SMALL, CONFIG, DEVICE. */
irgl_status irgl_batch_submit(const irgl_task *tasks, int32_t ntasks, void *ws, size_t ws_bytes,
                              const irgl_batch_config *cfg, void *stream, irgl_batch *out);

/* Wait for the batch (synchronizes its stream) and copy each task's
 * statistics, in task order, to per_task (HOST irgl_stats[ntasks], or NULL).
 * Returns IRGL_OK when the launch completed; per-task device errors are in
 * per_task[i].status. */
irgl_status irgl_batch_wait(irgl_batch b, irgl_stats *per_task);

/* Release the handle (waits for the batch first). */
irgl_status irgl_batch_free(irgl_batch b);

/* ---------------------------------------------------------------------
 * Pipes (Section 4.2, Compiling Pipe; Section 4.3, Compiling Kernel
 * Invocations).  A pipe program is a list of orchestration statements over
 * the library's kernel bodies, run by ONE outlined control kernel (a
 * cooperative persistent launch; every invocation is a device-function call
 * followed by a grid barrier).  All statements share the pipe context: the
 * incoming, outgoing and retry worklists `in`, `out`, `retry` (each of n
 * vertex ids).  An invocation of a body that uses worklists pops `in` and
 * pushes `out` (with cooperative conversion); afterwards `in` and `out` are
 * swapped.  A body that also uses `retry` is invoked again, with `in` and
 * `retry` swapped and `out` kept, while its retry list is non-empty; then
 * `in` and `out` are swapped.  A body that uses no worklist leaves them as
 * they are.
 *
 * Statements (irgl_pipe_op.op; a, b are arguments):
 *   IRGL_PIPE_INVOKE  a = body: one invocation (Invoke)
 *   IRGL_PIPE_ITERATE a = body: invocations until its worklist is empty, or,
 *                     for a body that returns a reduction, until it returns
 *                     false (Iterate)
 *   IRGL_PIPE_BEGIN   a = 0: a looping Pipe (its statements repeat while
 *                     `in` is non-empty at its END), a = 1: Pipe Once
 *   IRGL_PIPE_END     closes the innermost BEGIN
 *   IRGL_PIPE_IF      a = condition, b = the statement to continue at when it
 *                     is false (forward only): the consumer of a worklist is
 *                     chosen at run time (dynamic piping)
 *   IRGL_PIPE_JUMP    a = statement to continue at (forward only)
 *   IRGL_PIPE_INIT_SOURCE  `in` = [io->src] (the scalar worklist initializer);
 *                     BFS levels are reset to INF except level[src] = 0
 * Conditions: IRGL_COND_IN_EMPTY (`in` is empty), IRGL_COND_FRONTIER_LARGE
 * (`in` holds at least n / 16 vertices), IRGL_COND_RETURNED (the last
 * reduction returned true); IRGL_COND_NOT (or'ed in) negates.
 *
 * T_control (Section 4.3): each body has a set T_k of workgroup sizes it can
 * run with, from its class (ElasticBlock: any size up to the launch bound
 * of 1024; ShrinkableBlock: up to `block`; FixedBlock: exactly `block`) and
 * its LDS footprint (lds_base + lds_per_thread x size must fit the device's
 * per-workgroup LDS).  The control kernel of a program runs with the largest
 * size in the intersection of its bodies' sets; an empty intersection means
 * the pipe cannot be outlined (IRGL_ERR_CONFIG).  Sizes are powers of two
 * from 64 to 1024.
 * --------------------------------------------------------------------- */
enum {
    IRGL_PIPE_INVOKE = 0,
    IRGL_PIPE_ITERATE = 1,
    IRGL_PIPE_BEGIN = 2,
    IRGL_PIPE_END = 3,
    IRGL_PIPE_IF = 4,
    IRGL_PIPE_JUMP = 5,
    IRGL_PIPE_INIT_SOURCE = 6
};
enum { IRGL_COND_IN_EMPTY = 0, IRGL_COND_FRONTIER_LARGE = 1, IRGL_COND_RETURNED = 2 };
#define IRGL_COND_NOT 0x100

/* Kernel bodies a program may invoke. */
enum {
    IRGL_BODY_BFS_PUSH = 0,     /* top-down BFS level: pops `in`, labels unvisited out-neighbours
                                   with the next level, pushes them (nested edge parallelism) */
    IRGL_BODY_BFS_PULL = 1,     /* bottom-up BFS level (symmetric graphs): every unvisited vertex
                                   with a neighbour in the current level is labelled and pushed */
    IRGL_BODY_MST_INIT = 2,     /* Boruvka: every vertex its own component; pushes the vertices
                                   that have edges (worklist initializer from an array) */
    IRGL_BODY_MST_FINDMIN = 3,  /* pops `in`: a vertex's lightest edge to another component becomes
                                   the component's candidate inside a non-blocking Atomic section;
                                   the vertex is pushed to `out` when it had such an edge, or to
                                   `retry` when the section's lock was busy (Atomic ... Else) */
    IRGL_BODY_MST_HOOK = 4,     /* every component root hooks to the component at the other end of
                                   its candidate edge, which joins the forest */
    IRGL_BODY_MST_JUMP = 5,     /* pointer jumping over the hooks; returns Any(changed) */
    IRGL_BODY_MST_RELABEL = 6,  /* every vertex moves to its component's new root */
    IRGL_BODY_MST_MINID = 7,    /* smallest vertex id of every component */
    IRGL_BODY_MST_LABEL = 8,    /* component[v] = that smallest id */
    IRGL_BODY_COUNT = 9
};

#define IRGL_BLOCK_ELASTIC 0
#define IRGL_BLOCK_SHRINKABLE 1
#define IRGL_BLOCK_FIXED 2

typedef struct irgl_block_constraint {
    int32_t kind;            /* IRGL_BLOCK_* */
    int32_t block;           /* ShrinkableBlock: largest size; FixedBlock: the size; Elastic: ignored */
    int32_t lds_base;        /* LDS bytes per workgroup ... */
    int32_t lds_per_thread;  /* ... plus this many per thread */
} irgl_block_constraint;

typedef struct irgl_pipe_op {
    int32_t op;
    int32_t a;
    int32_t b;
    int32_t reserved;
} irgl_pipe_op;

typedef struct irgl_pipe_io {
    int32_t src;             /* source of IRGL_PIPE_INIT_SOURCE */
    uint32_t *level;         /* BFS bodies: DEVICE uint32[n] (output) */
    int32_t *component;      /* MST bodies: DEVICE int32[n] (output: smallest vertex id of the tree) */
    uint8_t *in_forest;      /* MST bodies: DEVICE uint8[m] (output: 1 on both entries of forest edges) */
    uint64_t *weight;        /* MST bodies: DEVICE uint64[1] (output: forest weight) */
    int32_t *trace;          /* DEVICE int32[trace_len] or NULL: the body of each invocation */
    uint32_t trace_len;
    int32_t block;           /* 0 = the largest size of T_control; else a member of it */
    uint32_t max_invocations; /* safety cap (0 = 8 n + 64): IRGL_ERR_ITERATION_LIMIT */
    uint32_t watchdog_ms;    /* 0 = 20000 */
    int32_t grid;            /* workgroups (0 = co-resident limit) */
    uint32_t force_retry;    /* test knob: 1 = in the first round of every MST_FINDMIN invocation
                                the vertices with odd ids take the Else branch (retry) as if
                                their lock were busy; results are unchanged */
} irgl_pipe_io;

/* T_control of a set of constraints for a per-workgroup LDS limit (bytes):
 * the largest power-of-two size in [64, 1024] that every constraint admits,
 * or IRGL_ERR_CONFIG when none does.  Host-only. */
irgl_status irgl_control_block(const irgl_block_constraint *k, int32_t nk, int32_t lds_limit, int32_t *block);
/* The constraint of a library body (from its launch bound and LDS layout).  Host-only. */
irgl_status irgl_pipe_body_constraint(int32_t body, irgl_block_constraint *out);
/* Structural check of a program: known statements, conditions and bodies,
 * balanced BEGIN/END (at most 8 deep), forward targets in range, ITERATE of
 * bodies that use a worklist or return a reduction, and at least one
 * invocation inside every looping Pipe.  Host-only (IRGL_ERR_INVALID_ARGUMENT). */
irgl_status irgl_pipe_check(const irgl_pipe_op *prog, int32_t nops);
/* T_control of a program's bodies; lds_limit 0 = the current device's. */
irgl_status irgl_pipe_control_block(const irgl_pipe_op *prog, int32_t nops, int32_t requested, int32_t lds_limit,
                                    int32_t *block);
/* Device workspace bytes of a program on g. */
irgl_status irgl_pipe_workspace_bytes(irgl_graph g, const irgl_pipe_op *prog, int32_t nops, size_t *bytes);
/* Run a program on g (caller's vertex ids) asynchronously on `stream`; the
 * program is copied during the call.  The outputs a program's bodies need
 * must be given in io (INVALID_ARGUMENT otherwise); BFS_PULL and the MST
 * bodies need a symmetric graph (IRGL_SYMMETRIC; CONFIG otherwise), the MST
 * bodies weights (NO_WEIGHTS).  Device-side errors are in dstats->status.
 * stats: iterations = invocations, items = popped worklist items, edges =
 * scanned CSR entries, max_frontier = largest `in`. */
irgl_status irgl_pipe_run(irgl_graph g, const irgl_pipe_op *prog, int32_t nops, const irgl_pipe_io *io, void *ws,
                          size_t ws_bytes, void *stream, irgl_stats *dstats);

/* ---------------------------------------------------------------------
 * Open batches (serving): the teams of a persistent server kernel take
 * tasks from a ring in host pinned memory WHILE the kernel runs, so a
 * request that arrives while others are on the GPU starts as soon as a team
 * is free and overlaps them (continuous batching).  A task on a graph with
 * at least cfg->gang_edges edges is a gang task: when it reaches the head of
 * the ring, every team joins it after its current task and the whole grid
 * runs it.  The kernel ends (all teams together) after `idle_ms` without
 * work or at close; irgl_batch_enqueue and irgl_batch_poll relaunch it when
 * work is pending.  Calls on one server must come from one host thread.
 * --------------------------------------------------------------------- */
typedef struct irgl_server_s *irgl_server;

/* Device workspace bytes of a server able to run tasks on any of graphs[]. */
irgl_status irgl_batch_open_bytes(const irgl_graph *graphs, int32_t ngraphs,
                                  const irgl_batch_config *cfg, int32_t ring_cap, size_t *bytes);

/* Create a server (launches nothing yet).  graphs[]: every graph a task may
 * use (each team's scratch is sized for the largest graph below the gang
 * threshold, one gang region for the largest at or above it).  ring_cap:
 * descriptors in flight (queued, running, or finished and not yet polled)
 * at most.  idle_ms: 0 = 50; at most a quarter of the watchdog
 * (IRGL_ERR_CONFIG otherwise).  ws: device workspace of at least
 * irgl_batch_open_bytes(...).  The server owns small pinned host buffers. */
irgl_status irgl_batch_open(const irgl_graph *graphs, int32_t ngraphs, const irgl_batch_config *cfg,
                            int32_t ring_cap, uint32_t idle_ms, void *ws, size_t ws_bytes, void *stream,
                            irgl_server *out);

/* Queue one task; *ticket identifies it (tickets count up from 0).  Ticket t
 * uses ring slot t % ring_cap, which is free once ticket t - ring_cap has been
 * reported done by irgl_batch_poll; otherwise IRGL_ERR_BUSY (poll, then
 * retry).  Asynchronous. */
irgl_status irgl_batch_enqueue(irgl_server s, const irgl_task *task, uint64_t *ticket);

/* *done = 1 and *st = the task's statistics when the task has finished (its
 * outputs are then visible to the host and other streams), else *done = 0.
 * A ticket stays pollable until its slot is reused; polling it after that,
 * or polling a ticket never issued, is IRGL_ERR_INVALID_ARGUMENT.
 * Relaunches the server kernel if it has ended with work pending. */
irgl_status irgl_batch_poll(irgl_server s, uint64_t ticket, irgl_stats *st, int32_t *done);

/* Server kernel launches so far (*launches), and how many of them gave up
 * at their start check (*gave_up): the grid barrier needs every workgroup
 * resident, so a launch whose workgroups are not all running within a few
 * milliseconds (a kernel on another stream holds part of the device) ends
 * before it claims any descriptor, and the next irgl_batch_enqueue or
 * irgl_batch_poll launches it again.  Diagnostics only. */
irgl_status irgl_batch_launches(irgl_server s, uint64_t *launches, uint64_t *gave_up);

/* Stop the server kernel, wait for it and release the handle. */
irgl_status irgl_batch_close(irgl_server s);

/* ---------------------------------------------------------------------
 * Minimum spanning forest by Boruvka's algorithm: the workload of the
 * Atomic construct (Section 3, the find-minimum-cross-component-edge
 * kernel, whose atomic section updates a component's lightest weight and
 * its edge together).  Rounds of find-min-edge over the vertices that still
 * have a cross-component edge, hooking, and pointer jumping run in one
 * cooperative launch with the grid barrier between phases.  Edges are
 * ordered by (weight, smaller endpoint, larger endpoint), so the forest is
 * unique.  The graph must be symmetric (every edge stored in both
 * directions with the same weight) with rows sorted by destination (as
 * the library's generators and irgl_graph_upload produce them; unsorted
 * rows are correct but slower); results refer to the caller's vertex ids
 * and CSR entries, also for a relabelled upload.
 * --------------------------------------------------------------------- */

/* How the atomic section is compiled. */
#define IRGL_LOCK_PACKED 0u /* the two words form one 64-bit key (weight << 32 | edge),
                               updated by one 64-bit atomicMin (default) */
#define IRGL_LOCK_SPIN 1u   /* Atomic, blocking: a compare-and-swap lock per component
                               taken in a divergence-safe retry loop */
#define IRGL_LOCK_TICKET 2u /* Atomic under a ticket lock per component */

typedef struct irgl_mst_config {
    int32_t block;        /* 256, 512 (default) or 1024 */
    int32_t grid;         /* workgroups; 0 = co-resident limit */
    uint32_t lock;        /* IRGL_LOCK_* */
    uint32_t watchdog_ms; /* bound of every barrier and lock wait (default 20000) */
    uint32_t barrier;     /* IRGL_BARRIER_* */
} irgl_mst_config;

/* Device workspace bytes of irgl_mst on graph g. */
irgl_status irgl_mst_workspace_bytes(irgl_graph g, size_t *bytes);

/* Minimum spanning forest of g (weights required unless g has no edges).  weight: DEVICE uint64[1],
 * the forest weight.  component: DEVICE int32[n] or NULL: the smallest vertex
 * id of each vertex's tree.  in_forest: DEVICE uint8[m] or NULL: 1 for both
 * stored directions of every forest edge, else 0.  ws: at least
 * irgl_mst_workspace_bytes.  dstats (DEVICE, optional): iterations = rounds,
 * items = worklist vertices summed over rounds, edges = CSR entries scanned,
 * frontier_edges = forest edges.  Asynchronous on `stream`.  Errors:
 * IRGL_ERR_NO_WEIGHTS, IRGL_ERR_CONFIG (block / lock / barrier),
 * IRGL_ERR_TOO_LARGE (m >= 2^31), IRGL_ERR_WORKSPACE_TOO_SMALL; on the device
 * (in dstats.status) IRGL_ERR_INVALID_GRAPH for an edge without its reverse,
 * IRGL_ERR_WATCHDOG for a wait past the limit. */
irgl_status irgl_mst(irgl_graph g, uint64_t *weight, int32_t *component, uint8_t *in_forest, void *ws,
                     size_t ws_bytes, void *stream, irgl_stats *dstats, const irgl_mst_config *cfg);

/* ---------------------------------------------------------------------
 * Delaunay mesh refinement: the workload of the Exclusive construct
 * (Section 3, Exclusive: the refine kernel, whose item must own every
 * triangle of its bad triangle's cavity and every triangle bordering it;
 * the locks are taken in three phases, race / priority check / check,
 * separated by grid barriers, and an item that loses goes back to the
 * worklist) and of the Pipe of the DMR main loop (Section 4.2: identify
 * the bad triangles once, then a looping Pipe of refine and incremental
 * identification among the triangles refine created, then one more
 * identification as a sanity check), all in ONE cooperative launch.
 *
 * The mesh triangulates the unit square [0,1]^2 and is Delaunay on entry
 * (the generators in meshgen.py build such meshes).  A triangle needs work
 * when its smallest angle is below the bound or when one of its boundary
 * edges is encroached (its opposite vertex sees it at more than 90
 * degrees).  Refinement inserts the circumcentre of a bad triangle, or, when
 * that point falls outside the domain or inside the diametral circle of a
 * boundary edge, the midpoint of that edge; the new point's cavity is
 * re-triangulated (Bowyer-Watson), so the mesh stays Delaunay.  On success
 * no triangle needs work; the result is not unique (it depends on the
 * order of insertions).
 * --------------------------------------------------------------------- */
typedef struct irgl_mesh {
    double *pts;    /* DEVICE float64[pcap][2]: x, y; the first npts in use */
    int32_t *tri;   /* DEVICE int32[tcap][4]: v0, v1, v2 (counter-clockwise), live flag */
    int32_t *nbr;   /* DEVICE int32[tcap][4]: entry i = the triangle across edge
                       (v_i, v_(i+1) mod 3), -1 on the domain boundary; entry 3 unused */
    int32_t npts;   /* points in use on entry (>= 3) */
    int32_t ntri;   /* triangle slots in use on entry (>= 1), all live */
    int32_t pcap;   /* capacity of pts (rows) */
    int32_t tcap;   /* capacity of tri and nbr (rows), below 2^30 */
} irgl_mesh;

typedef struct irgl_dmr_config {
    double min_angle;          /* quality bound in degrees, in (0, 60); 0 = 30 */
    int32_t block;             /* 64, 128 or 256 (default) threads per workgroup */
    int32_t grid;              /* workgroups; 0 = co-resident limit */
    uint32_t max_invocations;  /* safety cap of kernel invocations (0 = 100000) */
    uint32_t watchdog_ms;      /* bound of every barrier wait (0 = 20000) */
    uint32_t barrier;          /* IRGL_BARRIER_* */
    uint32_t reserved;
} irgl_dmr_config;

/* Written by the device when the refinement ends. */
typedef struct irgl_dmr_stats {
    int32_t status;          /* irgl_status of the run */
    uint32_t invocations;    /* kernel invocations of the pipe */
    uint32_t rounds;         /* Exclusive rounds (three phases each) over all refine invocations */
    int32_t block;
    int32_t grid;
    uint32_t reserved;
    uint64_t refined;        /* worklist items popped by refine */
    uint64_t conflicts;      /* items that lost their Exclusive section (Else: retried) */
    uint32_t inserted;       /* circumcentres inserted */
    uint32_t splits;         /* boundary edges split at their midpoint */
    int32_t npts;            /* points in use at the end */
    int32_t ntri;            /* triangle slots in use at the end (all live) */
    uint32_t final_bad;      /* triangles needing work found by the final identification (0 on success) */
    uint32_t max_cavity;     /* largest cavity re-triangulated */
} irgl_dmr_stats;

/* Device workspace bytes of irgl_dmr_refine on a mesh of this capacity:
 * the pipe's two worklists, the lock and push-stamp words (one per triangle
 * slot) and the control block.  Errors: INVALID_ARGUMENT (null pointers,
 * npts < 3, ntri < 1, capacities below the counts or at least 2^30). */
irgl_status irgl_dmr_workspace_bytes(const irgl_mesh *m, size_t *bytes);

/* Refine *m in place, asynchronously on `stream`: points are appended after
 * npts (the input points keep their indices and coordinates), triangles are
 * rewritten in their slots and appended after ntri; the final counts are in
 * dstats (DEVICE irgl_dmr_stats, optional).  ws: DEVICE, at least
 * irgl_dmr_workspace_bytes.  Errors: as irgl_dmr_workspace_bytes,
 * WORKSPACE_TOO_SMALL, CONFIG (angle, block, grid, barrier); on the device
 * (dstats.status) OVERFLOW when the point or triangle capacity or a cavity
 * bound (64 triangles) is exceeded, ITERATION_LIMIT, WATCHDOG, INTERNAL when
 * a geometric step fails (a point location that does not end, a cavity that
 * is not star-shaped); the mesh is then not valid. */
irgl_status irgl_dmr_refine(const irgl_mesh *m, void *ws, size_t ws_bytes, const irgl_dmr_config *cfg, void *stream,
                            irgl_dmr_stats *dstats);

#ifdef __cplusplus
}
#endif

#endif /* IRGL_H */
