/*
 * bfs.h -- C ABI of libbfsmi, a single-GPU (gfx950) level-synchronous
 * breadth-first search.
 *
 * The search is the local frontier expansion of Bisson, Bernaschi and
 * Mastrostefano, "Parallel Distributed Breadth First Search on the Kepler
 * Architecture" (2014), run by one GPU over the whole graph:
 *   - per level, an exclusive scan of the frontier vertices' degrees and a
 *     search of that cumulative array that maps every frontier edge to a
 *     thread (Section 3.4, the mapping formula and Algorithm 3; multi-edge
 *     threads, Section 3.4.1);
 *   - a visited bitmap with one bit per vertex, probed with a plain read and
 *     claimed with an atomic OR whose returned word picks the single winner
 *     that sets the vertex's level and predecessor (Algorithm 3);
 *   - compaction of the winners into the next frontier queue (Algorithm 3,
 *     the per-destination counter, here one queue and one counter);
 *   - a bitmap form of the frontier, used when the frontier list would be
 *     longer than the bitmap (threshold T = ceil(V / 32) vertices,
 *     Section 5), converted back to a list by ballot/prefix compaction.
 * Conventions (Algorithm 2 initialisation): level[root] = 0,
 * parent[root] = root, unreached vertices have level -1 and parent -1.
 *
 * All functions return an int status.  No C++ exception crosses the ABI.
 * The message of the last error on the calling thread is bfs_last_error().
 *
 * Memory ownership: the caller owns every device buffer.  A graph handle
 * borrows the CSR arrays and the workspace until bfs_graph_destroy().  The
 * library allocates no device memory on the search path; it allocates a
 * small pinned host block per graph handle at creation.
 *
 * Streams: hip_stream is a hipStream_t passed as void* (NULL = the null
 * stream).  bfs_run / bfs_run_batch enqueue on that stream and return after
 * the stream's work for the call has completed.
 */
#ifndef BFSMI_BFS_H
#define BFSMI_BFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define BFS_OK             0
#define BFS_PENDING        1   /* bfs_poll: the query has not finished      */
#define BFS_ERR_INVALID   -1   /* null pointer, bad size or out-of-range id  */
#define BFS_ERR_NO_DEVICE -2   /* no usable HIP device                        */
#define BFS_ERR_HIP       -3   /* a HIP runtime call failed                   */
#define BFS_ERR_WORKSPACE -4   /* workspace smaller than bfs_workspace_bytes  */
#define BFS_ERR_DEPTH     -5   /* a batch level does not fit int8 (> 127)     */
#define BFS_ERR_BUSY      -6   /* the graph handle is in use by another call  */
#define BFS_ERR_BUDGET    -7   /* a server graph can never fit the arena      */
#define BFS_ERR_TICKET    -8   /* unknown or already collected ticket         */

/* Flags for bfs_workspace_bytes / bfs_graph_create. */
#define BFS_VALIDATE_CSR  0x1u /* check offsets and column ids on creation    */
#define BFS_WS_BATCH      0x2u /* also reserve the multi-source batch arrays  */
#define BFS_DEGREE_ORDER  0x4u /* search on a degree-ordered internal copy of
                                  the CSR (built on the GPU at creation, kept
                                  in the workspace: + 64 V + 8 nnz bytes,
                                  + 64 V more with BFS_WS_BATCH),
                                  each row grouped by id range with per-row
                                  counts for the row prefix skip
                                  (BFS_OPT_ROW_SKIP); results are still in the
                                  caller's ids                              */

/* Options for bfs_set_option (tuning knobs; defaults are sensible). */
#define BFS_OPT_EDGES_PER_THREAD 1 /* 1, 2, 4 or 8 frontier edges per thread    */
#define BFS_OPT_FRONTIER_MODE    2 /* 0 auto (list/bitmap by threshold),
                                      1 list only, 2 bitmap whenever possible */
#define BFS_OPT_LOOP_DRIVER      3 /* 0 (default) or 2: runs of small levels
                                      (frontier <= 65536 vertices, none of
                                      degree > 8192) run in one persistent
                                      launch with a grid barrier per level,
                                      one control-block read per run; 1: every
                                      level from the host, one read per level */
#define BFS_OPT_BATCH_TILE       4 /* edges per workgroup in the batch kernels:
                                      256, 512, 1024 or 2048                  */
#define BFS_OPT_GRID_WGS         5 /* workgroups per CU for grid-stride kernels */
#define BFS_OPT_PROFILE          6 /* 1: time each kernel class with HIP events
                                      (fills the *_ms fields of bfs_stats)    */
#define BFS_OPT_VISITED_SUMMARY  7 /* before heavy levels, summarise the visited
                                      bitmap so the expansion's early visited
                                      test skips most bitmap loads:
                                      0 off, 1 fully visited id prefix,
                                      2 (default) prefix + one LDS bit per
                                      fully visited block of ids              */
#define BFS_OPT_ROW_SKIP         8 /* degree-ordered graphs: 1 (default) lets a
                                      heavy level's degree scan drop each
                                      frontier row's leading block of edges
                                      into the fully visited id prefix (the
                                      early visited test of Section 5 applied
                                      to whole row prefixes: levels and
                                      parents are unchanged, edges_scanned
                                      still counts the dropped edges); needs
                                      BFS_OPT_VISITED_SUMMARY >= 1; 0 off    */
#define BFS_OPT_DIRECTION        9 /* 0 (default) top-down only; 1 direction-
                                      optimizing: a dense level is searched
                                      bottom-up (each unvisited vertex looks
                                      for a visited neighbour, the variant the
                                      paper's related work discusses), with
                                      the switches of Beamer et al.: to
                                      bottom-up when the frontier's edges
                                      times alpha exceed the unvisited
                                      vertices' edges (while the frontier
                                      grows), back for good when the
                                      frontier times beta is below V and
                                      shrinking.
                                      Levels and valid parents are unchanged;
                                      fewer edges are examined
                                      (bfs_stats.edges_examined).  Needs a
                                      symmetric CSR (checked at creation;
                                      BFS_ERR_INVALID otherwise)             */
#define BFS_OPT_DO_ALPHA        10 /* alpha, 1..1000 (default 14)           */
#define BFS_OPT_DO_BETA         11 /* beta, 1..1000 (default 24)            */
#define BFS_OPT_LOOP_LIMIT      12 /* largest frontier (vertices) the
                                      persistent small-level loop takes and
                                      keeps: 64..65536 (default 65536)     */
#define BFS_OPT_CLAIM_MODE      13 /* degree-ordered graphs: how a level whose
                                      next frontier takes the bitmap form
                                      records the vertices it finds.  0: the
                                      atomicOr claim on the visited bitmap of
                                      Algorithm 3; 2: each vertex found gets a
                                      byte flag (a plain byte store, read
                                      first; no atomics) and a parent from
                                      the frontier, and the flags become
                                      bitmap bits when the frontier is
                                      compacted; 1 (default): 2 when V is at
                                      most 2^25, else 2 for the levels that
                                      start with at least V/16 vertices
                                      visited and 0 for the others.  Levels
                                      whose next frontier is
                                      a list always claim with atomicOr.
                                      Every mode gives the same levels and
                                      valid parents                          */
#define BFS_OPT_XCD_SLICES      15 /* degree-ordered graphs: 1 (default) runs the
                                      early host-driven levels of graphs with
                                      at least 2^23 vertices (frontier and
                                      visited set both at most V/64) as XCD-
                                      sliced levels: the ids are dealt to 8
                                      slices by 1024-id blocks (one line of
                                      the visited bitmap each), every row is
                                      also stored grouped by slice, and
                                      workgroup b of the expansion takes only
                                      edges into slice b mod 8, so the XCD it
                                      runs on probes one eighth of the
                                      bitmap.  0 off; 2 every host-driven
                                      level whose frontier has at most V/8
                                      vertices.  Same levels, valid parents  */

typedef struct bfs_graph bfs_graph;
typedef struct bfs_server bfs_server;

typedef struct bfs_stats {
    int32_t levels;         /* number of non-empty frontiers, root's included   */
    int32_t bitmap_levels;  /* levels whose next frontier used the bitmap form  */
    int64_t reached;        /* vertices reached (sum of frontier sizes)         */
    int64_t edges_scanned;  /* sum of out-degrees of reached vertices           */
    double  device_ms;      /* stream time of the call (HIP events)             */
    /* With BFS_OPT_PROFILE: summed stream time of each kernel class
     * (scan_ms includes the visited summary before heavy levels;
     * compact_ms the bitmap -> queue compaction and, under degree order,
     * the final pass that writes the caller-ordered outputs).            */
    double  init_ms, scan_ms, expand_ms, compact_ms;
    int32_t expand_launches;
    int32_t device_loop_levels; /* levels run inside the device-side loop      */
    /* Algorithmic bytes of the host-driven expansion kernels: per level
     * 4 * edges streamed (column ids; edges dropped by the row prefix skip
     * are not streamed) + 20 * frontier entries (queue entry, its
     * cumulative degree, its row offset) + 4 per discovered vertex for its
     * parent + 8 per discovered vertex in list mode (queue slot, level).  */
    int64_t expand_bytes;
    /* The same launches' share of the search's algorithmic bytes (the
     * roofline numerator): 4 * every frontier edge of those levels, the
     * ones the row prefix skip drops included (their column ids are what
     * the method reads), + 4 per discovered vertex for its level + 4 more
     * for its parent when parents are requested.                         */
    int64_t expand_alg_bytes;
    int32_t bottom_up_levels; /* levels searched bottom-up (BFS_OPT_DIRECTION) */
    int32_t pad0;
    /* Neighbour ids the search's kernels actually read: the column ids the
     * top-down expansions streamed (row-skipped edges excluded) plus the
     * neighbours the bottom-up steps probed.                              */
    int64_t edges_examined;
} bfs_stats;

/* Thread-local message of the last failing call ("" if none). */
const char *bfs_last_error(void);

/* Library ABI version (major * 100 + minor). */
int bfs_version(void);

/*
 * Device workspace needed by a graph with V vertices and nnz directed CSR
 * entries: the per-search arrays of Section 3.1 (visited bitmap of
 * ceil(V/32) words, frontier queues, level and predecessor by search id)
 * and the degree scan of Section 3.4.  Pure host arithmetic: never touches
 * the device.
 *   V    : 1 .. 2^31 - 1;  nnz : 0 .. 2^62
 *   flags: BFS_WS_BATCH adds the batch arrays (3 * 8 * V bytes, and 64 * V
 *   more with BFS_DEGREE_ORDER: the batch rows by internal id).
 * Errors: BFS_ERR_INVALID for out-of-range sizes or a null bytes pointer.
 */
int bfs_workspace_bytes(int32_t V, int64_t nnz, uint32_t flags, size_t *bytes);

/*
 * Create a graph handle over a CSR that is already in device memory.  The
 * CSR row of u lists u's out-neighbours, i.e. the paper's CSC column of u
 * (Section 3.1); creation-time work (checks, the degree-ordered relabel and
 * row grouping) stands where the paper partitions the graph before timing
 * starts (Section 4).
 *   d_row_offsets: int64[V + 1], d_row_offsets[0] = 0, non-decreasing,
 *                  d_row_offsets[V] = nnz (device, borrowed)
 *   d_col        : int32[nnz] neighbour ids in [0, V) (device, borrowed)
 *   d_workspace  : >= bfs_workspace_bytes(V, nnz, flags) bytes, 256-byte
 *                  aligned (device, borrowed)
 * The graph may be directed; the search follows out-edges.  Duplicates and
 * self-loops are legal.  With BFS_VALIDATE_CSR the offsets and ids are
 * checked on the device (BFS_ERR_INVALID on failure).  Synchronous.
 * Errors: BFS_ERR_INVALID, BFS_ERR_WORKSPACE, BFS_ERR_NO_DEVICE, BFS_ERR_HIP.
 */
int bfs_graph_create(bfs_graph **g, int32_t V, int64_t nnz,
                     const int64_t *d_row_offsets, const int32_t *d_col,
                     void *d_workspace, size_t ws_bytes, uint32_t flags,
                     void *hip_stream);

/* Release the handle (not the borrowed buffers).  NULL is a no-op. */
int bfs_graph_destroy(bfs_graph *g);

/* Set a tuning option (BFS_OPT_*).  BFS_ERR_INVALID for unknown keys or
 * values. */
int bfs_set_option(bfs_graph *g, int key, int64_t value);
int bfs_get_option(bfs_graph *g, int key, int64_t *value);

/*
 * Single-root search: the level loop of Algorithm 2 on one processor, each
 * level the degree scan and edge -> thread map of Section 3.4 (multi-edge
 * threads, Section 3.4.1), the claim of Algorithm 3 and the list / bitmap
 * frontier of Section 5; Algorithm 2's initialisation fixes the outputs'
 * conventions.
 *   root     : 0 <= root < V
 *   d_levels : int32[V] (device, caller-owned), written completely
 *   d_parents: int32[V] (device) or NULL to skip predecessors
 *   st       : nullable
 * Returns after the search has completed on hip_stream.  A handle runs one
 * search at a time: a concurrent call returns BFS_ERR_BUSY.
 */
int bfs_run(bfs_graph *g, int32_t root, int32_t *d_levels, int32_t *d_parents,
            void *hip_stream, bfs_stats *st);

/*
 * Multi-source batch: n_roots independent searches run together, one bit of
 * a 64-bit mask per root and vertex, the union frontier expanded once per
 * level with the scan and edge -> thread map of Section 3.4; each lane's
 * levels are those of its own single-root search (Algorithm 2).  Needs a graph created with BFS_WS_BATCH.
 *   h_roots : int32[n_roots] (host), each in [0, V); repeats are allowed
 *   n_roots : 1 .. 64
 *   d_levels: int8[n_roots][V] (device, row-major by root), written
 *             completely; -1 = unreached
 * BFS_ERR_DEPTH if some root's search goes deeper than 127 levels (the rows
 * are then incomplete).  st->reached / edges_scanned describe the union.
 */
int bfs_run_batch(bfs_graph *g, const int32_t *h_roots, int32_t n_roots,
                  int8_t *d_levels, void *hip_stream, bfs_stats *st);

/*
 * Allocation-free single-root search, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same search as bfs_run on a plain
 * (not degree-ordered) CSR, with no graph handle: every scratch array lives
 * in one static device array of 32 MiB per device, held from the library's
 * load until the process ends.  The call makes no device or pinned-host
 * allocation and creates no events or streams.
 *   d_row_offsets, d_col: the CSR as for bfs_graph_create (device, read
 *                         only); offsets and column ids are checked on
 *                         every call (BFS_ERR_INVALID)
 *   root, d_levels, d_parents, st: as for bfs_run; st->device_ms is the
 *                         host wall time of the call
 * Size limit: the scratch needs about 32.25 * V + nnz / 64 + 2.2 MB bytes
 * (V <= 524288 with nnz <= 2^28 always fits); larger inputs return
 * BFS_ERR_WORKSPACE before any device work.
 * Runs on the calling thread's current device; all pointers must be that
 * device's.  Calls that overlap on one device share the array and race:
 * serialise them.  Each call rewrites what it uses (the last call's
 * contents are never read).
 */
int bfs_run_noalloc(int32_t V, int64_t nnz, const int64_t *d_row_offsets,
                    const int32_t *d_col, int32_t root, int32_t *d_levels,
                    int32_t *d_parents, void *hip_stream, bfs_stats *st);

/* ---------------------------------------------------------------------- */
/* In-GPU 2D blocking: the search of Algorithm 2 run by an R x C grid of
 * virtual processors inside one GPU (Section 2.2 partitioning; local index
 * maps LOCAL_ROW / LOCAL_COL / ROW2COL of Section 3.1; the expansion of
 * Algorithm 3 with destinations grouped by owner column; the frontier
 * update of Section 3.5; list or bitmap messages by the threshold of
 * Section 5).  Vertex block p = j*R + i (B ids, B = ceil(V / RC) rounded up
 * to a multiple of 32) is owned by processor (i, j); processor (i, j) holds
 * the edges from column block j into row blocks m*R + i.  The column
 * (expand) and row (fold) exchanges are device-local.  Processor p's kernels
 * run on XCD p mod 8, so its bitmap of C*B local rows stays in one L2.   */

typedef struct bfs_grid2d bfs_grid2d;

/* bfs_grid2d_run msg_mode */
#define BFS_2D_MSG_AUTO   0  /* per message, a list unless longer than the
                                bitmap of the destination block (Section 5) */
#define BFS_2D_MSG_LIST   1  /* lists only                                  */
#define BFS_2D_MSG_BITMAP 2  /* bitmaps only (the bitmap-emitting expansion
                                and update kernels every level)             */

typedef struct bfs_grid2d_stats {
    int32_t levels;        /* non-empty frontiers, the root's included        */
    int32_t list_levels;   /* (processor, level) expansions that kept lists   */
    int64_t reached;
    int64_t edges_scanned; /* sum of out-degrees of reached vertices          */
    double  device_ms;
    /* column (expand) exchange: each front to the R - 1 others of its column */
    int64_t expand_list_msgs, expand_bitmap_msgs, expand_bytes;
    int64_t expand_list_only_bytes;   /* the same fronts sent as lists only   */
    /* row (fold) exchange: each processor to the C - 1 others of its row     */
    int64_t fold_list_msgs, fold_bitmap_msgs, fold_bytes;
    int64_t fold_list_only_bytes;     /* the same rows sent as lists only     */
    int64_t updated;       /* rows accepted by the frontier-update kernel     */
} bfs_grid2d_stats;

/*
 * Workspace of a 2D handle (pure host arithmetic).  R, C >= 1 with R * C in
 * {1, 2, 4} or a multiple of 8 up to 64.  About 8 R V (segment offsets) +
 * 4 nnz (local rows) + 24 R V (scan of the replicated column fronts) +
 * 8 C V (predecessor tables and outgoing lists) bytes.
 * Errors: BFS_ERR_INVALID.
 */
int bfs_grid2d_workspace_bytes(int32_t V, int64_t nnz, int32_t R, int32_t C,
                               size_t *bytes);

/*
 * Partition a device CSR (as for bfs_graph_create, borrowed for the call
 * only) into the R x C processors' local matrices, kept in d_workspace
 * (>= bfs_grid2d_workspace_bytes, 256-byte aligned, borrowed until
 * destroy).  Offsets and column ids are checked (BFS_ERR_INVALID).
 * Synchronous.  Errors: BFS_ERR_INVALID, BFS_ERR_WORKSPACE,
 * BFS_ERR_NO_DEVICE, BFS_ERR_HIP.
 */
int bfs_grid2d_create(bfs_grid2d **g, int32_t V, int64_t nnz,
                      const int64_t *d_row_offsets, const int32_t *d_col,
                      int32_t R, int32_t C, void *d_workspace, size_t ws_bytes,
                      void *hip_stream);

/* Release the handle (not the workspace).  NULL is a no-op. */
int bfs_grid2d_destroy(bfs_grid2d *g);

/*
 * Single-root search on the processor grid (Algorithm 2).  Outputs and
 * conventions as bfs_run: d_levels int32[V] (device, written completely),
 * d_parents int32[V] or NULL; predecessors of vertices found by another
 * processor are resolved at the end from the finder's table (delayed
 * predecessor exchange).  msg_mode: BFS_2D_MSG_*.  Synchronous; a handle
 * runs one search at a time (BFS_ERR_BUSY).
 */
int bfs_grid2d_run(bfs_grid2d *g, int32_t root, int32_t msg_mode,
                   int32_t *d_levels, int32_t *d_parents, void *hip_stream,
                   bfs_grid2d_stats *st);

/* ---------------------------------------------------------------------- */
/* Serving: a resident pool of graphs, queries admitted by an HBM budget and
 * batched per graph into multi-source lanes at level boundaries.          */

/* bfs_server_config.flags */
#define BFS_SRV_NO_PERSISTENT 0x1u /* deep graphs' rounds use the separate level
                                      kernels only (no persistent kernel)   */

typedef struct bfs_server_config {
    int32_t max_lanes;       /* lanes per graph batch, 1 .. 64 (default 64)   */
    int32_t max_inflight;    /* graphs with a running batch at once (>= 1)    */
    uint32_t flags;          /* BFS_SRV_* (default 0)                         */
    uint32_t reserved;       /* 0                                              */
} bfs_server_config;

typedef struct bfs_timing {
    int64_t submit_ns;  /* steady-clock times in nanoseconds */
    int64_t admit_ns;
    int64_t done_ns;
    int32_t levels;     /* depth of the query's search + 1 */
    int32_t lanes_in_batch;
} bfs_timing;

/*
 * Create a server over a caller-owned device arena of arena_bytes (the HBM
 * budget for per-graph batch state and per-query outputs).  cfg nullable.
 * Each query's result is its own single-root search's levels (Algorithm 2);
 * the server batches queries of one graph as lanes of bfs_run_batch's
 * multi-source search.
 */
int bfs_server_create(bfs_server **s, void *d_arena, size_t arena_bytes,
                      const bfs_server_config *cfg);

/* Register a graph (created without BFS_WS_BATCH is fine); the server does
 * not own it.  BFS_ERR_BUDGET if this graph's batch state can never fit. */
int bfs_server_add_graph(bfs_server *s, bfs_graph *g, int32_t *graph_id);

/* Enqueue a single-root query; non-blocking.  *ticket identifies it. */
int bfs_submit(bfs_server *s, int32_t graph_id, int32_t root, uint64_t *ticket);

/*
 * Poll a query.  BFS_PENDING while it runs.  On BFS_OK, if dst_levels is not
 * NULL, writes the int32[V] levels of the query's graph into it (-1 =
 * unreached), fills *t if not NULL, and retires the ticket.  dst_levels may
 * be host memory or device memory of the server's device.  A device buffer
 * is filled by a widening kernel on the device's default (null) stream, so
 * it is ordered after work the caller queued there, and never crosses
 * PCIe.  The call returns after the levels are written (under load that
 * kernel can wait about a millisecond behind other graphs' work in the
 * shared hardware queues, so a client that must keep submitting on time
 * should poll from another thread).  BFS_ERR_TICKET for unknown or retired
 * tickets.
 */
int bfs_poll(bfs_server *s, uint64_t ticket, int32_t *dst_levels, bfs_timing *t);

/*
 * Completion queue: moves up to max_tickets tickets of queries that have
 * finished (successfully or not) since the last call into tickets[] and
 * sets *n_out.  Each finished ticket is reported exactly once, so a client
 * polls only what is done instead of every outstanding ticket.  Reported
 * tickets stay valid for bfs_poll.
 */
int bfs_server_completed(bfs_server *s, uint64_t *tickets, int32_t max_tickets,
                         int32_t *n_out);

typedef struct bfs_server_stats {
    uint64_t submitted;    /* queries accepted by bfs_submit                  */
    uint64_t completed;    /* queries finished, failed ones included          */
    uint64_t failed;
    uint64_t rounds;       /* level rounds launched (either kind)             */
    uint64_t levels;       /* levels launched, summed over graph batches      */
    uint64_t lane_levels;  /* sum over launched levels of the live lanes      */
    uint64_t batches;      /* batch states created (arena allocations)        */
    uint64_t joins;        /* queries admitted into a lane                    */
    double   device_ms;    /* device time of all rounds, summed over streams  */
    uint64_t arena_peak;   /* peak arena bytes in use                         */
    uint64_t persistent_rounds; /* rounds run by the persistent level kernel  */
    uint64_t wide_rounds;  /* deep-graph rounds given to the captured level
                              kernels because the union frontier outgrew the
                              persistent kernel's limits                      */
} bfs_server_stats;

/* Counters since bfs_server_create (a consistent snapshot). */
int bfs_server_get_stats(bfs_server *s, bfs_server_stats *out);

/* Block until every submitted query has finished.  Finished results hold
 * arena memory until bfs_poll collects them, so queries can be left that no
 * memory will ever admit; when no batch is running and the next query's
 * batch state plus its result does not fit, drain returns BFS_ERR_BUDGET
 * (poll the finished tickets, then drain again) instead of blocking. */
int bfs_server_drain(bfs_server *s);

/* Stop the worker thread and release the server (graphs stay valid). */
int bfs_server_destroy(bfs_server *s);

#ifdef __cplusplus
}
#endif

#endif /* BFSMI_BFS_H */
