// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfsmi {

constexpr int kWG = 256;              // threads per workgroup (4 wave64)
constexpr int kScanItems = 8;         // frontier entries per thread in the scan
constexpr int kScanChunk = kWG * kScanItems;
constexpr int kBitmapWordsPerWG = kWG; // words per workgroup in bitmap->list
constexpr int kMaxEPT = 8;
constexpr int kMinTile = kWG;         // smallest edge tile (EPT = 1)
constexpr int kSummaryMaxWords = 2048; // visited summary: <= 8 KB of LDS
constexpr int kSkipLow = 16;          // row prefix skip thresholds 2^(16 + i) ...
constexpr int kSkipLevels = 10;       // ... for i = 0..9
constexpr int kBigTiles = 16;         // scan: an entry spanning this many tiles or more ...
constexpr int kBigTileList = 256;     // ... is queued (up to this many per block) for the workgroup
// XCD slices of the id space: the visited bitmap's 128-byte lines (1024 ids
// each) dealt round-robin to eight slices; workgroup b of a launch runs on
// XCD b mod 8, so an expansion whose workgroups b only probe slice b mod 8
// keeps each XCD's probes within one eighth of the bitmap (its own L2).
constexpr int kXcdSlices = 8;
constexpr int32_t kSliceMinV = 1 << 17;  // automatic sliced levels from this many vertices
constexpr int32_t kSliceHot = 1 << 13;   // ids below: dealt to slices by row, not by id
__host__ __device__ __forceinline__ int xcd_slice(int32_t v) { return (v >> 10) & (kXcdSlices - 1); }

// Flag claims (BFS_OPT_CLAIM_MODE 1) are used at every bitmap level up to
// this many vertices (one flag byte per vertex, probed at random; measured
// faster than the atomic claim of Algorithm 3 on R-MAT 16-25).
constexpr int32_t kFlagAutoMaxV = 1 << 25;

// Per-level control block in device memory.  The host reads it back once
// per level; the kernels read the fields they need directly.
struct alignas(64) Ctrl {
    int64_t r;           // edges of the current frontier (sum of degrees)
    int32_t ntiles;      // ceil(r / tile)
    int32_t bitmap_out;  // 1: next frontier produced in bitmap form
    uint32_t qn_count;   // size of the next frontier
    int32_t qlen;        // size of the current frontier
    int32_t level;       // depth being discovered
    int32_t done;        // device loop: set when the frontier is empty
    int64_t r_total;     // device loop: edges scanned so far
    int64_t reached;     // device loop: vertices reached so far
    int32_t levels;      // device loop: levels completed
    int32_t bitmap_levels;
    int32_t err;         // set when a guard trips (never expected)
    int32_t full_prefix; // every id below it is visited (visited summary)
    int32_t overflow;    // batch: a level did not fit the output type
    int32_t sparse;      // batch: this level's union frontier is small (see msbfs.hip)
    int32_t sparse_limit;  // batch: frontier sizes up to this count as small
    int32_t pad2;
    uint64_t alive;      // batch: OR of the lanes that found vertices this level
    uint64_t last_alive; // batch: alive of the last completed level
    int8_t* out8;        // batch: output rows (read by the device each launch)
    // single-root persistent loop (smallloop.hip)
    int32_t steps;       // levels completed in the loop
    int32_t pad3;
    int64_t skipped;     // edges the degree scan dropped (row prefix skip)
    int32_t fp_cand;     // batch: first id some live lane has not seen (prefix search)
    int32_t pad4;
    // bottom-up steps (bottomup.hip)
    uint32_t bu_found;   // vertices found by the step
    int32_t pad5;
    int64_t bu_deg;      // their degree sum
    int64_t bu_edges;    // neighbours the step probed
    int64_t next_deg;    // degree sum of the next frontier, when the bitmap compaction is asked for it
};


// ---- single-root kernels (frontier.hip) ----
// fill == 0: only the root's level / parent entries (degree order; the
// finish pass masks unvisited vertices).
hipError_t launch_init(hipStream_t s, int32_t V, int32_t W, int32_t root,
                       const int32_t* rank, int32_t* level, int32_t* parent,
                       uint32_t* vis, uint32_t* vis_old, int32_t* Q, Ctrl* ctrl,
                       int grid_cap, int fill, uint8_t* found = nullptr);

// Degree scan of the frontier Q: deg, cumul (exclusive, cumul[qlen] = r),
// rowstart[k] = off[Q[k]], uidv[k] = uid_map ? uid_map[Q[k]] : Q[k], and
// tile_k (the entry holding each tile's first edge).  With skip (the row
// prefix skip counts, [kSkipLevels][V]) each entry drops the leading block
// of its row that points below the largest threshold not above
// ctrl->full_prefix; deg and rowstart then describe the rest of the row and
// the dropped edges are added to ctrl->skipped.
hipError_t launch_scan(hipStream_t s, const int32_t* Q, int32_t qlen, const int64_t* off,
                       const int32_t* uid_map, int32_t* deg, int64_t* rowstart, int32_t* uidv,
                       int64_t* bsum, int64_t* cumul, int32_t* tile_k, int64_t tile_cap,
                       int tile, int64_t bitmap_threshold, int allow_bitmap, Ctrl* ctrl,
                       const int32_t* skip = nullptr, int32_t V = 0);

// Same scan with the frontier size taken from ctrl->qlen (fixed grid,
// grid-stride); every kernel returns at once when ctrl->done is set.
hipError_t launch_scan_dev(hipStream_t s, int grid, const int32_t* Q, const int64_t* off,
                           const int32_t* uid_map, int32_t* deg, int64_t* rowstart, int32_t* uidv,
                           int64_t* bsum, int64_t* cumul, int32_t* tile_k, int64_t tile_cap,
                           int tile, Ctrl* ctrl, const int32_t* skip = nullptr, int32_t V = 0);

// Expansion of one level (Algorithm 3); level / parent by search id, the
// level only in list mode (bitmap mode: launch_bitmap_to_queue writes it).
hipError_t launch_expand(hipStream_t s, int ept, int grid, int32_t V, const int64_t* rowstart,
                         const int32_t* uidv, const int64_t* cumul, const int32_t* tile_k,
                         const int32_t* col,
                         const uint32_t* summary, int32_t summary_words, int32_t shift,
                         int use_prefix, uint32_t* vis, uint32_t* vis_old, int32_t* level,
                         int32_t* parent, int32_t lvl, int32_t* Qn, Ctrl* ctrl,
                         uint8_t* found = nullptr, int32_t slice_q = 0);
// XCD-sliced level: the scan of launch_scan over 8 * qlen entries, entry
// s * qlen + k being slice s's group of frontier entry k's row in the
// slice-grouped rows (offsets xo); then launch_expand with slice_q = qlen on
// those rows.  Needs 8 * qlen <= V.
hipError_t launch_slice_scan(hipStream_t s, int grid, const int32_t* Q, int32_t qlen,
                             const int64_t* off, const uint32_t* xo, const int32_t* uid_map,
                             int32_t* deg, int64_t* rowstart, int32_t* uidv, int64_t* bsum,
                             int64_t* cumul, int32_t* tile_k, int64_t tile_cap, int tile,
                             int64_t bitmap_threshold, int allow_bitmap, Ctrl* ctrl);

// Single-root persistent loop for runs of small levels (smallloop.hip).
// Zeroed by the host before each launch.
// The grid barrier's counter and the per-level counters sit on separate
// 128-byte lines, so the barrier's polling does not queue behind the
// counters' atomics.
// Zero before a search's first launch; each launch leaves it zero again.
struct SmallSync {
    uint32_t arrive;   // grid barrier: arrivals (only grows within a launch)
    uint32_t leave;    // workgroups that have finished (the last one re-zeroes the block)
    uint32_t pad0[30];
    uint32_t qn[3];    // next-frontier size, by level mod 3
    uint32_t pad1[29];
    int32_t md[3];     // largest degree in the next frontier
    int32_t pad2[29];
    int64_t rn[3];     // edges of the next frontier
    int64_t edges;     // edges the launch expanded (to ctrl->r_total at the end)
    int64_t pad3[12];
};
// Row start, degree and caller id of each frontier entry, one set per
// queue (cap entries each), written by the workgroup that claims the vertex
// so the next level need not look them up.
struct SmallSide {
    int64_t* off[2];
    int32_t* deg[2];
    int32_t* id[2];
    int32_t cap;
};
int small_loop_blocks();
// qlen < 0: the frontier size is read from ctrl->qn_count (the previous
// host-driven level's output); the loop then runs no level when it is 0 or
// above qlimit.
hipError_t launch_small_levels(hipStream_t s, int grid, int32_t V, const int64_t* off,
                               const int32_t* col, const int32_t* orig, uint32_t* vis,
                               uint32_t* vis_old, int32_t* Qa, int32_t* Qb, int32_t* level,
                               int32_t* parent, SmallSync* sy, SmallSide side, Ctrl* ctrl,
                               int32_t qlen, int32_t lvl, int32_t qlimit, int64_t rlimit,
                               int32_t dlimit);

// Visited summary before a heavy level: ctrl->full_prefix and one bit per
// block of 2^shift ids (set when the whole block is visited); clears
// ctrl->skipped for the level's degree scan.
hipError_t launch_visited_summary(hipStream_t s, int grid, int32_t V, int32_t W,
                                  const uint32_t* vis, int32_t shift, int32_t nblocks,
                                  uint32_t* summary, Ctrl* ctrl);

// Resident expansion workgroups per CU for this configuration.
int expand_blocks_per_cu(int ept, int summary_words);

// deg_off non-null: also adds the degrees of the new frontier's vertices
// (from these row offsets) to ctrl->next_deg.
hipError_t launch_bitmap_to_queue(hipStream_t s, int grid, int32_t V, int32_t W, uint32_t* vis,
                                  uint32_t* vis_old, int32_t* Qn, int32_t* level, int32_t lvl,
                                  Ctrl* ctrl, const int64_t* deg_off = nullptr,
                                  uint8_t* found = nullptr);

// Degree order: caller-ordered outputs from the internal-id ones.
hipError_t launch_finish(hipStream_t s, int grid, int32_t V, const int32_t* rank,
                         const uint32_t* vis, const int32_t* lvl_int, const int32_t* par_int,
                         int32_t* level, int32_t* parent);

// ---- direction-optimizing search (bottomup.hip) ----
// One bottom-up step discovering depth lvl: vis_old := vis, the visited
// summary of that snapshot, then every unvisited vertex takes its first
// visited neighbour as parent (orig maps it to the caller's id when non-null);
// new bits go to vis.  Counts land in ctrl->bu_found / bu_deg / bu_edges;
// ctrl->bitmap_out = 1 and qn_count = 0 so launch_bitmap_to_queue can turn
// the step's vertices into a queue.
// Only ids below V_scan are candidates (ids at or above it have no
// neighbour; V_scan = V when that is not known).
hipError_t launch_bottom_up(hipStream_t s, int grid, int32_t V, int32_t V_scan, int32_t W,
                            const int64_t* off, const int32_t* col, const int32_t* orig,
                            uint32_t* vis, uint32_t* vis_old, int32_t* level, int32_t* parent,
                            int32_t lvl, Ctrl* ctrl, int summary_grid, int32_t summary_shift,
                            int32_t summary_blocks, uint32_t* summary);
// Adds the number of vertices with a neighbour to *out.
hipError_t launch_count_nonzero_degree(hipStream_t s, int grid, int32_t V, const int64_t* off,
                                       uint32_t* out);
// Wrapping sums of two hashes of every (u, v) and of every (v, u) into
// sums[0..1] and sums[2..3] (the caller zeroes them).
hipError_t launch_symmetry_sums(hipStream_t s, int grid, int32_t V, const int64_t* off,
                                const int32_t* col, unsigned long long* sums);

// ---- multi-source batch (msbfs.hip) ----
// The two masks of a vertex that the expansion tests together.
struct alignas(16) SeenNext {
    uint64_t seen;  // lanes that reached the vertex
    uint64_t next;  // lanes that found it during the current level
};

// Lanes are bits of a 64-bit mask per vertex: seen (reached), front (this
// level's frontier), next (found during this level).  All launches read
// their sizes from ctrl and return at once when ctrl->done is set.
// out_int non-null: the levels write int8 rows by internal id into out_int
// (no fill) and launch_ms_reorder produces the caller's rows out8 at the end;
// else they write out8 directly (filled with -1 here).
hipError_t launch_ms_init(hipStream_t s, int grid, int32_t V, const int32_t* h_roots_dev,
                          int32_t n_roots, const int32_t* rank, SeenNext* sn, uint64_t* front,
                          uint32_t* touched, int8_t* out8, int8_t* out_int, int32_t* Q,
                          Ctrl* ctrl);
hipError_t launch_ms_reorder(hipStream_t s, int grid, int32_t V, int32_t n_roots,
                             const int32_t* rank, const SeenNext* sn, const int8_t* out_int,
                             int8_t* out8);
// skip non-null (batch on a degree-ordered graph): after each level the
// longest id prefix that every live lane has seen is found (ctrl->full_prefix)
// and the next level's scan drops each row's block below the largest cut
// 2^(16 + i) inside it (the row prefix skip); the dropped edges go to
// ctrl->skipped.
hipError_t launch_ms_level(hipStream_t s, int scan_grid, int expand_grid, int fin_grid,
                           int ept, int32_t V, int64_t tile_cap, const int64_t* off,
                           const int32_t* col, const int32_t* orig, const int32_t* Q,
                           int32_t* Qn, int32_t* deg, int64_t* rowstart, int32_t* uidv,
                           int64_t* bsum, int64_t* cumul,
                           int32_t* tile_k, SeenNext* sn, uint64_t* front,
                           uint32_t* touched, int16_t* const* lane_out,
                           const int32_t* lane_start, Ctrl* ctrl,
                           const int32_t* skip = nullptr, int prefix_grid = 0);
int ms_expand_blocks_per_cu(int ept);

// Serving lanes (msbfs.hip).  lane_out: device table of 64 int16 result
// pointers; lane_start: device int32[64]; join: device int32 pairs
// (root, lane).
hipError_t launch_srv_reset(hipStream_t s, int grid, int32_t V, SeenNext* sn, uint64_t* front,
                            uint32_t* touched, Ctrl* ctrl);
hipError_t launch_srv_clear(hipStream_t s, int grid, int32_t V, SeenNext* sn, uint64_t mask);
hipError_t launch_fill16(hipStream_t s, int grid, int16_t* p, int64_t n, int16_t val);
hipError_t launch_widen16(hipStream_t s, int grid, const int16_t* src, int32_t* dst, int64_t n,
                          int32_t* maxp);
hipError_t launch_srv_join(hipStream_t s, int32_t V, int32_t n_join, const int32_t* join,
                           const int32_t* rank, SeenNext* sn, uint64_t* front,
                           int16_t* const* lane_out, int32_t* lane_start, int32_t* Q, Ctrl* ctrl);

// Persistent multi-source levels for serving batches (msloop.hip).  Zero
// before the first launch (the host clears it with the batch state); each
// launch leaves it zero again.
struct MsSync {
    uint32_t arrive;     // grid barrier: arrivals (only grows within a launch)
    uint32_t leave;      // workgroups that have finished (the last one re-zeroes the block)
    uint32_t pad0[30];   // the counters below sit on other lines
    uint32_t fn[3];      // found-list size, by level mod 3
    uint32_t qn[3];      // next-frontier size
    int32_t md[3];       // largest degree in the next frontier
    int32_t pad;
    int64_t rn[3];       // edges of the next frontier
    uint64_t alive[3];   // lanes that found vertices
};
int ms_small_loop_blocks();
// Runs up to max_levels serving levels (OUT16 outputs) from ctrl's state;
// ctrl->steps = levels run; the frontier ends in Qa; found is int32[V]
// scratch.  h_ctrl (pinned host memory, or null) receives a copy of the
// final control block.
hipError_t launch_ms_small_levels(hipStream_t s, int grid, int32_t V, const int64_t* off,
                                  const int32_t* col, const int32_t* orig, SeenNext* sn,
                                  uint64_t* front, int32_t* Qa, int32_t* Qb, int32_t* found,
                                  int16_t* const* lane_out, const int32_t* lane_start,
                                  MsSync* sy, Ctrl* ctrl, Ctrl* h_ctrl, int32_t max_levels,
                                  int32_t qlimit, int64_t rlimit, int32_t dlimit);

// Degree-ordered internal relabelling (relabel.hip).  rank[v] is v's
// internal id (vertices in non-increasing degree order, ties arbitrary),
// orig[rank[v]] = v; off_r / col_r is the CSR in internal ids (row x is
// the row of orig[x], neighbours mapped through rank).
hipError_t build_degree_order(hipStream_t s, int32_t V, int64_t nnz, const int64_t* off,
                              const int32_t* col, int32_t* rank, int32_t* orig,
                              int64_t* off_r, int32_t* col_r, int32_t* deg_tmp,
                              int64_t* rowstart_tmp, int32_t* uid_tmp,
                              int64_t* bsum_tmp, int32_t* tile_k, int64_t tile_cap,
                              uint32_t* hist_tmp, Ctrl* ctrl, int grid_cap);

hipError_t launch_validate_csr(hipStream_t s, int32_t V, int64_t nnz,
                               const int64_t* off, const int32_t* col,
                               int32_t* bad_flag, int32_t* maxdeg, int check_col);

// Row prefix skip (rowskip.hip): col_out = each row of col_in partitioned
// by the id ranges cut at 2^(16 + i); skip[i * V + x] = neighbours of row x
// below 2^(16 + i), i < kSkipLevels.
hipError_t build_row_skip(hipStream_t s, int32_t V, const int64_t* off, const int32_t* col_in,
                          int32_t* col_out, int32_t* skip, int grid);
// XCD slices (rowskip.hip): col_out = each row of col_in grouped by
// xcd_slice (stable), xo[x * 8 + s] = offset of slice s's group in row x.
hipError_t build_slice_rows(hipStream_t s, int32_t V, const int64_t* off, const int32_t* col_in,
                            int32_t* col_out, uint32_t* xo, int grid);

}  // namespace bfsmi
