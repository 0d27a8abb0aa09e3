// Host-side runtime structures behind the C ABI.
#pragma once

#include <atomic>
#include <string>

#include "../../include/bfs.h"
#include "bfs_internal.h"

namespace bfsmi {

// Record a message for bfs_last_error() and return the status code.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int ok();

#define BFS_HIP_TRY(expr)                                  \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return ::bfsmi::hip_fail(_e, #expr); \
    } while (0)

// Carving of the caller's workspace.  Every region is 256-byte aligned.
struct WsLayout {
    size_t vis, vis_old, q0, q1, deg, rowstart, suid, cumul, bsum, tile_k, ctrl, scratch, sync, sside, summary;
    size_t ms_sn, ms_front, ms_ctrl, ms_roots, ms_touched;
    size_t rank, orig, off_r, col_r, hist, col_tmp, skip, lvl_int, par_int, ms_out;
    size_t found, xo;
    size_t total;
};
WsLayout ws_layout(int32_t V, int64_t nnz, uint32_t flags);

}  // namespace bfsmi

struct bfs_graph {
    int32_t V = 0;
    int64_t nnz = 0;
    int32_t W = 0;  // bitmap words
    const int64_t* off = nullptr;
    const int32_t* col = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t flags = 0;
    int device = 0;
    int num_cus = 0;
    int32_t maxdeg = 0;
    bfsmi::WsLayout L{};

    uint32_t* vis = nullptr;
    uint32_t* vis_old = nullptr;
    int32_t* q[2] = {nullptr, nullptr};
    int32_t* deg = nullptr;
    int64_t* rowstart = nullptr;  // per frontier entry: row start in s_off
    int32_t* suid = nullptr;      // per frontier entry: id reported as parent
    int64_t* cumul = nullptr;
    int64_t* bsum = nullptr;
    int32_t* tile_k = nullptr;
    bfsmi::Ctrl* ctrl = nullptr;
    int32_t* scratch = nullptr;  // small device scratch (create-time checks)
    uint32_t* summary = nullptr; // visited summary: one bit per block of ids
    int32_t summary_shift = 10, summary_blocks = 0, summary_words = 0;
    bfsmi::SeenNext* ms_sn = nullptr;  // seen and next masks, side by side
    uint64_t* ms_front = nullptr;
    bfsmi::Ctrl* ms_ctrl = nullptr;
    int32_t* ms_roots = nullptr;       // device copy of the batch roots (64)
    uint32_t* ms_touched = nullptr;    // batch: vertices found this level (sparse levels)

    // the CSR the search runs on: the caller's, or the degree-ordered copy
    const int64_t* s_off = nullptr;
    const int32_t* s_col = nullptr;
    int32_t* rank = nullptr;  // caller id -> internal id (degree order only)
    int32_t* orig = nullptr;  // internal id -> caller id (degree order only)
    int32_t* skip = nullptr;  // row prefix skip counts [kSkipLevels][V] (degree order only)
    int32_t* lvl_int = nullptr;  // level by internal id during a search (degree order only)
    int32_t* par_int = nullptr;  // parent (caller id) by internal id (degree order only)
    int8_t* ms_out = nullptr;    // batch: int8 rows by internal id (degree order + batch)
    uint8_t* found = nullptr;    // flag claims: one byte per id (degree order only)
    uint32_t* xo = nullptr;      // XCD slices: per row, the offset of each slice's group
    int32_t* col_x = nullptr;    // XCD slices: rows grouped by slice (degree order only)

    bfsmi::Ctrl* h_ctrl = nullptr;      // pinned host mirror
    bfsmi::Ctrl* h_ms_ctrl = nullptr;   // pinned host mirror
    hipStream_t cap_stream = nullptr;   // private stream for graph capture
    hipGraphExec_t ms_graph = nullptr;  // captured batch levels
    int ms_graph_ept = 0;
    int ms_graph_skip = 0;              // row skip setting the batch levels were captured with
    bfsmi::SmallSync* small_sync = nullptr;  // persistent small-level loop: barrier, counters
    bfsmi::SmallSide small_side{};            // ... and its frontier entries' row data
    int small_grid = 0;                       // its workgroups (0: not available)
    int32_t* h_roots = nullptr;         // pinned staging for batch roots
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t pev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // per-kernel timing

    // options
    int ept = 4;
    int frontier_mode = 0;  // 0 auto, 1 list only, 2 bitmap whenever possible
    int loop_driver = 0;    // 0 auto (persistent loop for runs of small levels), 1 host only
    int batch_tile = 1024;  // edges per workgroup in the batch expansion
    int grid_wgs = 8;
    int profile = 0;
    int use_summary = 2;
    int row_skip = 1;
    int32_t small_limit = 1 << 16;  // largest frontier the persistent loop runs (<= 65536)
    int direction = 0;      // 1: direction-optimizing (bottom-up steps on dense levels)
    int do_alpha = 14;      // top-down -> bottom-up when frontier edges * alpha > unvisited edges
    int do_beta = 24;       // bottom-up -> top-down when frontier * beta < V and shrinking
    int symmetric = 0;      // the CSR equals its transpose (checked at creation)
    int32_t v_active = 0;   // degree order: internal ids below it have a neighbour (else V)
    int xcd_slices = 1;     // 0 off, 1 auto, 2 whenever the frontier fits (8 * qlen <= V)
    int claim_mode = 1;     // bitmap levels: 0 atomic claims, 1 flag claims up to
                            // kFlagAutoMaxV vertices, 2 flag claims
    std::atomic<int> busy{0};
};

namespace bfsmi {

// Points the handle's arrays into the workspace ws laid out as L (and sets
// the visited summary's block size from g->V).
void bind_workspace(bfs_graph* g, char* ws, const WsLayout& L, uint32_t flags);

// Single-root level loop on a bound handle; the caller holds the handle and
// has made its device current.
int run_host_loop(bfs_graph* g, int32_t root, int32_t* levels, int32_t* parents,
                  hipStream_t s, bfs_stats* st);

// Workgroups of the persistent small-level loop on a device with num_cus
// compute units (0: the loop is not available).
int small_loop_grid(int num_cus);

}  // namespace bfsmi
