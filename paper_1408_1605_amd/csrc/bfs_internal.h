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
    int32_t pad[3];
};

// Multi-source batch control block.
struct alignas(64) MsCtrl {
    int64_t r;
    int32_t ntiles;
    uint32_t qn_count;     // union frontier size of the next level
    uint64_t alive;        // OR of new bits found in this level (lanes alive)
    int32_t overflow;      // a level exceeded the output type
    int32_t pad[7];
};

// ---- single-root kernels (frontier.hip) ----
hipError_t launch_init(hipStream_t s, int32_t V, int32_t W, int32_t root,
                       int32_t* level, int32_t* parent, uint32_t* vis,
                       uint32_t* vis_old, int32_t* Q, Ctrl* ctrl, int grid_cap);

hipError_t launch_scan(hipStream_t s, const int32_t* Q, int32_t qlen,
                       const int64_t* off, int32_t* deg, int64_t* bsum,
                       int64_t* cumul, int32_t* tile_k, int64_t tile_cap, int tile,
                       int64_t bitmap_threshold, int allow_bitmap, Ctrl* ctrl);

hipError_t launch_expand(hipStream_t s, int ept, int grid, int32_t V, const int32_t* Q,
                         const int64_t* cumul, const int32_t* tile_k,
                         const int64_t* off, const int32_t* col, uint32_t* vis,
                         uint32_t* vis_old, int32_t* level, int32_t* parent,
                         int32_t lvl, int32_t* Qn, Ctrl* ctrl);

hipError_t launch_bitmap_to_queue(hipStream_t s, int grid, int32_t V, int32_t W,
                                  uint32_t* vis, uint32_t* vis_old,
                                  int32_t* Qn, int32_t* level, int32_t lvl,
                                  Ctrl* ctrl);

hipError_t launch_validate_csr(hipStream_t s, int32_t V, int64_t nnz,
                               const int64_t* off, const int32_t* col,
                               int32_t* bad_flag, int32_t* maxdeg, int check_col);

// Device-resident level loop for small frontiers: one cooperative launch
// that runs levels until the frontier is empty or exceeds small_limit
// entries / edges.  Returns the HIP status of the launch.
hipError_t launch_small_loop(hipStream_t s, int grid, const int64_t* off,
                             const int32_t* col, uint32_t* vis,
                             uint32_t* vis_old, int32_t* level,
                             int32_t* parent, int32_t* Qa, int32_t* Qb,
                             int64_t* cumul, Ctrl* ctrl, int32_t small_limit,
                             int64_t edge_limit);
int small_loop_max_grid(int device);

}  // namespace bfsmi
