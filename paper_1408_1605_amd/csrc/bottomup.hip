// Bottom-up steps of the direction-optimizing search (the variant the paper
// discusses among related work: a level is searched from the unvisited
// vertices, each looking for one neighbour in the frontier, instead of from
// the frontier's edges), and the symmetry check that guards it.
//
// A bottom-up step for depth lvl runs over every vertex id that has a
// neighbour (under degree order the ids below the count of such vertices).  An unvisited
// vertex scans its row in stored order and stops at the first neighbour that
// was visited when the step began; that neighbour is its parent.  At the
// start of the step the visited set is exactly the vertices of depth
// <= lvl - 1, and an unvisited vertex (depth >= lvl) has no neighbour of
// depth <= lvl - 2 in a symmetric graph, so any visited neighbour lies in
// the frontier (depth lvl - 1): probing the visited bitmap is the frontier
// test, and the visited summary's fully visited id prefix answers it without
// a load.  Under degree order each row lists its lowest ids (the hubs) first.
//
// The visited bitmap is read from vis_old, a copy taken when the step
// begins and not written during it; the new bits go to vis, each wave
// writing the two words of its own 64 vertices.  Afterwards vis & ~vis_old is
// the next frontier, as after a top-down level in bitmap form.
#include <algorithm>

#include "bfs_internal.h"
#include "wave_ops.h"

namespace bfsmi {

// vis_old := vis (the snapshot the step probes); clears the step's counters.
__global__ __launch_bounds__(kWG) void k_bu_begin(int32_t W, const uint32_t* __restrict__ vis,
                                                  uint32_t* __restrict__ vis_old, int32_t lvl,
                                                  Ctrl* __restrict__ ctrl)
{
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < W; i += stride) {
        const uint32_t x = vis[i];
        if (vis_old[i] != x) vis_old[i] = x;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->qn_count = 0;
        ctrl->bitmap_out = 1;  // a switch back converts vis & ~vis_old to a queue
        ctrl->level = lvl;
        ctrl->bu_found = 0;
        ctrl->bu_deg = 0;
        ctrl->bu_edges = 0;
        ctrl->next_deg = 0;
    }
}

// One wave per 64 consecutive vertex ids (two bitmap words).
__global__ __launch_bounds__(kWG) void k_bottom_up(int32_t V, int32_t V_scan, int32_t W,
                                                   const int64_t* __restrict__ off,
                                                   const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ orig,
                                                   uint32_t* __restrict__ vis,
                                                   const uint32_t* __restrict__ snap,
                                                   int32_t* __restrict__ level,
                                                   int32_t* __restrict__ parent, int32_t lvl,
                                                   Ctrl* __restrict__ ctrl)
{
    constexpr int U = 4;  // neighbours probed together
    const int lane = __lane_id();
    const int32_t fp = ctrl->full_prefix;
    const int64_t nunits = ((int64_t)V_scan + 63) / 64;
    const int64_t nwaves = (int64_t)gridDim.x * (kWG / 64);
    uint32_t found_n = 0;
    int64_t found_deg = 0, examined = 0;
    for (int64_t unit = (int64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6); unit < nunits;
         unit += nwaves) {
        const int64_t v = unit * 64 + lane;
        const int64_t w0 = unit * 2;
        bool visited = true;
        if (v < V_scan) visited = (snap[v >> 5] >> (v & 31)) & 1u;
        int32_t par = -1;
        int64_t deg = 0;
        if (!visited) {
            const int64_t a = off[v], b = off[v + 1];
            deg = b - a;
            for (int64_t e = a; e < b && par < 0; e += U) {
                int32_t u[U];
                bool hit[U];
#pragma unroll
                for (int k = 0; k < U; ++k) u[k] = e + k < b ? col[e + k] : -1;
#pragma unroll
                for (int k = 0; k < U; ++k)
                    hit[k] = u[k] >= 0 && (u[k] < fp || ((snap[u[k] >> 5] >> (u[k] & 31)) & 1u));
                int64_t seen = b - e < U ? b - e : U;
#pragma unroll
                for (int k = U - 1; k >= 0; --k) {
                    if (hit[k]) {
                        par = u[k];
                        seen = k + 1;
                    }
                }
                examined += seen;
            }
        }
        const bool got = par >= 0;
        const uint64_t mask = __ballot(got);
        if (got) {
            level[v] = lvl;
            if (parent) parent[v] = orig ? orig[par] : par;
            found_deg += deg;
        }
        found_n += got ? 1u : 0u;
        const uint32_t lo = (uint32_t)mask, hi = (uint32_t)(mask >> 32);
        if (lane == 0 && lo) vis[w0] = snap[w0] | lo;
        if (lane == 32 && hi && w0 + 1 < W) vis[w0 + 1] = snap[w0 + 1] | hi;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        found_n += __shfl_xor(found_n, d, 64);
        found_deg += __shfl_xor(found_deg, d, 64);
        examined += __shfl_xor(examined, d, 64);
    }
    if (lane == 0) {
        if (found_n) atomicAdd(&ctrl->bu_found, found_n);
        if (found_deg) atomicAdd((unsigned long long*)&ctrl->bu_deg, (unsigned long long)found_deg);
        if (examined) atomicAdd((unsigned long long*)&ctrl->bu_edges, (unsigned long long)examined);
    }
}

// Vertices with at least one neighbour (creation time: under degree order
// they are exactly the internal ids below the count, so a bottom-up step
// need not look at the rest, which no search can reach).
__global__ __launch_bounds__(kWG) void k_count_nonzero_degree(int32_t V,
                                                              const int64_t* __restrict__ off,
                                                              uint32_t* __restrict__ out)
{
    uint32_t n = 0;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < V; v += stride)
        n += off[v + 1] > off[v] ? 1u : 0u;
    for (int d = 32; d >= 1; d >>= 1) n += __shfl_xor(n, d, 64);
    if (__lane_id() == 0 && n) atomicAdd(out, n);
}

hipError_t launch_count_nonzero_degree(hipStream_t s, int grid, int32_t V, const int64_t* off,
                                       uint32_t* out)
{
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_count_nonzero_degree, dim3(grid), dim3(kWG), 0, s, V, off, out);
    return hipGetLastError();
}

hipError_t launch_bottom_up(hipStream_t s, int grid, int32_t V, int32_t V_scan, int32_t W,
                            const int64_t* off, const int32_t* col, const int32_t* orig,
                            uint32_t* vis, uint32_t* vis_old, int32_t* level, int32_t* parent,
                            int32_t lvl, Ctrl* ctrl, int summary_grid, int32_t summary_shift,
                            int32_t summary_blocks, uint32_t* summary)
{
    if (grid < 1) grid = 1;
    const int64_t wgrid = std::min<int64_t>(grid, ((int64_t)W + kWG - 1) / kWG);
    hipLaunchKernelGGL(k_bu_begin, dim3((unsigned)std::max<int64_t>(wgrid, 1)), dim3(kWG), 0, s, W,
                       vis, vis_old, lvl, ctrl);
    hipError_t e = launch_visited_summary(s, summary_grid, V, W, vis_old, summary_shift,
                                          summary_blocks, summary, ctrl);
    if (e != hipSuccess) return e;
    if (V_scan < 0 || V_scan > V) V_scan = V;
    const int64_t units = ((int64_t)V_scan + 63) / 64;
    const int64_t bgrid = std::min<int64_t>(grid, (units + 3) / 4);
    hipLaunchKernelGGL(k_bottom_up, dim3((unsigned)std::max<int64_t>(bgrid, 1)), dim3(kWG), 0, s,
                       V, V_scan, W, off, col, orig, vis, vis_old, level, parent, lvl, ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Symmetry check at graph creation: the CSR is symmetric iff its edge
// multiset equals its reverse.  Both multisets are summarised by wrapping
// 64-bit sums of a mixed hash of (u, v) and of (v, u), two independent
// hashes each; equal sums are taken as symmetric (a non-symmetric CSR passes
// only if both pairs of 64-bit sums collide).  The mixing function is the
// SplitMix64 finaliser (Steele, Lea and Flood, 2014).

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kWG) void k_symmetry_sums(int32_t V, const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ col,
                                                       unsigned long long* __restrict__ sums)
{
    const int lane = __lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (kWG / 64);
    uint64_t f1 = 0, f2 = 0, r1 = 0, r2 = 0;
    for (int64_t u = (int64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6); u < V; u += nwaves) {
        const int64_t a = off[u], b = off[u + 1];
        for (int64_t e = a + lane; e < b; e += 64) {
            const uint64_t v = (uint32_t)col[e];
            const uint64_t fw = ((uint64_t)u << 32) | v, rv = (v << 32) | (uint64_t)u;
            f1 += mix64(fw);
            r1 += mix64(rv);
            f2 += mix64(fw ^ 0x5851f42d4c957f2dull);
            r2 += mix64(rv ^ 0x5851f42d4c957f2dull);
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        f1 += __shfl_xor(f1, d, 64);
        f2 += __shfl_xor(f2, d, 64);
        r1 += __shfl_xor(r1, d, 64);
        r2 += __shfl_xor(r2, d, 64);
    }
    if (lane == 0) {
        atomicAdd(&sums[0], (unsigned long long)f1);
        atomicAdd(&sums[1], (unsigned long long)f2);
        atomicAdd(&sums[2], (unsigned long long)r1);
        atomicAdd(&sums[3], (unsigned long long)r2);
    }
}

hipError_t launch_symmetry_sums(hipStream_t s, int grid, int32_t V, const int64_t* off,
                                const int32_t* col, unsigned long long* sums)
{
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_symmetry_sums, dim3(grid), dim3(kWG), 0, s, V, off, col, sums);
    return hipGetLastError();
}

}  // namespace bfsmi
