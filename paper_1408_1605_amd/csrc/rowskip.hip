// Row prefix skip for the degree-ordered graph (built at graph creation).
//
// With degree-ordered ids the vertices that most edges point to own the
// lowest ids, and before a heavy level the visited summary finds a prefix of
// ids that is entirely visited: the early visited test of Section 5 rejects
// every edge into it.  If each row lists its neighbours below 2^16 first,
// then those in [2^16, 2^17), and so on, the edges into a fully visited
// prefix of at least 2^(16 + i) ids are a leading block of the row whose
// length is known in advance, and the level's degree scan can drop that
// block: the expansion never loads those column ids.
//
// Creation partitions every relabelled row into the eleven id ranges
//   [0, 2^16), [2^16, 2^17), ..., [2^24, 2^25), [2^25, V)
// (stable within a range) and records, for each threshold t_i = 2^(16 + i),
// i = 0..9, the number of the row's neighbours below t_i.  Levels and
// parents do not change: a skipped edge points to an already visited
// vertex, and the edge is still counted in the search's edge total.
#include "bfs_internal.h"
#include "wave_ops.h"

namespace bfsmi {

constexpr int kRanges = kSkipLevels + 1;

__device__ __forceinline__ int id_range(int32_t y)
{
    // number of thresholds 2^(16 + i) that y reaches
    const int lz = __clz(y);  // y > 0: its highest set bit is 31 - lz
    const int b = y < (1 << kSkipLow) ? 0 : 31 - lz - kSkipLow + 1;
    return b < kSkipLevels ? b : kSkipLevels;
}

// One wave per row (grid-stride over rows): count the row's ids per range
// with ballots, then write each range's ids in input order behind the
// ranges below it.  skip is laid out [kSkipLevels][V].
__global__ __launch_bounds__(kWG) void k_row_partition(int32_t V, const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ col_in,
                                                       int32_t* __restrict__ col_out,
                                                       int32_t* __restrict__ skip)
{
    const int lane = __lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (kWG / 64);
    for (int64_t x = (int64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6); x < V; x += nwaves) {
        const int64_t a = off[x], b = off[x + 1];
        int64_t cnt[kRanges];
#pragma unroll
        for (int k = 0; k < kRanges; ++k) cnt[k] = 0;
        for (int64_t e0 = a; e0 < b; e0 += 64) {
            const int64_t e = e0 + lane;
            const int rg = e < b ? id_range(col_in[e]) : -1;
#pragma unroll
            for (int k = 0; k < kRanges; ++k) cnt[k] += __popcll(__ballot(rg == k));
        }
        int64_t cur[kRanges];
        int64_t run = a;
#pragma unroll
        for (int k = 0; k < kRanges; ++k) {
            cur[k] = run;
            run += cnt[k];
        }
        if (lane < kSkipLevels) {
            int64_t s = 0;
#pragma unroll
            for (int k = 0; k < kSkipLevels; ++k) s += k <= lane ? cnt[k] : 0;
            skip[(int64_t)lane * V + x] = (int32_t)s;
        }
        for (int64_t e0 = a; e0 < b; e0 += 64) {
            const int64_t e = e0 + lane;
            const int32_t y = e < b ? col_in[e] : 0;
            const int rg = e < b ? id_range(y) : -1;
#pragma unroll
            for (int k = 0; k < kRanges; ++k) {
                const uint64_t m = __ballot(rg == k);
                if (rg == k) col_out[cur[k] + lanes_below(m)] = y;
                cur[k] += __popcll(m);
            }
        }
    }
}

// XCD slices: slice(y) = (y >> 10) & 7 (one 128-byte line of the visited
// bitmap per 1024 ids, the lines dealt round-robin to the eight slices),
// except for the ids below kSliceHot, the hubs most edges point at: their
// few bitmap lines stay in every L2, and they join slice x mod 8 of row x
// so that no slice gets all of the densest lines' edges.
// One wave per row: the row's ids grouped by slice (stable), xo[x * 8 + s]
// = the offset of slice s's group within the row.
__device__ __forceinline__ int row_slice(int32_t y, int64_t x)
{
    return y < kSliceHot ? (int)(x & (kXcdSlices - 1)) : xcd_slice(y);
}

__global__ __launch_bounds__(kWG) void k_slice_partition(int32_t V, const int64_t* __restrict__ off,
                                                         const int32_t* __restrict__ col_in,
                                                         int32_t* __restrict__ col_out,
                                                         uint32_t* __restrict__ xo)
{
    const int lane = __lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (kWG / 64);
    for (int64_t x = (int64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6); x < V; x += nwaves) {
        const int64_t a = off[x], b = off[x + 1];
        int64_t cnt[kXcdSlices];
#pragma unroll
        for (int k = 0; k < kXcdSlices; ++k) cnt[k] = 0;
        for (int64_t e0 = a; e0 < b; e0 += 64) {
            const int64_t e = e0 + lane;
            const int sl = e < b ? row_slice(col_in[e], x) : -1;
#pragma unroll
            for (int k = 0; k < kXcdSlices; ++k) cnt[k] += __popcll(__ballot(sl == k));
        }
        int64_t cur[kXcdSlices];
        int64_t run = a;
#pragma unroll
        for (int k = 0; k < kXcdSlices; ++k) {
            cur[k] = run;
            run += cnt[k];
        }
        if (lane < kXcdSlices) {
            int64_t st = 0;
#pragma unroll
            for (int k = 0; k < kXcdSlices; ++k) st += k < lane ? cnt[k] : 0;
            xo[x * kXcdSlices + lane] = (uint32_t)st;
        }
        for (int64_t e0 = a; e0 < b; e0 += 64) {
            const int64_t e = e0 + lane;
            const int32_t y = e < b ? col_in[e] : 0;
            const int sl = e < b ? row_slice(y, x) : -1;
#pragma unroll
            for (int k = 0; k < kXcdSlices; ++k) {
                const uint64_t m = __ballot(sl == k);
                if (sl == k) col_out[cur[k] + lanes_below(m)] = y;
                cur[k] += __popcll(m);
            }
        }
    }
}

hipError_t build_slice_rows(hipStream_t s, int32_t V, const int64_t* off, const int32_t* col_in,
                            int32_t* col_out, uint32_t* xo, int grid)
{
    int64_t g = ((int64_t)V + kWG / 64 - 1) / (kWG / 64);
    if (g > grid) g = grid;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_slice_partition, dim3((unsigned)g), dim3(kWG), 0, s, V, off, col_in,
                       col_out, xo);
    return hipGetLastError();
}

hipError_t build_row_skip(hipStream_t s, int32_t V, const int64_t* off, const int32_t* col_in,
                          int32_t* col_out, int32_t* skip, int grid)
{
    int64_t g = ((int64_t)V + kWG / 64 - 1) / (kWG / 64);
    if (g > grid) g = grid;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_row_partition, dim3((unsigned)g), dim3(kWG), 0, s, V, off, col_in,
                       col_out, skip);
    return hipGetLastError();
}

}  // namespace bfsmi
