// Degree-ordered internal relabelling, built on the GPU at graph creation.
//
// Vertices get internal ids in non-increasing order of degree class (a
// counting sort by class: degrees 0 to 3 on their own, above that four
// classes per power of two, given by the two bits after the leading one).
// The highest-degree vertices then own the lowest ids, so the visited bits
// that most frontier edges probe sit in a few contiguous words (and the
// visited summary's fully visited prefix covers them after the first
// levels).  Within a class, each run of 4096 consecutive caller ids gets one
// contiguous range of internal ids (order inside the run arbitrary), which
// keeps the end-of-search reordering pass local; the coarse classes keep
// the number of such ranges per run small.  The relabelled CSR keeps every
// row's neighbours in the input's order, mapped through rank.
// Graph creation is not part of a search's timed region (the paper starts
// its clock after partitioning the graph, Section 4).
#include "bfs_internal.h"
#include "tile_map.h"
#include "wave_ops.h"

namespace bfsmi {

constexpr int kDegBuckets = 256;
constexpr int kScatterChunk = kWG * 16;  // vertices per workgroup iteration
constexpr int kRelabelEPT = 4;

// Bucket 0 holds the highest degree class.
__device__ __forceinline__ int32_t deg_bucket(int64_t d)
{
    int32_t c;
    if (d < 4) {
        c = (int32_t)d;
    } else {
        const int hb = 63 - __clzll((unsigned long long)d);  // >= 2
        c = 4 + (hb - 2) * 4 + (int32_t)((d >> (hb - 2)) & 3);
    }
    if (c > kDegBuckets - 1) c = kDegBuckets - 1;
    return kDegBuckets - 1 - c;
}

__global__ __launch_bounds__(kWG) void k_deg_hist(int32_t V, const int64_t* __restrict__ off,
                                                  uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[kDegBuckets];
    for (int i = threadIdx.x; i < kDegBuckets; i += kWG) h[i] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < V; v += stride)
        atomicAdd(&h[deg_bucket(off[v + 1] - off[v])], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kDegBuckets; i += kWG)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// hist[0..kDegBuckets) := exclusive scan; hist[kDegBuckets..2x) := 0 (cursors)
__global__ __launch_bounds__(kWG) void k_deg_hist_scan(uint32_t* __restrict__ hist)
{
    __shared__ uint32_t s_wave[kWG / 64];
    uint32_t carry = 0;
    for (int b0 = 0; b0 < kDegBuckets; b0 += kWG) {
        const int b = b0 + threadIdx.x;
        const uint32_t x = hist[b];
        uint32_t tot;
        const uint32_t ex = wg_exclusive_scan<uint32_t>(x, &tot, s_wave);
        hist[b] = carry + ex;
        hist[kDegBuckets + b] = 0;
        carry += tot;
    }
}

__global__ __launch_bounds__(kWG) void k_deg_scatter(int32_t V, const int64_t* __restrict__ off,
                                                     const uint32_t* __restrict__ bstart,
                                                     uint32_t* __restrict__ cursor,
                                                     int32_t* __restrict__ rank,
                                                     int32_t* __restrict__ orig)
{
    __shared__ uint32_t h[kDegBuckets];
    constexpr int PER = kScatterChunk / kWG;
    for (int64_t c0 = (int64_t)blockIdx.x * kScatterChunk; c0 < V;
         c0 += (int64_t)gridDim.x * kScatterChunk) {
        for (int i = threadIdx.x; i < kDegBuckets; i += kWG) h[i] = 0;
        __syncthreads();
        int32_t b[PER];
        uint32_t local[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int64_t v = c0 + j * kWG + threadIdx.x;
            b[j] = -1;
            local[j] = 0;
            if (v < V) {
                b[j] = deg_bucket(off[v + 1] - off[v]);
                local[j] = atomicAdd(&h[b[j]], 1u);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kDegBuckets; i += kWG)
            if (h[i]) h[i] = atomicAdd(&cursor[i], h[i]);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (b[j] >= 0) {
                const int32_t v = (int32_t)(c0 + j * kWG + threadIdx.x);
                const int32_t x = (int32_t)(bstart[b[j]] + h[b[j]] + local[j]);
                rank[v] = x;
                orig[x] = v;
            }
        }
        __syncthreads();
    }
}

// col_r[e] = rank[col[off[orig[x]] + j]] for the j-th entry of internal row
// x, e = off_r[x] + j: the edge mapping of the search, with the identity
// frontier Q = orig over all vertices.
__global__ __launch_bounds__(kWG) void k_relabel_copy(const int64_t* __restrict__ rowstart,
                                                      const int32_t* __restrict__ uidv,
                                                      const int64_t* __restrict__ off_r,
                                                      const int32_t* __restrict__ tile_k,
                                                      const int32_t* __restrict__ col,
                                                      const int32_t* __restrict__ rank,
                                                      int32_t* __restrict__ col_r,
                                                      const Ctrl* __restrict__ ctrl)
{
    __shared__ TileLds<kRelabelEPT> L;
    const int64_t r = ctrl->r;
    const int32_t ntiles = ctrl->ntiles;
    StageRegs<kRelabelEPT> cur =
        fetch_stage<kRelabelEPT>(blockIdx.x, ntiles, off_r, rowstart, uidv, tile_k);
    for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int32_t uid[kRelabelEPT], v[kRelabelEPT];
        bool ok[kRelabelEPT];
        int64_t e[kRelabelEPT];
        map_tile<kRelabelEPT>(L, cur, r, off_r, rowstart, uidv, col, uid, v, ok, e);
        cur = fetch_stage<kRelabelEPT>(tile + gridDim.x, ntiles, off_r, rowstart, uidv, tile_k);
#pragma unroll
        for (int j = 0; j < kRelabelEPT; ++j)
            if (ok[j]) col_r[e[j]] = rank[v[j]];
        __syncthreads();
    }
}

hipError_t build_degree_order(hipStream_t s, int32_t V, int64_t nnz, const int64_t* off,
                              const int32_t* col, int32_t* rank, int32_t* orig, int64_t* off_r,
                              int32_t* col_r, int32_t* deg_tmp, int64_t* rowstart_tmp,
                              int32_t* uid_tmp, int64_t* bsum_tmp, int32_t* tile_k,
                              int64_t tile_cap, uint32_t* hist_tmp, Ctrl* ctrl, int grid_cap)
{
    hipError_t e = hipMemsetAsync(hist_tmp, 0, 2 * kDegBuckets * sizeof(uint32_t), s);
    if (e != hipSuccess) return e;
    int64_t g1 = ((int64_t)V + kWG - 1) / kWG;
    if (g1 > grid_cap) g1 = grid_cap;
    hipLaunchKernelGGL(k_deg_hist, dim3((unsigned)g1), dim3(kWG), 0, s, V, off, hist_tmp);
    hipLaunchKernelGGL(k_deg_hist_scan, dim3(1), dim3(kWG), 0, s, hist_tmp);
    int64_t g2 = ((int64_t)V + kScatterChunk - 1) / kScatterChunk;
    if (g2 > grid_cap) g2 = grid_cap;
    hipLaunchKernelGGL(k_deg_scatter, dim3((unsigned)g2), dim3(kWG), 0, s, V, off, hist_tmp,
                       hist_tmp + kDegBuckets, rank, orig);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // off_r = exclusive scan of deg(orig[x]) with tile heads for the copy
    e = launch_scan(s, orig, V, off, nullptr, deg_tmp, rowstart_tmp, uid_tmp, bsum_tmp, off_r,
                    tile_k, tile_cap, kWG * kRelabelEPT, (int64_t)1 << 62, 0, ctrl);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_relabel_copy, dim3((unsigned)grid_cap), dim3(kWG), 0, s, rowstart_tmp,
                       uid_tmp, off_r, tile_k, col, rank, col_r, ctrl);
    (void)nnz;
    return hipGetLastError();
}

}  // namespace bfsmi
