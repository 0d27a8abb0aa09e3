// Single-root frontier expansion kernels for gfx950 (wave64, 256-thread
// workgroups).
//
// One BFS level is (Section 3.4 of the paper, one GPU over the whole graph):
//   scan   : d_k = deg(Q[k]); cumul = exclusive_scan(d)      (k_scan_*)
//   expand : every frontier edge e is mapped to the frontier entry
//            k = max{l : cumul[l] <= e} and its neighbour
//            v = col[off[Q[k]] + e - cumul[k]]; v's bit in the visited bitmap
//            is probed with a plain load and claimed with atomicOr; the
//            thread whose returned word lacked the bit is the only winner
//            and sets parent[v] = Q[k] (and level[v] in list mode)
//            (Algorithm 3)                                    (k_expand)
//   next   : list mode: winners append to the next queue (one atomicAdd per
//            wave); bitmap mode: the next frontier is the set of bits that
//            turned on during the level, compacted to a vertex-ordered list
//            that also sets level[v] with coalesced stores
//            (Section 5)                                      (k_bitmap_to_queue)
#include "bfs_internal.h"

namespace bfsmi {

// Number of set bits of mask in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan over the 256 threads of a workgroup; *total receives the
// sum.  s_wave must hold kWG / 64 elements.  Contains two barriers: every
// thread of the workgroup must call it.
template <typename T>
__device__ __forceinline__ T wg_exclusive_scan(T x, T* total, T* s_wave)
{
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const T incl = wave_inclusive_scan(x);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWG / 64; ++w) {
        const T t = s_wave[w];
        if (w < wave) before += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return before + incl - x;
}

// ---------------------------------------------------------------------------
// Initialisation (Algorithm 2): level = -1, parent = -1, bitmap = 0, then the
// root: level 0, parent = root, its visited bit, frontier = {root}.

__global__ __launch_bounds__(kWG) void k_init(int32_t V, int32_t W, int32_t root,
                                              int32_t* __restrict__ level,
                                              int32_t* __restrict__ parent,
                                              uint32_t* __restrict__ vis,
                                              uint32_t* __restrict__ vis_old,
                                              int32_t* __restrict__ Q, Ctrl* __restrict__ ctrl,
                                              int vec)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t done = 0;
    if (vec) {
        // 16-byte stores; both arrays are 16-byte aligned (checked on host)
        const int64_t V4 = V / 4;
        int4* l4 = reinterpret_cast<int4*>(level);
        int4* p4 = reinterpret_cast<int4*>(parent);
        for (int64_t i = tid; i < V4; i += stride) {
            int4 lv = make_int4(-1, -1, -1, -1);
            int4 pv = lv;
            const int64_t b = i * 4;
            if (root >= b && root < b + 4) {
                const int c = (int)(root - b);
                if (c == 0) { lv.x = 0; pv.x = root; }
                if (c == 1) { lv.y = 0; pv.y = root; }
                if (c == 2) { lv.z = 0; pv.z = root; }
                if (c == 3) { lv.w = 0; pv.w = root; }
            }
            l4[i] = lv;
            if (parent) p4[i] = pv;
        }
        done = V4 * 4;
    }
    for (int64_t v = done + tid; v < V; v += stride) {
        level[v] = v == root ? 0 : -1;
        if (parent) parent[v] = v == root ? root : -1;
    }
    const int64_t rw = root >> 5;
    const uint32_t rb = 1u << (root & 31);
    for (int64_t i = tid; i < W; i += stride) {
        const uint32_t w = i == rw ? rb : 0u;
        vis[i] = w;
        vis_old[i] = w;
    }
    if (tid == 0) {
        Q[0] = root;
        ctrl->r = 0;
        ctrl->ntiles = 0;
        ctrl->bitmap_out = 0;
        ctrl->qn_count = 0;
        ctrl->qlen = 1;
        ctrl->level = 1;
        ctrl->done = 0;
        ctrl->r_total = 0;
        ctrl->reached = 1;
        ctrl->levels = 1;
        ctrl->bitmap_levels = 0;
        ctrl->err = 0;
    }
}

hipError_t launch_init(hipStream_t s, int32_t V, int32_t W, int32_t root, int32_t* level,
                       int32_t* parent, uint32_t* vis, uint32_t* vis_old, int32_t* Q,
                       Ctrl* ctrl, int grid_cap)
{
    const bool vec = ((uintptr_t)level % 16 == 0) &&
                     (parent == nullptr || (uintptr_t)parent % 16 == 0);
    int64_t work = (int64_t)(vec ? V / 4 : V);
    if (W > work) work = W;
    int64_t grid = (work + kWG - 1) / kWG;
    if (grid > grid_cap) grid = grid_cap;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_init, dim3((unsigned)grid), dim3(kWG), 0, s, V, W, root, level, parent,
                       vis, vis_old, Q, ctrl, vec ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Degree scan: deg, block sums, scan of block sums, per-entry cumul and
// tile heads (tile_k[t] = frontier entry holding edge t * tile).

__global__ __launch_bounds__(kWG) void k_scan_reduce(const int32_t* __restrict__ Q, int32_t qlen,
                                                     const int64_t* __restrict__ off,
                                                     int32_t* __restrict__ deg,
                                                     int64_t* __restrict__ bsum)
{
    __shared__ int64_t s_wave[kWG / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int64_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t k = base + j * kWG + threadIdx.x;
        if (k < qlen) {
            const int32_t u = Q[k];
            const int64_t d = off[u + 1] - off[u];
            deg[k] = (int32_t)d;
            sum += d;
        }
    }
    int64_t tot;
    wg_exclusive_scan<int64_t>(sum, &tot, s_wave);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kWG) void k_scan_top(int64_t* __restrict__ bsum, int32_t nblk,
                                                  int32_t qlen, int64_t tile_cap, int32_t tile,
                                                  int64_t bitmap_threshold, int allow_bitmap,
                                                  int64_t* __restrict__ cumul,
                                                  int32_t* __restrict__ tile_k,
                                                  Ctrl* __restrict__ ctrl)
{
    __shared__ int64_t s_wave[kWG / 64];
    int64_t carry = 0;
    for (int32_t b0 = 0; b0 < nblk; b0 += kWG) {
        const int32_t b = b0 + threadIdx.x;
        const int64_t x = b < nblk ? bsum[b] : 0;
        int64_t tot;
        const int64_t ex = wg_exclusive_scan<int64_t>(x, &tot, s_wave);
        if (b < nblk) bsum[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        int64_t r = carry;
        int64_t nt = (r + tile - 1) / tile;
        if (nt > tile_cap) {  // more edges than the graph holds: refuse
            ctrl->err = 1;
            r = 0;
            nt = 0;
        }
        const int32_t ntiles = (int32_t)nt;
        ctrl->r = r;
        ctrl->ntiles = ntiles;
        ctrl->qlen = qlen;
        ctrl->bitmap_out = (allow_bitmap == 2 && r > 0) || (allow_bitmap == 1 && r > bitmap_threshold);
        ctrl->qn_count = 0;
        cumul[qlen] = r;
        tile_k[ntiles] = qlen - 1;
    }
}

__global__ __launch_bounds__(kWG) void k_scan_down(const int32_t* __restrict__ deg, int32_t qlen,
                                                   const int64_t* __restrict__ bsum,
                                                   int64_t tile_cap,
                                                   int32_t tile, int64_t* __restrict__ cumul,
                                                   int32_t* __restrict__ tile_k)
{
    __shared__ int64_t s_wave[kWG / 64];
    // +1 word of padding every 8 entries keeps the strided reads conflict-light
    __shared__ int32_t s_deg[kScanChunk + kScanChunk / kScanItems];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int32_t li = j * kWG + threadIdx.x;
        const int64_t k = base + li;
        s_deg[li + li / kScanItems] = k < qlen ? deg[k] : 0;
    }
    __syncthreads();
    int64_t local[kScanItems];
    int64_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int32_t li = threadIdx.x * kScanItems + j;
        local[j] = sum;
        sum += s_deg[li + li / kScanItems];
    }
    int64_t tot;
    const int64_t ex = wg_exclusive_scan<int64_t>(sum, &tot, s_wave);
    const int64_t start = bsum[blockIdx.x] + ex;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int32_t li = threadIdx.x * kScanItems + j;
        const int64_t k = base + li;
        if (k < qlen) {
            const int64_t c = start + local[j];
            cumul[k] = c;
            const int32_t d = s_deg[li + li / kScanItems];
            if (d > 0) {
                const int64_t t0 = (c + tile - 1) / tile;
                int64_t t1 = (c + d - 1) / tile;
                if (t1 >= tile_cap) t1 = tile_cap - 1;
                for (int64_t t = t0; t <= t1; ++t) tile_k[t] = (int32_t)k;
            }
        }
    }
}

hipError_t launch_scan(hipStream_t s, const int32_t* Q, int32_t qlen, const int64_t* off,
                       int32_t* deg, int64_t* bsum, int64_t* cumul, int32_t* tile_k,
                       int64_t tile_cap, int tile, int64_t bitmap_threshold, int allow_bitmap,
                       Ctrl* ctrl)
{
    const int32_t nblk = (int32_t)(((int64_t)qlen + kScanChunk - 1) / kScanChunk);
    if (nblk > 0) {
        hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kWG), 0, s, Q, qlen, off, deg, bsum);
    }
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kWG), 0, s, bsum, nblk, qlen, tile_cap, tile,
                       bitmap_threshold, allow_bitmap, cumul, tile_k, ctrl);
    if (nblk > 0) {
        hipLaunchKernelGGL(k_scan_down, dim3(nblk), dim3(kWG), 0, s, deg, qlen, bsum, tile_cap,
                           tile, cumul, tile_k);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Frontier expansion.  A workgroup owns a tile of TILE = 256 * EPT
// consecutive frontier edges [e0, e0 + TILE).  The frontier entries that
// overlap the tile, [tile_k[t], tile_k[t + 1]], are staged in LDS; each
// thread binary-searches the staged cumulative degrees once for its first
// slot and advances linearly over EPT consecutive slots (Section 3.4.1),
// recording slot -> entry in LDS.  The edges are then visited with a slot
// stride of 256 so that the column loads of a wave are contiguous.

template <int EPT>
__global__ __launch_bounds__(kWG) void k_expand(int32_t V, const int32_t* __restrict__ Q,
                                                const int64_t* __restrict__ cumul,
                                                const int32_t* __restrict__ tile_k,
                                                const int64_t* __restrict__ off,
                                                const int32_t* __restrict__ col,
                                                uint32_t* __restrict__ vis,
                                                uint32_t* __restrict__ vis_old,
                                                int32_t* __restrict__ level,
                                                int32_t* __restrict__ parent, int32_t lvl,
                                                int32_t* __restrict__ Qn,
                                                Ctrl* __restrict__ ctrl)
{
    constexpr int TILE = kWG * EPT;
    __shared__ int32_t s_cum[TILE + 1];
    __shared__ int32_t s_u[TILE + 1];
    __shared__ int64_t s_base[TILE + 1];
    __shared__ uint16_t s_map[TILE];

    const int64_t r = ctrl->r;
    const int32_t ntiles = ctrl->ntiles;
    const bool list_out = ctrl->bitmap_out == 0;

    for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t e0 = (int64_t)tile * TILE;
        const int64_t rem = r - e0;
        const int32_t n_e = rem < TILE ? (int32_t)rem : TILE;
        const int32_t k_lo = tile_k[tile];
        const int32_t k_hi = tile_k[tile + 1];
        const int32_t n_k = k_hi - k_lo + 1;

        int32_t uu[EPT], vv[EPT];
        bool ok[EPT];
        if (n_k <= TILE + 1) {
            for (int32_t i = threadIdx.x; i < n_k; i += kWG) {
                const int32_t k = k_lo + i;
                const int32_t u = Q[k];
                const int64_t c = cumul[k];
                const int64_t rel = c - e0;
                s_cum[i] = rel > 0 ? (int32_t)rel : 0;
                s_u[i] = u;
                s_base[i] = off[u] - c;
            }
            __syncthreads();
            const int32_t s0 = threadIdx.x * EPT;
            if (s0 < n_e) {
                int32_t lo = 0, hi = n_k - 1;  // s_cum[0] == 0 <= s0
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (s_cum[mid] <= s0) lo = mid;
                    else hi = mid - 1;
                }
                int32_t i = lo;
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    const int32_t sl = s0 + j;
                    if (sl < n_e) {
                        while (i + 1 < n_k && s_cum[i + 1] <= sl) ++i;
                        s_map[sl] = (uint16_t)i;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const int32_t sl = threadIdx.x + j * kWG;
                ok[j] = sl < n_e;
                uu[j] = 0;
                vv[j] = 0;
                if (ok[j]) {
                    const int32_t i = s_map[sl];
                    uu[j] = s_u[i];
                    vv[j] = __builtin_nontemporal_load(col + (s_base[i] + e0 + sl));
                }
            }
        } else {
            // More frontier entries than tile slots (zero-degree entries):
            // search the global cumulative array for each edge.
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const int32_t sl = threadIdx.x + j * kWG;
                ok[j] = sl < n_e;
                uu[j] = 0;
                vv[j] = 0;
                if (ok[j]) {
                    const int64_t e = e0 + sl;
                    int32_t lo = k_lo, hi = k_hi;
                    while (lo < hi) {
                        const int32_t mid = lo + ((hi - lo + 1) >> 1);
                        if (cumul[mid] <= e) lo = mid;
                        else hi = mid - 1;
                    }
                    const int32_t u = Q[lo];
                    uu[j] = u;
                    vv[j] = col[off[u] + (e - cumul[lo])];
                }
            }
        }

        // Visit: probe (plain load; a stale word only lets more threads try
        // the atomic), then claim.
        uint32_t wd[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) wd[j] = ok[j] ? vis[vv[j] >> 5] : 0xffffffffu;
        bool win[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            win[j] = false;
            const uint32_t m = 1u << (vv[j] & 31);
            if (ok[j] && !(wd[j] & m)) {
                const uint32_t old = atomicOr(vis + (vv[j] >> 5), m);
                win[j] = !(old & m);
            }
        }
        if (parent) {
#pragma unroll
            for (int j = 0; j < EPT; ++j)
                if (win[j]) parent[vv[j]] = uu[j];
        }
        if (list_out) {
            uint64_t mask[EPT];
            uint32_t total = 0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                mask[j] = __ballot(win[j]);
                total += (uint32_t)__popcll(mask[j]);
            }
            if (total) {
                uint32_t base = 0;
                if (__lane_id() == 0) base = atomicAdd(&ctrl->qn_count, total);
                base = __shfl(base, 0, 64);
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    if (win[j]) {
                        const int32_t v = vv[j];
                        const uint32_t pos = base + lanes_below(mask[j]);
                        if (pos < (uint32_t)V) Qn[pos] = v;
                        else ctrl->err = 2;
                        level[v] = lvl;
                        atomicOr(vis_old + (v >> 5), 1u << (v & 31));
                    }
                    base += (uint32_t)__popcll(mask[j]);
                }
            }
        }
        __syncthreads();
    }
}

hipError_t launch_expand(hipStream_t s, int ept, int grid, int32_t V, const int32_t* Q,
                         const int64_t* cumul,
                         const int32_t* tile_k, const int64_t* off, const int32_t* col,
                         uint32_t* vis, uint32_t* vis_old, int32_t* level, int32_t* parent,
                         int32_t lvl, int32_t* Qn, Ctrl* ctrl)
{
    if (grid < 1) grid = 1;
    switch (ept) {
    case 1:
        hipLaunchKernelGGL(k_expand<1>, dim3(grid), dim3(kWG), 0, s, V, Q, cumul, tile_k, off, col,
                           vis, vis_old, level, parent, lvl, Qn, ctrl);
        break;
    case 2:
        hipLaunchKernelGGL(k_expand<2>, dim3(grid), dim3(kWG), 0, s, V, Q, cumul, tile_k, off, col,
                           vis, vis_old, level, parent, lvl, Qn, ctrl);
        break;
    case 4:
        hipLaunchKernelGGL(k_expand<4>, dim3(grid), dim3(kWG), 0, s, V, Q, cumul, tile_k, off, col,
                           vis, vis_old, level, parent, lvl, Qn, ctrl);
        break;
    case 8:
        hipLaunchKernelGGL(k_expand<8>, dim3(grid), dim3(kWG), 0, s, V, Q, cumul, tile_k, off, col,
                           vis, vis_old, level, parent, lvl, Qn, ctrl);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Bitmap form of the next frontier: F = vis & ~vis_old (the bits that turned
// on during this level), vis_old := vis, and F compacted in vertex order to
// the next queue.  A workgroup handles 256 words (8192 vertices); thread j
// of pass p looks at vertex p * 256 + j of the block, so level stores and
// queue stores of a wave are contiguous.

__global__ __launch_bounds__(kWG) void k_bitmap_to_queue(int32_t V, int32_t W,
                                                         uint32_t* __restrict__ vis,
                                                         uint32_t* __restrict__ vis_old,
                                                         int32_t* __restrict__ Qn,
                                                         int32_t* __restrict__ level,
                                                         int32_t lvl, Ctrl* __restrict__ ctrl)
{
    if (!ctrl->bitmap_out) return;
    __shared__ uint32_t s_f[kBitmapWordsPerWG];
    __shared__ uint32_t s_off[kBitmapWordsPerWG];
    __shared__ uint32_t s_wave[kWG / 64];
    __shared__ uint32_t s_base;
    const int64_t nblocks = ((int64_t)W + kBitmapWordsPerWG - 1) / kBitmapWordsPerWG;
    for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const int64_t i = blk * kBitmapWordsPerWG + threadIdx.x;
        uint32_t f = 0;
        if (i < W) {
            const uint32_t a = vis[i];
            const uint32_t b = vis_old[i];
            f = a & ~b;
            if (f) vis_old[i] = a;
        }
        uint32_t tot;
        const uint32_t ex = wg_exclusive_scan<uint32_t>((uint32_t)__popc(f), &tot, s_wave);
        s_f[threadIdx.x] = f;
        s_off[threadIdx.x] = ex;
        if (threadIdx.x == 0) s_base = tot ? atomicAdd(&ctrl->qn_count, tot) : 0u;
        __syncthreads();
        if (tot) {
            const uint32_t base = s_base;
            const int64_t vbase = blk * kBitmapWordsPerWG * 32;
#pragma unroll 4
            for (int p = 0; p < 32; ++p) {
                const int32_t local = p * kWG + threadIdx.x;
                const uint32_t w = s_f[local >> 5];
                const uint32_t bit = local & 31;
                if ((w >> bit) & 1u) {
                    const int32_t v = (int32_t)(vbase + local);
                    const uint32_t rank = s_off[local >> 5] + (uint32_t)__popc(w & ((1u << bit) - 1u));
                    if (base + rank < (uint32_t)V) Qn[base + rank] = v;
                    else ctrl->err = 3;
                    level[v] = lvl;
                }
            }
        }
        __syncthreads();
    }
}

hipError_t launch_bitmap_to_queue(hipStream_t s, int grid, int32_t V, int32_t W, uint32_t* vis,
                                  uint32_t* vis_old, int32_t* Qn, int32_t* level, int32_t lvl,
                                  Ctrl* ctrl)
{
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_bitmap_to_queue, dim3(grid), dim3(kWG), 0, s, V, W, vis, vis_old, Qn,
                       level, lvl, ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CSR checks for graph creation: offsets start at 0, end at nnz, never
// decrease; every column id is in [0, V).  Also the maximum degree.

__global__ __launch_bounds__(kWG) void k_validate_csr(int32_t V, int64_t nnz,
                                                      const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ col,
                                                      int32_t* __restrict__ bad,
                                                      int32_t* __restrict__ maxdeg, int check_col)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t mybad = 0;
    int64_t mymax = 0;
    for (int64_t v = tid; v < V; v += stride) {
        const int64_t a = off[v], b = off[v + 1];
        if (b < a) mybad |= 1;
        if (b - a > mymax) mymax = b - a;
    }
    if (tid == 0 && (off[0] != 0 || off[V] != nnz)) mybad |= 2;
    if (check_col) {
        for (int64_t e = tid; e < nnz; e += stride) {
            const int32_t c = col[e];
            if (c < 0 || c >= V) mybad |= 4;
        }
    }
    if (mybad) atomicOr(bad, mybad);
    if (mymax > 0) atomicMax(maxdeg, (int32_t)(mymax > 0x7fffffff ? 0x7fffffff : mymax));
}

hipError_t launch_validate_csr(hipStream_t s, int32_t V, int64_t nnz, const int64_t* off,
                               const int32_t* col, int32_t* bad_flag, int32_t* maxdeg,
                               int check_col)
{
    hipLaunchKernelGGL(k_validate_csr, dim3(1024), dim3(kWG), 0, s, V, nnz, off, col, bad_flag,
                       maxdeg, check_col);
    return hipGetLastError();
}

}  // namespace bfsmi
