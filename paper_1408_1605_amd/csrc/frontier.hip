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
//            and sets level[v] and parent[v] = Q[k]  (Algorithm 3)  (k_expand)
//   next   : list mode: winners append to the next queue (one atomicAdd per
//            wave); bitmap mode: the next frontier is the set of bits that
//            turned on during the level, compacted to an id-ordered list
//            (Section 5)                                      (k_bitmap_to_queue)
#include "bfs_internal.h"
#include "tile_map.h"
#include "wave_ops.h"

namespace bfsmi {

// ---------------------------------------------------------------------------
// Initialisation (Algorithm 2): level = -1, parent = -1, bitmap = 0, then the
// root: level 0, parent = root, its visited bit, frontier = {root}.  level
// and parent are indexed by search id (the internal id under degree order,
// where the root's slot is rank[root]); the root's parent value is its
// caller id.  With fill == 0 (degree order) only the root's entries are
// written: k_finish reads level / parent only for visited vertices.

__global__ __launch_bounds__(kWG) void k_init(int32_t V, int32_t W, int32_t root,
                                              const int32_t* __restrict__ rank,
                                              int32_t* __restrict__ level,
                                              int32_t* __restrict__ parent,
                                              uint32_t* __restrict__ vis,
                                              uint32_t* __restrict__ vis_old,
                                              int32_t* __restrict__ Q, Ctrl* __restrict__ ctrl,
                                              int vec, int fill, uint4* __restrict__ found16,
                                              int64_t n_found16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t rin = rank ? rank[root] : root;  // the root's search id
    int64_t done = fill ? 0 : V;
    if (!fill && tid == 0) {
        level[rin] = 0;
        if (parent) parent[rin] = root;
    }
    if (fill && vec) {
        // 16-byte stores; both arrays are 16-byte aligned (checked on host)
        const int64_t V4 = V / 4;
        int4* l4 = reinterpret_cast<int4*>(level);
        int4* p4 = reinterpret_cast<int4*>(parent);
        for (int64_t i = tid; i < V4; i += stride) {
            int4 lv = make_int4(-1, -1, -1, -1);
            int4 pv = lv;
            const int64_t b = i * 4;
            if (rin >= b && rin < b + 4) {
                const int c = (int)(rin - b);
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
        level[v] = v == rin ? 0 : -1;
        if (parent) parent[v] = v == rin ? root : -1;
    }
    for (int64_t i = tid; i < n_found16; i += stride) found16[i] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t rw = rin >> 5;
    const uint32_t rb = 1u << (rin & 31);
    for (int64_t i = tid; i < W; i += stride) {
        const uint32_t w = i == rw ? rb : 0u;
        vis[i] = w;
        vis_old[i] = w;
    }
    if (tid == 0) {
        Q[0] = rin;
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
        ctrl->skipped = 0;
    }
}

hipError_t launch_init(hipStream_t s, int32_t V, int32_t W, int32_t root, const int32_t* rank,
                       int32_t* level, int32_t* parent, uint32_t* vis, uint32_t* vis_old,
                       int32_t* Q, Ctrl* ctrl, int grid_cap, int fill, uint8_t* found)
{
    const bool vec = ((uintptr_t)level % 16 == 0) &&
                     (parent == nullptr || (uintptr_t)parent % 16 == 0);
    // the flags are padded to whole words: W * 32 bytes
    const int64_t n_found16 = found ? (int64_t)W * 2 : 0;
    int64_t work = fill ? (int64_t)(vec ? V / 4 : V) : 0;
    if (W > work) work = W;
    if (n_found16 > work) work = n_found16;
    int64_t grid = (work + kWG - 1) / kWG;
    if (grid > grid_cap) grid = grid_cap;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_init, dim3((unsigned)grid), dim3(kWG), 0, s, V, W, root, rank, level,
                       parent, vis, vis_old, Q, ctrl, vec ? 1 : 0, fill,
                       reinterpret_cast<uint4*>(found), n_found16);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Degree scan: deg, block sums, scan of block sums, per-entry cumul and
// tile heads (tile_k[t] = frontier entry holding edge t * tile).

// With dev != 0 the frontier size comes from ctrl->qlen and the kernels
// return at once when ctrl->done is set, so a fixed-size launch sequence can
// be replayed for any level (device-driven loops, graph capture); the block
// loops are grid-stride in both modes.

__global__ __launch_bounds__(kWG) void k_scan_reduce(const int32_t* __restrict__ Q, int32_t qlen_arg,
                                                     const int64_t* __restrict__ off,
                                                     const int32_t* __restrict__ uid_map,
                                                     int32_t* __restrict__ deg,
                                                     int64_t* __restrict__ rowstart,
                                                     int32_t* __restrict__ uidv,
                                                     int64_t* __restrict__ bsum,
                                                     Ctrl* __restrict__ ctrl, int dev,
                                                     const int32_t* __restrict__ skip, int32_t V)
{
    __shared__ int64_t s_wave[kWG / 64];
    if (dev && ctrl->done) return;
    const int32_t qlen = dev ? ctrl->qlen : qlen_arg;
    const int64_t nblk = ((int64_t)qlen + kScanChunk - 1) / kScanChunk;
    // row prefix skip: the largest threshold 2^(16 + i) below which every
    // id is visited (uniform across the grid: full_prefix is set before)
    const int32_t* sk = nullptr;
    if (skip) {
        const int32_t fp = ctrl->full_prefix;
        int lv = -1;
#pragma unroll
        for (int i = 0; i < kSkipLevels; ++i)
            if (fp >= (1 << (kSkipLow + i))) lv = i;
        if (lv >= 0) sk = skip + (int64_t)lv * V;
    }
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t base = blk * kScanChunk;
        int64_t sum = 0, dropped = 0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const int64_t k = base + j * kWG + threadIdx.x;
            if (k < qlen && !Q) {
                sum += deg[k];  // entries prefilled (k_slice_entries)
            } else if (k < qlen) {
                const int32_t u = Q[k];
                int64_t a = off[u];
                int64_t d = off[u + 1] - a;
                if (sk) {
                    const int32_t n = sk[u];
                    a += n;
                    d -= n;
                    dropped += n;
                }
                deg[k] = (int32_t)d;
                rowstart[k] = a;
                uidv[k] = uid_map ? uid_map[u] : u;
                sum += d;
            }
        }
        int64_t tot;
        wg_exclusive_scan<int64_t>(sum, &tot, s_wave);
        if (threadIdx.x == 0) bsum[blk] = tot;
        if (sk) {
            int64_t dtot;
            wg_exclusive_scan<int64_t>(dropped, &dtot, s_wave);
            if (threadIdx.x == 0 && dtot) atomicAdd((unsigned long long*)&ctrl->skipped,
                                                    (unsigned long long)dtot);
        }
    }
}

__global__ __launch_bounds__(kWG) void k_scan_top(int64_t* __restrict__ bsum, int32_t qlen_arg,
                                                  int64_t tile_cap, int32_t tile,
                                                  int64_t bitmap_threshold, int allow_bitmap,
                                                  int64_t* __restrict__ cumul,
                                                  int32_t* __restrict__ tile_k,
                                                  Ctrl* __restrict__ ctrl, int dev)
{
    __shared__ int64_t s_wave[kWG / 64];
    if (dev && ctrl->done) return;
    const int32_t qlen = dev ? ctrl->qlen : qlen_arg;
    const int32_t nblk = (int32_t)(((int64_t)qlen + kScanChunk - 1) / kScanChunk);
    // kTopItems consecutive block sums per thread and pass: a heavy level
    // has thousands of blocks, and each pass costs two barriers
    constexpr int kTopItems = 8;
    int64_t carry = 0;
    for (int32_t b0 = 0; b0 < nblk; b0 += kWG * kTopItems) {
        int64_t x[kTopItems];
        int64_t sum = 0;
#pragma unroll
        for (int i = 0; i < kTopItems; ++i) {
            const int32_t b = b0 + threadIdx.x * kTopItems + i;
            x[i] = b < nblk ? bsum[b] : 0;
            sum += x[i];
        }
        int64_t tot;
        int64_t run = carry + wg_exclusive_scan<int64_t>(sum, &tot, s_wave);
#pragma unroll
        for (int i = 0; i < kTopItems; ++i) {
            const int32_t b = b0 + threadIdx.x * kTopItems + i;
            if (b < nblk) bsum[b] = run;
            run += x[i];
        }
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
        ctrl->next_deg = 0;
        ctrl->r_total += r;
        cumul[qlen] = r;
        tile_k[ntiles] = qlen - 1;
    }
}

__global__ __launch_bounds__(kWG) void k_scan_down(const int32_t* __restrict__ deg, int32_t qlen_arg,
                                                   const int64_t* __restrict__ bsum,
                                                   int64_t tile_cap,
                                                   int32_t tile, int64_t* __restrict__ cumul,
                                                   int32_t* __restrict__ tile_k,
                                                   const Ctrl* __restrict__ ctrl, int dev)
{
    __shared__ int64_t s_wave[kWG / 64];
    // +1 word of padding every 8 entries keeps the strided reads conflict-light
    __shared__ int32_t s_deg[kScanChunk + kScanChunk / kScanItems];
    __shared__ int64_t s_cum[kScanChunk];  // transposes the stores
    // entries whose edges cover many tiles (hubs) have their tile heads
    // written by the whole workgroup instead of by their own thread
    __shared__ int64_t s_big_t0[kBigTileList], s_big_t1[kBigTileList];
    __shared__ int32_t s_big_k[kBigTileList];
    __shared__ int32_t s_nbig;
    if (dev && ctrl->done) return;
    const int32_t qlen = dev ? ctrl->qlen : qlen_arg;
    const int64_t nblk = ((int64_t)qlen + kScanChunk - 1) / kScanChunk;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t base = blk * kScanChunk;
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
        if (threadIdx.x == 0) s_nbig = 0;
        int64_t tot;
        const int64_t ex = wg_exclusive_scan<int64_t>(sum, &tot, s_wave);  // barriers inside
        const int64_t start = bsum[blk] + ex;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const int32_t li = threadIdx.x * kScanItems + j;
            const int64_t k = base + li;
            const int64_t c = start + local[j];
            s_cum[li] = c;
            if (k < qlen) {
                const int32_t d = s_deg[li + li / kScanItems];
                if (d > 0) {
                    const int64_t t0 = (c + tile - 1) / tile;
                    int64_t t1 = (c + d - 1) / tile;
                    if (t1 >= tile_cap) t1 = tile_cap - 1;
                    bool mine = true;
                    if (t1 - t0 >= kBigTiles) {
                        const int32_t slot = atomicAdd(&s_nbig, 1);
                        if (slot < kBigTileList) {
                            s_big_t0[slot] = t0;
                            s_big_t1[slot] = t1;
                            s_big_k[slot] = (int32_t)k;
                            mine = false;
                        }
                    }
                    if (mine)
                        for (int64_t t = t0; t <= t1; ++t) tile_k[t] = (int32_t)k;
                }
            }
        }
        __syncthreads();
        const int32_t nbig = min(s_nbig, kBigTileList);
        for (int32_t b = 0; b < nbig; ++b) {
            const int32_t k = s_big_k[b];
            for (int64_t t = s_big_t0[b] + threadIdx.x; t <= s_big_t1[b]; t += kWG) tile_k[t] = k;
        }
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const int32_t li = j * kWG + threadIdx.x;
            if (base + li < qlen) cumul[base + li] = s_cum[li];
        }
        __syncthreads();  // s_deg and s_cum are reused by the next block
    }
}

// XCD-sliced level: frontier entry k becomes the eight entries s * qlen + k
// (s = 0..7), the slice-s group of its row (grouped rows col_x, offsets xo;
// row starts as in off), so one scan over 8 * qlen entries numbers the
// edges slice by slice.
__global__ __launch_bounds__(kWG) void k_slice_entries(const int32_t* __restrict__ Q, int32_t qlen,
                                                       const int64_t* __restrict__ off,
                                                       const uint32_t* __restrict__ xo,
                                                       const int32_t* __restrict__ uid_map,
                                                       int32_t* __restrict__ deg,
                                                       int64_t* __restrict__ rowstart,
                                                       int32_t* __restrict__ uidv)
{
    for (int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x; k < qlen;
         k += (int64_t)gridDim.x * kWG) {
        const int32_t u = Q[k];
        const int64_t a = off[u];
        const uint32_t d = (uint32_t)(off[u + 1] - a);
        const uint4 lo = *reinterpret_cast<const uint4*>(xo + (int64_t)u * kXcdSlices);
        const uint4 hi = *reinterpret_cast<const uint4*>(xo + (int64_t)u * kXcdSlices + 4);
        const uint32_t st[kXcdSlices + 1] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w, d};
        const int32_t id = uid_map ? uid_map[u] : u;
#pragma unroll
        for (int s = 0; s < kXcdSlices; ++s) {
            const int64_t i = (int64_t)s * qlen + k;
            deg[i] = (int32_t)(st[s + 1] - st[s]);
            rowstart[i] = a + st[s];
            uidv[i] = id;
        }
    }
}

hipError_t launch_slice_scan(hipStream_t s, int grid, const int32_t* Q, int32_t qlen,
                             const int64_t* off, const uint32_t* xo, const int32_t* uid_map,
                             int32_t* deg, int64_t* rowstart, int32_t* uidv, int64_t* bsum,
                             int64_t* cumul, int32_t* tile_k, int64_t tile_cap, int tile,
                             int64_t bitmap_threshold, int allow_bitmap, Ctrl* ctrl)
{
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_slice_entries, dim3(grid), dim3(kWG), 0, s, Q, qlen, off, xo, uid_map, deg,
                       rowstart, uidv);
    // the scan proper over the 8 * qlen prefilled entries (Q == nullptr)
    return launch_scan(s, nullptr, kXcdSlices * qlen, off, nullptr, deg, rowstart, uidv, bsum,
                       cumul, tile_k, tile_cap, tile, bitmap_threshold, allow_bitmap, ctrl);
}

hipError_t launch_scan(hipStream_t s, const int32_t* Q, int32_t qlen, const int64_t* off,
                       const int32_t* uid_map, int32_t* deg, int64_t* rowstart, int32_t* uidv,
                       int64_t* bsum, int64_t* cumul, int32_t* tile_k, int64_t tile_cap,
                       int tile, int64_t bitmap_threshold, int allow_bitmap, Ctrl* ctrl,
                       const int32_t* skip, int32_t V)
{
    const int32_t nblk = (int32_t)(((int64_t)qlen + kScanChunk - 1) / kScanChunk);
    if (nblk > 0) {
        hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kWG), 0, s, Q, qlen, off, uid_map, deg,
                           rowstart, uidv, bsum, ctrl, 0, skip, V);
    }
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kWG), 0, s, bsum, qlen, tile_cap, tile,
                       bitmap_threshold, allow_bitmap, cumul, tile_k, ctrl, 0);
    if (nblk > 0) {
        hipLaunchKernelGGL(k_scan_down, dim3(nblk), dim3(kWG), 0, s, deg, qlen, bsum, tile_cap,
                           tile, cumul, tile_k, ctrl, 0);
    }
    return hipGetLastError();
}

hipError_t launch_scan_dev(hipStream_t s, int grid, const int32_t* Q, const int64_t* off,
                           const int32_t* uid_map, int32_t* deg, int64_t* rowstart, int32_t* uidv,
                           int64_t* bsum, int64_t* cumul, int32_t* tile_k, int64_t tile_cap,
                           int tile, Ctrl* ctrl, const int32_t* skip, int32_t V)
{
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3(grid), dim3(kWG), 0, s, Q, 0, off, uid_map, deg,
                       rowstart, uidv, bsum, ctrl, 1, skip, V);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kWG), 0, s, bsum, 0, tile_cap, tile,
                       (int64_t)1 << 62, 0, cumul, tile_k, ctrl, 1);
    hipLaunchKernelGGL(k_scan_down, dim3(grid), dim3(kWG), 0, s, deg, 0, bsum, tile_cap, tile,
                       cumul, tile_k, ctrl, 1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Visited summary for the expansion's early test (a two-level bitmap).
//
// Before a heavy level, k_visited_summary records (a) full_prefix: every
// vertex id below it is already visited, and (b) one bit per block of
// 2^shift ids that is set when the whole block is visited.  Both only ever
// under-report (bits are only set during a search), so "summary says
// visited" implies the bitmap bit is set and the paper's early test would
// return.  With degree-ordered ids the highest-degree vertices, which most
// frontier edges point to, fill the lowest ids, and at the heaviest level
// most probes are answered by a register compare or an LDS bit.

// One workgroup per summary word: 32 blocks of 2^shift ids.  Thread t of
// the workgroup checks P = 2^(shift-8) consecutive bitmap words, so 8
// consecutive threads cover one block; no atomics, one plain store per word.
__global__ __launch_bounds__(kWG) void k_visited_summary(int32_t V, int32_t W,
                                                         const uint32_t* __restrict__ vis,
                                                         int32_t shift, int32_t nwords,
                                                         uint32_t* __restrict__ summary)
{
    __shared__ uint32_t s_bits[kWG / 64];
    const int32_t P = 1 << (shift - 8);
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    for (int32_t sw = blockIdx.x; sw < nwords; sw += gridDim.x) {
        const int64_t w0 = ((int64_t)sw * kWG + threadIdx.x) * P;
        uint32_t open_any = 0;
        for (int32_t j = 0; j < P; ++j) {
            const int64_t w = w0 + j;
            const uint32_t x = w < W ? vis[w] : 0u;
            const int64_t lo = w * 32;
            uint32_t valid = 0xffffffffu;  // ids at or beyond V count as visited
            if (lo + 32 > V) valid = lo >= V ? 0u : ((1u << (V - lo)) - 1u);
            open_any |= ~x & valid;
        }
        uint32_t grp = open_any ? 1u : 0u;
        grp |= __shfl_xor(grp, 1, 64);
        grp |= __shfl_xor(grp, 2, 64);
        grp |= __shfl_xor(grp, 4, 64);
        const uint64_t full = __ballot(grp == 0);
        // lanes 0, 8, .., 56 hold blocks 8*wave .. 8*wave+7 of this word
        uint32_t bits = 0;
        for (int i = 0; i < 8; ++i) bits |= (uint32_t)((full >> (8 * i)) & 1ull) << i;
        if (lane == 0) s_bits[wave] = bits << (8 * wave);
        __syncthreads();
        if (threadIdx.x == 0) summary[sw] = s_bits[0] | s_bits[1] | s_bits[2] | s_bits[3];
        __syncthreads();
    }
}

// full_prefix = first unvisited id: the first block whose summary bit is
// clear, then the first open bit in that block's words.  One workgroup.
__global__ __launch_bounds__(kWG) void k_visited_prefix(int32_t V, int32_t W,
                                                        const uint32_t* __restrict__ vis,
                                                        int32_t shift, int32_t nwords,
                                                        const uint32_t* __restrict__ summary,
                                                        Ctrl* __restrict__ ctrl)
{
    __shared__ int32_t s_min;
    if (threadIdx.x == 0) {
        s_min = 0x7fffffff;
        ctrl->skipped = 0;  // the degree scan that follows adds its dropped edges
    }
    __syncthreads();
    int32_t first_word = 0x7fffffff;
    for (int32_t i = threadIdx.x; i < nwords; i += kWG)
        if (summary[i] != 0xffffffffu) { first_word = i; break; }
    atomicMin(&s_min, first_word);
    __syncthreads();
    const int32_t sw = s_min;
    __syncthreads();
    if (sw == 0x7fffffff) {
        if (threadIdx.x == 0) ctrl->full_prefix = V;  // everything visited
        return;
    }
    const uint32_t bits = summary[sw];
    const int32_t b = sw * 32 + __builtin_ctz(~bits);  // first non-full block
    const int64_t wlo = ((int64_t)b << shift) >> 5;
    const int64_t whi = (((int64_t)b + 1) << shift) >> 5;
    if (threadIdx.x == 0) s_min = 0x7fffffff;
    __syncthreads();
    for (int64_t w = wlo + threadIdx.x; w < whi; w += kWG) {
        const uint32_t x = w < W ? vis[w] : 0u;
        const int64_t lo = w * 32;
        uint32_t valid = 0xffffffffu;
        if (lo + 32 > V) valid = lo >= V ? 0u : ((1u << (V - lo)) - 1u);
        const uint32_t open = ~x & valid;
        if (open) atomicMin(&s_min, (int32_t)(lo + __builtin_ctz(open)));
    }
    __syncthreads();
    if (threadIdx.x == 0) ctrl->full_prefix = s_min == 0x7fffffff ? V : s_min;
}

hipError_t launch_visited_summary(hipStream_t s, int grid, int32_t V, int32_t W,
                                  const uint32_t* vis, int32_t shift, int32_t nblocks,
                                  uint32_t* summary, Ctrl* ctrl)
{
    const int32_t nwords = (nblocks + 31) / 32;
    if (grid < 1) grid = 1;
    if (grid > nwords) grid = nwords;
    hipLaunchKernelGGL(k_visited_summary, dim3(grid), dim3(kWG), 0, s, V, W, vis, shift, nwords,
                       summary);
    hipLaunchKernelGGL(k_visited_prefix, dim3(1), dim3(kWG), 0, s, V, W, vis, shift, nwords,
                       summary, ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Frontier expansion (Algorithm 3).  Edge slots come from map_tile (the
// cumulative-degree search of Section 3.4, one search per EPT edges).
//
// Vertex ids inside the search may be internal (degree-ordered) ids: level
// and parent are then indexed by internal id (k_finish reorders them) and
// uidv holds each frontier entry's caller id, the parent value.  When
// summary_words > 0, the visited summary of this level is copied into LDS
// and answers the early test before any bitmap load.

template <int EPT>
__global__ __launch_bounds__(kWG) void k_expand(int32_t V, const int64_t* __restrict__ rowstart,
                                                const int32_t* __restrict__ uidv,
                                                const int64_t* __restrict__ cumul,
                                                const int32_t* __restrict__ tile_k,
                                                const int32_t* __restrict__ col,
                                                const uint32_t* __restrict__ summary,
                                                int32_t summary_words, int32_t shift,
                                                int use_prefix,
                                                uint32_t* __restrict__ vis,
                                                uint32_t* __restrict__ vis_old,
                                                int32_t* __restrict__ level,
                                                int32_t* __restrict__ parent, int32_t lvl,
                                                int32_t* __restrict__ Qn,
                                                Ctrl* __restrict__ ctrl,
                                                uint8_t* __restrict__ found, int32_t slice_q)
{
    __shared__ TileLds<EPT> L;
    extern __shared__ uint32_t s_sum[];

    const int64_t r = ctrl->r;
    const int32_t ntiles = ctrl->ntiles;
    const bool list_out = ctrl->bitmap_out == 0;
    // flag claims: a bitmap level marks its vertices with byte stores
    // instead of claiming bits (below)
    const bool flags = found != nullptr && !list_out;
    const int32_t skip_below = use_prefix ? ctrl->full_prefix : 0;
    // XCD-sliced level (slice_q > 0: the scan numbered the edges slice by
    // slice, slice s owning edges [cumul[s * slice_q], cumul[(s + 1) *
    // slice_q])): workgroup b takes slice b mod 8 only, so the XCD it runs
    // on probes one eighth of the bitmap; tiles on a slice boundary are
    // shared by both slices, each taking its own edges
    int32_t t_first = blockIdx.x, t_end = ntiles, t_step = gridDim.x;
    int64_t e_lo = 0, e_hi = r;
    if (slice_q > 0) {
        constexpr int64_t TILE = TileLds<EPT>::TILE;
        const int sl = blockIdx.x & (kXcdSlices - 1);
        e_lo = cumul[(int64_t)sl * slice_q];
        e_hi = cumul[(int64_t)(sl + 1) * slice_q];
        t_step = gridDim.x / kXcdSlices;
        t_first = (int32_t)(e_lo / TILE) + (int32_t)(blockIdx.x / kXcdSlices);
        t_end = (int32_t)((e_hi + TILE - 1) / TILE);
        if (t_end > ntiles) t_end = ntiles;
    }
    if (t_first >= t_end) return;  // whole workgroup: uniform

    StageRegs<EPT> cur = fetch_stage<EPT>(t_first, t_end, cumul, rowstart, uidv, tile_k);
    for (int32_t w = threadIdx.x; w < summary_words; w += kWG) s_sum[w] = summary[w];
    __syncthreads();

    for (int32_t tile = t_first; tile < t_end; tile += t_step) {
        int32_t uu[EPT], vv[EPT];
        bool ok[EPT];
        int64_t ee[EPT];
        map_tile<EPT>(L, cur, r, cumul, rowstart, uidv, col, uu, vv, ok, ee);
        if (slice_q > 0) {
#pragma unroll
            for (int j = 0; j < EPT; ++j) ok[j] = ok[j] && ee[j] >= e_lo && ee[j] < e_hi;
        }

        // Early visited test: summary (register / LDS), else a plain load of
        // the bitmap word (a stale word only lets more threads try the atomic).
        bool known[EPT];
        uint32_t wd[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int32_t v = vv[j];
            known[j] = !ok[j] || v < skip_below;
            if (!known[j] && summary_words > 0) {
                const uint32_t b = (uint32_t)v >> shift;
                known[j] = (s_sum[b >> 5] >> (b & 31)) & 1u;
            }
            if (!known[j]) wd[j] = vis[v >> 5];
        }
        // the next tile's staging loads overlap this tile's probes and claims
        cur = fetch_stage<EPT>(tile + t_step, t_end, cumul, rowstart, uidv, tile_k);
        bool need[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) need[j] = !known[j] && !(wd[j] & (1u << (vv[j] & 31)));
        if (flags) {
            // A bitmap level needs no exactly-once claim: its next frontier is
            // the set of flagged vertices, taken by k_bitmap_to_queue.  A
            // vertex not visited before the level gets its flag byte set
            // (byte stores never disturb neighbouring flags, so no atomic is
            // needed) and a parent from the frontier; when several threads
            // flag it in the same level, each stores a valid parent and one
            // of them remains.  The flag is read first so that most repeat
            // visits store nothing.  Before that, the visited word just read
            // is stored back with the vertex's bit as a hint: later probes
            // of the same XCD (its L2 holds the line) then stop at the
            // visited bit.  The store is a plain one, so two hints to one
            // word may overwrite each other; that only loses hints (the
            // flags are the level's result, and the compaction rebuilds the
            // word from them), never a bit set before the level, which every
            // stored value carries.
            uint8_t fl[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j)
                if (need[j]) vis[vv[j] >> 5] = wd[j] | (1u << (vv[j] & 31));
#pragma unroll
            for (int j = 0; j < EPT; ++j) fl[j] = need[j] ? found[vv[j]] : (uint8_t)1;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                if (!fl[j]) {
                    found[vv[j]] = 1;
                    if (parent) __builtin_nontemporal_store(uu[j], parent + vv[j]);
                }
            }
            __syncthreads();
            continue;
        }
        // claims: issue every atomic before using any result
        uint32_t old[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            if (need[j]) old[j] = atomicOr(vis + (vv[j] >> 5), 1u << (vv[j] & 31));
        bool win[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) win[j] = need[j] && !(old[j] & (1u << (vv[j] & 31)));
        // outputs by search id; in bitmap mode k_bitmap_to_queue writes the
        // level while it walks the new vertices in id order
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (win[j]) {
                if (list_out) level[vv[j]] = lvl;
                // written once per search, read back only at its end
                if (parent) __builtin_nontemporal_store(uu[j], parent + vv[j]);
            }
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
                        atomicOr(vis_old + (v >> 5), 1u << (v & 31));
                    }
                    base += (uint32_t)__popcll(mask[j]);
                }
            }
        }
        __syncthreads();
    }
}

hipError_t launch_expand(hipStream_t s, int ept, int grid, int32_t V, const int64_t* rowstart,
                         const int32_t* uidv, const int64_t* cumul, const int32_t* tile_k,
                         const int32_t* col, const uint32_t* summary,
                         int32_t summary_words, int32_t shift, int use_prefix, uint32_t* vis,
                         uint32_t* vis_old, int32_t* level, int32_t* parent, int32_t lvl,
                         int32_t* Qn, Ctrl* ctrl, uint8_t* found, int32_t slice_q)
{
    if (slice_q > 0) grid = grid / kXcdSlices * kXcdSlices;  // every slice the same workgroups
    if (grid < 1) grid = slice_q > 0 ? kXcdSlices : 1;
    if (summary_words < 0 || summary == nullptr) summary_words = 0;
    const size_t dyn = (size_t)summary_words * 4;
#define BFS_EXPAND_CASE(E)                                                                        \
    case E:                                                                                      \
        hipLaunchKernelGGL(k_expand<E>, dim3(grid), dim3(kWG), dyn, s, V, rowstart, uidv, cumul,  \
                           tile_k, col, summary, summary_words, shift, use_prefix, vis,           \
                           vis_old,                                                              \
                           level, parent,                                                        \
                           lvl, Qn, ctrl, found, slice_q);                                       \
        break;
    switch (ept) {
        BFS_EXPAND_CASE(1)
        BFS_EXPAND_CASE(2)
        BFS_EXPAND_CASE(4)
        BFS_EXPAND_CASE(8)
    default:
        return hipErrorInvalidValue;
    }
#undef BFS_EXPAND_CASE
    return hipGetLastError();
}

int expand_blocks_per_cu(int ept, int summary_words)
{
    int n = 0;
    const size_t dyn = (size_t)(summary_words > 0 ? summary_words : 0) * 4;
    hipError_t e = hipErrorInvalidValue;
    switch (ept) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_expand<1>, kWG, dyn); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_expand<2>, kWG, dyn); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_expand<4>, kWG, dyn); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_expand<8>, kWG, dyn); break;
    default: break;
    }
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

// ---------------------------------------------------------------------------
// Bitmap form of the next frontier: F = vis & ~vis_old (the bits that turned
// on during this level), vis_old := vis, and F compacted in vertex order to
// the next queue, with level[v] = lvl for each v in F.  A workgroup handles
// 256 words (8192 vertices); thread j of pass p looks at vertex p * 256 + j
// of the block, so level stores and queue stores of a wave are contiguous.

__global__ __launch_bounds__(kWG) void k_bitmap_to_queue(int32_t V, int32_t W,
                                                         uint32_t* __restrict__ vis,
                                                         uint32_t* __restrict__ vis_old,
                                                         int32_t* __restrict__ Qn,
                                                         int32_t* __restrict__ level,
                                                         int32_t lvl, Ctrl* __restrict__ ctrl,
                                                         const int64_t* __restrict__ deg_off,
                                                         uint4* __restrict__ found16)
{
    if (!ctrl->bitmap_out) return;
    __shared__ uint32_t s_f[kBitmapWordsPerWG];
    __shared__ uint32_t s_off[kBitmapWordsPerWG];
    __shared__ uint32_t s_wave[kWG / 64];
    __shared__ uint32_t s_base;
    int64_t dsum = 0;  // degrees of the new vertices this thread wrote
    const int64_t nblocks = ((int64_t)W + kBitmapWordsPerWG - 1) / kBitmapWordsPerWG;
    for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const int64_t i = blk * kBitmapWordsPerWG + threadIdx.x;
        uint32_t f = 0;
        if (i < W) {
            uint32_t a = vis[i];
            if (found16) {
                // the level's flag bytes (0 or 1) of this word's 32 ids
                // become bits; the flags are cleared for the next level
                const uint4 x = found16[2 * i], y = found16[2 * i + 1];
                const uint32_t q[8] = {x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
                uint32_t pf = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t z = q[k];
                    pf |= ((z & 1u) | ((z >> 7) & 2u) | ((z >> 14) & 4u) | ((z >> 21) & 8u)) << (4 * k);
                }
                if (pf) {
                    a |= pf;
                    vis[i] = a;
                    found16[2 * i] = make_uint4(0u, 0u, 0u, 0u);
                    found16[2 * i + 1] = make_uint4(0u, 0u, 0u, 0u);
                }
            }
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
                    if (deg_off) dsum += deg_off[v + 1] - deg_off[v];
                }
            }
        }
        __syncthreads();
    }
    if (deg_off) {
        for (int d = 32; d >= 1; d >>= 1) dsum += __shfl_xor(dsum, d, 64);
        if (__lane_id() == 0 && dsum)
            atomicAdd((unsigned long long*)&ctrl->next_deg, (unsigned long long)dsum);
    }
}

hipError_t launch_bitmap_to_queue(hipStream_t s, int grid, int32_t V, int32_t W, uint32_t* vis,
                                  uint32_t* vis_old, int32_t* Qn, int32_t* level, int32_t lvl,
                                  Ctrl* ctrl, const int64_t* deg_off, uint8_t* found)
{
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_bitmap_to_queue, dim3(grid), dim3(kWG), 0, s, V, W, vis, vis_old, Qn,
                       level, lvl, ctrl, deg_off, reinterpret_cast<uint4*>(found));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Degree order: the search keeps level and parent by internal id (the
// winners' and the compaction's stores then stay within the search's own id
// space); one pass at the end writes the caller-ordered outputs: for x =
// rank[c], level[c] = lvl_int[x] and parent[c] = par_int[x] if x is visited,
// else -1 (the internal arrays are only written for visited vertices).  The
// stores are coalesced, and the gathers stay local: the relabelling hands
// each run of 4096 consecutive caller ids one contiguous id range per
// degree bucket.

// A workgroup takes whole 4096-id chunks (the relabelling's unit), so a
// chunk's gathers reuse lines in one CU's caches instead of being spread
// over the XCDs' L2s.
constexpr int kFinishChunk = 4096;

__global__ __launch_bounds__(kWG) void k_finish(int32_t V, const int32_t* __restrict__ rank,
                                                const uint32_t* __restrict__ vis,
                                                const int32_t* __restrict__ lvl_int,
                                                const int32_t* __restrict__ par_int,
                                                int32_t* __restrict__ level,
                                                int32_t* __restrict__ parent, int vec)
{
    constexpr int kPer = kFinishChunk / kWG;  // ids per thread and chunk
    const int64_t nchunks = ((int64_t)V + kFinishChunk - 1) / kFinishChunk;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t c0 = ch * kFinishChunk;
        if (vec && c0 + kFinishChunk <= V) {
            // a whole chunk: thread t owns ids c0 + 4 t + 1024 j + (0..3);
            // every load of the chunk is issued before the first is used
            int4 x[kPer / 4];
#pragma unroll
            for (int j = 0; j < kPer / 4; ++j)
                x[j] = *reinterpret_cast<const int4*>(rank + c0 + j * 4 * kWG + 4 * threadIdx.x);
            uint32_t w[kPer];
#pragma unroll
            for (int j = 0; j < kPer / 4; ++j) {
                w[4 * j + 0] = vis[x[j].x >> 5];
                w[4 * j + 1] = vis[x[j].y >> 5];
                w[4 * j + 2] = vis[x[j].z >> 5];
                w[4 * j + 3] = vis[x[j].w >> 5];
            }
            int32_t l[kPer], p[kPer];
#pragma unroll
            for (int j = 0; j < kPer / 4; ++j) {
                const int32_t xs[4] = {x[j].x, x[j].y, x[j].z, x[j].w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bool on = (w[4 * j + k] >> (xs[k] & 31)) & 1u;
                    l[4 * j + k] = on ? lvl_int[xs[k]] : -1;
                    p[4 * j + k] = (on && parent) ? par_int[xs[k]] : -1;
                }
            }
#pragma unroll
            for (int j = 0; j < kPer / 4; ++j) {
                const int64_t c = c0 + j * 4 * kWG + 4 * threadIdx.x;
                *reinterpret_cast<int4*>(level + c) =
                    make_int4(l[4 * j], l[4 * j + 1], l[4 * j + 2], l[4 * j + 3]);
                if (parent)
                    *reinterpret_cast<int4*>(parent + c) =
                        make_int4(p[4 * j], p[4 * j + 1], p[4 * j + 2], p[4 * j + 3]);
            }
            continue;
        }
#pragma unroll 4
        for (int j = 0; j < kPer; ++j) {
            const int64_t c = c0 + j * kWG + threadIdx.x;
            if (c < V) {
                const int32_t x = rank[c];
                int32_t l = -1, p = -1;
                if ((vis[x >> 5] >> (x & 31)) & 1u) {
                    l = lvl_int[x];
                    if (parent) p = par_int[x];
                }
                level[c] = l;
                if (parent) parent[c] = p;
            }
        }
    }
}

hipError_t launch_finish(hipStream_t s, int grid, int32_t V, const int32_t* rank,
                         const uint32_t* vis, const int32_t* lvl_int, const int32_t* par_int,
                         int32_t* level, int32_t* parent)
{
    const int64_t nchunks = ((int64_t)V + kFinishChunk - 1) / kFinishChunk;
    if (grid > nchunks) grid = (int)nchunks;
    if (grid < 1) grid = 1;
    // 16-byte rank loads and output stores when the caller's arrays allow
    const bool vec = (uintptr_t)rank % 16 == 0 && (uintptr_t)level % 16 == 0 &&
                     (parent == nullptr || (uintptr_t)parent % 16 == 0);
    hipLaunchKernelGGL(k_finish, dim3(grid), dim3(kWG), 0, s, V, rank, vis, lvl_int, par_int,
                       level, parent, vec ? 1 : 0);
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
