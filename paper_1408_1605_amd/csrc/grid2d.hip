// In-GPU 2D blocking: the paper's R x C processor grid (Section 2.2,
// Figure 1; local data structures Section 3.1; Algorithms 2 and 3; the
// frontier update of Section 3.5; list/bitmap messages of Section 5), run by
// R * C virtual processors inside one GPU.
//
// Vertices are split into R*C blocks of B ids (B a multiple of 32).  Virtual
// processor P(i, j) owns vertex block j*R + i and holds the edges (u, v) with
// u in column block j (ids [j*R*B, (j+1)*R*B)) and v in the row blocks
// m*R + i, m = 0..C-1.  Its local indices follow Section 3.1:
//   LOCAL_COL(u) = u - j*R*B                        (its R*B local columns)
//   LOCAL_ROW(v) = (v / B / R) * B + v % B          (its C*B local rows)
//   ROW2COL(r)   = i*B + r % B                      (a row it owns, as a column)
// The processor with index p = j*R + i is the one that owns vertex block p.
//
// One level (Algorithm 2):
//   expand (column exchange)  k2_gather: each column's frontier is the
//       concatenation of the R fronts of its processors; a front travels as a
//       list of local columns or, when longer than its bitmap, as the B-bit
//       bitmap of the owner's block, unpacked by ballot/prefix compaction;
//   expand_frontier           k2_scan_* + k2_expand: per processor, an
//       exclusive scan of the local degrees of the column frontier and the
//       edge -> thread map of Algorithm 3 (EPT = 4, Section 3.4.1); claims in
//       the processor's own bitmap of C*B local rows; each winner is grouped
//       by tgtj = its owner's column, local ones get their level, every winner
//       gets its predecessor;
//   fold (row exchange)       k2_update: each processor receives, from the
//       C-1 others of its grid row, the rows they discovered in its block,
//       each message a list or the sender's bitmap of that block (Section 5);
//       the frontier-update kernel (Section 3.5) claims them in its own
//       bitmap, sets their level and records the sender's column as the
//       predecessor;
//   next front                k2_front: the rows of the owner's block that
//       turned on during the level, kept as a list or as a bitmap.
// At the end k2_finish resolves the predecessors of remotely found vertices
// from the sender's table (the delayed predecessor exchange).
//
// Single-GPU specifics: the exchanges are device-local (the column list is
// gathered once per column and read by its R processors; a receiver reads
// the sender's outgoing list, or the sender's bitmap words, in place), and
// workgroup b of the processor-bound kernels runs on XCD b mod 8 and serves
// only processors p with p mod 8 = b mod 8 (R*C >= 8) or the processor
// (b mod 8) mod R*C (R*C < 8), so each processor's bitmap is probed from one
// XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <new>

#include "runtime.h"
#include "tile_map.h"
#include "wave_ops.h"

namespace bfsmi {
namespace g2 {

constexpr int kMaxP = 64;
constexpr int kEPT = 4;
constexpr int kTile = kWG * kEPT;  // edges per expansion tile
constexpr int kChunk = kScanChunk; // entries per scan block
constexpr int kListUnit = 2048;    // list entries per gather unit
constexpr int kSlots = 8;          // XCDs

// Host-computed description of the grid (fixed) and of the level, copied to
// the device before each level.
struct Plan {
    int32_t V, R, C, RC, B, WB;      // WB = B / 32 bitmap words per block
    int32_t root, pad0;
    int32_t porder[kMaxP];           // processors in slot order
    int32_t ppos[kMaxP];             // position of processor p in porder
    int32_t slot_pos[kSlots + 1];    // slot x holds positions [slot_pos[x], slot_pos[x+1])
    int32_t lvl, msg_mode;
    int32_t nfront[kMaxP];           // front size by processor
    int32_t fform[kMaxP];            // front form: 0 list, 1 bitmap
    int64_t segoff[kMaxP];           // where front p lands in its column's gathered list
    int64_t afb[kMaxP + 1];          // column j's gathered list starts at afb[j]
    int64_t eb[kMaxP + 1];           // entries of porder position t start at eb[t]
    int32_t cb[kMaxP + 1];           // scan blocks of position t start at cb[t]
    int32_t ub[kMaxP + 1];           // gather units of processor p start at ub[p]
};

// Device control block; the head (up to tstart) is read back every level.
struct Ctl {
    int32_t err, total_tiles;
    uint32_t nfront[kMaxP];          // next front size by processor
    int32_t listmode[kMaxP];         // this level's expansion appends lists
    int64_t rp[kMaxP];               // this level's edges by processor
    unsigned long long fold_list_msgs, fold_bitmap_msgs, fold_bytes, fold_vertices, updated;
    int32_t tstart[kMaxP + 1];       // tiles of porder position t: [tstart[t], tstart[t+1])
    int64_t estart[kMaxP + 1];       // edge numbering of position t starts at estart[t]
    uint32_t segcnt[kMaxP];          // gather: reservations in front p's segment
    uint32_t dcnt[kMaxP * kMaxP];    // list lengths by (sender p, destination column m)
};
constexpr size_t kCtlHead = offsetof(Ctl, tstart);

constexpr int kMsgAuto = 0, kMsgList = 1, kMsgBitmap = 2;

// Which processors workgroup blockIdx.x serves (see the file comment): the
// porder positions [first, end) and its index among the nw workgroups that
// share them.
struct SlotWork {
    int32_t first, end, widx, nw;
};

__device__ __forceinline__ SlotWork slot_work(const Plan& pl)
{
    const int32_t x = blockIdx.x % kSlots, k = blockIdx.x / kSlots, K = gridDim.x / kSlots;
    SlotWork s;
    if (pl.RC >= kSlots) {
        s.first = pl.slot_pos[x];
        s.end = pl.slot_pos[x + 1];
        s.widx = k;
        s.nw = K;
    } else {
        const int32_t p = x % pl.RC;
        s.first = pl.ppos[p];
        s.end = s.first + 1;
        s.widx = (x / pl.RC) * K + k;
        s.nw = (kSlots / pl.RC) * K;
    }
    return s;
}

// largest t in [lo, hi) with a[t] <= x (a non-decreasing, a[lo] <= x)
template <typename T>
__device__ __forceinline__ int32_t last_le(const T* a, int32_t lo, int32_t hi, T x)
{
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Partitioning at creation (Section 2.2): each CSR row u is split, stably,
// into R segments by the grid row i = (v / B) % R of its neighbours; segment
// i of row u is column LOCAL_COL(u) of P(i, u / (R*B))'s local matrix, and
// its entries are stored as LOCAL_ROW(v).  off2[u*R + i] is the segment's
// start (the segments of a row are consecutive, so off2 is a CSR over the
// pseudo-rows u*R + i).  One wave per row.

__global__ __launch_bounds__(kWG) void k2_part_count(int32_t V, int64_t nnz, int32_t R, int32_t B,
                                                     const int64_t* __restrict__ off,
                                                     const int32_t* __restrict__ col,
                                                     int64_t* __restrict__ off2)
{
    const int lane = __lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (kWG / 64);
    for (int64_t u = (int64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6); u < V; u += nwaves) {
        const int64_t a = off[u], b = off[u + 1];
        int64_t my = 0;  // lane i < R: neighbours in grid row i
        for (int64_t e0 = a; e0 < b; e0 += 64) {
            const int64_t e = e0 + lane;
            const int32_t gi = e < b ? (col[e] / B) % R : -1;
            for (int32_t i = 0; i < R; ++i) {
                const uint64_t m = __ballot(gi == i);
                if (lane == i) my += __popcll(m);
            }
        }
        const int64_t incl = wave_inclusive_scan<int64_t>(my);
        if (lane < R) off2[u * R + lane] = a + incl - my;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) off2[(int64_t)V * R] = nnz;
}

__global__ __launch_bounds__(kWG) void k2_part_scatter(int32_t V, int32_t R, int32_t B,
                                                       const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ col,
                                                       const int64_t* __restrict__ off2,
                                                       int32_t* __restrict__ lrow)
{
    const int lane = __lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (kWG / 64);
    for (int64_t u = (int64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6); u < V; u += nwaves) {
        const int64_t a = off[u], b = off[u + 1];
        int64_t next = lane < R ? off2[u * R + lane] : 0;  // lane i: next slot of segment i
        for (int64_t e0 = a; e0 < b; e0 += 64) {
            const int64_t e = e0 + lane;
            const int32_t v = e < b ? col[e] : 0;
            const int32_t blk = v / B;
            const int32_t gi = e < b ? blk % R : -1;
            const int32_t lr = (blk / R) * B + (v - blk * B);
            for (int32_t i = 0; i < R; ++i) {
                const uint64_t m = __ballot(gi == i);
                const int64_t base = __shfl(next, i, 64);
                if (gi == i) lrow[base + lanes_below(m)] = lr;
                if (lane == i) next += __popcll(m);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Initialisation (Algorithm 2 lines 1-10): level = -1, bitmaps = 0; the
// owner of the root sets its level, predecessor and visited bit, and its
// front holds ROW2COL of the root.

__global__ __launch_bounds__(kWG) void k2_init(int32_t V, int32_t root, int32_t* __restrict__ level,
                                               uint32_t* __restrict__ bm,
                                               uint32_t* __restrict__ bm_old, int64_t nwords,
                                               int64_t root_word, uint32_t root_bit,
                                               int32_t* __restrict__ pred, int64_t root_pred,
                                               int32_t* __restrict__ dst, int64_t root_slot,
                                               int32_t root_col, Ctl* __restrict__ ctl)
{
    const int64_t stride = (int64_t)gridDim.x * kWG;
    const int64_t tid = (int64_t)blockIdx.x * kWG + threadIdx.x;
    for (int64_t v = tid; v < V; v += stride) level[v] = v == root ? 0 : -1;
    for (int64_t w = tid; w < nwords; w += stride) {
        const uint32_t x = w == root_word ? root_bit : 0u;
        bm[w] = x;
        bm_old[w] = x;
    }
    if (tid == 0) {
        pred[root_pred] = root;
        dst[root_slot] = root_col;
        ctl->err = 0;
        ctl->fold_list_msgs = ctl->fold_bitmap_msgs = ctl->fold_bytes = 0;
        ctl->fold_vertices = ctl->updated = 0;
    }
    if (tid < kMaxP) ctl->segcnt[tid] = 0;
}

// ---------------------------------------------------------------------------
// Expand exchange: column j's list = the R fronts of P(0..R-1, j).  A list
// front is copied; a bitmap front is unpacked (ballot/prefix compaction,
// one reservation per workgroup in the front's segment).

__global__ __launch_bounds__(kWG) void k2_gather(const Plan* __restrict__ plp,
                                                 const int32_t* __restrict__ dst,
                                                 const uint32_t* __restrict__ fbm,
                                                 int32_t* __restrict__ af, Ctl* __restrict__ ctl)
{
    __shared__ uint32_t s_wave[kWG / 64];
    __shared__ uint32_t s_base;
    const Plan& pl = *plp;
    const int32_t R = pl.R, C = pl.C, B = pl.B, WB = pl.WB;
    const int32_t U = pl.ub[pl.RC];
    for (int32_t u = blockIdx.x; u < U; u += gridDim.x) {
        const int32_t p = last_le<int32_t>(pl.ub, 0, pl.RC, u);
        const int32_t k = u - pl.ub[p];
        const int32_t i = p % R, j = p / R;
        const int64_t seg = pl.segoff[p];
        if (pl.fform[p] == 0) {
            const int32_t* src = dst + ((int64_t)p * C + j) * B;
            const int32_t n = pl.nfront[p];
            const int32_t e1 = min(n, (k + 1) * kListUnit);
            for (int32_t e = k * kListUnit + threadIdx.x; e < e1; e += kWG) af[seg + e] = src[e];
        } else {
            const int32_t w = k * kWG + threadIdx.x;
            uint32_t f = w < WB ? fbm[(int64_t)p * WB + w] : 0u;
            uint32_t tot;
            const uint32_t ex = wg_exclusive_scan<uint32_t>((uint32_t)__popc(f), &tot, s_wave);
            if (threadIdx.x == 0) s_base = tot ? atomicAdd(&ctl->segcnt[p], tot) : 0u;
            __syncthreads();
            int64_t at = seg + s_base + ex;
            const int32_t c0 = i * B + w * 32;
            while (f) {
                af[at++] = c0 + __builtin_ctz(f);
                f &= f - 1;
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Degree scan over every processor's column frontier (Section 3.4).  Entry
// k of porder position t is the column-list entry c: its local degree is the
// length of segment i of row u = j*R*B + c, its parent value u.  Each
// processor's edge numbering starts on a tile boundary, so a tile never
// spans two processors.

__global__ __launch_bounds__(kWG) void k2_scan_reduce(const Plan* __restrict__ plp,
                                                      const int32_t* __restrict__ af,
                                                      const int64_t* __restrict__ off2,
                                                      int32_t* __restrict__ deg,
                                                      int64_t* __restrict__ rowstart,
                                                      int32_t* __restrict__ uidv,
                                                      int64_t* __restrict__ bsum)
{
    __shared__ int64_t s_wave[kWG / 64];
    const Plan& pl = *plp;
    const int32_t R = pl.R, RB = pl.R * pl.B;
    const int32_t nch = pl.cb[pl.RC];
    for (int32_t cid = blockIdx.x; cid < nch; cid += gridDim.x) {
        const int32_t t = last_le<int32_t>(pl.cb, 0, pl.RC, cid);
        const int32_t p = pl.porder[t];
        const int32_t i = p % R, j = p / R;
        const int64_t colbase = pl.afb[j];
        const int64_t n = pl.afb[j + 1] - colbase;
        const int64_t l0 = (int64_t)(cid - pl.cb[t]) * kChunk;
        int64_t sum = 0;
#pragma unroll
        for (int jj = 0; jj < kScanItems; ++jj) {
            const int64_t kl = l0 + jj * kWG + threadIdx.x;
            if (kl < n) {
                const int32_t u = j * RB + af[colbase + kl];
                const int64_t pr = (int64_t)u * R + i;
                const int64_t a = off2[pr];
                const int64_t d = off2[pr + 1] - a;
                const int64_t k = pl.eb[t] + kl;
                deg[k] = (int32_t)d;
                rowstart[k] = a;
                uidv[k] = u;
                sum += d;
            }
        }
        int64_t tot;
        wg_exclusive_scan<int64_t>(sum, &tot, s_wave);
        if (threadIdx.x == 0) bsum[cid] = tot;
    }
}

// One workgroup: block sums -> block starts, processor by processor, each
// processor's numbering rounded up to a whole tile; per-processor edge
// counts and list modes; counters of the level cleared.
__global__ __launch_bounds__(kWG) void k2_scan_top(const Plan* __restrict__ plp,
                                                   int64_t* __restrict__ bsum,
                                                   int64_t* __restrict__ cumul,
                                                   int32_t* __restrict__ tile_k, int64_t tile_cap,
                                                   Ctl* __restrict__ ctl)
{
    __shared__ int64_t s_wave[kWG / 64];
    const Plan& pl = *plp;
    const int64_t list_limit = (int64_t)pl.C * pl.WB;  // words of the processor's bitmap
    int64_t run = 0;
    for (int32_t t = 0; t < pl.RC; ++t) {
        const int64_t start = run;
        int64_t carry = start;
        for (int32_t b0 = pl.cb[t]; b0 < pl.cb[t + 1]; b0 += kWG) {
            const int32_t b = b0 + threadIdx.x;
            const int64_t x = b < pl.cb[t + 1] ? bsum[b] : 0;
            int64_t tot;
            const int64_t ex = wg_exclusive_scan<int64_t>(x, &tot, s_wave);
            if (b < pl.cb[t + 1]) bsum[b] = carry + ex;
            carry += tot;
        }
        const int64_t rp = carry - start;
        run = start + (rp + kTile - 1) / kTile * kTile;
        if (threadIdx.x == 0) {
            const int32_t p = pl.porder[t];
            ctl->estart[t] = start;
            ctl->tstart[t] = (int32_t)(start / kTile);
            ctl->rp[p] = rp;
            ctl->listmode[p] = pl.msg_mode == kMsgList ? 1
                             : pl.msg_mode == kMsgBitmap ? 0 : (rp <= list_limit ? 1 : 0);
        }
    }
    if (threadIdx.x == 0) {
        int64_t nt = run / kTile;
        if (nt > tile_cap) {  // more edges than the graph holds: refuse
            ctl->err = 1;
            nt = 0;
        }
        ctl->estart[pl.RC] = run;
        ctl->tstart[pl.RC] = (int32_t)nt;
        ctl->total_tiles = (int32_t)nt;
        const int64_t ne = pl.eb[pl.RC];
        cumul[ne] = run;
        tile_k[nt] = ne > 0 ? (int32_t)(ne - 1) : 0;
    }
    for (int32_t x = threadIdx.x; x < pl.RC * pl.C; x += kWG) ctl->dcnt[x] = 0;
    if (threadIdx.x < kMaxP) {
        ctl->nfront[threadIdx.x] = 0;
        ctl->segcnt[threadIdx.x] = 0;
    }
}

__global__ __launch_bounds__(kWG) void k2_scan_down(const Plan* __restrict__ plp,
                                                    const int32_t* __restrict__ deg,
                                                    const int64_t* __restrict__ bsum,
                                                    int64_t tile_cap, int64_t* __restrict__ cumul,
                                                    int32_t* __restrict__ tile_k)
{
    __shared__ int64_t s_wave[kWG / 64];
    __shared__ int32_t s_deg[kChunk + kChunk / kScanItems];
    __shared__ int64_t s_cum[kChunk];
    const Plan& pl = *plp;
    const int32_t nch = pl.cb[pl.RC];
    for (int32_t cid = blockIdx.x; cid < nch; cid += gridDim.x) {
        const int32_t t = last_le<int32_t>(pl.cb, 0, pl.RC, cid);
        const int64_t k0 = pl.eb[t] + (int64_t)(cid - pl.cb[t]) * kChunk;
        const int64_t kend = pl.eb[t + 1];
#pragma unroll
        for (int jj = 0; jj < kScanItems; ++jj) {
            const int32_t li = jj * kWG + threadIdx.x;
            const int64_t k = k0 + li;
            s_deg[li + li / kScanItems] = k < kend ? deg[k] : 0;
        }
        __syncthreads();
        int64_t local[kScanItems];
        int64_t sum = 0;
#pragma unroll
        for (int jj = 0; jj < kScanItems; ++jj) {
            const int32_t li = threadIdx.x * kScanItems + jj;
            local[jj] = sum;
            sum += s_deg[li + li / kScanItems];
        }
        int64_t tot;
        const int64_t ex = wg_exclusive_scan<int64_t>(sum, &tot, s_wave);
        const int64_t start = bsum[cid] + ex;
#pragma unroll
        for (int jj = 0; jj < kScanItems; ++jj) {
            const int32_t li = threadIdx.x * kScanItems + jj;
            const int64_t k = k0 + li;
            const int64_t c = start + local[jj];
            s_cum[li] = c;
            if (k < kend) {
                const int32_t d = s_deg[li + li / kScanItems];
                if (d > 0) {
                    const int64_t t0 = (c + kTile - 1) / kTile;
                    int64_t t1 = (c + d - 1) / kTile;
                    if (t1 >= tile_cap) t1 = tile_cap - 1;
                    for (int64_t tt = t0; tt <= t1; ++tt) tile_k[tt] = (int32_t)k;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < kScanItems; ++jj) {
            const int32_t li = jj * kWG + threadIdx.x;
            if (k0 + li < kend) cumul[k0 + li] = s_cum[li];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Frontier expansion of every processor (Algorithm 3): plain-read probe of
// the processor's bitmap, atomicOr claim, tgtj = LOCAL_ROW / B; a winner's
// predecessor is set, its level too when the processor owns it.  In list
// mode winners are appended to the processor's outgoing list for column
// tgtj (own rows as ROW2COL, forming the processor's next front), one LDS
// counter per column and one global reservation per column and tile.

__global__ __launch_bounds__(kWG) void k2_expand(const Plan* __restrict__ plp,
                                                 Ctl* __restrict__ ctl,
                                                 const int64_t* __restrict__ rowstart,
                                                 const int32_t* __restrict__ uidv,
                                                 const int64_t* __restrict__ cumul,
                                                 const int32_t* __restrict__ tile_k,
                                                 const int32_t* __restrict__ lrow,
                                                 uint32_t* __restrict__ bm,
                                                 int32_t* __restrict__ pred,
                                                 int32_t* __restrict__ dst,
                                                 int32_t* __restrict__ level)
{
    constexpr int EPT = kEPT;
    __shared__ TileLds<EPT> L;
    __shared__ int32_t s_tstart[kMaxP + 1];
    __shared__ int64_t s_rend[kMaxP];
    __shared__ uint32_t s_cnt[kMaxP];
    __shared__ uint32_t s_base[kMaxP];
    const Plan& pl = *plp;
    const int32_t R = pl.R, C = pl.C, B = pl.B, WB = pl.WB, lvl = pl.lvl;
    const SlotWork sw = slot_work(pl);
    if (threadIdx.x <= pl.RC) s_tstart[threadIdx.x] = ctl->tstart[threadIdx.x];
    if (threadIdx.x < pl.RC)
        s_rend[threadIdx.x] = ctl->estart[threadIdx.x] + ctl->rp[pl.porder[threadIdx.x]];
    __syncthreads();
    const int32_t A = s_tstart[sw.first], E = s_tstart[sw.end];
    int32_t tile = A + sw.widx;
    if (tile >= E) return;  // uniform over the workgroup
    StageRegs<EPT> cur = fetch_stage<EPT>(tile, E, cumul, rowstart, uidv, tile_k);
    for (; tile < E; tile += sw.nw) {
        const int32_t t = last_le<int32_t>(s_tstart, sw.first, sw.end, tile);
        const int32_t p = pl.porder[t];
        const int32_t i = p % R, j = p / R;
        const bool list = ctl->listmode[p] != 0;
        uint32_t* bmp = bm + (int64_t)p * C * WB;
        int32_t* prp = pred + (int64_t)p * C * B;
        if (threadIdx.x < C) s_cnt[threadIdx.x] = 0;
        int32_t uu[EPT], vv[EPT];
        bool ok[EPT];
        int64_t ee[EPT];
        map_tile<EPT>(L, cur, s_rend[t], cumul, rowstart, uidv, lrow, uu, vv, ok, ee);
        uint32_t wd[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) wd[q] = ok[q] ? bmp[vv[q] >> 5] : 0xffffffffu;
        cur = fetch_stage<EPT>(tile + sw.nw, E, cumul, rowstart, uidv, tile_k);
        bool need[EPT];
        uint32_t old[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            need[q] = ok[q] && !(wd[q] & (1u << (vv[q] & 31)));
            if (need[q]) old[q] = atomicOr(bmp + (vv[q] >> 5), 1u << (vv[q] & 31));
        }
        int32_t tg[EPT];
        uint32_t slot[EPT];
        bool win[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            win[q] = need[q] && !(old[q] & (1u << (vv[q] & 31)));
            tg[q] = win[q] ? vv[q] / B : 0;
            if (win[q]) {
                prp[vv[q]] = uu[q];
                if (tg[q] == j) level[(int64_t)(j * R + i) * B + (vv[q] - j * B)] = lvl;
                if (list) slot[q] = atomicAdd(&s_cnt[tg[q]], 1u);
            }
        }
        __syncthreads();
        if (list) {
            if (threadIdx.x < C) {
                const uint32_t n = s_cnt[threadIdx.x];
                s_base[threadIdx.x] = n ? atomicAdd(&ctl->dcnt[p * C + threadIdx.x], n) : 0u;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                if (win[q]) {
                    const uint32_t pos = s_base[tg[q]] + slot[q];
                    const int32_t val = tg[q] == j ? i * B + (vv[q] - j * B) : vv[q];
                    if (pos < (uint32_t)B) dst[((int64_t)p * C + tg[q]) * B + pos] = val;
                    else ctl->err = 2;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Fold exchange and frontier update (Section 3.5): receiver P(i, m) takes
// the rows the other processors of grid row i found in its block m.  A
// message is the sender's list when the sender kept one and it is not
// longer than the block's bitmap (Section 5), else the sender's bitmap words
// of block m that turned on this level.  An unvisited received row is
// claimed with atomicOr in the receiver's bitmap (a bitmap message claims a
// whole word at once: sender and receiver number the block's rows alike);
// the winner sets its level, records the sender's column as its predecessor
// (-2 - column) and, in list mode, appends it to the receiver's next front
// (one reservation per wave).

__device__ __forceinline__ bool fold_is_list(const Plan& pl, const Ctl* ctl, int32_t p, int32_t m)
{
    if (!ctl->listmode[p]) return false;  // the sender kept no lists
    if (pl.msg_mode == kMsgList) return true;
    return ctl->dcnt[p * pl.C + m] <= (uint32_t)pl.WB;
}

__global__ __launch_bounds__(kWG) void k2_update(const Plan* __restrict__ plp,
                                                 Ctl* __restrict__ ctl,
                                                 uint32_t* __restrict__ bm,
                                                 const uint32_t* __restrict__ bm_old,
                                                 int32_t* __restrict__ pred,
                                                 int32_t* __restrict__ dst,
                                                 int32_t* __restrict__ level)
{
    const Plan& pl = *plp;
    const int32_t R = pl.R, C = pl.C, B = pl.B, WB = pl.WB, lvl = pl.lvl;
    const SlotWork sw = slot_work(pl);
    const int64_t pw = (int64_t)C * WB;  // bitmap words per processor
    const int64_t step = (int64_t)sw.nw * kWG;
    uint32_t accepted = 0, carried = 0;
    for (int32_t t = sw.first; t < sw.end; ++t) {
        const int32_t q = pl.porder[t];
        const int32_t i = q % R, m = q / R;
        uint32_t* bmq = bm + (int64_t)q * pw;
        int32_t* prq = pred + (int64_t)q * C * B;
        const bool qlist = ctl->listmode[q] != 0;
        int32_t* qfront = dst + ((int64_t)q * C + m) * B;
        uint32_t* qcnt = &ctl->dcnt[q * C + m];
        const int64_t vbase = (int64_t)(m * R + i) * B - (int64_t)m * B;  // v = vbase + r
        const int32_t cbase = i * B - m * B;                              // ROW2COL(r) = cbase + r
        for (int32_t jj = 0; jj < C; ++jj) {
            if (jj == m) continue;
            const int32_t p = jj * R + i;
            if (fold_is_list(pl, ctl, p, m)) {
                // list message: one row per thread, one claim each; the
                // workgroup walks the list in uniform steps so a wave's
                // winners append with one reservation
                const int64_t n = ctl->dcnt[p * C + m];
                const int32_t* src = dst + ((int64_t)p * C + m) * B;
                for (int64_t e0 = (int64_t)sw.widx * kWG; e0 < n; e0 += step) {
                    const int64_t e = e0 + threadIdx.x;
                    bool win = false;
                    int32_t r = 0;
                    if (e < n) {
                        r = src[e];
                        const uint32_t bit = 1u << (r & 31);
                        if (!(bmq[r >> 5] & bit)) win = !(atomicOr(bmq + (r >> 5), bit) & bit);
                    }
                    if (win) {
                        level[vbase + r] = lvl;
                        prq[r] = -2 - jj;
                        accepted++;
                    }
                    if (qlist) {
                        const uint64_t mask = __ballot(win);
                        uint32_t base = 0;
                        if (__lane_id() == 0 && mask) base = atomicAdd(qcnt, (uint32_t)__popcll(mask));
                        base = __shfl(base, 0, 64);
                        if (win) {
                            const uint32_t pos = base + lanes_below(mask);
                            if (pos < (uint32_t)B) qfront[pos] = cbase + r;
                            else ctl->err = 3;
                        }
                    }
                }
            } else {
                // bitmap message: the sender's words of block m that turned on
                // this level; sender and receiver number the block's rows the
                // same way, so a word is claimed with one atomicOr
                const uint32_t* a = bm + (int64_t)p * pw + (int64_t)m * WB;
                const uint32_t* b = bm_old + (int64_t)p * pw + (int64_t)m * WB;
                uint32_t* rq = bmq + (int64_t)m * WB;
                for (int64_t w0 = (int64_t)sw.widx * kWG; w0 < WB; w0 += step) {
                    const int64_t w = w0 + threadIdx.x;
                    uint32_t got = 0;
                    if (w < WB) {
                        const uint32_t f = a[w] & ~b[w];
                        carried += __popc(f);
                        const uint32_t open = f & ~rq[w];
                        if (open) got = open & ~atomicOr(rq + w, open);
                    }
                    const uint32_t ng = (uint32_t)__popc(got);
                    accepted += ng;
                    uint32_t at = 0;
                    if (qlist) {
                        // wave-wide prefix of the new rows, one reservation per wave
                        const uint32_t incl = wave_inclusive_scan<uint32_t>(ng);
                        uint32_t base = 0;
                        const uint32_t tot = __shfl(incl, 63, 64);
                        if (__lane_id() == 63 && tot) base = atomicAdd(qcnt, tot);
                        at = __shfl(base, 63, 64) + incl - ng;
                    }
                    const int32_t r0 = m * B + (int32_t)w * 32;
                    while (got) {
                        const int32_t r = r0 + __builtin_ctz(got);
                        got &= got - 1;
                        level[vbase + r] = lvl;
                        prq[r] = -2 - jj;
                        if (qlist) {
                            if (at < (uint32_t)B) qfront[at] = cbase + r;
                            else ctl->err = 3;
                            at++;
                        }
                    }
                }
            }
        }
    }
    // one counter update per wave
    for (int d = 32; d >= 1; d >>= 1) {
        accepted += __shfl_xor(accepted, d, 64);
        carried += __shfl_xor(carried, d, 64);
    }
    if (__lane_id() == 0) {
        if (accepted) atomicAdd(&ctl->updated, (unsigned long long)accepted);
        if (carried) atomicAdd(&ctl->fold_vertices, (unsigned long long)carried);
    }
}

// ---------------------------------------------------------------------------
// Next front: the rows of the owner's block that turned on during the level
// (its own expansion's and the update's), kept as a B-bit bitmap (fbm) and
// counted; every processor's bitmap is then copied to bm_old, which makes
// the next level's bitmap messages the bits found during that level.
// Workgroup 0 also adds up this level's fold messages and their bytes.

__global__ __launch_bounds__(kWG) void k2_front(const Plan* __restrict__ plp,
                                                Ctl* __restrict__ ctl,
                                                const uint32_t* __restrict__ bm,
                                                uint32_t* __restrict__ bm_old,
                                                uint32_t* __restrict__ fbm)
{
    const Plan& pl = *plp;
    const int32_t R = pl.R, C = pl.C, WB = pl.WB;
    const SlotWork sw = slot_work(pl);
    const int64_t pw = (int64_t)C * WB;
    for (int32_t t = sw.first; t < sw.end; ++t) {
        const int32_t q = pl.porder[t];
        const int32_t m = q / R;
        const uint32_t* a = bm + (int64_t)q * pw;
        uint32_t* b = bm_old + (int64_t)q * pw;
        uint32_t cnt = 0;
        for (int64_t w = (int64_t)sw.widx * kWG + threadIdx.x; w < pw; w += (int64_t)sw.nw * kWG) {
            const uint32_t x = a[w], y = b[w];
            if (w >= (int64_t)m * WB && w < (int64_t)(m + 1) * WB) {
                const uint32_t f = x & ~y;
                fbm[(int64_t)q * WB + (w - (int64_t)m * WB)] = f;
                cnt += __popc(f);
            }
            if (x != y) b[w] = x;
        }
        for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
        if (__lane_id() == 0 && cnt) atomicAdd(&ctl->nfront[q], cnt);
    }
    if (blockIdx.x == 0 && C > 1) {
        unsigned long long nl = 0, nb = 0, bytes = 0;
        for (int32_t x = threadIdx.x; x < pl.RC * C; x += kWG) {
            const int32_t p = x / C, m = x % C;
            if (m == p / R) continue;
            if (fold_is_list(pl, ctl, p, m)) {
                nl++;
                bytes += 4ull * ctl->dcnt[x];
            } else {
                nb++;
                bytes += 4ull * WB;
            }
        }
        for (int d = 32; d >= 1; d >>= 1) {
            nl += __shfl_xor(nl, d, 64);
            nb += __shfl_xor(nb, d, 64);
            bytes += __shfl_xor(bytes, d, 64);
        }
        if (__lane_id() == 0) {
            if (nl) atomicAdd(&ctl->fold_list_msgs, nl);
            if (nb) atomicAdd(&ctl->fold_bitmap_msgs, nb);
            if (bytes) atomicAdd(&ctl->fold_bytes, bytes);
        }
    }
}

// ---------------------------------------------------------------------------
// Predecessors: a vertex found by its owner's expansion has its source in
// the owner's table; one received in the fold has the sender's column there,
// and the source in the sender's table at the same local row.

__global__ __launch_bounds__(kWG) void k2_finish(int32_t V, int32_t R, int32_t C, int32_t B,
                                                 int32_t root, const int32_t* __restrict__ level,
                                                 const int32_t* __restrict__ pred,
                                                 int32_t* __restrict__ parent)
{
    const int64_t stride = (int64_t)gridDim.x * kWG;
    const int64_t pstride = (int64_t)C * B;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < V; v += stride) {
        int32_t out = -1;
        if (v == root) {
            out = root;
        } else if (level[v] > 0) {
            const int32_t blk = (int32_t)(v / B);
            const int32_t i = blk % R, m = blk / R;
            const int32_t r = m * B + (int32_t)(v - (int64_t)blk * B);
            const int32_t x = pred[(int64_t)(m * R + i) * pstride + r];
            out = x >= 0 ? x : pred[(int64_t)((-2 - x) * R + i) * pstride + r];
        }
        parent[v] = out;
    }
}

int expand_occupancy()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k2_expand, kWG, 0) != hipSuccess || n < 1)
        n = 1;
    return n;
}

}  // namespace g2
}  // namespace bfsmi

using namespace bfsmi;
using namespace bfsmi::g2;

struct bfs_grid2d {
    int32_t V = 0, R = 1, C = 1, RC = 1, B = 32, WB = 1;
    int64_t nnz = 0;
    int device = 0;
    int num_cus = 256;
    int expand_grid = 0, slot_grid = 0;
    int64_t tile_cap = 0;
    char* ws = nullptr;
    int64_t* off2 = nullptr;
    int32_t* lrow = nullptr;
    uint32_t* bm = nullptr;
    uint32_t* bm_old = nullptr;
    int32_t* pred = nullptr;
    int32_t* dst = nullptr;
    uint32_t* fbm = nullptr;
    int32_t* af = nullptr;
    int32_t* deg = nullptr;
    int64_t* rowstart = nullptr;
    int32_t* uidv = nullptr;
    int64_t* cumul = nullptr;
    int64_t* bsum = nullptr;
    int32_t* tile_k = nullptr;
    Ctl* ctl = nullptr;
    Plan* plan = nullptr;    // device copy
    Plan* h_plan = nullptr;  // pinned host
    Ctl* h_ctl = nullptr;    // pinned host (head only is read back)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::atomic<int> busy{0};
};

namespace {

struct Layout2 {
    size_t off2, lrow, bm, bm_old, pred, dst, fbm, af, deg, rowstart, uidv, cumul, bsum, tile_k,
        ctl, plan, total;
};

bool grid_ok(int32_t R, int32_t C)
{
    if (R < 1 || C < 1) return false;
    const int64_t rc = (int64_t)R * C;
    if (rc > kMaxP) return false;
    return rc == 1 || rc == 2 || rc == 4 || rc % kSlots == 0;
}

int32_t block_size(int32_t V, int32_t RC)
{
    const int64_t b = ((int64_t)V + RC - 1) / RC;
    return (int32_t)((b + 31) / 32 * 32);
}

Layout2 layout2(int32_t V, int64_t nnz, int32_t R, int32_t C)
{
    Layout2 L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p = (p + bytes + 255) / 256 * 256;
        return at;
    };
    const int64_t RC = (int64_t)R * C;
    const int64_t B = block_size(V, (int32_t)RC);
    const int64_t Np = RC * B;                 // padded vertex count
    const int64_t words = RC * C * (B / 32);   // all processors' bitmaps
    const int64_t entries = (int64_t)R * Np;   // column lists, replicated R times at most
    const int64_t chunks = entries / kChunk + RC + 1;
    const int64_t tiles = (nnz + kTile - 1) / kTile + RC + 2;
    L.off2 = take(((size_t)V * R + 1) * 8);
    L.lrow = take((size_t)std::max<int64_t>(nnz, 1) * 4);
    L.bm = take((size_t)words * 4);
    L.bm_old = take((size_t)words * 4);
    L.pred = take((size_t)RC * C * B * 4);
    L.dst = take((size_t)RC * C * B * 4);
    L.fbm = take((size_t)RC * (B / 32) * 4);
    L.af = take((size_t)Np * 4);
    L.deg = take((size_t)entries * 4);
    L.rowstart = take((size_t)entries * 8);
    L.uidv = take((size_t)entries * 4);
    L.cumul = take((size_t)(entries + 1) * 8);
    L.bsum = take((size_t)chunks * 8);
    L.tile_k = take((size_t)tiles * 4);
    L.ctl = take(sizeof(Ctl));
    L.plan = take(sizeof(Plan));
    L.total = p;
    return L;
}

struct Busy2 {
    bfs_grid2d* g;
    bool held = false;
    explicit Busy2(bfs_grid2d* gg) : g(gg)
    {
        int e = 0;
        held = g->busy.compare_exchange_strong(e, 1);
    }
    ~Busy2()
    {
        if (held) g->busy.store(0);
    }
};

struct Dev2 {
    int prev = -1;
    explicit Dev2(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~Dev2()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int run2d(bfs_grid2d* g, int32_t root, int32_t msg_mode, int32_t* levels, int32_t* parents,
          hipStream_t s, bfs_grid2d_stats* st)
{
    Plan& P = *g->h_plan;
    const int32_t R = g->R, C = g->C, RC = g->RC, B = g->B, WB = g->WB;
    const int64_t pw = (int64_t)C * WB;
    P.msg_mode = msg_mode;
    P.root = root;

    // the root's owner, local row and column
    const int32_t rblk = root / B;
    const int32_t ri = rblk % R, rm = rblk / R;
    const int32_t rq = rm * R + ri;
    const int32_t rrow = rm * B + (root - rblk * B);
    const int32_t rcol = ri * B + (root - rblk * B);
    BFS_HIP_TRY(hipEventRecord(g->ev0, s));
    {
        const int64_t work = std::max<int64_t>(g->V, (int64_t)RC * pw);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((work + kWG - 1) / kWG,
                                                                      (int64_t)g->num_cus * 8));
        hipLaunchKernelGGL(k2_init, dim3(grid), dim3(kWG), 0, s, g->V, root, levels, g->bm,
                           g->bm_old, (int64_t)RC * pw, (int64_t)rq * pw + (rrow >> 5),
                           1u << (rrow & 31), g->pred, (int64_t)rq * C * B + rrow, g->dst,
                           ((int64_t)rq * C + rm) * B, rcol, g->ctl);
        BFS_HIP_TRY(hipGetLastError());
    }
    for (int p = 0; p < RC; ++p) {
        P.nfront[p] = p == rq ? 1 : 0;
        P.fform[p] = 0;
    }
    bfs_grid2d_stats acc{};
    int64_t reached = 1, edges = 0;
    int32_t nlevels = 1;
    int32_t lvl = 1;
    const int cap = g->num_cus * 8;
    while (true) {
        // column lists and the scan's entry / block / gather-unit tables
        int64_t ncol[kMaxP] = {0};
        int64_t total = 0;
        for (int p = 0; p < RC; ++p) {
            ncol[p / R] += P.nfront[p];
            total += P.nfront[p];
        }
        if (total == 0) break;
        P.afb[0] = 0;
        for (int j = 0; j < C; ++j) {
            P.afb[j + 1] = P.afb[j] + ncol[j];
            int64_t at = P.afb[j];
            for (int i = 0; i < R; ++i) {
                P.segoff[j * R + i] = at;
                at += P.nfront[j * R + i];
            }
        }
        P.eb[0] = 0;
        P.cb[0] = 0;
        for (int t = 0; t < RC; ++t) {
            const int64_t n = ncol[P.porder[t] / R];
            P.eb[t + 1] = P.eb[t] + n;
            P.cb[t + 1] = P.cb[t] + (int32_t)((n + kChunk - 1) / kChunk);
        }
        P.ub[0] = 0;
        for (int p = 0; p < RC; ++p) {
            int32_t units = 0;
            if (P.nfront[p] > 0)
                units = P.fform[p] ? (WB + kWG - 1) / kWG : (P.nfront[p] + kListUnit - 1) / kListUnit;
            P.ub[p + 1] = P.ub[p] + units;
            if (R > 1) {  // the front goes to the R - 1 other processors of its column
                acc.expand_list_msgs += P.fform[p] ? 0 : R - 1;
                acc.expand_bitmap_msgs += P.fform[p] ? R - 1 : 0;
                acc.expand_bytes += (int64_t)(R - 1) * (P.fform[p] ? 4ll * WB : 4ll * P.nfront[p]);
                acc.expand_list_only_bytes += (int64_t)(R - 1) * 4 * P.nfront[p];
            }
        }
        P.lvl = lvl;
        BFS_HIP_TRY(hipMemcpyAsync(g->plan, g->h_plan, sizeof(Plan), hipMemcpyHostToDevice, s));
        if (P.ub[RC] > 0)
            hipLaunchKernelGGL(k2_gather, dim3(std::min(P.ub[RC], cap)), dim3(kWG), 0, s, g->plan,
                               g->dst, g->fbm, g->af, g->ctl);
        const int32_t nch = P.cb[RC];
        if (nch > 0)
            hipLaunchKernelGGL(k2_scan_reduce, dim3(std::min(nch, cap)), dim3(kWG), 0, s, g->plan,
                               g->af, g->off2, g->deg, g->rowstart, g->uidv, g->bsum);
        hipLaunchKernelGGL(k2_scan_top, dim3(1), dim3(kWG), 0, s, g->plan, g->bsum, g->cumul,
                           g->tile_k, g->tile_cap, g->ctl);
        if (nch > 0)
            hipLaunchKernelGGL(k2_scan_down, dim3(std::min(nch, cap)), dim3(kWG), 0, s, g->plan,
                               g->deg, g->bsum, g->tile_cap, g->cumul, g->tile_k);
        hipLaunchKernelGGL(k2_expand, dim3(g->expand_grid), dim3(kWG), 0, s, g->plan, g->ctl,
                           g->rowstart, g->uidv, g->cumul, g->tile_k, g->lrow, g->bm, g->pred,
                           g->dst, levels);
        if (C > 1)
            hipLaunchKernelGGL(k2_update, dim3(g->slot_grid), dim3(kWG), 0, s, g->plan, g->ctl,
                               g->bm, g->bm_old, g->pred, g->dst, levels);
        hipLaunchKernelGGL(k2_front, dim3(g->slot_grid), dim3(kWG), 0, s, g->plan, g->ctl, g->bm,
                           g->bm_old, g->fbm);
        BFS_HIP_TRY(hipGetLastError());
        BFS_HIP_TRY(hipMemcpyAsync(g->h_ctl, g->ctl, kCtlHead, hipMemcpyDeviceToHost, s));
        BFS_HIP_TRY(hipStreamSynchronize(s));
        const Ctl& c = *g->h_ctl;
        if (c.err) return fail(BFS_ERR_HIP, "internal guard tripped in the 2D search (code %d)", c.err);
        int64_t found = 0;
        for (int p = 0; p < RC; ++p) {
            edges += c.rp[p];
            found += c.nfront[p];
            P.nfront[p] = (int32_t)c.nfront[p];
            const bool keep_list = c.listmode[p] && (msg_mode == kMsgList || c.nfront[p] <= (uint32_t)WB);
            P.fform[p] = keep_list ? 0 : 1;
            acc.list_levels += c.listmode[p] ? 1 : 0;
        }
        if (found == 0) break;
        reached += found;
        nlevels++;
        lvl++;
    }
    if (parents) {
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((g->V + kWG - 1) / kWG, cap));
        hipLaunchKernelGGL(k2_finish, dim3(grid), dim3(kWG), 0, s, g->V, R, C, B, root, levels,
                           g->pred, parents);
        BFS_HIP_TRY(hipGetLastError());
    }
    BFS_HIP_TRY(hipEventRecord(g->ev1, s));
    BFS_HIP_TRY(hipEventSynchronize(g->ev1));
    if (st) {
        const Ctl& c = *g->h_ctl;  // the last level's read-back holds the totals
        *st = acc;
        st->levels = nlevels;
        st->reached = reached;
        st->edges_scanned = edges;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g->ev0, g->ev1) != hipSuccess) ms = 0.f;
        st->device_ms = ms;
        st->fold_list_msgs = (int64_t)c.fold_list_msgs;
        st->fold_bitmap_msgs = (int64_t)c.fold_bitmap_msgs;
        st->fold_bytes = (int64_t)c.fold_bytes;
        st->updated = (int64_t)c.updated;
        // as lists only: the list messages as sent, plus one word per row
        // that a bitmap message carried
        st->fold_list_only_bytes = st->fold_bytes -
                                   4 * (int64_t)WB * (int64_t)c.fold_bitmap_msgs +
                                   4 * (int64_t)c.fold_vertices;
    }
    return ok();
}

}  // namespace

extern "C" {

int bfs_grid2d_workspace_bytes(int32_t V, int64_t nnz, int32_t R, int32_t C, size_t* bytes)
{
    if (!bytes) return fail(BFS_ERR_INVALID, "bytes is NULL");
    if (V < 1) return fail(BFS_ERR_INVALID, "V must be >= 1 (got %d)", V);
    if (nnz < 0 || nnz > ((int64_t)1 << 40)) return fail(BFS_ERR_INVALID, "nnz out of range");
    if (!grid_ok(R, C))
        return fail(BFS_ERR_INVALID, "R * C must be 1, 2, 4 or a multiple of 8 up to 64 (got %d x %d)",
                    R, C);
    *bytes = layout2(V, nnz, R, C).total;
    return ok();
}

int bfs_grid2d_create(bfs_grid2d** out, int32_t V, int64_t nnz, const int64_t* d_row_offsets,
                      const int32_t* d_col, int32_t R, int32_t C, void* d_workspace,
                      size_t ws_bytes, void* hip_stream)
{
    if (!out) return fail(BFS_ERR_INVALID, "out-pointer is NULL");
    *out = nullptr;
    size_t need = 0;
    const int rc = bfs_grid2d_workspace_bytes(V, nnz, R, C, &need);
    if (rc != BFS_OK) return rc;
    if (!d_row_offsets) return fail(BFS_ERR_INVALID, "row offsets pointer is NULL");
    if (!d_col && nnz > 0) return fail(BFS_ERR_INVALID, "column pointer is NULL");
    if (!d_workspace) return fail(BFS_ERR_INVALID, "workspace pointer is NULL");
    if ((uintptr_t)d_workspace % 256 != 0) return fail(BFS_ERR_INVALID, "workspace not 256-byte aligned");
    if (ws_bytes < need) return fail(BFS_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(BFS_ERR_NO_DEVICE, "no HIP device");
    int dev = 0;
    BFS_HIP_TRY(hipGetDevice(&dev));
    bfs_grid2d* g = new (std::nothrow) bfs_grid2d();
    if (!g) return fail(BFS_ERR_INVALID, "out of host memory");
    auto bail = [&](int code) {
        bfs_grid2d_destroy(g);
        return code;
    };
    g->V = V;
    g->nnz = nnz;
    g->R = R;
    g->C = C;
    g->RC = R * C;
    g->B = block_size(V, R * C);
    g->WB = g->B / 32;
    g->device = dev;
    const Layout2 L = layout2(V, nnz, R, C);
    char* w = static_cast<char*>(d_workspace);
    g->ws = w;
    g->off2 = reinterpret_cast<int64_t*>(w + L.off2);
    g->lrow = reinterpret_cast<int32_t*>(w + L.lrow);
    g->bm = reinterpret_cast<uint32_t*>(w + L.bm);
    g->bm_old = reinterpret_cast<uint32_t*>(w + L.bm_old);
    g->pred = reinterpret_cast<int32_t*>(w + L.pred);
    g->dst = reinterpret_cast<int32_t*>(w + L.dst);
    g->fbm = reinterpret_cast<uint32_t*>(w + L.fbm);
    g->af = reinterpret_cast<int32_t*>(w + L.af);
    g->deg = reinterpret_cast<int32_t*>(w + L.deg);
    g->rowstart = reinterpret_cast<int64_t*>(w + L.rowstart);
    g->uidv = reinterpret_cast<int32_t*>(w + L.uidv);
    g->cumul = reinterpret_cast<int64_t*>(w + L.cumul);
    g->bsum = reinterpret_cast<int64_t*>(w + L.bsum);
    g->tile_k = reinterpret_cast<int32_t*>(w + L.tile_k);
    g->ctl = reinterpret_cast<Ctl*>(w + L.ctl);
    g->plan = reinterpret_cast<Plan*>(w + L.plan);
    g->tile_cap = (nnz + kTile - 1) / kTile + g->RC + 1;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    g->num_cus = cus;
    {
        const int per_cu = std::min(8, expand_occupancy());
        const int grid = std::max(kSlots, cus * per_cu / kSlots * kSlots);
        g->expand_grid = grid;
        g->slot_grid = std::max(kSlots, cus * 4 / kSlots * kSlots);
    }
    hipError_t e = hipHostMalloc((void**)&g->h_plan, sizeof(Plan) + sizeof(Ctl), hipHostMallocDefault);
    if (e != hipSuccess) return bail(hip_fail(e, "hipHostMalloc"));
    g->h_ctl = reinterpret_cast<Ctl*>(reinterpret_cast<char*>(g->h_plan) + sizeof(Plan));
    if ((e = hipEventCreate(&g->ev0)) != hipSuccess || (e = hipEventCreate(&g->ev1)) != hipSuccess)
        return bail(hip_fail(e, "hipEventCreate"));

    // fixed part of the plan: processors in slot order
    Plan& P = *g->h_plan;
    std::memset(&P, 0, sizeof(Plan));
    P.V = V;
    P.R = R;
    P.C = C;
    P.RC = g->RC;
    P.B = g->B;
    P.WB = g->WB;
    int n = 0;
    if (g->RC >= kSlots) {
        for (int x = 0; x < kSlots; ++x) {
            P.slot_pos[x] = n;
            for (int p = x; p < g->RC; p += kSlots) {
                P.ppos[p] = n;
                P.porder[n++] = p;
            }
        }
        P.slot_pos[kSlots] = n;
    } else {
        for (int p = 0; p < g->RC; ++p) {
            P.ppos[p] = p;
            P.porder[p] = p;
        }
        for (int x = 0; x <= kSlots; ++x) P.slot_pos[x] = 0;
    }

    // CSR checks, then the partition
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int32_t* flags = reinterpret_cast<int32_t*>(g->ctl);  // scratch before the first search
    int32_t h[2] = {0, 0};
    e = hipMemcpyAsync(flags, h, sizeof(h), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_validate_csr(s, V, nnz, d_row_offsets, d_col, flags, flags + 1, 1);
    if (e == hipSuccess) e = hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(hip_fail(e, "CSR check"));
    if (h[0] & 3) return bail(fail(BFS_ERR_INVALID, "row offsets are not a valid CSR (code %d)", h[0]));
    if (h[0] & 4) return bail(fail(BFS_ERR_INVALID, "a column id is outside [0, V)"));
    const int pgrid = cus * 8;
    hipLaunchKernelGGL(k2_part_count, dim3(pgrid), dim3(kWG), 0, s, V, nnz, R, g->B, d_row_offsets,
                       d_col, g->off2);
    hipLaunchKernelGGL(k2_part_scatter, dim3(pgrid), dim3(kWG), 0, s, V, R, g->B, d_row_offsets,
                       d_col, g->off2, g->lrow);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(hip_fail(e, "2D partition"));
    *out = g;
    return ok();
}

int bfs_grid2d_destroy(bfs_grid2d* g)
{
    if (!g) return ok();
    if (g->h_plan) (void)hipHostFree(g->h_plan);
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
    delete g;
    return ok();
}

int bfs_grid2d_run(bfs_grid2d* g, int32_t root, int32_t msg_mode, int32_t* d_levels,
                   int32_t* d_parents, void* hip_stream, bfs_grid2d_stats* st)
{
    if (!g) return fail(BFS_ERR_INVALID, "grid handle is NULL");
    if (root < 0 || root >= g->V) return fail(BFS_ERR_INVALID, "root %d outside [0, %d)", root, g->V);
    if (!d_levels) return fail(BFS_ERR_INVALID, "levels pointer is NULL");
    if (msg_mode < kMsgAuto || msg_mode > kMsgBitmap)
        return fail(BFS_ERR_INVALID, "message mode must be 0, 1 or 2");
    Busy2 busy(g);
    if (!busy.held) return fail(BFS_ERR_BUSY, "grid handle is in use");
    Dev2 dg(g->device);
    return run2d(g, root, msg_mode, d_levels, d_parents, static_cast<hipStream_t>(hip_stream), st);
}

}  // extern "C"
