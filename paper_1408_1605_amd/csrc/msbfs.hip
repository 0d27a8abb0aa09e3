// Multi-source batch search: up to 64 independent searches in one pass.
//
// Lane b of a 64-bit mask per vertex belongs to root b.  seen[v] holds the
// lanes that reached v, front[v] the lanes for which v is in this level's
// frontier, next[v] the lanes that found v during this level; seen and next
// sit side by side (SeenNext), so one 16-byte load tests both.  A level is
// the paper's frontier expansion (Section 3.4) run once over the union
// frontier {v : front[v] != 0}: the same degree scan and edge -> thread
// mapping, with the visited test and claim done on whole masks,
//   next[v] |= front[u] & ~(seen[v] | next[v])   (64-bit atomic OR, no
//   return value, skipped when no lane is new),
// then a finalize pass turns next into the new frontier (new = next & ~seen),
// writes level L into row b of the output for every new lane b, and
// compacts the union frontier.  Lanes never interact, so each row equals the
// single-root search from its root.
//
// When the union frontier is small (at most V/64 vertices: deep, narrow
// searches such as grids), the expansion also marks each vertex it finds in
// a touched bitmap, the old frontier's masks are cleared through the queue,
// and the finalize pass only does work for touched vertices, so a level
// costs O(frontier + V/32) instead of O(V).
//
// Every launch reads its sizes from ctrl and returns at once when
// ctrl->done is set, so a fixed sequence of levels can be captured in a
// hipGraph and replayed until the frontier is empty.
#include "bfs_internal.h"
#include "tile_map.h"
#include "wave_ops.h"

namespace bfsmi {

__global__ __launch_bounds__(kWG) void k_ms_clear(int32_t V, int32_t n_roots,
                                                  SeenNext* __restrict__ sn,
                                                  uint64_t* __restrict__ front,
                                                  uint32_t* __restrict__ touched,
                                                  int8_t* __restrict__ out8, int vec)
{
    const int64_t stride = (int64_t)gridDim.x * kWG;
    const int64_t tid = (int64_t)blockIdx.x * kWG + threadIdx.x;
    for (int64_t v = tid; v < V; v += stride) {
        sn[v] = SeenNext{0ull, 0ull};
        front[v] = 0;
    }
    for (int64_t w = tid; w < ((int64_t)V + 31) / 32; w += stride) touched[w] = 0;
    const int64_t nbytes = (int64_t)n_roots * V;
    int64_t done = 0;
    if (vec) {
        int4* o4 = reinterpret_cast<int4*>(out8);
        const int4 m1 = make_int4(-1, -1, -1, -1);
        for (int64_t i = tid; i < nbytes / 16; i += stride) o4[i] = m1;
        done = nbytes / 16 * 16;
    }
    for (int64_t i = done + tid; i < nbytes; i += stride) out8[i] = -1;
}

// out8: the rows the level kernels write (ctrl->out8): the caller's rows,
// or with internal_rows the internal-id rows that k_ms_reorder turns into
// the caller's at the end.
__global__ __launch_bounds__(kWG) void k_ms_roots(int32_t V, int32_t n_roots,
                                                  const int32_t* __restrict__ roots,
                                                  const int32_t* __restrict__ rank,
                                                  SeenNext* __restrict__ sn,
                                                  uint64_t* __restrict__ front,
                                                  int8_t* __restrict__ out8, int internal_rows,
                                                  int32_t* __restrict__ Q,
                                                  Ctrl* __restrict__ ctrl)
{
    __shared__ int32_t s_x[64];
    __shared__ int32_t s_n;
    const int b = threadIdx.x;
    if (b == 0) s_n = 0;
    if (b < n_roots) {
        const int32_t r = roots[b];
        s_x[b] = rank ? rank[r] : r;
        out8[(int64_t)b * V + (internal_rows ? s_x[b] : r)] = 0;
    }
    __syncthreads();
    if (b < n_roots) {
        const int32_t x = s_x[b];
        uint64_t lanes = 0;
        bool first = true;
        for (int c = 0; c < n_roots; ++c) {
            if (s_x[c] == x) {
                lanes |= 1ull << c;
                if (c < b) first = false;
            }
        }
        if (first) {
            sn[x].seen = lanes;
            front[x] = lanes;
            Q[atomicAdd(&s_n, 1)] = x;
        }
    }
    __syncthreads();
    if (b == 0) {
        ctrl->qlen = s_n;
        ctrl->qn_count = 0;
        ctrl->level = 1;
        ctrl->done = 0;
        ctrl->err = 0;
        ctrl->overflow = 0;
        ctrl->r = 0;
        ctrl->ntiles = 0;
        ctrl->r_total = 0;
        ctrl->reached = s_n;
        ctrl->levels = 1;
        ctrl->alive = 0;
        ctrl->last_alive = 0;
        ctrl->out8 = out8;
        ctrl->full_prefix = 0;
        ctrl->fp_cand = 0x7fffffff;
        ctrl->skipped = 0;
        ctrl->sparse_limit = V / 64;
        ctrl->sparse = s_n <= V / 64;
    }
}

hipError_t launch_ms_init(hipStream_t s, int grid, int32_t V, const int32_t* roots_dev,
                          int32_t n_roots, const int32_t* rank, SeenNext* sn, uint64_t* front,
                          uint32_t* touched, int8_t* out8, int8_t* out_int, int32_t* Q,
                          Ctrl* ctrl)
{
    if (grid < 1) grid = 1;
    // internal rows need no fill: the reorder reads only the lanes a vertex has seen
    int8_t* fill = out_int ? nullptr : out8;
    const int vec = ((uintptr_t)out8 % 16) == 0;
    hipLaunchKernelGGL(k_ms_clear, dim3(grid), dim3(kWG), 0, s, V, fill ? n_roots : 0, sn, front,
                       touched, fill, vec);
    hipLaunchKernelGGL(k_ms_roots, dim3(1), dim3(64), 0, s, V, n_roots, roots_dev, rank, sn, front,
                       out_int ? out_int : out8, out_int ? 1 : 0, Q, ctrl);
    return hipGetLastError();
}

// Batch with degree order: out8[b][c] = out_int[b][rank[c]] where lane b has
// seen c, else -1.  A workgroup takes runs of 4096 caller ids (the
// relabelling's unit, one contiguous internal range per degree class), so
// the gathers reuse lines; for a fixed lane the stores of a wave are
// contiguous.
constexpr int kReorderChunk = 4096;

__global__ __launch_bounds__(kWG) void k_ms_reorder(int32_t V, int32_t n_roots,
                                                    const int32_t* __restrict__ rank,
                                                    const SeenNext* __restrict__ sn,
                                                    const int8_t* __restrict__ out_int,
                                                    int8_t* __restrict__ out8)
{
    const int64_t nchunks = ((int64_t)V + kReorderChunk - 1) / kReorderChunk;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        for (int j = 0; j < kReorderChunk / kWG; ++j) {
            const int64_t c = ch * kReorderChunk + j * kWG + threadIdx.x;
            if (c >= V) continue;
            const int32_t x = rank[c];
            const uint64_t seen = sn[x].seen;
            for (int b = 0; b < n_roots; ++b) {
                const int8_t lv = ((seen >> b) & 1ull) ? out_int[(int64_t)b * V + x] : (int8_t)-1;
                out8[(int64_t)b * V + c] = lv;
            }
        }
    }
}

hipError_t launch_ms_reorder(hipStream_t s, int grid, int32_t V, int32_t n_roots,
                             const int32_t* rank, const SeenNext* sn, const int8_t* out_int,
                             int8_t* out8)
{
    const int64_t nchunks = ((int64_t)V + kReorderChunk - 1) / kReorderChunk;
    if (grid > nchunks) grid = (int)nchunks;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_ms_reorder, dim3(grid), dim3(kWG), 0, s, V, n_roots, rank, sn, out_int,
                       out8);
    return hipGetLastError();
}

template <int EPT>
__global__ __launch_bounds__(kWG) void k_ms_expand(const int64_t* __restrict__ rowstart,
                                                   const int32_t* __restrict__ uidv,
                                                   const int64_t* __restrict__ cumul,
                                                   const int32_t* __restrict__ tile_k,
                                                   const int32_t* __restrict__ col,
                                                   const uint64_t* __restrict__ front,
                                                   SeenNext* __restrict__ sn,
                                                   uint32_t* __restrict__ touched,
                                                   const Ctrl* __restrict__ ctrl)
{
    __shared__ TileLds<EPT> L;
    if (ctrl->done) return;
    const bool sparse = ctrl->sparse != 0;
    const int64_t r = ctrl->r;
    const int32_t ntiles = ctrl->ntiles;
    StageRegs<EPT> cur = fetch_stage<EPT>(blockIdx.x, ntiles, cumul, rowstart, uidv, tile_k);
    for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int32_t uu[EPT], vv[EPT];
        bool ok[EPT];
        int64_t ee[EPT];
        map_tile<EPT>(L, cur, r, cumul, rowstart, uidv, col, uu, vv, ok, ee);
        cur = fetch_stage<EPT>(tile + gridDim.x, ntiles, cumul, rowstart, uidv, tile_k);
        // one 16-byte load gives both masks of the target: lanes that have
        // seen it, and lanes already recorded for the next level (a stale
        // pair only lets more threads issue the atomic)
        uint64_t f[EPT], have[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) f[j] = ok[j] ? front[uu[j]] : 0ull;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            have[j] = ~0ull;
            if (f[j]) {
                const SeenNext p = sn[vv[j]];
                have[j] = p.seen | p.next;
            }
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint64_t nb = f[j] & ~have[j];
            if (nb) {
                (void)__hip_atomic_fetch_or(&sn[vv[j]].next, nb, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
                if (sparse)
                    (void)__hip_atomic_fetch_or(touched + (vv[j] >> 5), 1u << (vv[j] & 31),
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

constexpr int kFinItems = 8;  // vertices per thread and chunk in the finalize

__device__ __forceinline__ uint64_t wave_or64(uint64_t x)
{
    for (int d = 1; d < 64; d <<= 1) x |= __shfl_xor(x, d, 64);
    return x;
}

// OUT16 = false: batch output, int8 rows ctrl->out8[b][v] = level.
// OUT16 = true : serving output, lane b writes level - lane_start[b] into
//                its own int16 buffer lane_out[b] (caller ids).
template <bool OUT16>
__global__ __launch_bounds__(kWG) void k_ms_finalize(int32_t V, const int32_t* __restrict__ orig,
                                                     SeenNext* __restrict__ sn,
                                                     uint64_t* __restrict__ front,
                                                     uint32_t* __restrict__ touched,
                                                     int32_t* __restrict__ Qn,
                                                     int16_t* const* __restrict__ lane_out,
                                                     const int32_t* __restrict__ lane_start,
                                                     Ctrl* __restrict__ ctrl)
{
    constexpr int IT = kFinItems;
    __shared__ int16_t* s_out[64];
    __shared__ int32_t s_start[64];
    __shared__ uint32_t s_wave[kWG / 64];
    __shared__ uint32_t s_base;
    __shared__ uint64_t s_alive[kWG / 64];
    if (ctrl->done) return;
    const int32_t lvl = ctrl->level;
    const bool sparse = ctrl->sparse != 0;
    int8_t* __restrict__ out8 = ctrl->out8;
    if (OUT16) {
        // the lane tables, once per workgroup
        if (threadIdx.x < 64) {
            s_out[threadIdx.x] = lane_out[threadIdx.x];
            s_start[threadIdx.x] = lane_start[threadIdx.x];
        }
        __syncthreads();
    }
    // A workgroup takes chunks of kWG * IT vertices; each chunk reserves its
    // queue slots with one atomicAdd (a per-wave add on the one counter
    // would serialise tens of thousands of atomics per level).
    constexpr int64_t chunk = (int64_t)kWG * IT;
    uint64_t alive = 0;
    for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < V; c0 += (int64_t)gridDim.x * chunk) {
        uint64_t nw[IT];
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int64_t v = c0 + j * kWG + threadIdx.x;
            nw[j] = 0;
            bool hit = v < V;
            if (sparse && v < V) {
                // the 32 lanes of a word read it before its first lane clears it
                const uint32_t tw = touched[v >> 5];
                hit = (tw >> (v & 31)) & 1u;
                if ((v & 31) == 0 && tw) touched[v >> 5] = 0;
            }
            if (hit) {
                const SeenNext p = sn[v];
                if (p.next) {
                    nw[j] = p.next & ~p.seen;
                    sn[v] = SeenNext{p.seen | nw[j], 0ull};
                }
                front[v] = nw[j];
            }
            cnt += nw[j] ? 1u : 0u;
        }
        uint32_t tot;
        const uint32_t ex = wg_exclusive_scan<uint32_t>(cnt, &tot, s_wave);
        if (tot == 0) continue;  // uniform: no queue slots, no outputs
        if (threadIdx.x == 0) s_base = atomicAdd(&ctrl->qn_count, tot);
        __syncthreads();
        uint32_t pos = s_base + ex;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            if (!nw[j]) continue;
            const int64_t v = c0 + j * kWG + threadIdx.x;
            if (pos < (uint32_t)V) Qn[pos] = (int32_t)v;
            else ctrl->err = 4;
            ++pos;
            // each vertex writes only the lanes that reached it now
            const int64_t vo = orig ? orig[v] : v;
            if (OUT16) {
                for (uint64_t m = nw[j]; m; m &= m - 1) {
                    const int b = __builtin_ctzll(m);
                    const int32_t d = lvl - s_start[b];
                    if (d > 32767) ctrl->overflow = 1;
                    else if (s_out[b]) s_out[b][vo] = (int16_t)d;  // null: retired lane
                }
            } else if (lvl > 127) {
                ctrl->overflow = 1;
            } else if (orig) {
                for (uint64_t m = nw[j]; m; m &= m - 1)
                    out8[(int64_t)__builtin_ctzll(m) * V + vo] = (int8_t)lvl;
            }
            alive |= nw[j];
        }
        if (!OUT16 && !orig && lvl <= 127) {
            // rows by search id: lane b of a wave's vertices is one contiguous
            // (masked) store, lanes taken in the same order by every thread
#pragma unroll
            for (int j = 0; j < IT; ++j) {
                const int64_t v = c0 + j * kWG + threadIdx.x;
                for (uint64_t m = wave_or64(nw[j]); m; m &= m - 1) {
                    const int b = __builtin_ctzll(m);
                    if ((nw[j] >> b) & 1ull) out8[(int64_t)b * V + v] = (int8_t)lvl;
                }
            }
        }
        __syncthreads();  // s_base is rewritten by the next chunk
    }
    // one alive update per workgroup
    alive = wave_or64(alive);
    if (__lane_id() == 0) s_alive[threadIdx.x >> 6] = alive;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0;
        for (int w = 0; w < kWG / 64; ++w) a |= s_alive[w];
        if (a) atomicOr((unsigned long long*)&ctrl->alive, (unsigned long long)a);
    }
}

// Sparse levels: the old frontier's masks are cleared through the queue
// (after the expansion has read them, before the finalize writes new ones).
__global__ __launch_bounds__(kWG) void k_ms_clear_front(const int32_t* __restrict__ Q,
                                                        uint64_t* __restrict__ front,
                                                        const Ctrl* __restrict__ ctrl)
{
    if (ctrl->done || !ctrl->sparse) return;
    const int32_t qlen = ctrl->qlen;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x; k < qlen; k += stride) front[Q[k]] = 0;
}

// After a level's finalize: the first id, from the current prefix on, that
// some lane still searching (found vertices this level) has not seen.  Each
// workgroup takes 2048-id chunks in order and stops once a smaller candidate
// is known; k_ms_advance moves ctrl->full_prefix there (the prefix only
// grows: seen masks grow and the set of searching lanes shrinks).
constexpr int kPrefixChunk = kWG * 8;

__global__ __launch_bounds__(kWG) void k_ms_prefix(int32_t V, const SeenNext* __restrict__ sn,
                                                   Ctrl* __restrict__ ctrl)
{
    __shared__ int32_t s_min, s_known;
    if (ctrl->done) return;
    const uint64_t live = ctrl->alive;
    if (live == 0) return;  // the batch ends at this level
    const int32_t p0 = ctrl->full_prefix;
    for (int64_t c0 = (int64_t)p0 + (int64_t)blockIdx.x * kPrefixChunk; c0 < V;
         c0 += (int64_t)gridDim.x * kPrefixChunk) {
        if (threadIdx.x == 0) {
            s_min = 0x7fffffff;
            s_known = __hip_atomic_load(&ctrl->fp_cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (c0 >= s_known) break;  // uniform (one read, shared through LDS)
#pragma unroll
        for (int j = 0; j < kPrefixChunk / kWG; ++j) {
            const int64_t x = c0 + j * kWG + threadIdx.x;
            if (x < V && (sn[x].seen & live) != live) atomicMin(&s_min, (int32_t)x);
        }
        __syncthreads();
        const int32_t m = s_min;
        if (m != 0x7fffffff) {
            if (threadIdx.x == 0) atomicMin(&ctrl->fp_cand, m);
            break;  // uniform
        }
        __syncthreads();  // s_min is reset for the next chunk
    }
}

__global__ void k_ms_advance(Ctrl* __restrict__ ctrl, int32_t V, int prefix)
{
    if (ctrl->done) return;
    if (prefix) {
        // no candidate: every id from the old prefix on is seen by all live lanes
        const int32_t c = ctrl->fp_cand;
        ctrl->full_prefix = c < V ? c : V;
        ctrl->fp_cand = 0x7fffffff;
    }
    const uint32_t q = ctrl->qn_count;
    ctrl->sparse = (int32_t)q <= ctrl->sparse_limit;
    ctrl->last_alive = ctrl->alive;  // lanes that found vertices this level
    ctrl->alive = 0;
    ctrl->reached += q;
    ctrl->qlen = (int32_t)q;
    ctrl->qn_count = 0;
    if (q) ctrl->levels += 1;
    ctrl->level += 1;
    ctrl->done = (q == 0 || ctrl->overflow || ctrl->err) ? 1 : 0;
}

template <int EPT>
static void ms_expand_launch(hipStream_t s, int grid, const int64_t* rowstart, const int32_t* uidv,
                             const int64_t* cumul, const int32_t* tile_k, const int32_t* col,
                             const uint64_t* front, SeenNext* sn, uint32_t* touched,
                             const Ctrl* ctrl)
{
    hipLaunchKernelGGL(k_ms_expand<EPT>, dim3(grid), dim3(kWG), 0, s, rowstart, uidv, cumul, tile_k,
                       col, front, sn, touched, ctrl);
}

int ms_expand_blocks_per_cu(int ept)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (ept) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ms_expand<1>, kWG, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ms_expand<2>, kWG, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ms_expand<4>, kWG, 0); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ms_expand<8>, kWG, 0); break;
    default: break;
    }
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

hipError_t launch_ms_level(hipStream_t s, int scan_grid, int expand_grid, int fin_grid, int ept,
                           int32_t V, int64_t tile_cap, const int64_t* off, const int32_t* col,
                           const int32_t* orig, const int32_t* Q, int32_t* Qn, int32_t* deg,
                           int64_t* rowstart, int32_t* uidv, int64_t* bsum, int64_t* cumul,
                           int32_t* tile_k, SeenNext* sn, uint64_t* front, uint32_t* touched,
                           int16_t* const* lane_out, const int32_t* lane_start, Ctrl* ctrl,
                           const int32_t* skip, int prefix_grid)
{
    const bool prefix = skip != nullptr && prefix_grid > 0;
    hipError_t e = launch_scan_dev(s, scan_grid, Q, off, nullptr, deg, rowstart, uidv, bsum, cumul,
                                   tile_k, tile_cap, kWG * ept, ctrl, prefix ? skip : nullptr, V);
    if (e != hipSuccess) return e;
    if (expand_grid < 1) expand_grid = 1;
    switch (ept) {
    case 1: ms_expand_launch<1>(s, expand_grid, rowstart, uidv, cumul, tile_k, col, front, sn, touched, ctrl); break;
    case 2: ms_expand_launch<2>(s, expand_grid, rowstart, uidv, cumul, tile_k, col, front, sn, touched, ctrl); break;
    case 4: ms_expand_launch<4>(s, expand_grid, rowstart, uidv, cumul, tile_k, col, front, sn, touched, ctrl); break;
    case 8: ms_expand_launch<8>(s, expand_grid, rowstart, uidv, cumul, tile_k, col, front, sn, touched, ctrl); break;
    default: return hipErrorInvalidValue;
    }
    if (fin_grid < 1) fin_grid = 1;
    hipLaunchKernelGGL(k_ms_clear_front, dim3(scan_grid), dim3(kWG), 0, s, Q, front, ctrl);
    if (lane_out) {
        hipLaunchKernelGGL(k_ms_finalize<true>, dim3(fin_grid), dim3(kWG), 0, s, V, orig, sn,
                           front, touched, Qn, lane_out, lane_start, ctrl);
    } else {
        hipLaunchKernelGGL(k_ms_finalize<false>, dim3(fin_grid), dim3(kWG), 0, s, V, orig, sn,
                           front, touched, Qn, lane_out, lane_start, ctrl);
    }
    if (prefix)
        hipLaunchKernelGGL(k_ms_prefix, dim3(prefix_grid), dim3(kWG), 0, s, V, sn, ctrl);
    hipLaunchKernelGGL(k_ms_advance, dim3(1), dim3(1), 0, s, ctrl, V, prefix ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Serving: lanes join a running batch at a level boundary and retire when a
// level finds nothing for them.

__global__ __launch_bounds__(kWG) void k_srv_reset(int32_t V, SeenNext* __restrict__ sn,
                                                   uint64_t* __restrict__ front,
                                                   uint32_t* __restrict__ touched,
                                                   Ctrl* __restrict__ ctrl)
{
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < V; v += stride) {
        sn[v] = SeenNext{0ull, 0ull};
        front[v] = 0;
    }
    for (int64_t w = (int64_t)blockIdx.x * kWG + threadIdx.x; w < ((int64_t)V + 31) / 32; w += stride)
        touched[w] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->qlen = 0;
        ctrl->qn_count = 0;
        ctrl->level = 1;
        ctrl->done = 1;  // nothing to expand until a lane joins
        ctrl->err = 0;
        ctrl->overflow = 0;
        ctrl->r = 0;
        ctrl->ntiles = 0;
        ctrl->r_total = 0;
        ctrl->reached = 0;
        ctrl->levels = 0;
        ctrl->alive = 0;
        ctrl->last_alive = 0;
        ctrl->out8 = nullptr;
        ctrl->sparse_limit = V / 64;
        ctrl->sparse = 1;
    }
}

// Clear the retired lanes' bits from every vertex's seen mask.
__global__ __launch_bounds__(kWG) void k_srv_clear(int32_t V, SeenNext* __restrict__ sn,
                                                   uint64_t mask)
{
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < V; v += stride) {
        const uint64_t x = sn[v].seen;
        if (x & mask) sn[v].seen = x & ~mask;
    }
}

__global__ __launch_bounds__(kWG) void k_fill16(int16_t* __restrict__ p, int64_t n, int16_t val)
{
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) p[i] = val;
}

// dst[i] = src[i] widened to int32, and *maxp = max(*maxp, max src[i]):
// delivery of a serving result into a device buffer of the caller.
__global__ __launch_bounds__(kWG) void k_widen16(const int16_t* __restrict__ src,
                                                 int32_t* __restrict__ dst, int64_t n,
                                                 int32_t* __restrict__ maxp)
{
    const int64_t stride = (int64_t)gridDim.x * kWG;
    int32_t m = -1;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        const int32_t x = src[i];
        dst[i] = x;
        m = x > m ? x : m;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const int32_t o = __shfl_xor(m, d, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m >= 0) atomicMax(maxp, m);
}

// Lane join_lane[i] starts a search from join_root[i] (caller id).  Its
// root gets depth 0; its first expansion is the next level, so
// lane_start = level - 1.  Roots not yet in the union frontier are appended.
__global__ void k_srv_join(int32_t V, int32_t n_join, const int32_t* __restrict__ join,
                           const int32_t* __restrict__ rank, SeenNext* __restrict__ sn,
                           uint64_t* __restrict__ front, int16_t* const* __restrict__ lane_out,
                           int32_t* __restrict__ lane_start, int32_t* __restrict__ Q,
                           Ctrl* __restrict__ ctrl)
{
    // join[2 * i] = root, join[2 * i + 1] = lane; one wave, n_join <= 64
    __shared__ int32_t s_app;
    const int i = threadIdx.x;
    if (i == 0) s_app = 0;
    __syncthreads();
    const int32_t qlen = ctrl->qlen;
    if (i < n_join) {
        const int32_t r = join[2 * i];
        const int32_t b = join[2 * i + 1];
        const int32_t x = rank ? rank[r] : r;
        const uint64_t bit = 1ull << b;
        atomicOr((unsigned long long*)&sn[x].seen, (unsigned long long)bit);
        const uint64_t old = atomicOr((unsigned long long*)&front[x], (unsigned long long)bit);
        lane_out[b][r] = 0;
        lane_start[b] = ctrl->level - 1;
        if (old == 0) {
            const int32_t pos = qlen + atomicAdd(&s_app, 1);
            if (pos < V) Q[pos] = x;
            else ctrl->err = 5;
        }
    }
    __syncthreads();
    if (i == 0) {
        ctrl->qlen = qlen + s_app;
        ctrl->sparse = ctrl->qlen <= ctrl->sparse_limit;
        ctrl->done = 0;
    }
}

hipError_t launch_srv_reset(hipStream_t s, int grid, int32_t V, SeenNext* sn, uint64_t* front,
                            uint32_t* touched, Ctrl* ctrl)
{
    hipLaunchKernelGGL(k_srv_reset, dim3(grid), dim3(kWG), 0, s, V, sn, front, touched, ctrl);
    return hipGetLastError();
}

hipError_t launch_srv_clear(hipStream_t s, int grid, int32_t V, SeenNext* sn, uint64_t mask)
{
    hipLaunchKernelGGL(k_srv_clear, dim3(grid), dim3(kWG), 0, s, V, sn, mask);
    return hipGetLastError();
}

hipError_t launch_fill16(hipStream_t s, int grid, int16_t* p, int64_t n, int16_t val)
{
    hipLaunchKernelGGL(k_fill16, dim3(grid), dim3(kWG), 0, s, p, n, val);
    return hipGetLastError();
}

hipError_t launch_widen16(hipStream_t s, int grid, const int16_t* src, int32_t* dst, int64_t n,
                          int32_t* maxp)
{
    hipLaunchKernelGGL(k_widen16, dim3(grid), dim3(kWG), 0, s, src, dst, n, maxp);
    return hipGetLastError();
}

hipError_t launch_srv_join(hipStream_t s, int32_t V, int32_t n_join, const int32_t* join,
                           const int32_t* rank, SeenNext* sn, uint64_t* front,
                           int16_t* const* lane_out, int32_t* lane_start, int32_t* Q, Ctrl* ctrl)
{
    hipLaunchKernelGGL(k_srv_join, dim3(1), dim3(64), 0, s, V, n_join, join, rank, sn, front,
                       lane_out, lane_start, Q, ctrl);
    return hipGetLastError();
}

}  // namespace bfsmi
