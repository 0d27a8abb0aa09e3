// Persistent search for runs of small levels (single root).
//
// A level whose frontier holds a few thousand vertices does almost no work,
// but launching its kernels (degree scan, expansion, bookkeeping) costs a
// dispatch gap of several microseconds each; a 4096 x 4096 grid has
// thousands of such levels.  One persistent kernel of a few dozen
// workgroups (at most one per CU, so all are resident together) runs them
// back to back instead:
//   - each workgroup takes an equal slice of the frontier, stages the
//     slice's degrees, row starts and caller ids in LDS with a prefix sum,
//     and maps the slice's edges to threads by binary search in it
//     (Section 3.4, within the slice, so no grid-wide scan is needed);
//   - claims use the plain-read probe and atomicOr of Algorithm 3; winners
//     write level and parent and append to the next queue;
//   - one grid-wide barrier ends each level.
// The kernel hands the search back to the host when the next frontier, its
// edge count or its largest degree exceeds the limits the host passes, and
// ends the search when a frontier is empty.  Every barrier wait is bounded:
// a wait that does not end sets ctrl->err and every workgroup leaves.
#include "bfs_internal.h"
#include "wave_ops.h"

namespace bfsmi {

constexpr int kSmallEPT = 4;
constexpr int kSmallTile = kWG * kSmallEPT;
constexpr int kSmallStage = 1024;  // frontier entries staged per pass (4 per thread)
constexpr uint32_t kSpinCap = 1u << 24;

// Grid-wide barrier: thread 0 of each workgroup arrives on a counter; the
// last one resets it and advances the generation the others wait on.
// Device-scope fences order the level's queue and output writes.
__device__ __forceinline__ bool grid_sync(SmallSync* sy, uint32_t nwg, uint32_t* s_gen)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const uint32_t g = *s_gen;
        __threadfence();
        const uint32_t a = atomicAdd(&sy->arrive, 1u);
        if (a == nwg - 1) {
            atomicExch(&sy->arrive, 0u);
            __threadfence();
            atomicAdd(&sy->gen, 1u);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(&sy->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kSpinCap) {
                    ok = 0;
                    break;
                }
            }
        }
        __threadfence();
        *s_gen = g + 1;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

__global__ __launch_bounds__(kWG) void k_small_levels(
    int32_t V, const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const int32_t* __restrict__ orig, uint32_t* __restrict__ vis, uint32_t* __restrict__ vis_old,
    int32_t* __restrict__ Qa, int32_t* __restrict__ Qb, int32_t* __restrict__ level,
    int32_t* __restrict__ parent, SmallSync* __restrict__ sy, Ctrl* __restrict__ ctrl,
    int32_t qlen0, int32_t lvl0, int32_t qlimit, int64_t rlimit, int32_t dlimit)
{
    __shared__ int32_t s_cum[kSmallStage + 1];
    __shared__ int32_t s_uid[kSmallStage];
    __shared__ int64_t s_base[kSmallStage];
    __shared__ uint16_t s_map[kSmallTile];
    __shared__ int32_t s_wave[kWG / 64];
    __shared__ uint32_t s_gen;
    const uint32_t N = gridDim.x;
    const uint32_t w = blockIdx.x;
    const int t = threadIdx.x;
    if (t == 0) s_gen = 0;

    // The first frontier's size limits are checked before any level runs.
    {
        const int64_t k0 = (int64_t)qlen0 * w / N, k1 = (int64_t)qlen0 * (w + 1) / N;
        int64_t sum = 0;
        int32_t mx = 0;
        for (int64_t k = k0 + t; k < k1; k += kWG) {
            const int32_t u = Qa[k];
            const int64_t d = off[u + 1] - off[u];
            sum += d;
            mx = d > mx ? (int32_t)d : mx;
        }
        for (int o = 32; o >= 1; o >>= 1) {
            sum += __shfl_xor(sum, o, 64);
            const int32_t m2 = __shfl_xor(mx, o, 64);
            mx = m2 > mx ? m2 : mx;
        }
        if ((t & 63) == 0) {
            if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(&sy->rn[2]),
                               (unsigned long long)sum);
            if (mx) atomicMax(&sy->md[2], mx);
        }
    }
    if (!grid_sync(sy, N, &s_gen)) {
        if (t == 0) ctrl->err = 4;
        return;
    }
    {
        // slot 2 is next reset during level 1, after every workgroup read it
        const int64_t rn = __hip_atomic_load(&sy->rn[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t md = __hip_atomic_load(&sy->md[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (rn > rlimit || md > dlimit) {
            if (w == 0 && t == 0) {
                ctrl->done = 2;
                ctrl->qlen = qlen0;
                ctrl->level = lvl0;
                ctrl->steps = 0;
                ctrl->reached = 0;
                ctrl->levels = 0;
            }
            return;
        }
    }

    int32_t qlen = qlen0, lvl = lvl0, step = 0, par = 0, code = 0;
    int64_t my_edges = 0, reached = 0;
    while (true) {
        const int32_t* __restrict__ Q = par ? Qb : Qa;
        int32_t* __restrict__ Qn = par ? Qa : Qb;
        const int cs = step % 3;  // counters of this level
        if (w == 0 && t == 0) {
            // the next level's counters were last read two barriers ago
            const int nx = (step + 1) % 3;
            sy->qn[nx] = 0;
            sy->rn[nx] = 0;
            sy->md[nx] = 0;
        }
        const int64_t k0 = (int64_t)qlen * w / N, k1 = (int64_t)qlen * (w + 1) / N;
        for (int64_t s0 = k0; s0 < k1; s0 += kSmallStage) {
            const int32_t n = (int32_t)(k1 - s0 < kSmallStage ? k1 - s0 : kSmallStage);
            // stage 4 consecutive entries per thread, prefix sum of degrees
            int64_t a[4];
            int32_t d[4], id[4];
            int32_t tot = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int32_t i = t * 4 + m;
                a[m] = 0;
                d[m] = 0;
                id[m] = 0;
                if (i < n) {
                    const int32_t u = Q[s0 + i];
                    a[m] = off[u];
                    d[m] = (int32_t)(off[u + 1] - a[m]);
                    id[m] = orig ? orig[u] : u;
                }
                tot += d[m];
            }
            int32_t R;
            int32_t c = wg_exclusive_scan<int32_t>(tot, &R, s_wave);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int32_t i = t * 4 + m;
                if (i < n) {
                    s_cum[i] = c;
                    s_uid[i] = id[m];
                    s_base[i] = a[m] - c;
                }
                c += d[m];
            }
            if (t == 0) s_cum[n] = R;
            __syncthreads();
            my_edges += R;
            for (int32_t e0 = 0; e0 < R; e0 += kSmallTile) {
                const int32_t n_e = R - e0 < kSmallTile ? R - e0 : kSmallTile;
                // slots s0 .. s0+3 of this thread: entry = max{i : cum[i] <= slot}
                const int32_t sl0 = e0 + t * kSmallEPT;
                if (t * kSmallEPT < n_e) {
                    int32_t lo = 0;
                    for (int32_t st = 1 << (31 - __builtin_clz(n)); st > 0; st >>= 1) {
                        const int32_t x = lo + st;
                        if (x < n && s_cum[x] <= sl0) lo = x;
                    }
                    int32_t i = lo;
#pragma unroll
                    for (int j = 0; j < kSmallEPT; ++j) {
                        const int32_t sl = sl0 + j;
                        if (sl - e0 < n_e) {
                            while (i + 1 < n && s_cum[i + 1] <= sl) ++i;
                            s_map[sl - e0] = (uint16_t)i;
                        }
                    }
                }
                __syncthreads();
                int32_t vv[kSmallEPT], uu[kSmallEPT];
                bool ok[kSmallEPT];
#pragma unroll
                for (int j = 0; j < kSmallEPT; ++j) {
                    const int32_t sl = t + j * kWG;
                    ok[j] = sl < n_e;
                    const int32_t sc = ok[j] ? sl : n_e - 1;
                    const int32_t i = s_map[sc];
                    uu[j] = s_uid[i];
                    vv[j] = col[s_base[i] + e0 + sc];
                }
                uint32_t wd[kSmallEPT];
#pragma unroll
                for (int j = 0; j < kSmallEPT; ++j) wd[j] = ok[j] ? vis[vv[j] >> 5] : ~0u;
                bool need[kSmallEPT];
                uint32_t old[kSmallEPT];
#pragma unroll
                for (int j = 0; j < kSmallEPT; ++j) {
                    need[j] = ok[j] && !(wd[j] & (1u << (vv[j] & 31)));
                    old[j] = ~0u;
                    if (need[j]) old[j] = atomicOr(vis + (vv[j] >> 5), 1u << (vv[j] & 31));
                }
                int64_t dsum = 0;
                int32_t dmax = 0;
                bool win[kSmallEPT];
                uint64_t mask[kSmallEPT];
                uint32_t total = 0;
#pragma unroll
                for (int j = 0; j < kSmallEPT; ++j) {
                    win[j] = need[j] && !(old[j] & (1u << (vv[j] & 31)));
                    mask[j] = __ballot(win[j]);
                    total += (uint32_t)__popcll(mask[j]);
                }
                uint32_t base = 0;
                if (total && __lane_id() == 0) base = atomicAdd(&sy->qn[cs], total);
#pragma unroll
                for (int j = 0; j < kSmallEPT; ++j) {
                    int32_t dv = 0;
                    if (win[j]) {
                        const int32_t v = vv[j];
                        level[v] = lvl;
                        if (parent) parent[v] = uu[j];
                        dv = (int32_t)(off[v + 1] - off[v]);
                        atomicOr(vis_old + (v >> 5), 1u << (v & 31));
                    }
                    dsum += dv;
                    dmax = dv > dmax ? dv : dmax;
                }
                if (total) {
                    base = __shfl(base, 0, 64);
#pragma unroll
                    for (int j = 0; j < kSmallEPT; ++j) {
                        if (win[j]) {
                            const uint32_t pos = base + lanes_below(mask[j]);
                            if (pos < (uint32_t)V) Qn[pos] = vv[j];
                            else ctrl->err = 5;
                        }
                        base += (uint32_t)__popcll(mask[j]);
                    }
                }
                for (int o = 32; o >= 1; o >>= 1) {
                    dsum += __shfl_xor(dsum, o, 64);
                    const int32_t m2 = __shfl_xor(dmax, o, 64);
                    dmax = m2 > dmax ? m2 : dmax;
                }
                if (__lane_id() == 0) {
                    if (dsum) atomicAdd(reinterpret_cast<unsigned long long*>(&sy->rn[cs]),
                                        (unsigned long long)dsum);
                    if (dmax) atomicMax(&sy->md[cs], dmax);
                }
                __syncthreads();
            }
        }
        if (!grid_sync(sy, N, &s_gen)) {
            if (t == 0) ctrl->err = 4;
            code = 3;
            break;
        }
        const uint32_t qn = __hip_atomic_load(&sy->qn[cs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t rn = __hip_atomic_load(&sy->rn[cs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t md = __hip_atomic_load(&sy->md[cs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ++step;
        ++lvl;
        reached += qn;
        if (qn == 0) {
            code = 1;
            break;
        }
        qlen = (int32_t)qn;
        par ^= 1;
        if ((int32_t)qn > qlimit || rn > rlimit || md > dlimit) {
            code = 2;
            break;
        }
    }
    if (t == 0 && my_edges)
        atomicAdd(reinterpret_cast<unsigned long long*>(&ctrl->r_total), (unsigned long long)my_edges);
    if (w == 0 && t == 0 && code != 3) {
        ctrl->done = code;
        ctrl->qlen = qlen;
        ctrl->level = lvl;
        ctrl->steps = step;
        ctrl->reached = reached;
        ctrl->levels = code == 1 ? step - 1 : step;
    }
}

int small_loop_blocks()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_small_levels, kWG, 0) != hipSuccess)
        return 0;
    return n;
}

hipError_t launch_small_levels(hipStream_t s, int grid, int32_t V, const int64_t* off,
                               const int32_t* col, const int32_t* orig, uint32_t* vis,
                               uint32_t* vis_old, int32_t* Qa, int32_t* Qb, int32_t* level,
                               int32_t* parent, SmallSync* sy, Ctrl* ctrl, int32_t qlen,
                               int32_t lvl, int32_t qlimit, int64_t rlimit, int32_t dlimit)
{
    // An ordinary launch: the grid (at most one workgroup per CU) is small
    // enough to be resident at once, and a cooperative launch would make
    // the runtime stop overlapping later kernels of other streams.
    hipLaunchKernelGGL(k_small_levels, dim3(grid), dim3(kWG), 0, s, V, off, col, orig, vis, vis_old,
                       Qa, Qb, level, parent, sy, ctrl, qlen, lvl, qlimit, rlimit, dlimit);
    return hipGetLastError();
}

}  // namespace bfsmi
