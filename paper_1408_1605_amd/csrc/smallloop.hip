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
//   - on levels of at most 64K edges claims go straight to the atomicOr of
//     Algorithm 3 (the plain-read probe would add one dependent memory round
//     trip per level, and such levels are bound by round trips, not by
//     atomic throughput); levels with more edges probe first, since hub rows
//     would queue their claims on a few bitmap lines; winners write level
//     and parent, and append to the next queue with one reservation per
//     workgroup and tile;
//   - a winner also stores its row start, degree and caller id beside its
//     queue slot, so the next level stages its frontier without looking
//     them up in the CSR;
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
constexpr int64_t kSmallProbeEdges = 1 << 16;  // levels with more edges probe before claiming
static_assert(kWG == 256, "per-wave partials below assume four waves");

// Grid-wide barrier on a counter that only grows (reset to zero before the
// launch): barrier number k is passed once it reaches k * nwg.  Thread 0 of
// each workgroup arrives with a release add and waits with relaxed loads
// followed by an acquire fence.
__device__ __forceinline__ bool grid_sync(SmallSync* sy, uint32_t nwg, uint32_t* s_ep)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t target = (*s_ep + 1u) * nwg;
        uint32_t a = __hip_atomic_fetch_add(&sy->arrive, 1u, __ATOMIC_RELEASE,
                                            __HIP_MEMORY_SCOPE_AGENT) + 1u;
        int ok = 1;
        uint32_t spins = 0;
        while ((int32_t)(a - target) < 0) {
            __builtin_amdgcn_s_sleep(2);
            a = __hip_atomic_load(&sy->arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (++spins > kSpinCap) {
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ep += 1u;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// The levels; every workgroup returns from it exactly once.
__device__ __forceinline__ void small_levels_body(
    int32_t V, const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const int32_t* __restrict__ orig, uint32_t* __restrict__ vis, uint32_t* __restrict__ vis_old,
    int32_t* __restrict__ Qa, int32_t* __restrict__ Qb, int32_t* __restrict__ level,
    int32_t* __restrict__ parent, SmallSync* __restrict__ sy, SmallSide side,
    Ctrl* __restrict__ ctrl, int32_t qlen0, int32_t lvl0, int32_t qlimit, int64_t rlimit, int32_t dlimit)
{
    __shared__ int32_t s_cum[kSmallStage + 1];
    __shared__ int32_t s_uid[kSmallStage];
    __shared__ int64_t s_base[kSmallStage];
    __shared__ uint16_t s_map[kSmallTile];
    __shared__ int32_t s_wave[kWG / 64];
    __shared__ uint32_t s_wq[kWG / 64];
    __shared__ int64_t s_rs[kWG / 64];
    __shared__ int32_t s_rm[kWG / 64];
    __shared__ uint32_t s_qbase;
    __shared__ uint32_t s_epoch;
    const uint32_t N = gridDim.x;
    const uint32_t w = blockIdx.x;
    const int t = threadIdx.x;
    const int wave = t >> 6;
    if (t == 0) s_epoch = 0;
    // qlen0 < 0: launched right behind a host-driven level, whose next
    // frontier size is in ctrl->qn_count; an empty frontier ends the search
    // and one above the limits goes back to the host, both before any level
    if (qlen0 < 0) {
        qlen0 = (int32_t)ctrl->qn_count;
        if (qlen0 == 0 || qlen0 > qlimit || qlen0 > side.cap) {
            if (w == 0 && t == 0) {
                ctrl->done = qlen0 == 0 ? 1 : 2;
                ctrl->qlen = qlen0;
                ctrl->level = lvl0;
                ctrl->steps = 0;
                ctrl->reached = 0;
                ctrl->levels = 0;
            }
            return;
        }
    }

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
    if (!grid_sync(sy, N, &s_epoch)) {
        if (t == 0) ctrl->err = 4;
        return;
    }
    int64_t cur_rn;  // edges of the frontier being expanded
    {
        // slot 2 is next reset during level 1, after every workgroup read it
        const int64_t rn = __hip_atomic_load(&sy->rn[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cur_rn = rn;
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
        // from the second level on, every frontier entry carries its row start,
        // degree and caller id, written by the workgroup that claimed it
        const bool from_side = step > 0;
        const int64_t* __restrict__ in_off = side.off[par];
        const int32_t* __restrict__ in_deg = side.deg[par];
        const int32_t* __restrict__ in_id = side.id[par];
        int64_t* __restrict__ out_off = side.off[par ^ 1];
        int32_t* __restrict__ out_deg = side.deg[par ^ 1];
        int32_t* __restrict__ out_id = side.id[par ^ 1];
        const int cs = step % 3;  // counters of this level
        // a level with many edges reads the target's bitmap word first and
        // claims only unset bits: on hub rows the claims of a bare atomicOr
        // would queue on a few bitmap lines
        const bool probe = cur_rn > kSmallProbeEdges;
        if (w == 0 && t == 0) {
            // the next level's counters were last read two barriers ago
            const int nx = (step + 1) % 3;
            sy->qn[nx] = 0;
            sy->rn[nx] = 0;
            sy->md[nx] = 0;
        }
        int64_t dsum = 0;
        int32_t dmax = 0;
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
                    if (from_side) {
                        a[m] = in_off[s0 + i];
                        d[m] = in_deg[s0 + i];
                        id[m] = in_id[s0 + i];
                    } else
                    {
                        const int32_t u = Q[s0 + i];
                        a[m] = off[u];
                        d[m] = (int32_t)(off[u + 1] - a[m]);
                        id[m] = orig ? orig[u] : u;
                    }
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
                uint32_t old[kSmallEPT];
                if (probe) {
#pragma unroll
                    for (int j = 0; j < kSmallEPT; ++j) old[j] = ok[j] ? vis[vv[j] >> 5] : ~0u;
#pragma unroll
                    for (int j = 0; j < kSmallEPT; ++j)
                        if (!(old[j] & (1u << (vv[j] & 31))))
                            old[j] = atomicOr(vis + (vv[j] >> 5), 1u << (vv[j] & 31));
                } else {
#pragma unroll
                    for (int j = 0; j < kSmallEPT; ++j) {
                        old[j] = ~0u;
                        if (ok[j]) old[j] = atomicOr(vis + (vv[j] >> 5), 1u << (vv[j] & 31));
                    }
                }
                bool win[kSmallEPT];
                uint64_t mask[kSmallEPT];
                uint32_t total = 0;
#pragma unroll
                for (int j = 0; j < kSmallEPT; ++j) {
                    win[j] = ok[j] && !(old[j] & (1u << (vv[j] & 31)));
                    mask[j] = __ballot(win[j]);
                    total += (uint32_t)__popcll(mask[j]);
                }
                int64_t va[kSmallEPT];
                int32_t vd[kSmallEPT], vi[kSmallEPT];
#pragma unroll
                for (int j = 0; j < kSmallEPT; ++j) {
                    va[j] = 0;
                    vd[j] = 0;
                    vi[j] = 0;
                    if (win[j]) {
                        const int32_t v = vv[j];
                        level[v] = lvl;
                        if (parent) parent[v] = uu[j];
                        va[j] = off[v];
                        vd[j] = (int32_t)(off[v + 1] - va[j]);
                        vi[j] = orig ? orig[v] : v;
                        atomicOr(vis_old + (v >> 5), 1u << (v & 31));
                    }
                    dsum += vd[j];
                    dmax = vd[j] > dmax ? vd[j] : dmax;
                }
                // one queue reservation per workgroup and tile
                if (__lane_id() == 0) s_wq[wave] = total;
                __syncthreads();
                if (t == 0) {
                    const uint32_t all = s_wq[0] + s_wq[1] + s_wq[2] + s_wq[3];
                    s_qbase = all ? atomicAdd(&sy->qn[cs], all) : 0u;
                }
                __syncthreads();
                if (total) {
                    uint32_t base = s_qbase;
                    for (int k = 0; k < wave; ++k) base += s_wq[k];
#pragma unroll
                    for (int j = 0; j < kSmallEPT; ++j) {
                        if (win[j]) {
                            const uint32_t pos = base + lanes_below(mask[j]);
                            if (pos < (uint32_t)V) {
                                Qn[pos] = vv[j];
                                if (pos < (uint32_t)side.cap) {
                                    out_off[pos] = va[j];
                                    out_deg[pos] = vd[j];
                                    out_id[pos] = vi[j];
                                }
                            } else {
                                ctrl->err = 5;
                            }
                        }
                        base += (uint32_t)__popcll(mask[j]);
                    }
                }
                __syncthreads();
            }
        }
        // the next frontier's edges and largest degree: one update per workgroup
        for (int o = 32; o >= 1; o >>= 1) {
            dsum += __shfl_xor(dsum, o, 64);
            const int32_t m2 = __shfl_xor(dmax, o, 64);
            dmax = m2 > dmax ? m2 : dmax;
        }
        if (__lane_id() == 0) {
            s_rs[wave] = dsum;
            s_rm[wave] = dmax;
        }
        __syncthreads();
        if (t == 0) {
            const int64_t rs = s_rs[0] + s_rs[1] + s_rs[2] + s_rs[3];
            int32_t rm = s_rm[0];
            for (int k = 1; k < kWG / 64; ++k) rm = s_rm[k] > rm ? s_rm[k] : rm;
            if (rs) atomicAdd(reinterpret_cast<unsigned long long*>(&sy->rn[cs]),
                              (unsigned long long)rs);
            if (rm) atomicMax(&sy->md[cs], rm);
        }
        if (!grid_sync(sy, N, &s_epoch)) {
            if (t == 0) ctrl->err = 4;
            code = 3;
            break;
        }
        const uint32_t qn = __hip_atomic_load(&sy->qn[cs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t rn = __hip_atomic_load(&sy->rn[cs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t md = __hip_atomic_load(&sy->md[cs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cur_rn = rn;
        ++step;
        ++lvl;
        reached += qn;
        if (qn == 0) {
            code = 1;
            break;
        }
        qlen = (int32_t)qn;
        par ^= 1;
        if ((int32_t)qn > qlimit || (int32_t)qn > side.cap || rn > rlimit || md > dlimit) {
            code = 2;
            break;
        }
    }
    if (t == 0 && my_edges)
        atomicAdd(reinterpret_cast<unsigned long long*>(&sy->edges), (unsigned long long)my_edges);
    if (w == 0 && t == 0 && code != 3) {
        ctrl->done = code;
        ctrl->qlen = qlen;
        ctrl->level = lvl;
        ctrl->steps = step;
        ctrl->reached = reached;
        ctrl->levels = code == 1 ? step - 1 : step;
    }
}

// The launch leaves its sync block as it found it (zero), so it needs no
// clearing of its own: the workgroup that leaves last (after every other has
// stopped reading the block) publishes the edge total and clears the block.
__global__ __launch_bounds__(kWG) void k_small_levels(
    int32_t V, const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const int32_t* __restrict__ orig, uint32_t* __restrict__ vis, uint32_t* __restrict__ vis_old,
    int32_t* __restrict__ Qa, int32_t* __restrict__ Qb, int32_t* __restrict__ level,
    int32_t* __restrict__ parent, SmallSync* __restrict__ sy, SmallSide side,
    Ctrl* __restrict__ ctrl, int32_t qlen0, int32_t lvl0, int32_t qlimit, int64_t rlimit, int32_t dlimit)
{
    small_levels_body(V, off, col, orig, vis, vis_old, Qa, Qb, level, parent, sy, side, ctrl, qlen0,
                      lvl0, qlimit, rlimit, dlimit);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t k =
            __hip_atomic_fetch_add(&sy->leave, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (k == gridDim.x - 1) {
            ctrl->r_total = sy->edges;
            sy->arrive = 0;
            for (int i = 0; i < 3; ++i) {
                sy->qn[i] = 0;
                sy->md[i] = 0;
                sy->rn[i] = 0;
            }
            sy->edges = 0;
            sy->leave = 0;
        }
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
                               int32_t* parent, SmallSync* sy, SmallSide side, Ctrl* ctrl,
                               int32_t qlen, int32_t lvl, int32_t qlimit, int64_t rlimit,
                               int32_t dlimit)
{
    // An ordinary launch: the grid (at most one workgroup per CU) is small
    // enough to be resident at once, and a cooperative launch would make
    // the runtime stop overlapping later kernels of other streams.
    hipLaunchKernelGGL(k_small_levels, dim3(grid), dim3(kWG), 0, s, V, off, col, orig, vis, vis_old,
                       Qa, Qb, level, parent, sy, side, ctrl, qlen, lvl, qlimit, rlimit, dlimit);
    return hipGetLastError();
}

}  // namespace bfsmi
