// Persistent multi-source levels for serving batches on deep graphs.
//
// On a grid-like graph a serving batch runs thousands of levels whose union
// frontier holds a few thousand vertices.  As separate launches each level
// is seven kernels (degree scan, expansion, front clear, finalize, advance),
// and on a busy GPU every one of them waits behind other graphs' kernels in
// the shared hardware queues.  This kernel runs up to max_levels such levels
// in one launch of a few dozen workgroups, two grid barriers per level:
//   expand   : each workgroup takes an equal slice of the union frontier,
//              stages its entries (front mask, row start, prefix sum of
//              degrees) in LDS, clears their front masks, and maps the
//              slice's edges to threads by binary search in the prefix sum
//              (Section 3.4 within the slice).  Per edge u -> v the lanes
//              new to v are f = front[u] & ~(seen[v] | next[v]); they are
//              ORed into next[v] with a returning atomic, and the thread
//              that turns next[v] from zero to non-zero appends v to the
//              level's found list (so each vertex is listed once);
//   finalize : workgroups split the found list: new = next & ~seen, seen |=
//              new, next = 0, front = new, v appended to the next queue, and
//              each new lane b gets depth level - lane_start[b] in its
//              int16 result row (caller ids).
// The per-level bookkeeping is that of the separate launches (level, alive
// lanes, reached, done), so the host's round logic does not change.  The
// kernel stops when the batch is done, after max_levels levels, or before
// a level whose frontier, edge count or largest degree exceeds the limits
// (the host then runs that level with the ordinary kernels).  The final
// frontier is left in Qa.  The grid is small enough to be resident
// together; every barrier wait is bounded (ctrl->err on expiry).
#include "bfs_internal.h"
#include "wave_ops.h"

namespace bfsmi {

constexpr int kMsStage = 1024;           // frontier entries staged per pass
constexpr int kMsEPT = 4;                // edges per thread per pass
constexpr int kMsTile = kWG * kMsEPT;
constexpr uint32_t kMsSpinCap = 1u << 24;

// Grid-wide barrier on a counter that only grows (zeroed before each
// launch): barrier number k is passed once it reaches k * nwg.  Thread 0 of
// each workgroup arrives with a release add and waits with relaxed loads
// followed by an acquire fence.
__device__ __forceinline__ bool ms_grid_sync(MsSync* sy, uint32_t nwg, uint32_t* s_ep)
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
            if (++spins > kMsSpinCap) {
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

template <typename T>
__device__ __forceinline__ T ms_load(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kWG) void k_ms_small_levels(
    int32_t V, const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const int32_t* __restrict__ orig, SeenNext* __restrict__ sn, uint64_t* __restrict__ front,
    int32_t* __restrict__ Qa, int32_t* __restrict__ Qb, int32_t* __restrict__ found,
    int16_t* const* __restrict__ lane_out, const int32_t* __restrict__ lane_start,
    MsSync* __restrict__ sy, Ctrl* __restrict__ ctrl, int32_t max_levels, int32_t qlimit,
    int64_t rlimit, int32_t dlimit)
{
    __shared__ int32_t s_cum[kMsStage + 1];
    __shared__ uint64_t s_f[kMsStage];
    __shared__ int64_t s_base[kMsStage];
    __shared__ uint16_t s_map[kMsTile];
    __shared__ int32_t s_wave[kWG / 64];
    __shared__ int16_t* s_out[64];
    __shared__ int32_t s_start[64];
    __shared__ uint64_t s_alive[kWG / 64];
    __shared__ uint32_t s_epoch;
    const uint32_t N = gridDim.x;
    const uint32_t w = blockIdx.x;
    const int t = threadIdx.x;
    if (t == 0) s_epoch = 0;
    if (t < 64) {
        s_out[t] = lane_out[t];
        s_start[t] = lane_start[t];
    }
    if (w == 0 && t == 0) ctrl->steps = 0;  // levels run, set again at the end
    if (ctrl->done) return;  // uniform (rewritten only after the last barrier): nothing to run
    const int32_t qlen0 = ctrl->qlen;
    const int32_t lvl0 = ctrl->level;

    // limits of the first frontier, before anything is changed
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
    if (!ms_grid_sync(sy, N, &s_epoch)) {
        if (t == 0) ctrl->err = 6;
        return;
    }
    if (qlen0 > qlimit || ms_load(&sy->rn[2]) > rlimit || ms_load(&sy->md[2]) > dlimit)
        return;  // no level run: ctrl->steps stays 0, the rest of ctrl unchanged

    int32_t qlen = qlen0, lvl = lvl0, step = 0, par = 0;
    int64_t reached = 0;
    int32_t levels = 0;
    uint64_t last_alive = 0;
    bool done = false, failed = false;
    while (step < max_levels) {
        const int32_t* __restrict__ Q = par ? Qb : Qa;
        int32_t* __restrict__ Qn = par ? Qa : Qb;
        const int cs = step % 3;
        if (w == 0 && t == 0) {
            // the next level's slot was last read before the previous level's
            // first barrier
            const int nx = (step + 1) % 3;
            sy->fn[nx] = 0;
            sy->qn[nx] = 0;
            sy->md[nx] = 0;
            sy->rn[nx] = 0;
            sy->alive[nx] = 0;
        }
        // ---- expand
        const int64_t k0 = (int64_t)qlen * w / N, k1 = (int64_t)qlen * (w + 1) / N;
        for (int64_t s0 = k0; s0 < k1; s0 += kMsStage) {
            const int32_t n = (int32_t)(k1 - s0 < kMsStage ? k1 - s0 : kMsStage);
            int64_t a[4];
            int32_t d[4];
            uint64_t f[4];
            int32_t tot = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int32_t i = t * 4 + m;
                a[m] = 0;
                d[m] = 0;
                f[m] = 0;
                if (i < n) {
                    const int32_t u = Q[s0 + i];
                    f[m] = front[u];
                    front[u] = 0;  // this workgroup is the only reader of u's mask
                    a[m] = off[u];
                    d[m] = f[m] ? (int32_t)(off[u + 1] - a[m]) : 0;
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
                    s_f[i] = f[m];
                    s_base[i] = a[m] - c;
                }
                c += d[m];
            }
            if (t == 0) s_cum[n] = R;
            __syncthreads();
            for (int32_t e0 = 0; e0 < R; e0 += kMsTile) {
                const int32_t n_e = R - e0 < kMsTile ? R - e0 : kMsTile;
                const int32_t sl0 = e0 + t * kMsEPT;
                if (t * kMsEPT < n_e) {
                    int32_t lo = 0;
                    for (int32_t st = 1 << (31 - __builtin_clz(n)); st > 0; st >>= 1) {
                        const int32_t x = lo + st;
                        if (x < n && s_cum[x] <= sl0) lo = x;
                    }
                    int32_t i = lo;
#pragma unroll
                    for (int j = 0; j < kMsEPT; ++j) {
                        const int32_t sl = sl0 + j;
                        if (sl - e0 < n_e) {
                            while (i + 1 < n && s_cum[i + 1] <= sl) ++i;
                            s_map[sl - e0] = (uint16_t)i;
                        }
                    }
                }
                __syncthreads();
                int32_t vv[kMsEPT];
                uint64_t fm[kMsEPT], have[kMsEPT];
#pragma unroll
                for (int j = 0; j < kMsEPT; ++j) {
                    const int32_t sl = t + j * kWG;
                    const bool ok = sl < n_e;
                    const int32_t sc = ok ? sl : n_e - 1;
                    const int32_t i = s_map[sc];
                    fm[j] = ok ? s_f[i] : 0ull;
                    vv[j] = col[s_base[i] + e0 + sc];
                }
#pragma unroll
                for (int j = 0; j < kMsEPT; ++j) {
                    have[j] = ~0ull;
                    if (fm[j]) {
                        const SeenNext p = sn[vv[j]];
                        have[j] = p.seen | p.next;
                    }
                }
                bool first[kMsEPT];
#pragma unroll
                for (int j = 0; j < kMsEPT; ++j) {
                    const uint64_t nb = fm[j] & ~have[j];
                    first[j] = false;
                    if (nb) {
                        const uint64_t old = __hip_atomic_fetch_or(&sn[vv[j]].next, nb,
                                                                   __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT);
                        first[j] = old == 0;
                    }
                }
                uint64_t mask[kMsEPT];
                uint32_t total = 0;
#pragma unroll
                for (int j = 0; j < kMsEPT; ++j) {
                    mask[j] = __ballot(first[j]);
                    total += (uint32_t)__popcll(mask[j]);
                }
                if (total) {
                    uint32_t base = 0;
                    if (__lane_id() == 0) base = atomicAdd(&sy->fn[cs], total);
                    base = __shfl(base, 0, 64);
#pragma unroll
                    for (int j = 0; j < kMsEPT; ++j) {
                        if (first[j]) {
                            const uint32_t pos = base + lanes_below(mask[j]);
                            if (pos < (uint32_t)V) found[pos] = vv[j];
                            else ctrl->err = 7;
                        }
                        base += (uint32_t)__popcll(mask[j]);
                    }
                }
                __syncthreads();
            }
        }
        if (!ms_grid_sync(sy, N, &s_epoch)) {
            failed = true;
            break;
        }
        // ---- finalize (a vertex is listed at most once, so fn <= V)
        uint32_t fn = ms_load(&sy->fn[cs]);
        if (fn > (uint32_t)V) fn = (uint32_t)V;
        const int64_t f0 = (int64_t)fn * w / N, f1 = (int64_t)fn * (w + 1) / N;
        uint64_t alive = 0;
        int64_t dsum = 0;
        int32_t dmax = 0;
        for (int64_t i0 = f0; i0 < f1; i0 += kWG) {
            const int64_t i = i0 + t;
            uint64_t nw = 0;
            int32_t v = 0;
            if (i < f1) {
                v = found[i];
                const SeenNext p = sn[v];
                nw = p.next & ~p.seen;
                sn[v] = SeenNext{p.seen | nw, 0ull};
                front[v] = nw;
            }
            const bool app = nw != 0;
            const uint64_t m = __ballot(app);
            uint32_t base = 0;
            if (m && __lane_id() == 0) base = atomicAdd(&sy->qn[cs], (uint32_t)__popcll(m));
            base = __shfl(base, 0, 64);
            if (app) {
                const uint32_t pos = base + lanes_below(m);
                if (pos < (uint32_t)V) Qn[pos] = v;
                else ctrl->err = 8;
                const int32_t vo = orig ? orig[v] : v;
                for (uint64_t b = nw; b; b &= b - 1) {
                    const int k = __builtin_ctzll(b);
                    const int32_t dd = lvl - s_start[k];
                    if (dd > 32767) ctrl->overflow = 1;
                    else if (s_out[k]) s_out[k][vo] = (int16_t)dd;  // null: retired lane
                }
                alive |= nw;
                const int32_t dv = (int32_t)(off[v + 1] - off[v]);
                dsum += dv;
                dmax = dv > dmax ? dv : dmax;
            }
        }
        for (int o = 32; o >= 1; o >>= 1) {
            alive |= __shfl_xor(alive, o, 64);
            dsum += __shfl_xor(dsum, o, 64);
            const int32_t m2 = __shfl_xor(dmax, o, 64);
            dmax = m2 > dmax ? m2 : dmax;
        }
        if (__lane_id() == 0) {
            s_alive[t >> 6] = alive;
            if (dsum) atomicAdd(reinterpret_cast<unsigned long long*>(&sy->rn[cs]),
                                (unsigned long long)dsum);
            if (dmax) atomicMax(&sy->md[cs], dmax);
        }
        __syncthreads();
        if (t == 0) {
            uint64_t a = 0;
            for (int k = 0; k < kWG / 64; ++k) a |= s_alive[k];
            if (a) atomicOr(reinterpret_cast<unsigned long long*>(&sy->alive[cs]),
                            (unsigned long long)a);
        }
        if (!ms_grid_sync(sy, N, &s_epoch)) {
            failed = true;
            break;
        }
        // ---- the level's bookkeeping (as the separate advance does)
        const uint32_t qn = ms_load(&sy->qn[cs]);
        last_alive = ms_load(&sy->alive[cs]);
        const int64_t rn = ms_load(&sy->rn[cs]);
        const int32_t md = ms_load(&sy->md[cs]);
        const int32_t ovf = ms_load(&ctrl->overflow);
        const int32_t err = ms_load(&ctrl->err);
        ++step;
        ++lvl;
        reached += qn;
        if (qn) ++levels;
        qlen = (int32_t)qn;
        par ^= 1;
        if (qn == 0 || qn > (uint32_t)V || ovf || err) {
            if (qn > (uint32_t)V && t == 0) ctrl->err = 8;
            done = true;
            break;
        }
        if ((int32_t)qn > qlimit || rn > rlimit || md > dlimit) break;
    }
    if (failed) {
        if (t == 0) ctrl->err = 6;
        return;
    }
    // the frontier goes back to Qa (the ordinary level kernels start there)
    if (par) {
        for (int64_t k = (int64_t)w * kWG + t; k < qlen; k += (int64_t)N * kWG) Qa[k] = Qb[k];
    }
    if (w == 0 && t == 0) {
        ctrl->steps = step;
        if (step > 0) {
            ctrl->last_alive = last_alive;
            ctrl->alive = 0;
            ctrl->reached += reached;
            ctrl->levels += levels;
            ctrl->level = lvl;
            ctrl->qlen = qlen;
            ctrl->qn_count = 0;
            ctrl->sparse = qlen <= ctrl->sparse_limit;
            ctrl->done = done ? 1 : 0;
        }
    }
}

int ms_small_loop_blocks()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ms_small_levels, kWG, 0) != hipSuccess)
        return 0;
    return n;
}

hipError_t launch_ms_small_levels(hipStream_t s, int grid, int32_t V, const int64_t* off,
                                  const int32_t* col, const int32_t* orig, SeenNext* sn,
                                  uint64_t* front, int32_t* Qa, int32_t* Qb, int32_t* found,
                                  int16_t* const* lane_out, const int32_t* lane_start,
                                  MsSync* sy, Ctrl* ctrl, int32_t max_levels, int32_t qlimit,
                                  int64_t rlimit, int32_t dlimit)
{
    // an ordinary launch of a grid small enough to be resident at once
    hipLaunchKernelGGL(k_ms_small_levels, dim3(grid), dim3(kWG), 0, s, V, off, col, orig, sn, front,
                       Qa, Qb, found, lane_out, lane_start, sy, ctrl, max_levels, qlimit, rlimit,
                       dlimit);
    return hipGetLastError();
}

}  // namespace bfsmi
