// Persistent multi-source levels for serving batches on deep graphs.
//
// On a grid-like graph a serving batch runs thousands of levels whose union
// frontier holds a few thousand vertices.  As separate launches each level
// is seven kernels (degree scan, expansion, front clear, finalize, advance),
// and on a busy GPU every one of them waits behind other graphs' kernels in
// the shared hardware queues.  This kernel runs up to max_levels such levels
// in one launch of a few dozen workgroups, one grid barrier per level.
//
// A level's work is the expansion of the paper's Section 3.4 on lane masks:
// per edge u -> v the lanes new to v are f = mask(u) & ~(seen[v] | next[v]),
// ORed into next[v] with a returning atomic, and the thread that turns
// next[v] from zero to non-zero appends v to the level's candidate list (so
// each vertex is listed once); then each candidate is finalized: new =
// next & ~seen, seen |= new, next = 0, and each new lane b gets depth
// level - lane_start[b] in its int16 result row (caller ids).
//
// The finalize of one level and the expansion of the next run in the same
// phase: a workgroup finalizes its slice of the candidate list and expands
// the vertices that got new lanes right away (degree prefix sum in LDS,
// edges mapped to threads by binary search in it), so only one grid barrier
// separates levels.  The next masks and candidate lists come in two
// parities (sn[].next and front[]; the found and Qb lists): a phase
// finalizes one parity while its expansion fills the other, so a thread
// that finalizes v writes only v's own words of the parity it reads, and
// the seen masks it updates are read elsewhere only as a filter (a stale
// seen lets a spurious candidate through, which its finalize then drops).
//
// The kernel starts from the state the level kernels leave (frontier in Qa,
// lane masks in front) and leaves the same state when it stops: the round's
// last phase only finalizes, writing the frontier to Qa and its masks to
// front.  The per-level bookkeeping is that of the separate launches
// (level, alive lanes, reached, done), so the host's round logic does not
// change.  The kernel stops when the batch is done, after max_levels levels,
// or before expanding a frontier whose candidates (an upper bound on it),
// their edges or their largest degree exceed the limits; the host then
// runs that level with the ordinary kernels.  The grid is small enough to
// be resident together; every barrier wait is bounded (ctrl->err on
// expiry).
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

constexpr int kMsPer = kMsStage / kWG;  // staged entries per thread

// Stages n frontier entries, kMsPer per thread (row start a, degree d, lane
// mask f): the exclusive prefix of the degrees goes to s_cum (s_cum[n] = R,
// the stage's edges), the masks to s_f and the row starts less the prefix to
// s_base.  Returns R (uniform).
__device__ __forceinline__ int32_t ms_stage(int32_t n, const int64_t (&a)[kMsPer],
                                            const int32_t (&d)[kMsPer],
                                            const uint64_t (&f)[kMsPer], int32_t* s_cum,
                                            uint64_t* s_f, int64_t* s_base, int32_t* s_wave)
{
    const int t = threadIdx.x;
    int32_t tot = 0;
#pragma unroll
    for (int m = 0; m < kMsPer; ++m) tot += d[m];
    int32_t R;
    int32_t c = wg_exclusive_scan<int32_t>(tot, &R, s_wave);
#pragma unroll
    for (int m = 0; m < kMsPer; ++m) {
        const int32_t i = t * kMsPer + m;
        if (i < n) {
            s_cum[i] = c;
            s_f[i] = f[m];
            s_base[i] = a[m] - c;
        }
        c += d[m];
    }
    if (t == 0) s_cum[n] = R;
    __syncthreads();
    return R;
}

// Expands a staged set of n entries with R edges: edges go to threads by
// binary search in s_cum, kMsTile per pass.  Per edge u -> x the lanes new
// to x are f = mask(u) & ~(seen[x] | next[x] | front[x]), ORed into x's
// marks of parity tp (0: sn[x].next, 1: front[x]) with a returning atomic;
// the thread that turns those marks from zero to non-zero appends x to list
// (so x is listed once per level) and adds x's degree to the bounds rsum,
// rmax on the next frontier's edges.
__device__ __forceinline__ void ms_expand_staged(
    int32_t n, int32_t R, int32_t V, const int64_t* __restrict__ off,
    const int32_t* __restrict__ col, SeenNext* __restrict__ sn, uint64_t* __restrict__ front,
    int tp, int32_t* __restrict__ list, uint32_t* __restrict__ list_n, Ctrl* __restrict__ ctrl,
    const int32_t* s_cum, const uint64_t* s_f, const int64_t* s_base, uint16_t* s_map,
    int64_t& rsum, int32_t& rmax)
{
    const int t = threadIdx.x;
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
        // stale masks only let more threads issue the atomic
#pragma unroll
        for (int j = 0; j < kMsEPT; ++j) {
            have[j] = ~0ull;
            if (fm[j]) {
                const SeenNext p = sn[vv[j]];
                have[j] = p.seen | p.next | front[vv[j]];
            }
        }
        bool first[kMsEPT];
#pragma unroll
        for (int j = 0; j < kMsEPT; ++j) {
            const uint64_t nb = fm[j] & ~have[j];
            first[j] = false;
            if (nb) {
                uint64_t* mk = tp ? front + vv[j] : &sn[vv[j]].next;
                const uint64_t old =
                    __hip_atomic_fetch_or(mk, nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
            if (__lane_id() == 0) base = atomicAdd(list_n, total);
            base = __shfl(base, 0, 64);
#pragma unroll
            for (int j = 0; j < kMsEPT; ++j) {
                if (first[j]) {
                    const uint32_t pos = base + lanes_below(mask[j]);
                    if (pos < (uint32_t)V) list[pos] = vv[j];
                    else ctrl->err = 7;
                    const int32_t dv = (int32_t)(off[vv[j] + 1] - off[vv[j]]);
                    rsum += dv;
                    rmax = dv > rmax ? dv : rmax;
                }
                base += (uint32_t)__popcll(mask[j]);
            }
        }
        __syncthreads();
    }
}

// A phase's totals, one set of atomics per wave (alive: one per workgroup).
__device__ __forceinline__ void ms_phase_totals(MsSync* __restrict__ sy, int cs, uint64_t alive,
                                                uint32_t qcnt, int64_t rsum, int32_t rmax,
                                                uint64_t* s_alive)
{
    for (int o = 32; o >= 1; o >>= 1) {
        alive |= __shfl_xor(alive, o, 64);
        qcnt += __shfl_xor(qcnt, o, 64);
        rsum += __shfl_xor(rsum, o, 64);
        const int32_t m2 = __shfl_xor(rmax, o, 64);
        rmax = m2 > rmax ? m2 : rmax;
    }
    if (__lane_id() == 0) {
        s_alive[threadIdx.x >> 6] = alive;
        if (qcnt) atomicAdd(&sy->qn[cs], qcnt);
        if (rsum) atomicAdd(reinterpret_cast<unsigned long long*>(&sy->rn[cs]),
                            (unsigned long long)rsum);
        if (rmax) atomicMax(&sy->md[cs], rmax);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0;
        for (int k = 0; k < kWG / 64; ++k) a |= s_alive[k];
        if (a) atomicOr(reinterpret_cast<unsigned long long*>(&sy->alive[cs]),
                        (unsigned long long)a);
    }
}

// The levels; every workgroup returns from it exactly once.
__device__ __forceinline__ void ms_levels_body(
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
    if (max_levels < 1 || qlen0 > qlimit || ms_load(&sy->rn[2]) > rlimit ||
        ms_load(&sy->md[2]) > dlimit)
        return;  // no level run: ctrl->steps stays 0, the rest of ctrl unchanged

    // ---- phase 0: expand the entry frontier (Qa, lane masks in front, which
    // are cleared) into marks 0 (sn.next), candidates into list 0 (found)
    {
        const int64_t k0 = (int64_t)qlen0 * w / N, k1 = (int64_t)qlen0 * (w + 1) / N;
        int64_t rsum = 0;
        int32_t rmax = 0;
        for (int64_t s0 = k0; s0 < k1; s0 += kMsStage) {
            const int32_t n = (int32_t)(k1 - s0 < kMsStage ? k1 - s0 : kMsStage);
            int64_t a[kMsPer];
            int32_t d[kMsPer];
            uint64_t f[kMsPer];
#pragma unroll
            for (int m = 0; m < kMsPer; ++m) {
                const int32_t i = t * kMsPer + m;
                a[m] = 0;
                d[m] = 0;
                f[m] = 0;
                if (i < n) {
                    const int32_t u = Qa[s0 + i];
                    f[m] = front[u];
                    front[u] = 0;  // this workgroup is the only reader of u's mask
                    a[m] = off[u];
                    d[m] = f[m] ? (int32_t)(off[u + 1] - a[m]) : 0;
                }
            }
            const int32_t R = ms_stage(n, a, d, f, s_cum, s_f, s_base, s_wave);
            ms_expand_staged(n, R, V, off, col, sn, front, 0, found, &sy->fn[0], ctrl, s_cum, s_f,
                             s_base, s_map, rsum, rmax);
        }
        ms_phase_totals(sy, 0, 0ull, 0u, rsum, rmax, s_alive);
    }
    if (!ms_grid_sync(sy, N, &s_epoch)) {
        if (t == 0) ctrl->err = 6;
        return;
    }

    // ---- phase j >= 1: finalize the candidates of expansion j (found at
    // depth level lvl0 + j - 1) and, unless this is the round's last phase,
    // expand the new frontier at once (expansion j + 1).  Marks and lists
    // alternate by parity: phase j reads those of parity (j - 1) & 1 (every
    // candidate is listed there once, and its marks are cleared here) while
    // its expansion fills those of parity j & 1, cleared in phase j - 1.
    uint64_t last_alive = 0;
    int64_t reached = 0;
    int32_t levels = 0, qlen = 0, steps = 0;
    bool done = ms_load(&ctrl->err) != 0 || ms_load(&ctrl->overflow) != 0;
    bool failed = false;
    for (int32_t j = 1; !done; ++j) {
        const int pc = (j - 1) % 3, cs = j % 3;
        uint32_t fn = ms_load(&sy->fn[pc]);
        if (fn > (uint32_t)V) fn = (uint32_t)V;  // a vertex is listed at most once
        const bool last = j >= max_levels || (int32_t)fn > qlimit || ms_load(&sy->rn[pc]) > rlimit ||
                          ms_load(&sy->md[pc]) > dlimit;
        if (w == 0 && t == 0) {
            // slot (j + 1) % 3 was last read before the previous barrier
            const int nx = (j + 1) % 3;
            sy->fn[nx] = 0;
            sy->qn[nx] = 0;
            sy->md[nx] = 0;
            sy->rn[nx] = 0;
            sy->alive[nx] = 0;
        }
        const int sp = (j - 1) & 1;
        const int32_t* __restrict__ Lin = sp ? Qb : found;
        int32_t* __restrict__ Lout = sp ? found : Qb;
        const int32_t dl = lvl0 + j - 1;
        uint64_t alive = 0;
        uint32_t qcnt = 0;
        int64_t rsum = 0;
        int32_t rmax = 0;
        const int64_t f0 = (int64_t)fn * w / N, f1 = (int64_t)fn * (w + 1) / N;
        for (int64_t s0 = f0; s0 < f1; s0 += kMsStage) {
            const int32_t n = (int32_t)(f1 - s0 < kMsStage ? f1 - s0 : kMsStage);
            int64_t a[kMsPer];
            int32_t d[kMsPer], vx[kMsPer];
            uint64_t nw[kMsPer];
#pragma unroll
            for (int m = 0; m < kMsPer; ++m) {
                const int32_t i = t * kMsPer + m;
                a[m] = 0;
                d[m] = 0;
                nw[m] = 0;
                vx[m] = 0;
                if (i < n) {
                    const int32_t v = Lin[s0 + i];
                    if ((uint32_t)v >= (uint32_t)V) {
                        ctrl->err = 9;
                        continue;
                    }
                    vx[m] = v;
                    const SeenNext p = sn[v];
                    const uint64_t mk = sp ? front[v] : p.next;
                    a[m] = off[v];
                    const int64_t a1 = off[v + 1];
                    nw[m] = mk & ~p.seen;
                    // v's own slot only: other threads OR into the marks of
                    // the other parity meanwhile
                    if (sp) {
                        if (nw[m]) sn[v].seen = p.seen | nw[m];
                        front[v] = last ? nw[m] : 0ull;
                    } else {
                        sn[v] = SeenNext{p.seen | nw[m], 0ull};
                        if (last) front[v] = nw[m];
                    }
                    if (nw[m]) {
                        const int32_t vo = orig ? orig[v] : v;
                        for (uint64_t b = nw[m]; b; b &= b - 1) {
                            const int k = __builtin_ctzll(b);
                            const int32_t dd = dl - s_start[k];
                            if (dd > 32767) ctrl->overflow = 1;
                            else if (s_out[k]) s_out[k][vo] = (int16_t)dd;  // null: retired lane
                        }
                        alive |= nw[m];
                        d[m] = (int32_t)(a1 - a[m]);
                    }
                }
            }
            if (last) {
                // the new frontier goes to Qa, the form the level kernels take
                uint64_t mask[kMsPer];
                uint32_t total = 0;
#pragma unroll
                for (int m = 0; m < kMsPer; ++m) {
                    mask[m] = __ballot(nw[m] != 0);
                    total += (uint32_t)__popcll(mask[m]);
                }
                if (total) {
                    uint32_t base = 0;
                    if (__lane_id() == 0) base = atomicAdd(&sy->qn[cs], total);
                    base = __shfl(base, 0, 64);
#pragma unroll
                    for (int m = 0; m < kMsPer; ++m) {
                        if (nw[m]) {
                            const uint32_t pos = base + lanes_below(mask[m]);
                            if (pos < (uint32_t)V) Qa[pos] = vx[m];
                            else ctrl->err = 8;
                        }
                        base += (uint32_t)__popcll(mask[m]);
                    }
                }
            } else {
#pragma unroll
                for (int m = 0; m < kMsPer; ++m) qcnt += nw[m] ? 1u : 0u;
                const int32_t R = ms_stage(n, a, d, nw, s_cum, s_f, s_base, s_wave);
                ms_expand_staged(n, R, V, off, col, sn, front, j & 1, Lout, &sy->fn[cs], ctrl,
                                 s_cum, s_f, s_base, s_map, rsum, rmax);
            }
        }
        ms_phase_totals(sy, cs, alive, qcnt, rsum, rmax, s_alive);
        if (!ms_grid_sync(sy, N, &s_epoch)) {
            failed = true;
            break;
        }
        // ---- the level's bookkeeping (as the separate advance does)
        const uint32_t qn = ms_load(&sy->qn[cs]);
        last_alive = ms_load(&sy->alive[cs]);
        const int32_t ovf = ms_load(&ctrl->overflow);
        const int32_t err = ms_load(&ctrl->err);
        steps = j;
        reached += qn;
        if (qn) ++levels;
        qlen = (int32_t)qn;
        if (qn == 0 || qn > (uint32_t)V || ovf || err) {
            if (qn > (uint32_t)V && t == 0) ctrl->err = 8;
            done = true;
        } else if (last) {
            break;
        }
    }
    if (failed) {
        if (t == 0) ctrl->err = 6;
        return;
    }
    if (w == 0 && t == 0) {
        ctrl->steps = steps;
        if (steps > 0) {
            ctrl->last_alive = last_alive;
            ctrl->alive = 0;
            ctrl->reached += reached;
            ctrl->levels += levels;
            ctrl->level = lvl0 + steps;
            ctrl->qlen = qlen;
            ctrl->qn_count = 0;
            ctrl->sparse = qlen <= ctrl->sparse_limit;
            ctrl->done = done ? 1 : 0;
        }
    }
}

// The launch leaves its sync block as it found it (zero) and mirrors the
// control block into pinned host memory, so a round needs no clearing and
// no copy of its own: the workgroup that leaves last (after every other
// has stopped reading the sync block) does both.
static_assert(sizeof(Ctrl) % sizeof(int4) == 0, "the control block is copied in 16-byte words");

__global__ __launch_bounds__(kWG) void k_ms_small_levels(
    int32_t V, const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const int32_t* __restrict__ orig, SeenNext* __restrict__ sn, uint64_t* __restrict__ front,
    int32_t* __restrict__ Qa, int32_t* __restrict__ Qb, int32_t* __restrict__ found,
    int16_t* const* __restrict__ lane_out, const int32_t* __restrict__ lane_start,
    MsSync* __restrict__ sy, Ctrl* __restrict__ ctrl, Ctrl* __restrict__ h_ctrl,
    int32_t max_levels, int32_t qlimit, int64_t rlimit, int32_t dlimit)
{
    ms_levels_body(V, off, col, orig, sn, front, Qa, Qb, found, lane_out, lane_start, sy, ctrl,
                   max_levels, qlimit, rlimit, dlimit);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t k =
            __hip_atomic_fetch_add(&sy->leave, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (k == gridDim.x - 1) {
            sy->arrive = 0;
            for (int i = 0; i < 3; ++i) {
                sy->fn[i] = 0;
                sy->qn[i] = 0;
                sy->md[i] = 0;
                sy->rn[i] = 0;
                sy->alive[i] = 0;
            }
            sy->leave = 0;
            if (h_ctrl) {
                const int4* src = reinterpret_cast<const int4*>(ctrl);
                int4* dst = reinterpret_cast<int4*>(h_ctrl);
                for (int i = 0; i < (int)(sizeof(Ctrl) / sizeof(int4)); ++i) dst[i] = src[i];
                __threadfence_system();
            }
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
                                  MsSync* sy, Ctrl* ctrl, Ctrl* h_ctrl, int32_t max_levels,
                                  int32_t qlimit, int64_t rlimit, int32_t dlimit)
{
    // an ordinary launch of a grid small enough to be resident at once
    hipLaunchKernelGGL(k_ms_small_levels, dim3(grid), dim3(kWG), 0, s, V, off, col, orig, sn, front,
                       Qa, Qb, found, lane_out, lane_start, sy, ctrl, h_ctrl, max_levels, qlimit,
                       rlimit, dlimit);
    return hipGetLastError();
}

}  // namespace bfsmi
