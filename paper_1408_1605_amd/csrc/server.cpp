// C ABI: serving (bfs_server_*, bfs_submit, bfs_poll).
//
// A worker thread owns every device launch.  Each registered graph has its
// own stream; while a graph has queries, it runs a multi-source batch (the
// kernels of msbfs.hip) whose 64 lanes are filled from the graph's queue at
// level boundaries: a query joins a free lane with its root at depth 0 and
// lane_start = level - 1, the batch keeps expanding the union frontier of
// all live lanes, and a lane retires at the first level that finds nothing
// for it; its seen bits are then cleared before the lane is reused.  The
// batch state and each query's int16 result live in the caller's device
// arena; a graph's batch starts only when its state fits the free arena
// (admission by HBM budget), and a query joins only when its result fits.
// Different graphs' batches run concurrently on their streams.
//
// Admission into a running batch follows the graph's depth.  On a
// small-world graph every search touches most edges at its one or two
// widest levels; lanes that start together share those levels in one
// expansion, while a lane that joins later pays them again on its own.  So
// on such a graph new queries join only at the start of a batch (waves).
// On a deep graph (lanes live for many cheap levels) and on a small graph
// a query joins at the next level boundary (continuous batching).  The
// depth is learnt per graph from the lifetimes of retired lanes.
//
// The worker takes the server lock only to move queries and arena blocks;
// its HIP calls run unlocked, so submit/poll never wait behind a launch.
//
// Every graph has its own stream, and HIP maps a process's streams onto a
// few hardware queues (GPU_MAX_HW_QUEUES, 4 by default): a deep graph's
// round then waits behind other graphs' kernels in its queue.  Serving
// processes run with 8 hardware queues (the benchmark sets it before HIP
// starts); that, with the persistent rounds' wider limits, roughly halves
// the deep graphs' time per level in a mixed pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

namespace bfsmi {

static int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// First-fit allocator over the caller's arena (offsets, 256-byte aligned).
class Arena {
public:
    void init(char* base, size_t size)
    {
        base_ = base;
        size_ = size / 256 * 256;
        free_.clear();
        if (size_) free_[0] = size_;
    }
    char* alloc(size_t bytes)
    {
        bytes = align256(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_[off] = bytes;
                in_use_ += bytes;
                peak_ = std::max(peak_, in_use_);
                return base_ + off;
            }
        }
        return nullptr;
    }
    void release(char* p)
    {
        if (!p) return;
        const size_t off = (size_t)(p - base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t len = u->second;
        used_.erase(u);
        in_use_ -= len;
        size_t start = off;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + len) {
            len += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(off);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == off) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    size_t size() const { return size_; }
    size_t peak() const { return peak_; }

private:
    size_t in_use_ = 0, peak_ = 0;
    char* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;
    std::unordered_map<size_t, size_t> used_;
};

struct SrvQuery {
    int32_t graph = 0;
    int32_t root = 0;
    int64_t submit_ns = 0, admit_ns = 0, done_ns = 0;
    int32_t lanes = 0;
    int32_t levels = 0;         // depth + 1, from the lane's lifetime
    int16_t* result = nullptr;  // arena, int16[V]
    int state = 0;              // 0 pending, 1 running, 2 done, 3 failed
    int err = 0;
};

// Device state of one running batch, carved from one arena block.
struct SrvBatch {
    char* mem = nullptr;
    SeenNext* sn = nullptr;  // seen and next masks, side by side
    uint64_t* front = nullptr;
    uint32_t* touched = nullptr;
    int32_t* q[2] = {nullptr, nullptr};
    int32_t* deg = nullptr;
    int64_t* rowstart = nullptr;
    int32_t* suid = nullptr;
    int64_t* cumul = nullptr;
    int64_t* bsum = nullptr;
    int32_t* tile_k = nullptr;
    Ctrl* ctrl = nullptr;
    int16_t** lane_out = nullptr;  // device table of 64 result pointers
    int32_t* lane_start = nullptr; // device int32[64]
    int32_t* join = nullptr;       // device int32[128] (root, lane) pairs
    MsSync* msync = nullptr;       // persistent levels: barrier and counters
    uint64_t lane_ticket[64] = {};
    int64_t lane_age[64] = {};     // levels launched since the lane joined
    uint64_t active = 0;
    int parity = 0;                // stays 0: every replay runs an even number of levels
    bool in_flight = false;
    bool persist = false;          // the round in flight is the persistent kernel
    bool big_next = false;         // it stopped before a large level: next round uses the graphs
    int round_levels = 0;          // levels of the round in flight
    int64_t idle_since = 0;        // steady-clock ns when the batch went idle (0: busy)
    hipGraphExec_t round[3] = {nullptr, nullptr, nullptr};  // 2, 8, 32 levels
};

constexpr int kRoundLevels[3] = {2, 8, 32};
constexpr int64_t kIdleKeepNs = 100 * 1000 * 1000;  // idle batches kept 100 ms
constexpr double kDeepLife = 48.0;                  // lanes living longer: continuous joins
constexpr int32_t kSmallV = 1 << 16;                // graphs this small: continuous joins
// Persistent rounds on deep graphs (msloop.hip): workgroups per launch, at
// most this many launches in flight (all their workgroups must be resident
// together), and the level sizes they take.
constexpr int kMsGrid = 32;
constexpr int kMaxPersist = 8;
constexpr int32_t kMsQLimit = 1 << 17;
constexpr int64_t kMsRLimit = 1 << 19;
constexpr int32_t kMsDLimit = 8192;

struct SrvGraph {
    bfs_graph* g = nullptr;
    size_t state_bytes = 0;
    std::deque<uint64_t> pending;
    SrvBatch* batch = nullptr;     // worker thread only
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev = nullptr;  // round start / end (timing events)
    hipEvent_t ev_stage = nullptr;  // after staging copies that no round event follows
    bool stage_pending = false;     // ev_stage recorded and not yet seen complete
    Ctrl* h_ctrl = nullptr;        // pinned
    int16_t** h_lane_out = nullptr;  // pinned staging for the lane table
    int32_t* h_join = nullptr;     // pinned staging for joins
    double life = 0.0;             // smoothed lane lifetime in levels
    int64_t life_n = 0;
};

// What one worker step launches for a graph, decided under the lock and
// carried out without it.
struct StepPlan {
    bool fresh = false;      // batch created: reset its state, capture its rounds
    bool reset = false;      // device error or depth overflow: reset all lanes
    uint64_t clear = 0;      // retired lanes whose seen bits are cleared
    int n_join = 0;          // staged in h_join / h_lane_out
    bool table = false;      // upload h_lane_out (lanes retired or joined)
    int16_t* fill[64] = {};  // result buffers of the joining lanes
    int round = -1;          // round to replay, -1 none
    bool persist = false;    // run the round's levels in the persistent kernel
    bool release = false;    // idle too long: give the batch's memory back
};

static size_t batch_state_bytes(const bfs_graph* g)
{
    const size_t V = (size_t)g->V;
    const size_t nblk = (V + kScanChunk - 1) / kScanChunk;
    const size_t ntile = (size_t)((g->nnz + kMinTile - 1) / kMinTile);
    size_t b = 0;
    b += align256(V * 16) + 2 * align256(V * 8);  // seen+next, front, rowstart
    b += align256((V + 31) / 32 * 4);
    b += 4 * align256(V * 4);
    b += align256((V + 1) * 8);
    b += align256((nblk + 1) * 8);
    b += align256((ntile + 2) * 4);
    b += align256(sizeof(Ctrl)) + align256(64 * 8) + align256(64 * 4) + align256(128 * 4);
    b += align256(sizeof(MsSync));
    return b;
}

}  // namespace bfsmi

using namespace bfsmi;

struct bfs_server {
    Arena arena;
    int device = 0;
    bfs_server_config cfg{64, 8, 0};
    std::mutex mu;
    std::condition_variable cv;       // wakes the worker
    std::condition_variable idle_cv;  // signals drain()
    std::deque<SrvGraph> graphs;      // deque: references stay valid on growth
    std::unordered_map<uint64_t, SrvQuery> queries;
    std::vector<uint64_t> done_list;  // finished, not yet reported by bfs_server_completed
    std::atomic<int64_t> n_done_list{0};
    uint64_t next_ticket = 1;
    int64_t outstanding = 0;
    std::atomic<bool> stop{false};
    int worker_err = 0;
    // no batch exists and the next query's batch state plus its result does
    // not fit: only bfs_poll (which frees finished results) can make room
    bool stalled = false;
    int persist_inflight = 0;         // worker thread only
    int ms_grid = 0;                  // persistent round workgroups (0: not available)
    bfs_server_stats stats{};
    // result delivery (bfs_poll)
    std::mutex poll_mu;
    hipStream_t poll_stream = nullptr;
    int32_t* d_max = nullptr;         // arena, one int32
    int32_t* h_max = nullptr;         // pinned
    int16_t* h_stage = nullptr;       // pinned, int16[stage_elems]
    size_t stage_elems = 0;
    std::thread worker;
    void run();
    bool step_graph(SrvGraph& G);
    bool plan_step(SrvGraph& G, bool round_done, bool round_err, StepPlan& P);
    void execute(SrvGraph& G, const StepPlan& P);
    void set_err(int e)
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!worker_err) worker_err = e;
        idle_cv.notify_all();
    }
};

namespace {

int clampi(int64_t x, int lo, int hi) { return (int)std::max<int64_t>(lo, std::min<int64_t>(x, hi)); }

hipError_t enqueue_srv_level(const bfs_graph* g, SrvBatch* B, hipStream_t s, int parity)
{
    // grids sized by the graph: every kernel is grid-stride, so this only
    // trades idle workgroups on small graphs against parallelism on big ones
    const int ept = std::max(1, g->batch_tile / kWG);
    const int64_t tile_cap = (g->nnz + kMinTile - 1) / kMinTile + 1;
    const int scan = clampi(g->V / 8192, 8, g->num_cus * 2);
    const int expand = clampi(g->nnz / 4096, 16, g->num_cus * std::min(8, ms_expand_blocks_per_cu(ept)));
    const int fin = clampi(g->V / 4096, 8, g->num_cus * 4);
    return launch_ms_level(s, scan, expand, fin, ept, g->V, tile_cap, g->s_off, g->s_col, g->orig,
                           B->q[parity], B->q[parity ^ 1], B->deg, B->rowstart, B->suid, B->bsum,
                           B->cumul, B->tile_k, B->sn, B->front, B->touched,
                           B->lane_out, B->lane_start, B->ctrl);
}

// Capture kRoundLevels[i] levels of this batch into round[i].
int capture_rounds(const bfs_graph* g, SrvBatch* B, hipStream_t s)
{
    for (int i = 0; i < 3; ++i) {
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return BFS_ERR_HIP;
        hipError_t e = hipSuccess;
        for (int k = 0; k < kRoundLevels[i] && e == hipSuccess; ++k) e = enqueue_srv_level(g, B, s, k & 1);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (e == hipSuccess && e2 == hipSuccess)
            e = hipGraphInstantiate(&B->round[i], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            B->round[i] = nullptr;
            return BFS_ERR_HIP;
        }
    }
    return BFS_OK;
}

// Device side of releasing a batch (worker thread; the stream is idle or
// about to be): wait for the stream and destroy the captured rounds.
void drop_batch_device(SrvGraph& G)
{
    SrvBatch* B = G.batch;
    (void)hipStreamSynchronize(G.stream);
    for (auto& r : B->round)
        if (r) (void)hipGraphExecDestroy(r);
}

SrvBatch* carve_batch(char* mem, const bfs_graph* g)
{
    SrvBatch* B = new SrvBatch();
    B->mem = mem;
    char* p = mem;
    auto take = [&](size_t bytes) {
        char* at = p;
        p += align256(bytes);
        return at;
    };
    const size_t V = (size_t)g->V;
    B->sn = (SeenNext*)take(V * 16);
    B->front = (uint64_t*)take(V * 8);
    B->touched = (uint32_t*)take((V + 31) / 32 * 4);
    B->q[0] = (int32_t*)take(V * 4);
    B->q[1] = (int32_t*)take(V * 4);
    B->deg = (int32_t*)take(V * 4);
    B->rowstart = (int64_t*)take(V * 8);
    B->suid = (int32_t*)take(V * 4);
    B->cumul = (int64_t*)take((V + 1) * 8);
    B->bsum = (int64_t*)take(((V + kScanChunk - 1) / kScanChunk + 1) * 8);
    B->tile_k = (int32_t*)take((size_t)((g->nnz + kMinTile - 1) / kMinTile + 2) * 4);
    B->ctrl = (Ctrl*)take(sizeof(Ctrl));
    B->lane_out = (int16_t**)take(64 * 8);
    B->lane_start = (int32_t*)take(64 * 4);
    B->join = (int32_t*)take(128 * 4);
    B->msync = (MsSync*)take(sizeof(MsSync));
    return B;
}

}  // namespace

// Decide one step for graph G (server lock held).  Returns false when the
// graph has nothing to launch or to release.
bool bfs_server::plan_step(SrvGraph& G, bool round_done, bool round_err, StepPlan& P)
{
    const bfs_graph* g = G.g;
    SrvBatch* B = G.batch;
    char* first_res = nullptr;  // reserved with a fresh batch for its first query
    if (!B) {
        if (G.pending.empty()) return false;
        int running = 0;
        for (const auto& o : graphs) running += o.batch != nullptr && o.batch->idle_since == 0;
        if (running >= cfg.max_inflight) return false;
        // a batch starts only when its state and its first query's result
        // both fit: a batch that could admit nobody is never created
        const size_t res_bytes = (size_t)g->V * 2;
        auto take_both = [&](char** mem_out) {
            char* m = arena.alloc(G.state_bytes);
            char* r = m ? arena.alloc(res_bytes) : nullptr;
            if (m && !r) {
                arena.release(m);
                m = nullptr;
            }
            *mem_out = m;
            return r;
        };
        char* mem = nullptr;
        first_res = take_both(&mem);
        if (!mem) {
            // release idle batches of other graphs, then retry once
            for (auto& o : graphs)
                if (o.batch && o.batch->idle_since != 0 && !o.batch->in_flight) {
                    drop_batch_device(o);
                    arena.release(o.batch->mem);
                    delete o.batch;
                    o.batch = nullptr;
                }
            first_res = take_both(&mem);
        }
        if (!mem) {
            // over budget: wait for memory to free up.  Running batches free
            // theirs when their lanes end; with none left, only results that
            // bfs_poll collects can make room.
            bool any = false;
            for (const auto& o : graphs) any |= o.batch != nullptr;
            if (!any && !stalled) {
                stalled = true;
                idle_cv.notify_all();
            }
            return false;
        }
        stalled = false;
        B = carve_batch(mem, g);
        G.batch = B;
        P.fresh = true;
        ++stats.batches;
    }
    if (round_done) {
        const Ctrl& c = *G.h_ctrl;
        const bool bad = round_err || c.err || c.overflow;
        // a persistent round that stopped early without finishing left a large
        // level, and a round that ended on a frontier above half the
        // persistent kernel's limit is likely to meet one: the next round runs
        // the captured level kernels.  A persistent round that ran no level at
        // all left ctrl (last_alive included) as it was: no lane has ended.
        B->big_next = !c.done && ((B->persist && c.steps < B->round_levels) ||
                                  c.qlen > kMsQLimit / 2);
        const bool no_level = B->persist && c.steps == 0 && !c.done;
        const uint64_t retired =
            bad ? B->active : (no_level ? 0ull : (B->active & ~c.last_alive));
        const int64_t t = now_ns();
        for (int b = 0; b < 64; ++b) {
            if (!((retired >> b) & 1ull)) continue;
            auto it = queries.find(B->lane_ticket[b]);
            if (it != queries.end()) {
                SrvQuery& q = it->second;
                q.done_ns = t;
                q.state = bad ? 3 : 2;
                q.err = bad ? (c.overflow && !c.err && !round_err ? BFS_ERR_DEPTH : BFS_ERR_HIP) : 0;
                done_list.push_back(it->first);
                ++stats.completed;
                stats.failed += bad;
            }
            if (!bad) {
                const double life = (double)B->lane_age[b];
                G.life = G.life_n ? 0.75 * G.life + 0.25 * life : life;
                ++G.life_n;
            }
            --outstanding;
        }
        n_done_list.store((int64_t)done_list.size());
        B->active &= ~retired;
        if (retired) {
            if (bad) P.reset = true;
            else P.clear = retired;
            // the device lane table drops the retired lanes' result rows
            for (int b = 0; b < 64; ++b)
                if ((retired >> b) & 1ull) G.h_lane_out[b] = nullptr;
            P.table = true;
            idle_cv.notify_all();
        }
    }
    // boundary: fill free lanes from the queue (FIFO, while results fit)
    int64_t oldest = 0;
    for (int b = 0; b < 64; ++b)
        if ((B->active >> b) & 1ull) oldest = std::max(oldest, B->lane_age[b]);
    const bool deep = G.life_n > 0 && G.life > kDeepLife;
    const bool continuous = deep || g->V <= kSmallV;
    const uint64_t lane_cap = cfg.max_lanes >= 64 ? ~0ull : ((1ull << cfg.max_lanes) - 1);
    if (continuous || oldest == 0) {
        while (!G.pending.empty() && (~B->active & lane_cap)) {
            const uint64_t ticket = G.pending.front();
            SrvQuery& q = queries[ticket];
            char* res = first_res ? first_res : arena.alloc((size_t)g->V * 2);
            first_res = nullptr;
            if (!res) break;
            G.pending.pop_front();
            const int b = __builtin_ctzll(~B->active & lane_cap);
            B->active |= 1ull << b;
            B->lane_ticket[b] = ticket;
            B->lane_age[b] = 0;
            q.result = reinterpret_cast<int16_t*>(res);
            q.state = 1;
            q.admit_ns = now_ns();
            G.h_join[2 * P.n_join] = q.root;
            G.h_join[2 * P.n_join + 1] = b;
            G.h_lane_out[b] = q.result;
            P.fill[P.n_join] = q.result;
            ++P.n_join;
        }
        if (first_res) {  // not expected: a fresh batch always admits its first query
            arena.release(first_res);
            first_res = nullptr;
        }
        if (P.n_join) {
            const int lanes = __builtin_popcountll(B->active);
            for (int i = 0; i < P.n_join; ++i)
                queries[B->lane_ticket[G.h_join[2 * i + 1]]].lanes = lanes;
            stats.joins += P.n_join;
        }
    }
    if (!B->active) {
        // nothing running: keep the batch a little for the next query, then
        // release its arena memory
        const int64_t t = now_ns();
        if (B->idle_since == 0) B->idle_since = t;
        if (t - B->idle_since > kIdleKeepNs) P.release = true;
        return P.fresh || P.reset || P.clear || P.release;
    }
    B->idle_since = 0;
    // levels per replay: waves run 8 (most small-world searches end within
    // one replay; levels after every lane has ended exit at once); deep
    // graphs start with 2 and lengthen as their oldest lane ages
    const int ri = !deep ? 1 : (oldest < 32 ? 0 : (oldest < 256 ? 1 : 2));
    const int K = kRoundLevels[ri];
    P.round = ri;
    P.persist = deep && ms_grid > 0 && !B->big_next && persist_inflight < kMaxPersist;
    stats.persistent_rounds += P.persist;
    stats.wide_rounds += deep && ms_grid > 0 && B->big_next;
    ++stats.rounds;
    stats.levels += (uint64_t)K;
    stats.lane_levels += (uint64_t)K * (uint64_t)__builtin_popcountll(B->active);
    for (int b = 0; b < 64; ++b)
        if ((B->active >> b) & 1ull) B->lane_age[b] += K;
    return true;
}

// Carry out a plan (no lock held; only the worker touches G.batch).
void bfs_server::execute(SrvGraph& G, const StepPlan& P)
{
    const bfs_graph* g = G.g;
    SrvBatch* B = G.batch;
    bool bad = false;
    if (P.fresh) {
        bad |= launch_srv_reset(G.stream, g->num_cus * 4, g->V, B->sn, B->front, B->touched,
                                B->ctrl) != hipSuccess;
        bad |= capture_rounds(g, B, G.stream) != BFS_OK;
    }
    if (P.reset)
        bad |= launch_srv_reset(G.stream, g->num_cus * 4, g->V, B->sn, B->front, B->touched,
                                B->ctrl) != hipSuccess;
    if (P.fresh || P.reset)  // each persistent launch then leaves it zero
        bad |= hipMemsetAsync(B->msync, 0, sizeof(MsSync), G.stream) != hipSuccess;
    else if (P.clear)
        bad |= launch_srv_clear(G.stream, g->num_cus * 4, g->V, B->sn, P.clear) != hipSuccess;
    for (int i = 0; i < P.n_join; ++i)
        bad |= launch_fill16(G.stream, g->num_cus * 2, P.fill[i], g->V, (int16_t)-1) != hipSuccess;
    const bool staged = P.n_join || P.table;
    if (staged)
        bad |= hipMemcpyAsync(B->lane_out, G.h_lane_out, 64 * sizeof(int16_t*),
                              hipMemcpyHostToDevice, G.stream) != hipSuccess;
    if (P.n_join) {
        bad |= hipMemcpyAsync(B->join, G.h_join, (size_t)P.n_join * 2 * sizeof(int32_t),
                              hipMemcpyHostToDevice, G.stream) != hipSuccess;
        bad |= launch_srv_join(G.stream, g->V, P.n_join, B->join, g->rank, B->sn, B->front,
                               B->lane_out, B->lane_start, B->q[B->parity], B->ctrl) != hipSuccess;
    }
    if (staged && P.round < 0 && !P.release) {
        // no round event follows these copies: the pinned staging they read
        // must not be rewritten (next plan_step) before the stream has read it
        bad |= hipEventRecord(G.ev_stage, G.stream) != hipSuccess;
        G.stage_pending = true;
    }
    if (P.release) {
        drop_batch_device(G);
        G.stage_pending = false;  // the stream was synchronised
        {
            std::lock_guard<std::mutex> lk(mu);
            arena.release(B->mem);
        }
        delete B;
        G.batch = nullptr;
    } else if (P.round >= 0) {
        bad |= hipEventRecord(G.ev0, G.stream) != hipSuccess;
        B->persist = P.persist;
        B->round_levels = kRoundLevels[P.round];
        if (P.persist) {
            ++persist_inflight;
            // the kernel copies the control block into G.h_ctrl itself
            bad |= launch_ms_small_levels(G.stream, ms_grid, g->V, g->s_off, g->s_col, g->orig,
                                          B->sn, B->front, B->q[0], B->q[1], B->deg, B->lane_out,
                                          B->lane_start, B->msync, B->ctrl, G.h_ctrl,
                                          B->round_levels, kMsQLimit, kMsRLimit,
                                          kMsDLimit) != hipSuccess;
        } else {
            bad |= !B->round[P.round] || hipGraphLaunch(B->round[P.round], G.stream) != hipSuccess;
            bad |= hipMemcpyAsync(G.h_ctrl, B->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost,
                                  G.stream) != hipSuccess;
        }
        bad |= hipEventRecord(G.ev, G.stream) != hipSuccess;
        B->in_flight = true;
    }
    if (bad) set_err(BFS_ERR_HIP);
}

// One scheduling step for graph G; returns true when it launched work.
bool bfs_server::step_graph(SrvGraph& G)
{
    SrvBatch* B = G.batch;
    bool round_done = false, round_err = false;
    double round_ms = 0.0;
    if (G.stage_pending) {
        const hipError_t q = hipEventQuery(G.ev_stage);
        if (q == hipErrorNotReady) return false;
        if (q != hipSuccess) set_err(BFS_ERR_HIP);
        G.stage_pending = false;
    }
    if (B && B->in_flight) {
        const hipError_t q = hipEventQuery(G.ev);
        if (q == hipErrorNotReady) return false;
        if (q == hipSuccess) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, G.ev0, G.ev) == hipSuccess) round_ms = ms;
        } else {
            round_err = true;
            set_err(BFS_ERR_HIP);
        }
        B->in_flight = false;
        round_done = true;
        if (B->persist) --persist_inflight;
    }
    StepPlan P;
    {
        std::lock_guard<std::mutex> lk(mu);
        stats.device_ms += round_ms;
        if (!plan_step(G, round_done, round_err, P)) return false;
    }
    execute(G, P);
    return P.round >= 0;
}

void bfs_server::run()
{
    (void)hipSetDevice(device);
    std::vector<SrvGraph*> gl;
    while (!stop.load()) {
        {
            std::lock_guard<std::mutex> lk(mu);
            gl.clear();
            for (auto& G : graphs) gl.push_back(&G);
        }
        bool busy = false;
        for (SrvGraph* G : gl) busy |= step_graph(*G);
        if (busy) continue;
        std::unique_lock<std::mutex> lk(mu);
        bool waiting = false;
        for (const auto& G : graphs) waiting |= G.batch != nullptr || !G.pending.empty();
        if (waiting && !stalled) {
            // poll in-flight rounds at a fine grain (a busy poll was measured:
            // it slowed the other graphs' rounds more than it sped up these)
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        } else {
            cv.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

extern "C" {

int bfs_server_create(bfs_server** out, void* d_arena, size_t arena_bytes,
                      const bfs_server_config* cfg)
{
    if (!out) return fail(BFS_ERR_INVALID, "server out-pointer is NULL");
    *out = nullptr;
    if (!d_arena || arena_bytes < 4096) return fail(BFS_ERR_INVALID, "arena is NULL or too small");
    if ((uintptr_t)d_arena % 256) return fail(BFS_ERR_INVALID, "arena not 256-byte aligned");
    bfs_server_config c{64, 8, 0};
    if (cfg) {
        c = *cfg;
        if (c.max_lanes < 1 || c.max_lanes > 64) return fail(BFS_ERR_INVALID, "max_lanes must be 1..64");
        if (c.max_inflight < 1) return fail(BFS_ERR_INVALID, "max_inflight must be >= 1");
        if (c.flags & ~BFS_SRV_NO_PERSISTENT) return fail(BFS_ERR_INVALID, "unknown server flags");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(BFS_ERR_NO_DEVICE, "no HIP device");
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, d_arena) == hipSuccess && attr.type == hipMemoryTypeDevice)
        dev = attr.device;
    (void)hipGetLastError();
    bfs_server* s = new (std::nothrow) bfs_server();
    if (!s) return fail(BFS_ERR_INVALID, "out of host memory");
    s->cfg = c;
    s->device = dev;
    if (!(c.flags & BFS_SRV_NO_PERSISTENT) && ms_small_loop_blocks() > 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
        s->ms_grid = std::min(kMsGrid, cus);
    }
    // the first 256 bytes of the arena hold the delivery kernel's maximum
    s->d_max = static_cast<int32_t*>(d_arena);
    s->arena.init(static_cast<char*>(d_arena) + 256, arena_bytes - 256);
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(dev);
    hipError_t e = hipStreamCreateWithFlags(&s->poll_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_max, 256, hipHostMallocDefault);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        if (s->poll_stream) (void)hipStreamDestroy(s->poll_stream);
        delete s;
        return hip_fail(e, "server resources");
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return ok();
}

int bfs_server_add_graph(bfs_server* s, bfs_graph* g, int32_t* graph_id)
{
    if (!s || !g || !graph_id) return fail(BFS_ERR_INVALID, "NULL argument");
    SrvGraph G;
    G.g = g;
    G.state_bytes = batch_state_bytes(g);
    if (G.state_bytes + align256((size_t)g->V * 2) > s->arena.size())
        return fail(BFS_ERR_BUDGET, "graph needs %zu arena bytes, arena has %zu",
                    G.state_bytes + align256((size_t)g->V * 2), s->arena.size());
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    hipError_t e = hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&G.ev0);
    if (e == hipSuccess) e = hipEventCreate(&G.ev);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&G.ev_stage, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&G.h_ctrl, sizeof(Ctrl) + 64 * sizeof(int16_t*) + 128 * sizeof(int32_t),
                          hipHostMallocDefault);
    {
        // pinned staging for host-side delivery, sized for the largest graph
        std::lock_guard<std::mutex> pl(s->poll_mu);
        if (e == hipSuccess && (size_t)g->V > s->stage_elems) {
            int16_t* st = nullptr;
            e = hipHostMalloc((void**)&st, (size_t)g->V * 2, hipHostMallocDefault);
            if (e == hipSuccess) {
                if (s->h_stage) (void)hipHostFree(s->h_stage);
                s->h_stage = st;
                s->stage_elems = (size_t)g->V;
            }
        }
    }
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        if (G.stream) (void)hipStreamDestroy(G.stream);
        if (G.ev0) (void)hipEventDestroy(G.ev0);
        if (G.ev) (void)hipEventDestroy(G.ev);
        if (G.ev_stage) (void)hipEventDestroy(G.ev_stage);
        if (G.h_ctrl) (void)hipHostFree(G.h_ctrl);
        return hip_fail(e, "server graph resources");
    }
    G.h_lane_out = reinterpret_cast<int16_t**>(G.h_ctrl + 1);
    G.h_join = reinterpret_cast<int32_t*>(G.h_lane_out + 64);
    std::memset(G.h_lane_out, 0, 64 * sizeof(int16_t*));
    std::lock_guard<std::mutex> lk(s->mu);
    s->graphs.push_back(G);
    *graph_id = (int32_t)s->graphs.size() - 1;
    return ok();
}

int bfs_submit(bfs_server* s, int32_t graph_id, int32_t root, uint64_t* ticket)
{
    if (!s || !ticket) return fail(BFS_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop.load()) return fail(BFS_ERR_INVALID, "server is stopping");
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size())
        return fail(BFS_ERR_INVALID, "unknown graph id %d", graph_id);
    SrvGraph& G = s->graphs[graph_id];
    if (root < 0 || root >= G.g->V) return fail(BFS_ERR_INVALID, "root %d outside [0, %d)", root, G.g->V);
    const uint64_t t = s->next_ticket++;
    SrvQuery q;
    q.graph = graph_id;
    q.root = root;
    q.submit_ns = now_ns();
    s->queries.emplace(t, q);
    G.pending.push_back(t);
    ++s->outstanding;
    ++s->stats.submitted;
    *ticket = t;
    s->cv.notify_one();
    return ok();
}

int bfs_poll(bfs_server* s, uint64_t ticket, int32_t* dst_levels, bfs_timing* tm)
{
    if (!s) return fail(BFS_ERR_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->queries.find(ticket);
    if (it == s->queries.end()) return fail(BFS_ERR_TICKET, "unknown ticket %llu", (unsigned long long)ticket);
    const SrvQuery q = it->second;
    if (q.state < 2) return BFS_PENDING;
    const int32_t V = s->graphs[q.graph].g->V;
    lk.unlock();
    int rc = BFS_OK;
    int32_t levels = 0;
    if (q.state == 3) {
        rc = fail(q.err ? q.err : BFS_ERR_HIP, "query failed on the device");
    } else if (dst_levels) {
        std::lock_guard<std::mutex> pl(s->poll_mu);
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(s->device);
        hipPointerAttribute_t attr;
        const bool on_device = hipPointerGetAttributes(&attr, dst_levels) == hipSuccess &&
                               attr.type == hipMemoryTypeDevice && attr.device == s->device;
        (void)hipGetLastError();
        hipError_t e;
        if (on_device) {
            // the device's default stream: ordered after whatever the caller
            // queued there for this buffer
            hipStream_t ds = nullptr;
            e = hipMemsetAsync(s->d_max, 0xff, sizeof(int32_t), ds);
            if (e == hipSuccess) {
                const int grid = (int)std::min<int64_t>(((int64_t)V + 4095) / 4096, 1024);
                e = launch_widen16(ds, std::max(grid, 1), q.result, dst_levels, V, s->d_max);
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(s->h_max, s->d_max, sizeof(int32_t), hipMemcpyDeviceToHost, ds);
            if (e == hipSuccess) e = hipStreamSynchronize(ds);
            levels = *s->h_max + 1;
        } else {
            e = hipMemcpyAsync(s->h_stage, q.result, (size_t)V * 2, hipMemcpyDeviceToHost,
                               s->poll_stream);
            if (e == hipSuccess) e = hipStreamSynchronize(s->poll_stream);
            int32_t lv = -1;
            if (e == hipSuccess) {
                const int16_t* src = s->h_stage;
                for (int32_t v = 0; v < V; ++v) {
                    const int32_t x = src[v];
                    dst_levels[v] = x;
                    lv = x > lv ? x : lv;
                }
            }
            levels = lv + 1;
        }
        (void)hipSetDevice(prev);
        if (e != hipSuccess) return hip_fail(e, "result delivery");
    }
    if (tm) {
        tm->submit_ns = q.submit_ns;
        tm->admit_ns = q.admit_ns;
        tm->done_ns = q.done_ns;
        tm->lanes_in_batch = q.lanes ? q.lanes : 1;
        tm->levels = (dst_levels && q.state == 2) ? levels : 0;
    }
    lk.lock();
    it = s->queries.find(ticket);
    if (it != s->queries.end()) {
        s->arena.release(reinterpret_cast<char*>(it->second.result));
        s->queries.erase(it);
        s->stalled = false;  // the worker retries admission
    }
    s->cv.notify_one();
    return rc == BFS_OK ? ok() : rc;
}

int bfs_server_completed(bfs_server* s, uint64_t* tickets, int32_t max_tickets, int32_t* n_out)
{
    if (!s || !n_out || (max_tickets > 0 && !tickets) || max_tickets < 0)
        return fail(BFS_ERR_INVALID, "NULL argument or negative max_tickets");
    *n_out = 0;
    if (s->n_done_list.load() == 0 || max_tickets == 0) return ok();
    std::lock_guard<std::mutex> lk(s->mu);
    const size_t n = std::min<size_t>((size_t)max_tickets, s->done_list.size());
    std::copy(s->done_list.begin(), s->done_list.begin() + n, tickets);
    s->done_list.erase(s->done_list.begin(), s->done_list.begin() + n);
    s->n_done_list.store((int64_t)s->done_list.size());
    *n_out = (int32_t)n;
    return ok();
}

int bfs_server_get_stats(bfs_server* s, bfs_server_stats* out)
{
    if (!s || !out) return fail(BFS_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->arena_peak = (uint64_t)s->arena.peak();
    return ok();
}

int bfs_server_drain(bfs_server* s)
{
    if (!s) return fail(BFS_ERR_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->idle_cv.wait(lk, [s] {
        return s->outstanding <= 0 || s->worker_err != 0 || s->stalled;
    });
    if (s->worker_err) return fail(s->worker_err, "server worker failed");
    if (s->outstanding > 0)
        return fail(BFS_ERR_BUDGET,
                    "%lld queries cannot start: the arena is held by finished results that "
                    "have not been collected with bfs_poll",
                    (long long)s->outstanding);
    return ok();
}

int bfs_server_destroy(bfs_server* s)
{
    if (!s) return ok();
    s->stop.store(true);
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (auto& G : s->graphs) {
        if (G.stream) (void)hipStreamSynchronize(G.stream);
        if (G.batch) {
            drop_batch_device(G);
            s->arena.release(G.batch->mem);
            delete G.batch;
            G.batch = nullptr;
        }
        if (G.stream) (void)hipStreamDestroy(G.stream);
        if (G.ev0) (void)hipEventDestroy(G.ev0);
        if (G.ev) (void)hipEventDestroy(G.ev);
        if (G.ev_stage) (void)hipEventDestroy(G.ev_stage);
        if (G.h_ctrl) (void)hipHostFree(G.h_ctrl);
    }
    if (s->poll_stream) (void)hipStreamDestroy(s->poll_stream);
    if (s->h_max) (void)hipHostFree(s->h_max);
    if (s->h_stage) (void)hipHostFree(s->h_stage);
    (void)hipSetDevice(prev);
    delete s;
    return ok();
}

}  // extern "C"
