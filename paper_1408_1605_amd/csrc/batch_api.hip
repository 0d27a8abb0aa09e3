// C ABI: multi-source batch search (bfs_run_batch).
//
// The level loop runs on a private stream.  By default (loop driver 0 or 2)
// kLevelsPerGraph levels are captured once per graph handle into a hipGraph
// whose kernels read every size from the control block and return at once
// after the last level, so the host replays the graph and reads the control
// block once per replay.  Loop driver 1 launches level by level instead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "runtime.h"

using namespace bfsmi;

namespace bfsmi {

constexpr int kLevelsPerGraph = 4;  // even: the queue buffers alternate

int ensure_cap_stream(bfs_graph* g)
{
    if (g->cap_stream) return BFS_OK;
    hipError_t e = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    return BFS_OK;
}

struct BatchGrids {
    int ept, scan, expand, fin;
    int64_t tile_cap;
};

static BatchGrids batch_grids(bfs_graph* g)
{
    BatchGrids b;
    b.ept = std::max(1, g->batch_tile / kWG);
    b.scan = g->num_cus * 2;
    b.expand = g->num_cus * std::min(8, ms_expand_blocks_per_cu(b.ept));
    b.fin = g->num_cus * 8;
    b.tile_cap = (g->nnz + kMinTile - 1) / kMinTile + 1;
    return b;
}

// The levels write the int8 rows by search id (no orig): directly the
// caller's rows without degree order, else g->ms_out, reordered at the end.
// With degree order the levels also track the id prefix every searching
// lane has seen, and each scan drops the rows' blocks below it (the row
// prefix skip of the single-root search, over the batch's live lanes).
static hipError_t enqueue_level(bfs_graph* g, hipStream_t s, const BatchGrids& b, int parity)
{
    const bool skip = g->skip && g->row_skip;
    return launch_ms_level(s, b.scan, b.expand, b.fin, b.ept, g->V, b.tile_cap, g->s_off, g->s_col,
                           nullptr, g->q[parity], g->q[parity ^ 1], g->deg, g->rowstart, g->suid,
                           g->bsum, g->cumul,
                           g->tile_k, g->ms_sn, g->ms_front, g->ms_touched, nullptr,
                           nullptr, g->ms_ctrl, skip ? g->skip : nullptr,
                           skip ? g->num_cus * 2 : 0);
}

static int capture_batch_graph(bfs_graph* g, const BatchGrids& b)
{
    if (g->ms_graph && g->ms_graph_ept == b.ept && g->ms_graph_skip == g->row_skip) return BFS_OK;
    if (g->ms_graph) {
        (void)hipGraphExecDestroy(g->ms_graph);
        g->ms_graph = nullptr;
    }
    hipStream_t s = g->cap_stream;
    BFS_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int j = 0; j < kLevelsPerGraph && e == hipSuccess; ++j) e = enqueue_level(g, s, b, j & 1);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(e, "batch level capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&g->ms_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g->ms_graph = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    g->ms_graph_ept = b.ept;
    g->ms_graph_skip = g->row_skip;
    return BFS_OK;
}

}  // namespace bfsmi

namespace {
struct BusyGuardB {
    bfs_graph* g;
    bool held = false;
    explicit BusyGuardB(bfs_graph* gg) : g(gg)
    {
        int expect = 0;
        held = g->busy.compare_exchange_strong(expect, 1);
    }
    ~BusyGuardB()
    {
        if (held) g->busy.store(0);
    }
};
struct DeviceGuardB {
    int prev = -1;
    explicit DeviceGuardB(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuardB()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
float ms_between(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.f;
    return ms;
}
}  // namespace

extern "C" int bfs_run_batch(bfs_graph* g, const int32_t* h_roots, int32_t n_roots,
                             int8_t* d_levels, void* hip_stream, bfs_stats* st)
{
    if (!g) return fail(BFS_ERR_INVALID, "graph is NULL");
    if (!h_roots) return fail(BFS_ERR_INVALID, "roots pointer is NULL");
    if (n_roots < 1 || n_roots > 64) return fail(BFS_ERR_INVALID, "n_roots must be 1..64 (got %d)", n_roots);
    if (!d_levels) return fail(BFS_ERR_INVALID, "levels pointer is NULL");
    if (!g->ms_sn) return fail(BFS_ERR_INVALID, "graph was created without BFS_WS_BATCH");
    for (int i = 0; i < n_roots; ++i)
        if (h_roots[i] < 0 || h_roots[i] >= g->V)
            return fail(BFS_ERR_INVALID, "root %d (index %d) outside [0, %d)", h_roots[i], i, g->V);
    BusyGuardB busy(g);
    if (!busy.held) return fail(BFS_ERR_BUSY, "graph handle is in use");
    DeviceGuardB dg(g->device);
    int rc = ensure_cap_stream(g);
    if (rc != BFS_OK) return rc;
    hipStream_t caller = static_cast<hipStream_t>(hip_stream);
    BFS_HIP_TRY(hipStreamSynchronize(caller));  // the caller's prior work (e.g. d_levels)
    hipStream_t s = g->cap_stream;
    const BatchGrids b = batch_grids(g);

    std::memcpy(g->h_roots, h_roots, sizeof(int32_t) * (size_t)n_roots);
    BFS_HIP_TRY(hipEventRecord(g->ev0, s));
    BFS_HIP_TRY(hipMemcpyAsync(g->ms_roots, g->h_roots, sizeof(int32_t) * (size_t)n_roots,
                               hipMemcpyHostToDevice, s));
    BFS_HIP_TRY(launch_ms_init(s, g->num_cus * 8, g->V, g->ms_roots, n_roots, g->rank, g->ms_sn,
                               g->ms_front, g->ms_touched, d_levels, g->rank ? g->ms_out : nullptr,
                               g->q[0], g->ms_ctrl));
    const bool use_graph = g->loop_driver != 1;
    if (use_graph) {
        rc = capture_batch_graph(g, b);
        if (rc != BFS_OK) return rc;
    }
    // every launch of kLevelsPerGraph levels is followed by one read-back
    const int64_t max_rounds = (int64_t)g->V / (use_graph ? kLevelsPerGraph : 1) + 4;
    int64_t rounds = 0;
    int parity = 0;
    while (true) {
        if (use_graph) {
            BFS_HIP_TRY(hipGraphLaunch(g->ms_graph, s));
        } else {
            BFS_HIP_TRY(enqueue_level(g, s, b, parity));
            parity ^= 1;
        }
        BFS_HIP_TRY(hipMemcpyAsync(g->h_ms_ctrl, g->ms_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        BFS_HIP_TRY(hipStreamSynchronize(s));
        if (g->h_ms_ctrl->done) break;
        if (++rounds > max_rounds) return fail(BFS_ERR_HIP, "batch level loop did not terminate");
    }
    if (g->rank)
        BFS_HIP_TRY(launch_ms_reorder(s, g->num_cus * 8, g->V, n_roots, g->rank, g->ms_sn,
                                      g->ms_out, d_levels));
    BFS_HIP_TRY(hipEventRecord(g->ev1, s));
    BFS_HIP_TRY(hipEventSynchronize(g->ev1));
    const Ctrl& c = *g->h_ms_ctrl;
    if (c.err) return fail(BFS_ERR_HIP, "internal guard tripped in batch (code %d)", c.err);
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->levels = c.levels;
        st->reached = c.reached;
        st->edges_scanned = c.r_total + c.skipped;  // the skipped edges are part of the union
        st->device_ms = ms_between(g->ev0, g->ev1);
    }
    if (c.overflow) return fail(BFS_ERR_DEPTH, "a batch search is deeper than 127 levels");
    return ok();
}

// Serving entry points are defined in server.cpp.
