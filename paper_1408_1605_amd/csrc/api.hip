// C ABI: errors, workspace layout, graph handles and the single-root search
// driver (host-driven level loop, one 64-byte control read-back per level).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "runtime.h"

namespace bfsmi {

constexpr int32_t kSmallQ = 1 << 16;  // frontiers up to this size may run in the persistent loop
constexpr int32_t kSmallDeg = 8192;   // ... if no frontier vertex has a larger degree
constexpr int kSmallWGs = 32;         // workgroups of the persistent loop


static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(BFS_ERR_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

int ok()
{
    g_err[0] = 0;
    return BFS_OK;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Entries per set of the persistent loop's frontier row data: a frontier
// that continues in the loop holds at most kSmallQ vertices, and never more
// than V.
static int32_t small_side_cap(int32_t V) { return V < kSmallQ ? V : kSmallQ; }

WsLayout ws_layout(int32_t V, int64_t nnz, uint32_t flags)
{
    WsLayout L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p = align_up(p + bytes, 256);
        return at;
    };
    const size_t W = ((size_t)V + 31) / 32;
    const size_t nblk = ((size_t)V + kScanChunk - 1) / kScanChunk;
    const size_t ntile_max = (size_t)((nnz + kMinTile - 1) / kMinTile);
    L.vis = take(W * 4);
    L.vis_old = take(W * 4);
    L.q0 = take((size_t)V * 4);
    L.q1 = take((size_t)V * 4);
    L.deg = take((size_t)V * 4);
    L.rowstart = take((size_t)V * 8);
    L.suid = take((size_t)V * 4);
    L.cumul = take(((size_t)V + 1) * 8);
    L.bsum = take((nblk + 1) * 8);
    L.tile_k = take((ntile_max + 2) * 4);
    L.ctrl = take(sizeof(Ctrl));
    L.scratch = take(256);
    L.sync = take(sizeof(SmallSync));
    L.sside = take((size_t)small_side_cap(V) * 32);
    L.summary = take(kSummaryMaxWords * 4);
    if (flags & BFS_WS_BATCH) {
        L.ms_sn = take((size_t)V * 16);
        L.ms_front = take((size_t)V * 8);
        L.ms_ctrl = take(sizeof(Ctrl));
        L.ms_roots = take(64 * 4);
        L.ms_touched = take(W * 4);
    }
    if (flags & BFS_DEGREE_ORDER) {
        L.rank = take((size_t)V * 4);
        L.orig = take((size_t)V * 4);
        L.off_r = take(((size_t)V + 1) * 8);
        L.col_r = take((size_t)(nnz > 0 ? nnz : 1) * 4);
        L.hist = take(2 * 4096 * 4);
        L.col_tmp = take((size_t)(nnz > 0 ? nnz : 1) * 4);  // relabelled rows before grouping
        L.skip = take((size_t)kSkipLevels * V * 4);
        L.lvl_int = take((size_t)V * 4);
        L.par_int = take((size_t)V * 4);
        if (flags & BFS_WS_BATCH) L.ms_out = take((size_t)64 * V);  // batch rows by internal id
        L.found = take(W * 32);  // flag claims: one byte per id, padded to whole words
        L.xo = take((size_t)V * kXcdSlices * 4);  // XCD slices: group offsets per row
        // (the slice-grouped rows reuse col_tmp, free once creation is done)
    }
    L.total = p;
    return L;
}

int small_loop_grid(int num_cus)
{
    // the persistent small-level loop needs all its workgroups resident: at
    // most one per CU
    return small_loop_blocks() > 0 ? std::min(kSmallWGs, num_cus) : 0;
}

// Points the handle's arrays into the workspace ws laid out as L.
void bind_workspace(bfs_graph* g, char* ws, const WsLayout& L, uint32_t flags)
{
    g->L = L;
    g->vis = reinterpret_cast<uint32_t*>(ws + L.vis);
    g->vis_old = reinterpret_cast<uint32_t*>(ws + L.vis_old);
    g->q[0] = reinterpret_cast<int32_t*>(ws + L.q0);
    g->q[1] = reinterpret_cast<int32_t*>(ws + L.q1);
    g->deg = reinterpret_cast<int32_t*>(ws + L.deg);
    g->rowstart = reinterpret_cast<int64_t*>(ws + L.rowstart);
    g->suid = reinterpret_cast<int32_t*>(ws + L.suid);
    g->cumul = reinterpret_cast<int64_t*>(ws + L.cumul);
    g->bsum = reinterpret_cast<int64_t*>(ws + L.bsum);
    g->tile_k = reinterpret_cast<int32_t*>(ws + L.tile_k);
    g->ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
    g->scratch = reinterpret_cast<int32_t*>(ws + L.scratch);
    g->small_sync = reinterpret_cast<SmallSync*>(ws + L.sync);
    {
        const int32_t cap = small_side_cap(g->V);
        char* b = ws + L.sside;
        g->small_side.off[0] = reinterpret_cast<int64_t*>(b);
        g->small_side.off[1] = reinterpret_cast<int64_t*>(b + (size_t)cap * 8);
        g->small_side.deg[0] = reinterpret_cast<int32_t*>(b + (size_t)cap * 16);
        g->small_side.deg[1] = reinterpret_cast<int32_t*>(b + (size_t)cap * 20);
        g->small_side.id[0] = reinterpret_cast<int32_t*>(b + (size_t)cap * 24);
        g->small_side.id[1] = reinterpret_cast<int32_t*>(b + (size_t)cap * 28);
        g->small_side.cap = cap;
    }
    g->summary = reinterpret_cast<uint32_t*>(ws + L.summary);
    {
        // blocks of 2^shift ids, at most kSummaryMaxWords * 32 of them
        int shift = 10;
        while ((((int64_t)g->V + (1ll << shift) - 1) >> shift) > (int64_t)kSummaryMaxWords * 32) ++shift;
        g->summary_shift = shift;
        g->summary_blocks = (int32_t)(((int64_t)g->V + (1ll << shift) - 1) >> shift);
        g->summary_words = (g->summary_blocks + 31) / 32;
    }
    g->s_off = g->off;
    g->s_col = g->col;
    if (flags & BFS_DEGREE_ORDER) {
        g->rank = reinterpret_cast<int32_t*>(ws + L.rank);
        g->orig = reinterpret_cast<int32_t*>(ws + L.orig);
        g->s_off = reinterpret_cast<int64_t*>(ws + L.off_r);
        g->s_col = reinterpret_cast<int32_t*>(ws + L.col_r);
        g->skip = reinterpret_cast<int32_t*>(ws + L.skip);
        g->lvl_int = reinterpret_cast<int32_t*>(ws + L.lvl_int);
        g->par_int = reinterpret_cast<int32_t*>(ws + L.par_int);
        if (flags & BFS_WS_BATCH) g->ms_out = reinterpret_cast<int8_t*>(ws + L.ms_out);
        g->found = reinterpret_cast<uint8_t*>(ws + L.found);
        g->xo = reinterpret_cast<uint32_t*>(ws + L.xo);
        g->col_x = reinterpret_cast<int32_t*>(ws + L.col_tmp);
    }
    if (flags & BFS_WS_BATCH) {
        g->ms_sn = reinterpret_cast<SeenNext*>(ws + L.ms_sn);
        g->ms_front = reinterpret_cast<uint64_t*>(ws + L.ms_front);
        g->ms_ctrl = reinterpret_cast<Ctrl*>(ws + L.ms_ctrl);
        g->ms_roots = reinterpret_cast<int32_t*>(ws + L.ms_roots);
        g->ms_touched = reinterpret_cast<uint32_t*>(ws + L.ms_touched);
    }
}

}  // namespace bfsmi

using namespace bfsmi;

extern "C" {

const char* bfs_last_error(void) { return g_err; }

int bfs_version(void) { return 105; }

int bfs_workspace_bytes(int32_t V, int64_t nnz, uint32_t flags, size_t* bytes)
{
    if (!bytes) return fail(BFS_ERR_INVALID, "bytes is NULL");
    if (V < 1) return fail(BFS_ERR_INVALID, "V must be >= 1 (got %d)", V);
    if (nnz < 0 || nnz > ((int64_t)1 << 62)) return fail(BFS_ERR_INVALID, "nnz out of range");
    if (flags & ~(BFS_VALIDATE_CSR | BFS_WS_BATCH | BFS_DEGREE_ORDER))
        return fail(BFS_ERR_INVALID, "unknown flags");
    *bytes = ws_layout(V, nnz, flags).total;
    return ok();
}

int bfs_graph_create(bfs_graph** out, int32_t V, int64_t nnz, const int64_t* d_row_offsets,
                     const int32_t* d_col, void* d_workspace, size_t ws_bytes, uint32_t flags,
                     void* hip_stream)
{
    if (!out) return fail(BFS_ERR_INVALID, "graph out-pointer is NULL");
    *out = nullptr;
    if (V < 1) return fail(BFS_ERR_INVALID, "V must be >= 1 (got %d)", V);
    if (nnz < 0 || nnz > ((int64_t)1 << 62)) return fail(BFS_ERR_INVALID, "nnz out of range");
    if (!d_row_offsets) return fail(BFS_ERR_INVALID, "row offsets pointer is NULL");
    if (!d_col && nnz > 0) return fail(BFS_ERR_INVALID, "column pointer is NULL");
    if (!d_workspace) return fail(BFS_ERR_INVALID, "workspace pointer is NULL");
    if ((uintptr_t)d_workspace % 256 != 0) return fail(BFS_ERR_INVALID, "workspace not 256-byte aligned");
    if (flags & ~(BFS_VALIDATE_CSR | BFS_WS_BATCH | BFS_DEGREE_ORDER))
        return fail(BFS_ERR_INVALID, "unknown flags");
    const WsLayout L = ws_layout(V, nnz, flags);
    if (ws_bytes < L.total)
        return fail(BFS_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(BFS_ERR_NO_DEVICE, "no HIP device");
    int dev = 0;
    BFS_HIP_TRY(hipGetDevice(&dev));
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, d_workspace) == hipSuccess && attr.type == hipMemoryTypeDevice)
        dev = attr.device;
    (void)hipGetLastError();

    bfs_graph* g = new (std::nothrow) bfs_graph();
    if (!g) return fail(BFS_ERR_INVALID, "out of host memory");
    g->V = V;
    g->nnz = nnz;
    g->W = (int32_t)(((int64_t)V + 31) / 32);
    g->off = d_row_offsets;
    g->col = d_col;
    g->ws = static_cast<char*>(d_workspace);
    g->ws_bytes = ws_bytes;
    g->flags = flags;
    g->device = dev;
    bind_workspace(g, g->ws, L, flags);

    auto cleanup = [&](int code) {
        bfs_graph_destroy(g);
        return code;
    };
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(dev) != hipSuccess) return cleanup(fail(BFS_ERR_HIP, "hipSetDevice failed"));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipSetDevice(prev);
        return cleanup(fail(BFS_ERR_HIP, "hipGetDeviceProperties failed"));
    }
    g->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    g->small_grid = small_loop_grid(g->num_cus);

    // pinned host block: [Ctrl][Ctrl for the batch][64 batch roots]
    hipError_t e = hipHostMalloc((void**)&g->h_ctrl, 2 * sizeof(Ctrl) + 64 * sizeof(int32_t),
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipSetDevice(prev);
        return cleanup(hip_fail(e, "hipHostMalloc"));
    }
    g->h_ms_ctrl = g->h_ctrl + 1;
    g->h_roots = reinterpret_cast<int32_t*>(g->h_ctrl + 2);
    if ((e = hipEventCreate(&g->ev0)) != hipSuccess || (e = hipEventCreate(&g->ev1)) != hipSuccess) {
        (void)hipSetDevice(prev);
        return cleanup(hip_fail(e, "hipEventCreate"));
    }
    for (int i = 0; i < 5; ++i) {
        if ((e = hipEventCreate(&g->pev[i])) != hipSuccess) {
            (void)hipSetDevice(prev);
            return cleanup(hip_fail(e, "hipEventCreate"));
        }
    }

    // CSR checks (always computes the maximum degree; BFS_VALIDATE_CSR adds
    // the column-range check).
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int32_t* dflags = g->scratch;  // [0] bad bits, [1] max degree
    int32_t h[2] = {0, 0};
    e = hipMemcpyAsync(dflags, h, sizeof(h), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_validate_csr(s, V, nnz, d_row_offsets, d_col, dflags, dflags + 1,
                                1 /* column ids are always checked: a bad id would fault */);
    if (e == hipSuccess) e = hipMemcpyAsync(h, dflags, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipSetDevice(prev);
        return cleanup(hip_fail(e, "CSR check"));
    }
    if (h[0] & 3) {
        (void)hipSetDevice(prev);
        return cleanup(fail(BFS_ERR_INVALID, "row offsets are not a valid CSR (code %d)", h[0]));
    }
    if (h[0] & 4) {
        (void)hipSetDevice(prev);
        return cleanup(fail(BFS_ERR_INVALID, "a column id is outside [0, V)"));
    }
    g->maxdeg = h[1];
    {
        // symmetry (for the direction-optimizing mode): hash sums of the
        // edges and of the reversed edges
        unsigned long long* d_sums = reinterpret_cast<unsigned long long*>(
            reinterpret_cast<char*>(g->scratch) + 64);
        unsigned long long hs[4] = {0, 0, 0, 0};
        e = hipMemcpyAsync(d_sums, hs, sizeof(hs), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_symmetry_sums(s, g->num_cus * 8, V, d_row_offsets, d_col, d_sums);
        if (e == hipSuccess) e = hipMemcpyAsync(hs, d_sums, sizeof(hs), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipSetDevice(prev);
            return cleanup(hip_fail(e, "symmetry check"));
        }
        g->symmetric = hs[0] == hs[2] && hs[1] == hs[3];
    }
    if (flags & BFS_DEGREE_ORDER) {
        const int64_t tile_cap = (nnz + kMinTile - 1) / kMinTile + 1;
        int32_t* col_tmp = reinterpret_cast<int32_t*>(g->ws + L.col_tmp);
        e = build_degree_order(s, V, nnz, d_row_offsets, d_col, g->rank, g->orig,
                               const_cast<int64_t*>(g->s_off), col_tmp, g->deg, g->rowstart,
                               g->suid, g->bsum, g->tile_k, tile_cap,
                               reinterpret_cast<uint32_t*>(g->ws + L.hist), g->ctrl,
                               g->num_cus * 8);
        if (e == hipSuccess)
            e = build_row_skip(s, V, g->s_off, col_tmp, const_cast<int32_t*>(g->s_col), g->skip,
                               g->num_cus * 8);
        // the rows grouped by XCD slice, in col_tmp's space (free from here on)
        if (e == hipSuccess)
            e = build_slice_rows(s, V, g->s_off, g->s_col, g->col_x, g->xo, g->num_cus * 8);
        // internal ids run in non-increasing degree class, so the vertices
        // with a neighbour are exactly the ids below their count
        uint32_t* d_cnt = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(g->scratch) + 128);
        uint32_t h_cnt = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(d_cnt, &h_cnt, 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_count_nonzero_degree(s, g->num_cus * 8, V, g->s_off, d_cnt);
        if (e == hipSuccess) e = hipMemcpyAsync(&h_cnt, d_cnt, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipSetDevice(prev);
            return cleanup(hip_fail(e, "degree ordering"));
        }
        g->v_active = (int32_t)h_cnt;
    }
    (void)hipSetDevice(prev);
    *out = g;
    return ok();
}

int bfs_graph_destroy(bfs_graph* g)
{
    if (!g) return ok();
    if (g->ms_graph) (void)hipGraphExecDestroy(g->ms_graph);
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    if (g->h_ctrl) (void)hipHostFree(g->h_ctrl);
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
    for (int i = 0; i < 5; ++i)
        if (g->pev[i]) (void)hipEventDestroy(g->pev[i]);
    delete g;
    return ok();
}

int bfs_set_option(bfs_graph* g, int key, int64_t value)
{
    if (!g) return fail(BFS_ERR_INVALID, "graph is NULL");
    switch (key) {
    case BFS_OPT_EDGES_PER_THREAD:
        if (value != 1 && value != 2 && value != 4 && value != 8)
            return fail(BFS_ERR_INVALID, "edges per thread must be 1, 2, 4 or 8");
        g->ept = (int)value;
        break;
    case BFS_OPT_FRONTIER_MODE:
        if (value < 0 || value > 2) return fail(BFS_ERR_INVALID, "frontier mode must be 0..2");
        g->frontier_mode = (int)value;
        break;
    case BFS_OPT_LOOP_DRIVER:
        if (value < 0 || value > 2) return fail(BFS_ERR_INVALID, "loop driver must be 0..2");
        g->loop_driver = (int)value;
        break;
    case BFS_OPT_BATCH_TILE:
        if (value != 256 && value != 512 && value != 1024 && value != 2048)
            return fail(BFS_ERR_INVALID, "batch tile must be 256, 512, 1024 or 2048");
        g->batch_tile = (int)value;
        break;
    case BFS_OPT_GRID_WGS:
        if (value < 1 || value > 64) return fail(BFS_ERR_INVALID, "grid workgroups per CU must be 1..64");
        g->grid_wgs = (int)value;
        break;
    case BFS_OPT_PROFILE:
        if (value < 0 || value > 1) return fail(BFS_ERR_INVALID, "profile must be 0 or 1");
        g->profile = (int)value;
        break;
    case BFS_OPT_VISITED_SUMMARY:
        if (value < 0 || value > 2) return fail(BFS_ERR_INVALID, "visited summary must be 0, 1 or 2");
        g->use_summary = (int)value;
        break;
    case BFS_OPT_ROW_SKIP:
        if (value < 0 || value > 1) return fail(BFS_ERR_INVALID, "row skip must be 0 or 1");
        g->row_skip = (int)value;
        break;
    case BFS_OPT_LOOP_LIMIT:
        if (value < 64 || value > kSmallQ)
            return fail(BFS_ERR_INVALID, "loop limit must be 64..%d", kSmallQ);
        g->small_limit = (int32_t)value;
        break;
    case BFS_OPT_DIRECTION:
        if (value < 0 || value > 1) return fail(BFS_ERR_INVALID, "direction must be 0 or 1");
        if (value == 1 && !g->symmetric)
            return fail(BFS_ERR_INVALID,
                        "direction-optimizing search needs a symmetric CSR (this one is not)");
        g->direction = (int)value;
        break;
    case BFS_OPT_DO_ALPHA:
        if (value < 1 || value > 1000) return fail(BFS_ERR_INVALID, "alpha must be 1..1000");
        g->do_alpha = (int)value;
        break;
    case BFS_OPT_DO_BETA:
        if (value < 1 || value > 1000) return fail(BFS_ERR_INVALID, "beta must be 1..1000");
        g->do_beta = (int)value;
        break;
    case BFS_OPT_CLAIM_MODE:
        if (value < 0 || value > 2) return fail(BFS_ERR_INVALID, "claim mode must be 0..2");
        g->claim_mode = (int)value;
        break;
    case BFS_OPT_XCD_SLICES:
        if (value < 0 || value > 2) return fail(BFS_ERR_INVALID, "XCD slices must be 0..2");
        g->xcd_slices = (int)value;
        break;
    default:
        return fail(BFS_ERR_INVALID, "unknown option %d", key);
    }
    return ok();
}

int bfs_get_option(bfs_graph* g, int key, int64_t* value)
{
    if (!g || !value) return fail(BFS_ERR_INVALID, "NULL argument");
    switch (key) {
    case BFS_OPT_EDGES_PER_THREAD: *value = g->ept; break;
    case BFS_OPT_FRONTIER_MODE: *value = g->frontier_mode; break;
    case BFS_OPT_LOOP_DRIVER: *value = g->loop_driver; break;
    case BFS_OPT_BATCH_TILE: *value = g->batch_tile; break;
    case BFS_OPT_GRID_WGS: *value = g->grid_wgs; break;
    case BFS_OPT_PROFILE: *value = g->profile; break;
    case BFS_OPT_VISITED_SUMMARY: *value = g->use_summary; break;
    case BFS_OPT_ROW_SKIP: *value = g->row_skip; break;
    case BFS_OPT_DIRECTION: *value = g->direction; break;
    case BFS_OPT_LOOP_LIMIT: *value = g->small_limit; break;
    case BFS_OPT_DO_ALPHA: *value = g->do_alpha; break;
    case BFS_OPT_DO_BETA: *value = g->do_beta; break;
    case BFS_OPT_CLAIM_MODE: *value = g->claim_mode; break;
    case BFS_OPT_XCD_SLICES: *value = g->xcd_slices; break;
    default: return fail(BFS_ERR_INVALID, "unknown option %d", key);
    }
    return ok();
}

}  // extern "C"

namespace {

struct BusyGuard {
    bfs_graph* g;
    bool held;
    explicit BusyGuard(bfs_graph* gg) : g(gg), held(false)
    {
        int expect = 0;
        held = g->busy.compare_exchange_strong(expect, 1);
    }
    ~BusyGuard()
    {
        if (held) g->busy.store(0);
    }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace bfsmi {

static float event_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.f;
    return ms;
}

// The level loop for one root: heavy levels are driven from the host (one
// control-block read per level, per-level choices of summary and frontier
// form); runs of small levels go to the device loop.  A handle without
// events (the allocation-free entry point) skips the event timing and
// profiling and ends with a stream synchronisation instead.
int run_host_loop(bfs_graph* g, int32_t root, int32_t* levels, int32_t* parents,
                         hipStream_t s, bfs_stats* st)
{
    const int tile = kWG * g->ept;
    const int64_t T = ((int64_t)g->V + 31) / 32;  // list longer than the bitmap
    const int allow_bitmap = g->frontier_mode == 1 ? 0 : (g->frontier_mode == 2 ? 2 : 1);
    const int grid_cap = g->num_cus * g->grid_wgs;
    // tile_k holds ceil(nnz / kMinTile) + 2 entries; ntiles + 1 must fit
    const int64_t tile_cap = (g->nnz + kMinTile - 1) / kMinTile + 1;
    const bool timed = g->ev0 != nullptr && g->ev1 != nullptr;
    const bool prof = timed && g->profile != 0;
    bfs_stats acc{};

    // under degree order the search writes level / parent by internal id and
    // k_finish reorders them into the caller's arrays at the end
    int32_t* lv_s = g->rank ? g->lvl_int : levels;
    int32_t* pa_s = parents ? (g->rank ? g->par_int : parents) : nullptr;
    if (timed) BFS_HIP_TRY(hipEventRecord(g->ev0, s));
    // flag claims (bitmap levels mark vertices with byte stores): the init
    // clears the flags of a search that may use them
    uint8_t* const flags = g->claim_mode != 0 ? g->found : nullptr;
    BFS_HIP_TRY(launch_init(s, g->V, g->W, root, g->rank, lv_s, pa_s, g->vis, g->vis_old,
                            g->q[0], g->ctrl, grid_cap, g->rank ? 0 : 1, flags));
    const int32_t sum_words = g->summary_words;
    const int xgrid_full = g->num_cus * std::min(g->grid_wgs, expand_blocks_per_cu(g->ept, 0));
    const int xgrid_sum = g->num_cus * std::min(g->grid_wgs, expand_blocks_per_cu(g->ept, sum_words));
    // profiling only records events; their times are read once the search
    // has completed, so a profiled search adds no waits of its own
    if (prof) BFS_HIP_TRY(hipEventRecord(g->pev[4], s));
    int32_t qlen = 1;
    int32_t lvl = 1;
    int cur = 0;
    int64_t reached = 1, edges = 0, xbytes = 0, xalg = 0;
    int32_t nlevels = 1, bitmap_levels = 0, xlaunches = 0, dev_levels = 0;
    const bool dev_ok = g->loop_driver != 1 && g->small_grid > 0;
    // the persistent loop's sync block: zero once per search (each launch
    // leaves it zero; the workspace's contents before the search are unknown)
    if (dev_ok) BFS_HIP_TRY(hipMemsetAsync(g->small_sync, 0, sizeof(SmallSync), s));
    bool dev_left = false;  // the persistent loop just handed a heavy level back
    // direction-optimizing mode: the degree sum of the frontier a bottom-up
    // step searches from, and the size of the frontier before it
    const bool dir_opt = g->direction != 0 && g->symmetric;
    bool bottom_up = false;
    bool bu_done = false;  // the search has switched back from bottom-up
    int64_t bu_front_deg = 0, bu_prev = 0, examined = 0;
    int32_t bu_levels = 0;
    const int nb_grid = (int)std::max<int64_t>(
        1, std::min<int64_t>(((int64_t)g->W + kBitmapWordsPerWG - 1) / kBitmapWordsPerWG, grid_cap));
    const int sum_grid = std::max(1, std::min(grid_cap, (g->summary_blocks + 31) / 32));
    while (true) {
        if (bottom_up) {
            // one bottom-up step discovering depth lvl
            BFS_HIP_TRY(launch_bottom_up(s, grid_cap, g->V, g->rank ? g->v_active : g->V, g->W,
                                         g->s_off, g->s_col, g->orig, g->vis, g->vis_old, lv_s,
                                         pa_s, lvl, g->ctrl, sum_grid, g->summary_shift,
                                         g->summary_blocks, g->summary));
            BFS_HIP_TRY(hipMemcpyAsync(g->h_ctrl, g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
            BFS_HIP_TRY(hipStreamSynchronize(s));
            const Ctrl& c = *g->h_ctrl;
            if (c.err) return fail(BFS_ERR_HIP, "internal guard tripped (code %d)", c.err);
            const int64_t found = c.bu_found;
            edges += bu_front_deg;  // the searched frontier's vertices are reached ones
            examined += c.bu_edges;
            bu_levels++;
            if (found == 0) break;
            reached += found;
            nlevels++;
            bitmap_levels++;
            bu_front_deg = c.bu_deg;
            const bool shrinking = found < bu_prev;
            bu_prev = found;
            if (found * g->do_beta < g->V && shrinking) {
                // back to top-down: the step's vertices (vis & ~vis_old) as
                // the next queue (the kernel rewrites their level, same value)
                BFS_HIP_TRY(launch_bitmap_to_queue(s, nb_grid, g->V, g->W, g->vis, g->vis_old,
                                                   g->q[cur ^ 1], lv_s, lvl, g->ctrl));
                cur ^= 1;
                qlen = (int32_t)found;
                bottom_up = false;
                bu_done = true;  // the frontier shrinks from here on: stay top-down
            }
            lvl++;
            continue;
        }
        if (dev_ok && !dev_left && qlen <= g->small_limit) {
            BFS_HIP_TRY(launch_small_levels(s, g->small_grid, g->V, g->s_off, g->s_col, g->orig,
                                            g->vis, g->vis_old, g->q[cur], g->q[cur ^ 1], lv_s,
                                            pa_s, g->small_sync, g->small_side, g->ctrl, qlen,
                                            lvl, g->small_limit,
                                            (int64_t)g->small_grid * kSmallDeg, kSmallDeg));
            BFS_HIP_TRY(hipMemcpyAsync(g->h_ctrl, g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
            BFS_HIP_TRY(hipStreamSynchronize(s));
            const Ctrl& c = *g->h_ctrl;
            if (c.err) return fail(BFS_ERR_HIP, "internal guard tripped (code %d)", c.err);
            reached += c.reached;
            nlevels += c.levels;
            edges += c.r_total;
            examined += c.r_total;
            dev_levels += c.steps;
            cur = (cur + c.steps) & 1;
            lvl = c.level;
            qlen = c.qlen;
            if (c.done == 1) break;  // the frontier ran empty
            dev_left = true;         // done == 2: the next level is the host's
            continue;
        }
        dev_left = false;
        const int32_t* Q = g->q[cur];
        int32_t* Qn = g->q[cur ^ 1];
        int64_t rmax = (int64_t)qlen * (int64_t)g->maxdeg;
        if (rmax > g->nnz) rmax = g->nnz;
        const int64_t tiles_ub = (rmax + tile - 1) / tile;
        // heavy levels get the visited summary (a cheap pass over the bitmap):
        // the fully visited prefix always, the LDS block bits in mode 2; it
        // runs before the degree scan so the scan can drop row prefixes
        const bool use_sum = g->use_summary > 0 && rmax > T;
        const bool lds_sum = use_sum && g->use_summary == 2;
        // XCD-sliced level: each XCD probes its eighth of the bitmap (for
        // early levels with few, high-degree frontier vertices: the level
        // after the hubs on large graphs); the row prefix skip is not used
        const bool sliced =
            g->xo && g->xcd_slices != 0 && !dir_opt && (int64_t)qlen * kXcdSlices <= g->V &&
            (g->xcd_slices == 2 ||
             (g->V >= kSliceMinV && reached * kXcdSlices <= (int64_t)g->V));
        const bool skip_rows = use_sum && g->skip && g->row_skip && !sliced;
        const int grid_cap_x = lds_sum ? xgrid_sum : xgrid_full;
        const int grid = sliced
            ? (int)std::max<int64_t>(kXcdSlices, std::min<int64_t>(
                  (tiles_ub + 2 * kXcdSlices) / kXcdSlices * kXcdSlices, grid_cap_x))
            : (int)std::max<int64_t>(1, std::min<int64_t>(tiles_ub, grid_cap_x));
        if (prof) BFS_HIP_TRY(hipEventRecord(g->pev[0], s));
        if (use_sum) {
            const int gs = std::max(1, std::min(grid_cap, (g->summary_blocks + 31) / 32));
            BFS_HIP_TRY(launch_visited_summary(s, gs, g->V, g->W, g->vis, g->summary_shift,
                                               g->summary_blocks, g->summary, g->ctrl));
        }
        if (sliced)
            BFS_HIP_TRY(launch_slice_scan(s, std::max(1, std::min(grid_cap, (qlen + kWG - 1) / kWG)),
                                          Q, qlen, g->s_off, g->xo, g->orig, g->deg, g->rowstart,
                                          g->suid, g->bsum, g->cumul, g->tile_k, tile_cap, tile, T,
                                          allow_bitmap, g->ctrl));
        else
            BFS_HIP_TRY(launch_scan(s, Q, qlen, g->s_off, g->orig, g->deg, g->rowstart, g->suid,
                                    g->bsum, g->cumul, g->tile_k, tile_cap, tile, T, allow_bitmap,
                                    g->ctrl, skip_rows ? g->skip : nullptr, g->V));
        if (dir_opt && !bu_done) {
            // the frontier's edge count decides the direction (Beamer et
            // al.): bottom-up when it exceeds the unvisited vertices' edges
            // divided by alpha; the scan is then not used
            BFS_HIP_TRY(hipMemcpyAsync(g->h_ctrl, g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
            BFS_HIP_TRY(hipStreamSynchronize(s));
            if (g->h_ctrl->err)
                return fail(BFS_ERR_HIP, "internal guard tripped (code %d)", g->h_ctrl->err);
            const int64_t mf = g->h_ctrl->r + (skip_rows ? g->h_ctrl->skipped : 0);
            const int64_t mu = g->nnz - edges - mf;
            if (mf * g->do_alpha > mu) {
                if (prof) {
                    BFS_HIP_TRY(hipEventRecord(g->pev[1], s));
                    BFS_HIP_TRY(hipEventSynchronize(g->pev[1]));
                    acc.scan_ms += event_ms(g->pev[0], g->pev[1]);
                }
                bottom_up = true;
                bu_front_deg = mf;
                bu_prev = qlen;
                continue;
            }
        }
        if (prof) BFS_HIP_TRY(hipEventRecord(g->pev[1], s));
        // flags for this level's bitmap form: always in mode 2; in mode 1
        // on graphs whose flags stay in the caches, at XCD-sliced levels
        // (each XCD then reads its eighth of the flags), and on larger
        // graphs once a sixteenth of the vertices is visited (most probes
        // then stop at the visited bit and few flags are read; measured per
        // level on R-MAT 26: faster there, slower than the atomics at an
        // unsliced level after the hubs)
        uint8_t* const lflags =
            (g->claim_mode == 2 ||
             (g->claim_mode == 1 && (g->V <= kFlagAutoMaxV || sliced ||
                                     reached * 16 >= (int64_t)g->V)))
                ? flags : nullptr;
        BFS_HIP_TRY(launch_expand(s, g->ept, grid, g->V, g->rowstart, g->suid, g->cumul,
                                  g->tile_k, sliced ? g->col_x : g->s_col, g->summary,
                                  lds_sum ? sum_words : 0, g->summary_shift, use_sum ? 1 : 0,
                                  g->vis, g->vis_old, lv_s, pa_s, lvl, Qn, g->ctrl, lflags,
                                  sliced ? qlen : 0));
        xlaunches++;
        if (prof) BFS_HIP_TRY(hipEventRecord(g->pev[2], s));
        const bool maybe_bitmap = (allow_bitmap == 2 && rmax > 0) || (allow_bitmap == 1 && rmax > T);
        if (maybe_bitmap) {
            const int64_t nb = ((int64_t)g->W + kBitmapWordsPerWG - 1) / kBitmapWordsPerWG;
            const int grid2 = (int)std::max<int64_t>(1, std::min<int64_t>(nb, grid_cap));
            // the direction-optimizing mode also sums the next frontier's
            // degrees, so the next level's direction is known without a scan
            BFS_HIP_TRY(launch_bitmap_to_queue(s, grid2, g->V, g->W, g->vis, g->vis_old, Qn, lv_s,
                                               lvl, g->ctrl, dir_opt ? g->s_off : nullptr, lflags));
        }
        if (prof) BFS_HIP_TRY(hipEventRecord(g->pev[3], s));
        // the persistent loop is queued right behind the level, before the
        // read-back: it takes the next frontier from the control block and
        // runs nothing when that is empty or too large, so a run of small
        // levels after a heavy one costs no extra host round trip
        const bool spec = dev_ok && !dir_opt;
        if (spec) {
            BFS_HIP_TRY(launch_small_levels(s, g->small_grid, g->V, g->s_off, g->s_col, g->orig,
                                            g->vis, g->vis_old, Qn, g->q[cur], lv_s, pa_s,
                                            g->small_sync, g->small_side, g->ctrl, -1, lvl + 1,
                                            g->small_limit, (int64_t)g->small_grid * kSmallDeg,
                                            kSmallDeg));
        }
        BFS_HIP_TRY(hipMemcpyAsync(g->h_ctrl, g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        BFS_HIP_TRY(hipStreamSynchronize(s));
        if (g->h_ctrl->err)
            return fail(BFS_ERR_HIP, "internal guard tripped (code %d)", g->h_ctrl->err);
        if (prof) {
            acc.scan_ms += event_ms(g->pev[0], g->pev[1]);
            acc.expand_ms += event_ms(g->pev[1], g->pev[2]);
            acc.compact_ms += event_ms(g->pev[2], g->pev[3]);
        }
        const int64_t r = g->h_ctrl->r;
        const uint32_t qn = g->h_ctrl->qn_count;
        const bool bm = g->h_ctrl->bitmap_out != 0;
        edges += r + (skip_rows ? g->h_ctrl->skipped : 0);
        examined += r;
        xbytes += 4 * r + 20 * (sliced ? kXcdSlices : 1) * (int64_t)qlen + (parents ? 4 : 0) * (int64_t)qn +
                  (bm ? 0 : 8 * (int64_t)qn);

        xalg += 4 * (r + (skip_rows ? g->h_ctrl->skipped : 0)) + (parents ? 8 : 4) * (int64_t)qn;
        if (qn == 0) break;
        if (bm) bitmap_levels++;
        reached += qn;
        nlevels++;
        qlen = (int32_t)qn;
        cur ^= 1;
        lvl++;
        if (spec) {
            // what the queued persistent loop did with the next frontier
            const Ctrl& c = *g->h_ctrl;
            dev_left = true;  // a frontier it handed back goes to the host path
            if (c.steps > 0) {
                reached += c.reached;
                nlevels += c.levels;
                edges += c.r_total;
                examined += c.r_total;
                dev_levels += c.steps;
                cur = (cur + c.steps) & 1;
                lvl = c.level;
                qlen = c.qlen;
                if (c.done == 1) break;  // the frontier ran empty
            }
            continue;
        }
        if (dir_opt && bm && !bu_done) {
            // the compaction summed the new frontier's degrees: decide its
            // level's direction now (Beamer et al.'s test)
            const int64_t mf = g->h_ctrl->next_deg;
            if (mf * g->do_alpha > g->nnz - edges - mf) {
                bottom_up = true;
                bu_front_deg = mf;
                bu_prev = qlen;
            }
        }
    }
    if (g->rank) {
        if (prof) BFS_HIP_TRY(hipEventRecord(g->pev[0], s));
        const int gf = (int)std::max<int64_t>(
            1, std::min<int64_t>(((int64_t)g->V + kWG - 1) / kWG, grid_cap));
        BFS_HIP_TRY(launch_finish(s, gf, g->V, g->rank, g->vis, g->lvl_int, pa_s, levels,
                                  parents));
        if (prof) BFS_HIP_TRY(hipEventRecord(g->pev[3], s));
    }
    if (timed) {
        BFS_HIP_TRY(hipEventRecord(g->ev1, s));
        BFS_HIP_TRY(hipEventSynchronize(g->ev1));
    } else {
        BFS_HIP_TRY(hipStreamSynchronize(s));
    }
    if (g->rank && prof) acc.compact_ms += event_ms(g->pev[0], g->pev[3]);
    if (prof) acc.init_ms = event_ms(g->ev0, g->pev[4]);
    if (st) {
        *st = acc;
        st->levels = nlevels;
        st->bitmap_levels = bitmap_levels;
        st->reached = reached;
        st->edges_scanned = edges;
        st->device_ms = timed ? event_ms(g->ev0, g->ev1) : 0.0;
        st->expand_launches = xlaunches;
        st->device_loop_levels = dev_levels;
        st->expand_bytes = xbytes;
        st->expand_alg_bytes = xalg;
        st->bottom_up_levels = bu_levels;
        st->edges_examined = examined;
    }
    return ok();
}

}  // namespace bfsmi

extern "C" int bfs_run(bfs_graph* g, int32_t root, int32_t* d_levels, int32_t* d_parents,
                       void* hip_stream, bfs_stats* st)
{
    if (!g) return fail(BFS_ERR_INVALID, "graph is NULL");
    if (root < 0 || root >= g->V) return fail(BFS_ERR_INVALID, "root %d outside [0, %d)", root, g->V);
    if (!d_levels) return fail(BFS_ERR_INVALID, "levels pointer is NULL");
    BusyGuard busy(g);
    if (!busy.held) return fail(BFS_ERR_BUSY, "graph handle is in use");
    DeviceGuard dg(g->device);
    return run_host_loop(g, root, d_levels, d_parents, static_cast<hipStream_t>(hip_stream), st);
}
