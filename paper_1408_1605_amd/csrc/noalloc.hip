// Allocation-free single-root search: bfs_run_noalloc.
//
// The same level loop as bfs_run on the caller's plain CSR, with every
// scratch array of the search (visited bitmaps, queues, degree scan,
// control block, persistent-loop state) carved out of one file-scope device
// array instead of a caller workspace.  The host side makes no device or
// pinned-host allocation and creates no events or streams: the control
// block is read back into a pageable per-device host mirror, and the CSR
// checks run on every call (their flags live in the same array).
//
// The array's host-side name is not a device address.  Each device's copy
// is located once, with that device current, by hipGetSymbolAddress, and
// only that address is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <chrono>
#include <mutex>

#include "runtime.h"

namespace bfsmi {
namespace {

constexpr size_t kNoAllocBytes = (size_t)32 << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

}  // namespace
}  // namespace bfsmi

static __device__ __align__(256) unsigned char scratch[bfsmi::kNoAllocBytes];

namespace bfsmi {
namespace {

struct NoAllocDevice {
    bool ready = false;
    char* base = nullptr;  // this device's copy of `scratch`
    int num_cus = 0;
    int small_grid = 0;
    Ctrl h_ctrl{};         // pageable host mirror of the control block
    int32_t h_flags[2] = {0, 0};
};

NoAllocDevice g_na[kMaxDevices];
std::mutex g_na_mu;

// Looks up this device's copy of the array (once per device, with the device
// current) and the launch sizes that depend on the device.
int noalloc_setup(int dev, NoAllocDevice** out)
{
    std::lock_guard<std::mutex> lk(g_na_mu);
    NoAllocDevice& d = g_na[dev];
    if (!d.ready) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || (uintptr_t)p % 256 != 0)
            return fail(BFS_ERR_HIP, "static scratch array has no usable device address");
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 1)
            cus = 256;
        d.base = static_cast<char*>(p);
        d.num_cus = cus;
        d.small_grid = small_loop_grid(cus);
        d.ready = true;
    }
    *out = &d;
    return BFS_OK;
}

}  // namespace
}  // namespace bfsmi

using namespace bfsmi;

extern "C" int bfs_run_noalloc(int32_t V, int64_t nnz, const int64_t* d_row_offsets,
                               const int32_t* d_col, int32_t root, int32_t* d_levels,
                               int32_t* d_parents, void* hip_stream, bfs_stats* st)
{
    if (V < 1) return fail(BFS_ERR_INVALID, "V must be >= 1 (got %d)", V);
    if (nnz < 0 || nnz > ((int64_t)1 << 62)) return fail(BFS_ERR_INVALID, "nnz out of range");
    if (!d_row_offsets) return fail(BFS_ERR_INVALID, "row offsets pointer is NULL");
    if (!d_col && nnz > 0) return fail(BFS_ERR_INVALID, "column pointer is NULL");
    if (!d_levels) return fail(BFS_ERR_INVALID, "levels pointer is NULL");
    if (root < 0 || root >= V) return fail(BFS_ERR_INVALID, "root %d outside [0, %d)", root, V);
    const WsLayout L = ws_layout(V, nnz, 0);
    if (L.total > kNoAllocBytes)
        return fail(BFS_ERR_WORKSPACE,
                    "V = %d, nnz = %lld need %zu bytes of scratch; the static array holds %zu",
                    V, (long long)nnz, L.total, kNoAllocBytes);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(BFS_ERR_NO_DEVICE, "no HIP device");
    if (dev < 0 || dev >= kMaxDevices) return fail(BFS_ERR_NO_DEVICE, "device %d out of range", dev);
    NoAllocDevice* d = nullptr;
    const int rc = noalloc_setup(dev, &d);
    if (rc != BFS_OK) return rc;

    // a handle on the stack over the static array (plain CSR, no events)
    bfs_graph g;
    g.V = V;
    g.nnz = nnz;
    g.W = (int32_t)(((int64_t)V + 31) / 32);
    g.off = d_row_offsets;
    g.col = d_col;
    g.ws = d->base;
    g.ws_bytes = kNoAllocBytes;
    g.flags = 0;
    g.device = dev;
    g.num_cus = d->num_cus;
    g.small_grid = d->small_grid;
    g.h_ctrl = &d->h_ctrl;
    bind_workspace(&g, d->base, L, 0);

    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // CSR checks and the largest degree (the level loop sizes its grids by it)
    d->h_flags[0] = d->h_flags[1] = 0;
    BFS_HIP_TRY(hipMemcpyAsync(g.scratch, d->h_flags, sizeof(d->h_flags), hipMemcpyHostToDevice, s));
    BFS_HIP_TRY(launch_validate_csr(s, V, nnz, d_row_offsets, d_col, g.scratch, g.scratch + 1, 1));
    BFS_HIP_TRY(hipMemcpyAsync(d->h_flags, g.scratch, sizeof(d->h_flags), hipMemcpyDeviceToHost, s));
    BFS_HIP_TRY(hipStreamSynchronize(s));
    if (d->h_flags[0] & 3) return fail(BFS_ERR_INVALID, "row offsets are not a valid CSR (code %d)", d->h_flags[0]);
    if (d->h_flags[0] & 4) return fail(BFS_ERR_INVALID, "a column id is outside [0, V)");
    g.maxdeg = d->h_flags[1];

    const int r = run_host_loop(&g, root, d_levels, d_parents, s, st);
    if (r == BFS_OK && st)
        st->device_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return r;
}
