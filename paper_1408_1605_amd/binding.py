"""Thin ctypes binding of libbfsmi.so (include/bfs.h).

Every function keeps the C name and only marshals arguments: device buffers
are torch tensors on the GPU (their data_ptr() is passed), streams are
torch.cuda streams (their cuda_stream handle is the hipStream_t).  All
search work runs in the library's HIP kernels; nothing here computes.
There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfsmi.so")

BFS_OK = 0
BFS_PENDING = 1
BFS_ERR_INVALID = -1
BFS_ERR_NO_DEVICE = -2
BFS_ERR_HIP = -3
BFS_ERR_WORKSPACE = -4
BFS_ERR_DEPTH = -5
BFS_ERR_BUSY = -6
BFS_ERR_BUDGET = -7
BFS_ERR_TICKET = -8

BFS_VALIDATE_CSR = 0x1
BFS_WS_BATCH = 0x2
BFS_DEGREE_ORDER = 0x4

BFS_OPT_EDGES_PER_THREAD = 1
BFS_OPT_FRONTIER_MODE = 2
BFS_OPT_LOOP_DRIVER = 3
BFS_OPT_BATCH_TILE = 4
BFS_OPT_GRID_WGS = 5
BFS_OPT_PROFILE = 6
BFS_OPT_VISITED_SUMMARY = 7
BFS_OPT_ROW_SKIP = 8
BFS_OPT_DIRECTION = 9
BFS_OPT_DO_ALPHA = 10
BFS_OPT_DO_BETA = 11
BFS_OPT_LOOP_LIMIT = 12
BFS_OPT_CLAIM_MODE = 13
BFS_OPT_XCD_SLICES = 15

BFS_SRV_NO_PERSISTENT = 0x1

BFS_2D_MSG_AUTO = 0
BFS_2D_MSG_LIST = 1
BFS_2D_MSG_BITMAP = 2

# Every symbol include/bfs.h declares.
EXPORTS = (
    "bfs_last_error", "bfs_version", "bfs_workspace_bytes", "bfs_graph_create",
    "bfs_graph_destroy", "bfs_set_option", "bfs_get_option", "bfs_run", "bfs_run_batch",
    "bfs_server_create", "bfs_server_add_graph", "bfs_submit", "bfs_poll",
    "bfs_server_completed", "bfs_server_get_stats", "bfs_server_drain", "bfs_server_destroy",
    "bfs_run_noalloc", "bfs_grid2d_workspace_bytes", "bfs_grid2d_create", "bfs_grid2d_destroy",
    "bfs_grid2d_run",
)


class BFSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("bfs error %d: %s" % (code, msg))
        self.code = code


class bfs_stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("bitmap_levels", ctypes.c_int32),
                ("reached", ctypes.c_int64), ("edges_scanned", ctypes.c_int64),
                ("device_ms", ctypes.c_double), ("init_ms", ctypes.c_double),
                ("scan_ms", ctypes.c_double), ("expand_ms", ctypes.c_double),
                ("compact_ms", ctypes.c_double), ("expand_launches", ctypes.c_int32),
                ("device_loop_levels", ctypes.c_int32), ("expand_bytes", ctypes.c_int64),
                ("expand_alg_bytes", ctypes.c_int64), ("bottom_up_levels", ctypes.c_int32),
                ("pad0", ctypes.c_int32), ("edges_examined", ctypes.c_int64)]


class bfs_server_config(ctypes.Structure):
    _fields_ = [("max_lanes", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class bfs_timing(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_int64), ("admit_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("lanes_in_batch", ctypes.c_int32)]


class bfs_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("levels", ctypes.c_uint64), ("lane_levels", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("joins", ctypes.c_uint64),
                ("device_ms", ctypes.c_double), ("arena_peak", ctypes.c_uint64),
                ("persistent_rounds", ctypes.c_uint64), ("wide_rounds", ctypes.c_uint64)]


class bfs_grid2d_stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("list_levels", ctypes.c_int32),
                ("reached", ctypes.c_int64), ("edges_scanned", ctypes.c_int64),
                ("device_ms", ctypes.c_double),
                ("expand_list_msgs", ctypes.c_int64), ("expand_bitmap_msgs", ctypes.c_int64),
                ("expand_bytes", ctypes.c_int64), ("expand_list_only_bytes", ctypes.c_int64),
                ("fold_list_msgs", ctypes.c_int64), ("fold_bitmap_msgs", ctypes.c_int64),
                ("fold_bytes", ctypes.c_int64), ("fold_list_only_bytes", ctypes.c_int64),
                ("updated", ctypes.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libbfsmi.so and declare the C signatures.  Raises if it is not
    built (run __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libbfsmi.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sz = ctypes.c_size_t
    sig = {
        "bfs_last_error": (ctypes.c_char_p, []),
        "bfs_version": (ctypes.c_int, []),
        "bfs_workspace_bytes": (ctypes.c_int, [i32, i64, u32, ctypes.POINTER(sz)]),
        "bfs_graph_create": (ctypes.c_int, [ctypes.POINTER(vp), i32, i64, vp, vp, vp, sz, u32, vp]),
        "bfs_graph_destroy": (ctypes.c_int, [vp]),
        "bfs_set_option": (ctypes.c_int, [vp, ctypes.c_int, i64]),
        "bfs_get_option": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(i64)]),
        "bfs_run": (ctypes.c_int, [vp, i32, vp, vp, vp, ctypes.POINTER(bfs_stats)]),
        "bfs_run_batch": (ctypes.c_int, [vp, ctypes.POINTER(i32), i32, vp, vp,
                                         ctypes.POINTER(bfs_stats)]),
        "bfs_server_create": (ctypes.c_int, [ctypes.POINTER(vp), vp, sz,
                                             ctypes.POINTER(bfs_server_config)]),
        "bfs_server_add_graph": (ctypes.c_int, [vp, vp, ctypes.POINTER(i32)]),
        "bfs_submit": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(ctypes.c_uint64)]),
        "bfs_poll": (ctypes.c_int, [vp, ctypes.c_uint64, vp, ctypes.POINTER(bfs_timing)]),
        "bfs_server_completed": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_uint64), i32,
                                                ctypes.POINTER(i32)]),
        "bfs_server_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(bfs_server_stats)]),
        "bfs_server_drain": (ctypes.c_int, [vp]),
        "bfs_server_destroy": (ctypes.c_int, [vp]),
        "bfs_run_noalloc": (ctypes.c_int, [i32, i64, vp, vp, i32, vp, vp, vp,
                                           ctypes.POINTER(bfs_stats)]),
        "bfs_grid2d_workspace_bytes": (ctypes.c_int, [i32, i64, i32, i32, ctypes.POINTER(sz)]),
        "bfs_grid2d_create": (ctypes.c_int, [ctypes.POINTER(vp), i32, i64, vp, vp, i32, i32, vp,
                                             sz, vp]),
        "bfs_grid2d_destroy": (ctypes.c_int, [vp]),
        "bfs_grid2d_run": (ctypes.c_int, [vp, i32, i32, vp, vp, vp,
                                          ctypes.POINTER(bfs_grid2d_stats)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code: int, allow=(BFS_OK,)) -> int:
    if code in allow:
        return code
    msg = load().bfs_last_error()
    raise BFSError(code, msg.decode() if msg else "")


def _ptr(t) -> int | None:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream) or None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None


def bfs_last_error() -> str:
    m = load().bfs_last_error()
    return m.decode() if m else ""


def bfs_version() -> int:
    return int(load().bfs_version())


def bfs_workspace_bytes(V: int, nnz: int, flags: int = 0) -> int:
    out = ctypes.c_size_t(0)
    _check(load().bfs_workspace_bytes(V, nnz, flags, ctypes.byref(out)))
    return int(out.value)


def bfs_graph_create(V: int, nnz: int, d_row_offsets, d_col, d_workspace, ws_bytes: int | None = None,
                     flags: int = 0, stream=None) -> int:
    """Returns the opaque handle (an int).  Tensors must live on the GPU."""
    h = ctypes.c_void_p(0)
    if ws_bytes is None:
        ws_bytes = d_workspace.numel() * d_workspace.element_size()
    _check(load().bfs_graph_create(ctypes.byref(h), V, nnz, _ptr(d_row_offsets), _ptr(d_col),
                                   _ptr(d_workspace), ws_bytes, flags, _stream(stream)))
    return int(h.value)


def bfs_graph_destroy(g: int) -> None:
    _check(load().bfs_graph_destroy(g))


def bfs_set_option(g: int, key: int, value: int) -> None:
    _check(load().bfs_set_option(g, key, value))


def bfs_get_option(g: int, key: int) -> int:
    v = ctypes.c_int64(0)
    _check(load().bfs_get_option(g, key, ctypes.byref(v)))
    return int(v.value)


def bfs_run(g: int, root: int, d_levels, d_parents=None, stream=None) -> bfs_stats:
    st = bfs_stats()
    _check(load().bfs_run(g, root, _ptr(d_levels), _ptr(d_parents), _stream(stream),
                          ctypes.byref(st)))
    return st


def bfs_run_noalloc(V: int, nnz: int, d_row_offsets, d_col, root: int, d_levels,
                    d_parents=None, stream=None) -> bfs_stats:
    st = bfs_stats()
    _check(load().bfs_run_noalloc(V, nnz, _ptr(d_row_offsets), _ptr(d_col), root, _ptr(d_levels),
                                  _ptr(d_parents), _stream(stream), ctypes.byref(st)))
    return st


def bfs_grid2d_workspace_bytes(V: int, nnz: int, R: int, C: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().bfs_grid2d_workspace_bytes(V, nnz, R, C, ctypes.byref(out)))
    return int(out.value)


def bfs_grid2d_create(V: int, nnz: int, d_row_offsets, d_col, R: int, C: int, d_workspace,
                      ws_bytes: int | None = None, stream=None) -> int:
    h = ctypes.c_void_p(0)
    if ws_bytes is None:
        ws_bytes = d_workspace.numel() * d_workspace.element_size()
    _check(load().bfs_grid2d_create(ctypes.byref(h), V, nnz, _ptr(d_row_offsets), _ptr(d_col),
                                    R, C, _ptr(d_workspace), ws_bytes, _stream(stream)))
    return int(h.value)


def bfs_grid2d_destroy(g: int) -> None:
    _check(load().bfs_grid2d_destroy(g))


def bfs_grid2d_run(g: int, root: int, d_levels, d_parents=None, msg_mode: int = BFS_2D_MSG_AUTO,
                   stream=None) -> bfs_grid2d_stats:
    st = bfs_grid2d_stats()
    _check(load().bfs_grid2d_run(g, root, msg_mode, _ptr(d_levels), _ptr(d_parents),
                                 _stream(stream), ctypes.byref(st)))
    return st


def bfs_run_batch(g: int, roots, d_levels, stream=None) -> bfs_stats:
    roots = [int(r) for r in roots]
    arr = (ctypes.c_int32 * max(len(roots), 1))(*roots)
    st = bfs_stats()
    _check(load().bfs_run_batch(g, arr, len(roots), _ptr(d_levels), _stream(stream),
                                ctypes.byref(st)))
    return st


def bfs_server_create(d_arena, arena_bytes: int | None = None, max_lanes: int = 64,
                      max_inflight: int = 8, flags: int = 0) -> int:
    h = ctypes.c_void_p(0)
    if arena_bytes is None:
        arena_bytes = d_arena.numel() * d_arena.element_size()
    cfg = bfs_server_config(max_lanes, max_inflight, flags, 0)
    _check(load().bfs_server_create(ctypes.byref(h), _ptr(d_arena), arena_bytes,
                                    ctypes.byref(cfg)))
    return int(h.value)


def bfs_server_add_graph(s: int, g: int) -> int:
    gid = ctypes.c_int32(-1)
    _check(load().bfs_server_add_graph(s, g, ctypes.byref(gid)))
    return int(gid.value)


def bfs_submit(s: int, graph_id: int, root: int) -> int:
    t = ctypes.c_uint64(0)
    _check(load().bfs_submit(s, graph_id, root, ctypes.byref(t)))
    return int(t.value)


def bfs_poll(s: int, ticket: int, dst_levels=None):
    """dst_levels: a host numpy int32[V] array, a device torch int32[V]
    tensor, or None.  Returns (status, bfs_timing) with status BFS_OK or
    BFS_PENDING."""
    tm = bfs_timing()
    if dst_levels is None:
        ptr = None
    elif hasattr(dst_levels, "data_ptr"):
        ptr = int(dst_levels.data_ptr())
    else:
        ptr = dst_levels.ctypes.data
    code = _check(load().bfs_poll(s, ticket, ptr, ctypes.byref(tm)), allow=(BFS_OK, BFS_PENDING))
    return code, tm


def bfs_server_completed(s: int, max_tickets: int = 4096) -> list:
    """Tickets finished since the last call (each reported once)."""
    n = ctypes.c_int32(0)
    m = max(1, int(max_tickets))
    buf = (ctypes.c_uint64 * m)()  # per call: client threads share nothing
    _check(load().bfs_server_completed(s, buf, m, ctypes.byref(n)))
    return list(buf[:n.value])


def bfs_server_get_stats(s: int) -> bfs_server_stats:
    st = bfs_server_stats()
    _check(load().bfs_server_get_stats(s, ctypes.byref(st)))
    return st


def bfs_server_drain(s: int) -> None:
    _check(load().bfs_server_drain(s))


def bfs_server_destroy(s: int) -> None:
    _check(load().bfs_server_destroy(s))


# ---------------------------------------------------------------------------
# Convenience: device-resident graph built from host CSR arrays.


@dataclass
class Graph:
    """A CSR graph resident in device memory plus its library handle.
    Owns the torch tensors it allocates (offsets, columns, workspace)."""
    V: int
    nnz: int
    off: object
    col: object
    ws: object
    handle: int

    @classmethod
    def from_csr(cls, off, col, flags: int = 0, device: str = "cuda", stream=None) -> "Graph":
        import numpy as np
        import torch
        off = np.ascontiguousarray(off, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        V = int(off.shape[0] - 1)
        nnz = int(off[-1])
        d_off = torch.from_numpy(off).to(device)
        d_col = torch.from_numpy(col if col.size else np.zeros(1, np.int32)).to(device)
        nbytes = bfs_workspace_bytes(V, nnz, flags)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        torch.cuda.synchronize()
        h = bfs_graph_create(V, nnz, d_off, d_col, ws, nbytes, flags, stream)
        return cls(V, nnz, d_off, d_col, ws, h)

    def run(self, root: int, levels=None, parents=None, want_parents: bool = True, stream=None):
        import torch
        if levels is None:
            levels = torch.empty(self.V, dtype=torch.int32, device=self.off.device)
        if parents is None and want_parents:
            parents = torch.empty(self.V, dtype=torch.int32, device=self.off.device)
        st = bfs_run(self.handle, root, levels, parents, stream)
        return levels, parents, st

    def run_batch(self, roots, levels=None, stream=None):
        import torch
        if levels is None:
            levels = torch.empty((len(roots), self.V), dtype=torch.int8, device=self.off.device)
        st = bfs_run_batch(self.handle, roots, levels, stream)
        return levels, st

    def set_option(self, key: int, value: int) -> None:
        bfs_set_option(self.handle, key, value)

    def get_option(self, key: int) -> int:
        return bfs_get_option(self.handle, key)

    def close(self) -> None:
        if self.handle:
            bfs_graph_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Grid2D:
    """A CSR partitioned over an R x C grid of virtual processors on one GPU
    (bfs_grid2d_*).  Owns its workspace tensor; the CSR tensors are needed
    only while the handle is created."""
    V: int
    nnz: int
    R: int
    C: int
    ws: object
    handle: int

    @classmethod
    def from_csr(cls, off, col, R: int, C: int, device: str = "cuda", stream=None) -> "Grid2D":
        import numpy as np
        import torch
        off = np.ascontiguousarray(off, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        V = int(off.shape[0] - 1)
        nnz = int(off[-1])
        d_off = torch.from_numpy(off).to(device)
        d_col = torch.from_numpy(col if col.size else np.zeros(1, np.int32)).to(device)
        nbytes = bfs_grid2d_workspace_bytes(V, nnz, R, C)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        torch.cuda.synchronize()
        h = bfs_grid2d_create(V, nnz, d_off, d_col, R, C, ws, nbytes, stream)
        torch.cuda.synchronize()
        del d_off, d_col
        return cls(V, nnz, R, C, ws, h)

    def run(self, root: int, msg_mode: int = BFS_2D_MSG_AUTO, want_parents: bool = True,
            levels=None, parents=None, stream=None):
        import torch
        dev = self.ws.device
        if levels is None:
            levels = torch.empty(self.V, dtype=torch.int32, device=dev)
        if parents is None and want_parents:
            parents = torch.empty(self.V, dtype=torch.int32, device=dev)
        st = bfs_grid2d_run(self.handle, root, levels, parents, msg_mode, stream)
        return levels, parents, st

    def close(self) -> None:
        if self.handle:
            bfs_grid2d_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
