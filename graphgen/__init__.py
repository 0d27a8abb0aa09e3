"""Seeded synthetic graph inputs (R-MAT and 2-D grids) in symmetric CSR form.

Both the CPU oracle and the GPU library take their inputs from here; this
module holds none of the breadth-first search itself.  The generator is
written in C (``graphgen.c``) and loaded with ctypes.

Workload recipe (the paper's benchmark graphs, Section 4 and Table 1): R-MAT
with quadrant probabilities A, B, C (D = 1 - A - B - C), edgefactor generated
edges per vertex, vertex ids relabelled by a keyed permutation, each edge
mirrored to make the graph undirected, self-loops dropped, duplicates merged,
rows sorted.  Row offsets are int64, column indices int32.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

# Defaults of the benchmark workloads.
RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19
EDGEFACTOR = 16


def graph_seed(scale: int) -> int:
    return 1000 + scale


def root_seed(scale: int) -> int:
    return 2000 + scale


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
             "-std=gnu11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.gg_rmat_csr.restype = ctypes.c_int64
        lib.gg_rmat_csr.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                    ctypes.c_int, i64p, i32p]
        lib.gg_grid_csr.restype = ctypes.c_int64
        lib.gg_grid_csr.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, i32p]
        lib.gg_pick_roots.restype = ctypes.c_int32
        lib.gg_pick_roots.argtypes = [ctypes.c_int32, i64p, ctypes.c_int32,
                                      ctypes.c_uint64, i32p]
        lib.gg_rmat_edges.restype = None
        lib.gg_rmat_edges.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                      ctypes.c_int, u32p, u32p]
        lib.gg_permute.restype = ctypes.c_uint32
        lib.gg_permute.argtypes = [ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64]
        lib.gg_splitmix64.restype = ctypes.c_uint64
        lib.gg_splitmix64.argtypes = [ctypes.c_uint64]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


@dataclass
class CSR:
    """Symmetric CSR graph: row r's neighbours are col[off[r]:off[r+1]]."""
    off: np.ndarray  # int64[V + 1]
    col: np.ndarray  # int32[nnz]
    name: str = ""

    @property
    def V(self) -> int:
        return int(self.off.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.off[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.off)


def rmat(scale: int, edgefactor: int = EDGEFACTOR, A: float = RMAT_A, B: float = RMAT_B,
         C: float = RMAT_C, seed: int | None = None, relabel: bool = True) -> CSR:
    """R-MAT graph, symmetrised, self-loops dropped, duplicates merged."""
    if seed is None:
        seed = graph_seed(scale)
    V = 1 << scale
    off = np.empty(V + 1, dtype=np.int64)
    # Upper bound before merging; pages past nnz are never touched.
    col = np.empty(2 * edgefactor * V, dtype=np.int32)
    nnz = _load().gg_rmat_csr(scale, edgefactor, A, B, C, seed & (2**64 - 1), int(relabel),
                              _ptr(off, ctypes.c_int64), _ptr(col, ctypes.c_int32))
    if nnz < 0:
        raise MemoryError("gg_rmat_csr failed (scale=%d)" % scale)
    return CSR(off, col[:nnz], name="rmat%d" % scale)


def rmat_edges(scale: int, n_edges: int, A: float = RMAT_A, B: float = RMAT_B,
               C: float = RMAT_C, seed: int = 0, relabel: bool = True):
    """The raw generated (src, dst) list, before symmetrisation."""
    src = np.empty(n_edges, dtype=np.uint32)
    dst = np.empty(n_edges, dtype=np.uint32)
    _load().gg_rmat_edges(scale, n_edges, A, B, C, seed & (2**64 - 1), int(relabel),
                          _ptr(src, ctypes.c_uint32), _ptr(dst, ctypes.c_uint32))
    return src, dst


def permute(v: int, scale: int, key: int) -> int:
    return int(_load().gg_permute(v, scale, key & (2**64 - 1)))


def splitmix64(z: int) -> int:
    return int(_load().gg_splitmix64(z & (2**64 - 1)))


def grid(w: int, h: int | None = None) -> CSR:
    """4-neighbour 2-D grid, id = row * w + column."""
    if h is None:
        h = w
    V = w * h
    off = np.empty(V + 1, dtype=np.int64)
    col = np.empty(max(2 * (2 * V - w - h), 1), dtype=np.int32)
    nnz = _load().gg_grid_csr(w, h, _ptr(off, ctypes.c_int64), _ptr(col, ctypes.c_int32))
    return CSR(off, col[:nnz], name="grid%dx%d" % (w, h))


def pick_roots(g: CSR, n: int, seed: int) -> np.ndarray:
    """n distinct roots, uniform among vertices with degree > 0."""
    out = np.empty(n, dtype=np.int32)
    got = _load().gg_pick_roots(g.V, _ptr(g.off, ctypes.c_int64), n, seed & (2**64 - 1),
                                _ptr(out, ctypes.c_int32))
    return out[:got]


def from_edges(V: int, src, dst, symmetric: bool = True) -> CSR:
    """CSR from an explicit edge list (small test graphs).  With symmetric
    set, each edge is mirrored; self-loops and duplicates are kept as given
    so tests can exercise them."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if symmetric:
        s = np.concatenate([src, dst])
        d = np.concatenate([dst, src])
    else:
        s, d = src, dst
    order = np.lexsort((d, s))
    s, d = s[order], d[order]
    off = np.zeros(V + 1, dtype=np.int64)
    np.add.at(off, s + 1, 1)
    off = np.cumsum(off).astype(np.int64)
    return CSR(off, d.astype(np.int32), name="edges")


def from_dense(adj) -> CSR:
    """CSR from a dense 0/1 adjacency matrix (row u lists u's out-neighbours)."""
    adj = np.asarray(adj, dtype=bool)
    V = adj.shape[0]
    off = np.zeros(V + 1, dtype=np.int64)
    off[1:] = np.cumsum(adj.sum(axis=1))
    col = np.nonzero(adj)[1].astype(np.int32)
    return CSR(off, col, name="dense")
