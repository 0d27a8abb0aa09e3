"""CPU oracle for the BFS path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library and its Python binding
never import it and share no code with it.

``bfs_oracle.c`` holds the quantity the paper's search computes (Algorithms 1
and 2: every reached vertex's level is its hop distance from the root) written
from its definition as a plain serial first-in first-out traversal, a
union-find connected-components routine, and a validator of the BFS-tree
invariants.  ``parallel.py`` runs many roots of the same graph at once in
forked worker processes (one serial search per worker) and caches results by
(CSR digest, root).  Everything here is integer arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

INVARIANTS = {
    0: "ok",
    1: "V1 root level/parent",
    2: "V2 parent is not a neighbour",
    3: "V3 parent level is not level-1",
    4: "V4 edge spans more than one level / reached-unreached edge",
    5: "V5 reached set differs from the root's component (cross-check)",
    6: "V6 unreached vertex with level/parent set",
}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (serial, -O3)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _bind(path: str):
    """Load an oracle shared library and declare its signatures."""
    lib = ctypes.CDLL(path)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_bfs.restype = ctypes.c_int32
    lib.oracle_bfs.argtypes = [ctypes.c_int32, i64p, i32p, ctypes.c_int32, i32p, i32p,
                               i64p, i64p]
    lib.oracle_components.restype = ctypes.c_int32
    lib.oracle_components.argtypes = [ctypes.c_int32, i64p, i32p, i32p]
    lib.oracle_validate.restype = ctypes.c_int32
    lib.oracle_validate.argtypes = [ctypes.c_int32, i64p, i32p, ctypes.c_int32, i32p, i32p,
                                    ctypes.c_int32, ctypes.c_int32, i32p, i32p]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _bind(_LIB)
    return _lib


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _csr(off, col):
    off = np.ascontiguousarray(off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return off, col


@dataclass
class BFSResult:
    level: np.ndarray           # int32[V], -1 = unreached
    parent: np.ndarray          # int32[V], -1 = unreached, parent[root] = root
    frontier_sizes: np.ndarray  # int64[nlevels], level 0 first
    edges_scanned: int          # sum of out-degrees over reached vertices

    @property
    def nlevels(self) -> int:
        return int(self.frontier_sizes.shape[0])

    @property
    def reached(self) -> int:
        return int(self.frontier_sizes.sum())


def bfs(off, col, root: int) -> BFSResult:
    """Hop distances (levels) and one valid parent per vertex from root,
    by a serial first-in first-out traversal."""
    off, col = _csr(off, col)
    V = off.shape[0] - 1
    if not 0 <= root < V:
        raise ValueError("root out of range")
    level = np.empty(V, dtype=np.int32)
    parent = np.empty(V, dtype=np.int32)
    fs = np.empty(V + 1, dtype=np.int64)
    scanned = ctypes.c_int64(0)
    n = _load().oracle_bfs(V, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32), int(root),
                           _p(level, ctypes.c_int32), _p(parent, ctypes.c_int32),
                           _p(fs, ctypes.c_int64), ctypes.byref(scanned))
    if n < 0:
        raise MemoryError("oracle_bfs failed")
    return BFSResult(level, parent, fs[:n].copy(), int(scanned.value))


def components(off, col) -> np.ndarray:
    """comp[v] = smallest vertex id in v's connected component (union-find)."""
    off, col = _csr(off, col)
    V = off.shape[0] - 1
    comp = np.empty(V, dtype=np.int32)
    if _load().oracle_components(V, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32),
                                 _p(comp, ctypes.c_int32)) != 0:
        raise MemoryError("oracle_components failed")
    return comp


def validate(off, col, root: int, level, parent, directed: bool = False,
             rows_sorted: bool = True, comp=None):
    """Check the BFS-tree invariants V1..V6. Returns (code, bad_vertex);
    code 0 means valid, see INVARIANTS for the others.  comp (the labels
    from components(), undirected graphs only) adds the V5 cross-check."""
    off, col = _csr(off, col)
    V = off.shape[0] - 1
    level = np.ascontiguousarray(level, dtype=np.int32)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    if level.shape[0] != V or parent.shape[0] != V:
        raise ValueError("level/parent length must be V")
    cptr = None
    if comp is not None:
        comp = np.ascontiguousarray(comp, dtype=np.int32)
        if comp.shape[0] != V:
            raise ValueError("comp length must be V")
        cptr = _p(comp, ctypes.c_int32)
    bad = ctypes.c_int32(-1)
    code = _load().oracle_validate(V, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32),
                                   int(root), _p(level, ctypes.c_int32),
                                   _p(parent, ctypes.c_int32), int(directed),
                                   int(rows_sorted), cptr, ctypes.byref(bad))
    if code < 0:
        raise ValueError("oracle_validate: bad arguments")
    return int(code), int(bad.value)


def levels_hist(level: np.ndarray) -> np.ndarray:
    """Count of vertices per level 0..max (unreached excluded)."""
    lv = level[level >= 0]
    return np.bincount(lv) if lv.size else np.zeros(0, dtype=np.int64)


def batch_levels_int8(off, col, roots) -> np.ndarray:
    """Per-root levels for a multi-source batch: int8[n_roots][V] with -1 for
    unreached, each row an independent single-root search.  Raises if any
    level exceeds 127."""
    rows = []
    for r in roots:
        lv = bfs(off, col, int(r)).level
        if lv.max(initial=-1) > 127:
            raise OverflowError("level exceeds int8")
        rows.append(lv.astype(np.int8))
    return np.stack(rows) if rows else np.zeros((0, np.asarray(off).shape[0] - 1), np.int8)
