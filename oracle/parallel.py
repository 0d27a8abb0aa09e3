"""Many roots of one graph at once -- TEST INFRASTRUCTURE ONLY (the same rule
as the rest of this package: only tests, the smoke check and the benchmark's
CPU-baseline leg may use it).

The serial routines of ``bfs_oracle.c`` run as ctypes foreign calls, which
release the interpreter lock, so a pool of threads runs one serial search per
host core with no process start-up and no copy of the graph.  Each search is
the plain serial oracle; nothing here splits one search over threads.

Results can be cached on disk by (CSR digest, root).  The digest is a
SHA-256 over the SHA-256 of each 64 MiB slice of the offsets and of the
column ids, so a multi-GiB graph is hashed on all threads.  Only the
oracle's own outputs are stored (levels, per-level counts, edges scanned).
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import _csr, bfs, validate

_SLICE = 64 << 20


def default_workers(n_items: int | None = None) -> int:
    """Threads for the pool: the host's cores, at most 16 (the CPU share of
    one GPU on the boxes this runs on), at most the number of items."""
    n = min(os.cpu_count() or 1, 16)
    if n_items is not None:
        n = min(n, max(int(n_items), 1))
    return max(n, 1)


def csr_digest(off, col, workers: int | None = None) -> str:
    off, col = _csr(off, col)
    views = []
    for a in (off, col):
        b = memoryview(a.reshape(-1).view(np.uint8))
        views.extend(b[i:i + _SLICE] for i in range(0, max(len(b), 1), _SLICE))

    def one(v):
        return hashlib.sha256(v).digest()

    with ThreadPoolExecutor(max_workers=workers or default_workers()) as ex:
        parts = list(ex.map(one, views))
    h = hashlib.sha256()
    h.update(np.array([off.shape[0] - 1, col.shape[0]], dtype=np.int64).tobytes())
    for p in parts:
        h.update(p)
    return h.hexdigest()


def cache_dir() -> str:
    return os.environ.get("BFSMI_ORACLE_CACHE") or os.path.join(tempfile.gettempdir(),
                                                                "bfsmi_oracle_cache")


@dataclass
class RootResult:
    root: int
    level: np.ndarray            # int32[V]
    frontier_sizes: np.ndarray   # int64[nlevels]
    edges_scanned: int
    seconds: float               # serial oracle time (0 when read from the cache)
    cached: bool

    @property
    def nlevels(self) -> int:
        return int(self.frontier_sizes.shape[0])

    @property
    def reached(self) -> int:
        return int(self.frontier_sizes.sum())


_SRC_TAG = None


def _source_tag() -> str:
    """Results are only reused by the same oracle source."""
    global _SRC_TAG
    if _SRC_TAG is None:
        from . import _SRC
        with open(_SRC, "rb") as f:
            _SRC_TAG = hashlib.sha256(f.read()).hexdigest()[:12]
    return _SRC_TAG


def _paths(digest: str, root: int):
    d = os.path.join(cache_dir(), digest[:32] + "_" + _source_tag())
    return d, os.path.join(d, "r%d.npy" % root), os.path.join(d, "r%d.json" % root)


def _load_cached(digest: str, root: int):
    _, pl, pj = _paths(digest, root)
    try:
        with open(pj) as f:
            meta = json.load(f)
        lv = np.load(pl, allow_pickle=False).astype(np.int32)
    except (OSError, ValueError, KeyError):
        return None
    return RootResult(root, lv, np.asarray(meta["frontier_sizes"], dtype=np.int64),
                      int(meta["edges_scanned"]), 0.0, True)


def _store(digest: str, res: RootResult) -> None:
    d, pl, pj = _paths(digest, res.root)
    try:
        os.makedirs(d, exist_ok=True)
        top = int(res.level.max(initial=-1))
        dt = np.int8 if top <= 127 else (np.int16 if top <= 32767 else np.int32)
        tmp = pl + ".tmp%d_%d" % (os.getpid(), res.root)
        with open(tmp, "wb") as f:
            np.save(f, res.level.astype(dt), allow_pickle=False)
        os.replace(tmp, pl)
        tmp = pj + ".tmp%d_%d" % (os.getpid(), res.root)
        with open(tmp, "w") as f:
            json.dump({"frontier_sizes": [int(x) for x in res.frontier_sizes],
                       "edges_scanned": int(res.edges_scanned)}, f)
        os.replace(tmp, pj)
    except OSError:
        pass  # a cache that cannot be written only costs time


def _one(off, col, root: int, digest: str | None, read: bool = True) -> RootResult:
    if digest is not None and read:
        hit = _load_cached(digest, root)
        if hit is not None:
            return hit
    t = time.perf_counter()
    r = bfs(off, col, root)
    dt = time.perf_counter() - t
    res = RootResult(int(root), r.level, r.frontier_sizes, r.edges_scanned, dt, False)
    if digest is not None:
        _store(digest, res)
    return res


def bfs_roots(off, col, roots, workers: int | None = None, cache: bool = True,
              fresh: bool = False, digest: str | None = None):
    """Oracle levels for every root, one serial search per thread.  With
    fresh, every search runs (for timing) and its result is still stored
    when cache is on.  Returns (results in root order, wall seconds,
    threads used)."""
    off, col = _csr(off, col)
    roots = [int(r) for r in roots]
    n = default_workers(len(roots)) if workers is None else max(1, min(workers, len(roots) or 1))
    if cache and digest is None:
        digest = csr_digest(off, col, n)
    dig = digest if cache else None
    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=n) as ex:
        out = list(ex.map(lambda r: _one(off, col, r, dig, not fresh), roots))
    return out, time.perf_counter() - t, n


@dataclass
class Check:
    root: int
    levels_equal: bool
    first_diff: list             # up to 8 vertex ids where the levels differ
    validate_code: int           # 0, or the failing invariant (parents given)
    bad_vertex: int
    reached: int
    nlevels: int
    edges_scanned: int
    oracle_seconds: float
    cached: bool

    @property
    def ok(self) -> bool:
        return self.levels_equal and self.validate_code == 0


def check_roots(off, col, items, workers: int | None = None, directed: bool = False,
                comp=None, cache: bool = True, digest: str | None = None):
    """items: (root, levels, parents or None) triples from the path under
    test.  For each, the oracle's levels must equal `levels` element by
    element, and (levels, parents) must pass the tree validator.  Runs on a
    pool of threads; returns one Check per item, in order."""
    off, col = _csr(off, col)
    items = list(items)
    n = default_workers(len(items)) if workers is None else max(1, min(workers, len(items) or 1))
    if cache and digest is None:
        digest = csr_digest(off, col, n)
    if not cache:
        digest = None

    def run(it):
        root, lv, pa = it
        ref = _one(off, col, int(root), digest)
        lv = np.asarray(lv).astype(np.int32, copy=False)
        eq = lv.shape == ref.level.shape and bool(np.array_equal(lv, ref.level))
        diff = [] if eq else [int(x) for x in np.nonzero(lv != ref.level)[0][:8]]
        code, bad = 0, -1
        if pa is not None:
            code, bad = validate(off, col, int(root), lv, pa, directed=directed, comp=comp)
        return Check(int(root), eq, diff, code, bad, ref.reached, ref.nlevels,
                     ref.edges_scanned, ref.seconds, ref.cached)

    with ThreadPoolExecutor(max_workers=n) as ex:
        return list(ex.map(run, items))
