"""Autotuner for the search's launch knobs.

Knobs: edges per thread (tile size), the visited-summary mode and
workgroups per CU for the single-root path, and the tile size of the batch
expansion.  Every candidate is first checked for parity: its levels (and
batch rows) must equal those of a reference configuration (list frontier,
one edge per thread, no summary) on the same roots, which the GPU tests pin
to the CPU oracle; only then is it timed.  The best configuration is cached
as JSON per (GPU architecture, graph class, scale).
"""
from __future__ import annotations

import json
import os
import time

from . import binding as B

CACHE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned")


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", "gpu").split(":")[0]


def cache_path(graph_class: str, scale: int) -> str:
    return os.path.join(CACHE_DIR, "%s_%s_%d.json" % (_arch(), graph_class, scale))


def _levels(G, root, lv):
    import torch
    B.bfs_run(G.handle, root, lv, None)
    torch.cuda.synchronize()
    return lv.clone()


def tune_single(G, roots, reps: int = 3, log=None):
    """Returns (best_config, table).  G is a binding.Graph."""
    import torch
    lv = torch.empty(G.V, dtype=torch.int32, device="cuda")
    saved = {k: B.bfs_get_option(G.handle, k) for k in
             (B.BFS_OPT_EDGES_PER_THREAD, B.BFS_OPT_VISITED_SUMMARY, B.BFS_OPT_FRONTIER_MODE,
              B.BFS_OPT_GRID_WGS)}
    # reference outputs
    B.bfs_set_option(G.handle, B.BFS_OPT_EDGES_PER_THREAD, 1)
    B.bfs_set_option(G.handle, B.BFS_OPT_VISITED_SUMMARY, 0)
    B.bfs_set_option(G.handle, B.BFS_OPT_FRONTIER_MODE, 1)
    ref = [_levels(G, r, lv) for r in roots]
    B.bfs_set_option(G.handle, B.BFS_OPT_FRONTIER_MODE, 0)
    table = []
    for ept in (1, 2, 4, 8):
        for summ in (0, 1, 2):
            for wgs in (4, 8):
                B.bfs_set_option(G.handle, B.BFS_OPT_EDGES_PER_THREAD, ept)
                B.bfs_set_option(G.handle, B.BFS_OPT_VISITED_SUMMARY, summ)
                B.bfs_set_option(G.handle, B.BFS_OPT_GRID_WGS, wgs)
                ok = all(bool(torch.equal(_levels(G, r, lv), x)) for r, x in zip(roots, ref))
                ms = None
                if ok:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        for r in roots:
                            B.bfs_run(G.handle, r, lv, None)
                    torch.cuda.synchronize()
                    ms = (time.perf_counter() - t0) * 1e3 / (reps * len(roots))
                row = {"ept": ept, "summary": summ, "grid_wgs": wgs, "parity": ok, "ms": ms}
                table.append(row)
                if log:
                    log("tune single %s" % row)
    for k, v in saved.items():
        B.bfs_set_option(G.handle, k, v)
    good = [t for t in table if t["parity"]]
    best = min(good, key=lambda t: t["ms"]) if good else None
    return best, table


def tune_batch(G, roots, reps: int = 2, log=None):
    """Batch tile size; G must have been created with BFS_WS_BATCH."""
    import torch
    out = torch.empty((len(roots), G.V), dtype=torch.int8, device="cuda")
    saved = B.bfs_get_option(G.handle, B.BFS_OPT_BATCH_TILE)
    B.bfs_set_option(G.handle, B.BFS_OPT_BATCH_TILE, 256)
    B.bfs_run_batch(G.handle, roots, out)
    torch.cuda.synchronize()
    ref = out.clone()
    table = []
    for tile in (256, 512, 1024, 2048):
        B.bfs_set_option(G.handle, B.BFS_OPT_BATCH_TILE, tile)
        B.bfs_run_batch(G.handle, roots, out)
        torch.cuda.synchronize()
        ok = bool(torch.equal(out, ref))
        ms = None
        if ok:
            t0 = time.perf_counter()
            for _ in range(reps):
                B.bfs_run_batch(G.handle, roots, out)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
        row = {"batch_tile": tile, "parity": ok, "ms": ms}
        table.append(row)
        if log:
            log("tune batch %s" % row)
    B.bfs_set_option(G.handle, B.BFS_OPT_BATCH_TILE, saved)
    good = [t for t in table if t["parity"]]
    best = min(good, key=lambda t: t["ms"]) if good else None
    return best, table


def save(graph_class: str, scale: int, result: dict) -> str:
    os.makedirs(CACHE_DIR, exist_ok=True)
    path = cache_path(graph_class, scale)
    with open(path, "w") as f:
        json.dump(result, f, indent=1)
    return path


def load_cached(graph_class: str, scale: int):
    path = cache_path(graph_class, scale)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def apply(G, cfg: dict) -> None:
    """Set a tuned single-root configuration on a graph handle."""
    if not cfg:
        return
    if "ept" in cfg:
        B.bfs_set_option(G.handle, B.BFS_OPT_EDGES_PER_THREAD, int(cfg["ept"]))
    if "summary" in cfg:
        B.bfs_set_option(G.handle, B.BFS_OPT_VISITED_SUMMARY, int(cfg["summary"]))
    if "grid_wgs" in cfg:
        B.bfs_set_option(G.handle, B.BFS_OPT_GRID_WGS, int(cfg["grid_wgs"]))
    if "batch_tile" in cfg:
        B.bfs_set_option(G.handle, B.BFS_OPT_BATCH_TILE, int(cfg["batch_tile"]))
