#!/usr/bin/env python3
"""Benchmark of the single-GPU BFS path.

Headline: GTEPS of single-root searches on R-MAT scale 26 (edgefactor 16,
A/B/C = 0.57/0.19/0.19, relabelled, symmetrised, deduplicated), one search
per step from seeded roots of degree > 0, inputs resident in HBM.  TEPS
counts the undirected edges of the traversed component (half the directed
CSR entries scanned) over the search time; the value is the harmonic mean
over the timed steps, as the paper reports TEPS (Section 4).

The JSON line also carries:
  roofline     -- the expansion kernel's algorithmic bytes / its summed
                  duration (HIP events around each launch, same stream),
                  against the MI355X HBM peak of 8 TB/s;
  cpu_baseline -- the serial CPU oracle on one root of the same graph, on
                  this host's cores (one thread), in GTEPS;
  batch, serve -- multi-source batch throughput and serving latency, when
                  those paths are enabled (--batch / --serve).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--scale S]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "GTEPS single-root at R-MAT scale 26; batched roots/sec; p99 query latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def harmonic_mean(xs):
    xs = [x for x in xs if x > 0]
    return len(xs) / sum(1.0 / x for x in xs) if xs else 0.0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def single_root(args, torch, np, graphgen, bfsmi):
    t = time.time()
    g = graphgen.rmat(args.scale)
    log("generated R-MAT scale %d: V=%d nnz=%d in %.1fs" % (args.scale, g.V, g.nnz, time.time() - t))
    roots = graphgen.pick_roots(g, args.roots, graphgen.root_seed(args.scale))
    t = time.time()
    flags = 0 if args.no_degree_order else bfsmi.BFS_DEGREE_ORDER
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=flags)
    log("uploaded and created graph handle (flags %d) in %.1fs" % (flags, time.time() - t))
    if args.summary >= 0:
        G.set_option(bfsmi.BFS_OPT_VISITED_SUMMARY, args.summary)
    if args.ept:
        G.set_option(bfsmi.BFS_OPT_EDGES_PER_THREAD, args.ept)
    G.set_option(bfsmi.BFS_OPT_PROFILE, 1)
    levels = torch.empty(g.V, dtype=torch.int32, device="cuda")
    parents = torch.empty(g.V, dtype=torch.int32, device="cuda")
    for i in range(args.warmup):
        bfsmi.bfs_run(G.handle, int(roots[i % len(roots)]), levels, parents)
    torch.cuda.synchronize()

    stats, times = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = int(roots[i % len(roots)])
        ts = time.perf_counter()
        st = bfsmi.bfs_run(G.handle, r, levels, parents)
        times.append(time.perf_counter() - ts)
        stats.append(st)
        log("step %d root %d: %.3f ms, levels %d (bitmap %d), reached %d, E_r %d, %.1f GTEPS"
            % (i, r, times[-1] * 1e3, st.levels, st.bitmap_levels, st.reached, st.edges_scanned,
               st.edges_scanned / 2 / times[-1] / 1e9))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0

    teps = [st.edges_scanned / 2 / dt / 1e9 for st, dt in zip(stats, times)]
    gteps = harmonic_mean(teps)
    x_bytes = sum(st.expand_bytes for st in stats)
    x_ms = sum(st.expand_ms for st in stats)
    x_launch = sum(st.expand_launches for st in stats)
    achieved = x_bytes / (x_ms * 1e-3) / 1e9 if x_ms > 0 else 0.0
    # whole-search algorithmic bytes: init 8.125 V, 32 per reached vertex,
    # 4 per scanned directed edge
    b_alg = [8.125 * g.V + 32 * st.reached + 4 * st.edges_scanned for st in stats]
    bfs_gbs = sum(b_alg) / sum(times) / 1e9
    breakdown = {k: round(sum(getattr(st, k) for st in stats) / len(stats), 4)
                 for k in ("init_ms", "scan_ms", "expand_ms", "compact_ms", "device_ms")}
    res = {
        "gteps": gteps,
        "ms_per_step": total * 1e3 / args.steps,
        "median_gteps": sorted(teps)[len(teps) // 2],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_expand<%d>" % bfsmi.bfs_get_option(G.handle, bfsmi.BFS_OPT_EDGES_PER_THREAD),
                     "launches": x_launch,
                     "avg_launch_ms": round(x_ms / max(x_launch, 1), 5),
                     "alg_bytes_per_launch": x_bytes // max(x_launch, 1)},
        "bfs_alg_gbs": round(bfs_gbs, 1),
        "bfs_roofline_frac": round(bfs_gbs / HBM_PEAK_GBS, 4),
        "breakdown_ms_per_root": breakdown,
        "levels": stats[0].levels if stats else 0,
        "reached": stats[0].reached if stats else 0,
        "edges_scanned": stats[0].edges_scanned if stats else 0,
    }

    if not args.no_cpu_baseline:
        import oracle
        r0 = int(roots[0])
        log("cpu baseline: serial oracle from root %d ..." % r0)
        ts = time.perf_counter()
        ref = oracle.bfs(g.off, g.col, r0)
        dt = time.perf_counter() - ts
        res["cpu_baseline"] = {"value": round(ref.edges_scanned / 2 / dt / 1e9, 5), "unit": "GTEPS",
                               "cores": 1, "kind": "oracle",
                               "sample": "1 root (%d) of the same R-MAT scale %d graph, serial C "
                                         "oracle, %.1f s" % (r0, args.scale, dt),
                               "cpu": cpu_model(), "host_cores": os.cpu_count()}
        bfsmi.bfs_run(G.handle, r0, levels, parents)
        torch.cuda.synchronize()
        lv = levels.cpu().numpy()
        res["parity_root0"] = bool(np.array_equal(lv, ref.level))
        log("parity of root %d vs oracle: %s" % (r0, res["parity_root0"]))
    G.close()
    return res, g


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--roots", type=int, default=16)
    ap.add_argument("--ept", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-degree-order", action="store_true")
    ap.add_argument("--summary", type=int, default=-1)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the single-GPU search has no "
              "multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    from __graft_entry__ import _ensure_built
    _ensure_built()
    import paper_1408_1605_amd as bfsmi

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    res, g = single_root(args, torch, np, graphgen, bfsmi)

    out = {
        "metric": METRIC,
        "value": round(res["gteps"], 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic R-MAT (seeded generator, Graph500 parameters), seeded roots",
        "config": {"workload": "rmat%d_single_root" % args.scale, "scale": args.scale,
                   "degree_order": not args.no_degree_order,
                   "edgefactor": 16, "A": 0.57, "B": 0.19, "C": 0.19, "V": g.V, "nnz": g.nnz,
                   "roots": args.roots, "levels_root0": res["levels"],
                   "reached_root0": res["reached"], "edges_scanned_root0": res["edges_scanned"]},
        "roofline": res["roofline"],
        "median_gteps": round(res["median_gteps"], 3),
        "bfs_alg_gbs": res["bfs_alg_gbs"],
        "bfs_roofline_frac": res["bfs_roofline_frac"],
        "breakdown_ms_per_root": res["breakdown_ms_per_root"],
        "context": {"paper_1xK20X_scale21_gteps": 1.13, "paper_4096xK20X_gteps": 830},
    }
    if "cpu_baseline" in res:
        out["cpu_baseline"] = res["cpu_baseline"]
        out["parity_root0"] = res["parity_root0"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
