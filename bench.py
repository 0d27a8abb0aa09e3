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
  grid         -- single-root searches on the 4096 x 4096 grid (GTEPS);
  batch        -- 64 roots in one multi-source batch on R-MAT scale 22:
                  roots/s, and the speedup over 64 one-at-a-time searches;
  serve        -- open-loop Poisson queries (2000/s) over 32 resident graphs
                  (24 R-MAT scales 14-22, 8 grids 256k x 256k): p50/p99
                  latency (completion - scheduled arrival) and completed QPS.

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


def kernel_source_hash():
    """Hash of the sources that define the expansion kernel and the row
    layout it reads; counter-derived traffic is only reported while it
    matches the hash recorded with it."""
    import hashlib
    h = hashlib.sha256()
    for f in ("frontier.hip", "tile_map.h", "wave_ops.h", "bfs_internal.h", "relabel.hip",
              "rowskip.hip"):
        with open(os.path.join(ROOT, "paper_1408_1605_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel_hash):
    """HBM bytes per expansion launch from profiles/k_expand_rmat26_traffic.txt
    (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None."""
    path = os.path.join(ROOT, "profiles", "k_expand_rmat26_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_hash:
        return None
    try:
        return int(float(vals["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


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
    tuned = None
    if args.autotune:
        from paper_1408_1605_amd import autotune
        tuned = autotune.load_cached("rmat", args.scale)
        if tuned is None:
            best, table = autotune.tune_single(G, [int(r) for r in roots[:4]], log=log)
            tuned = dict(best or {})
            autotune.save("rmat", args.scale, {"single": tuned, "table": table})
        else:
            tuned = tuned.get("single", {})
        autotune.apply(G, tuned)
        log("autotuned configuration: %s" % tuned)
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
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(kernel_source_hash()),
                     "source_hash": kernel_source_hash(),
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


def grid_section(args, torch, np, graphgen, bfsmi):
    """Single-root searches on the 4096 x 4096 4-neighbour grid (thousands
    of narrow levels): GTEPS and levels, 16 seeded roots."""
    w = args.grid_side
    g = graphgen.grid(w)
    rng = np.random.default_rng(2000 + w)
    roots = [int(x) for x in rng.choice(g.V, size=args.grid_roots, replace=False)]
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    lv = torch.empty(g.V, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.V, dtype=torch.int32, device="cuda")
    bfsmi.bfs_run(G.handle, roots[0], lv, pa)
    torch.cuda.synchronize()
    r0, c0 = divmod(roots[0], w)
    rr, cc = np.divmod(np.arange(g.V, dtype=np.int64), w)
    ok = bool(np.array_equal(lv.cpu().numpy(), np.abs(rr - r0) + np.abs(cc - c0)))
    teps, levels, times = [], [], []
    for r in roots:
        t0 = time.perf_counter()
        st = bfsmi.bfs_run(G.handle, r, lv, pa)
        dt = time.perf_counter() - t0
        times.append(dt)
        teps.append(st.edges_scanned / 2 / dt / 1e9)
        levels.append(st.levels)
    G.close()
    res = {"graph": "grid%dx%d" % (w, w), "roots": len(roots), "gteps": round(harmonic_mean(teps), 4),
           "ms_per_root": round(1e3 * sum(times) / len(times), 2),
           "levels_min": int(min(levels)), "levels_max": int(max(levels)),
           "root0_matches_manhattan": ok}
    log("grid: %s" % res)
    return res


def batch_section(args, torch, np, graphgen, bfsmi):
    """64 roots in one bfs_run_batch on R-MAT scale 22 vs 64 single-root
    searches one at a time (parents skipped) on the same GPU and graph."""
    scale = args.batch_scale
    g = graphgen.rmat(scale)
    roots = [int(r) for r in graphgen.pick_roots(g, 64, graphgen.root_seed(scale))]
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_WS_BATCH | bfsmi.BFS_DEGREE_ORDER)
    out = torch.empty((64, g.V), dtype=torch.int8, device="cuda")
    lv = torch.empty(g.V, dtype=torch.int32, device="cuda")
    for _ in range(2):
        bfsmi.bfs_run_batch(G.handle, roots, out)
    torch.cuda.synchronize()
    reps = args.batch_reps
    t0 = time.perf_counter()
    for _ in range(reps):
        st = bfsmi.bfs_run_batch(G.handle, roots, out)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    bfsmi.bfs_run(G.handle, roots[0], lv, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in roots:
        bfsmi.bfs_run(G.handle, r, lv, None)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    # rows vs the single-root path for a few roots (GPU against GPU; the
    # oracle comparisons live in the tests)
    ok = True
    rows = out.cpu().numpy()
    for i in (0, 31, 63):
        bfsmi.bfs_run(G.handle, roots[i], lv, None)
        torch.cuda.synchronize()
        ok &= bool(np.array_equal(rows[i].astype(np.int32), lv.cpu().numpy()))
    G.close()
    res = {"graph": "rmat%d" % scale, "n_roots": 64, "batch_ms": round(t_batch * 1e3, 3),
           "roots_per_s": round(64 / t_batch, 1), "sequential_roots_per_s": round(64 / t_seq, 1),
           "speedup_vs_sequential": round(t_seq / t_batch, 2), "union_levels": st.levels,
           "union_edges_scanned": st.edges_scanned, "rows_match_single_root": ok}
    log("batch: %s" % res)
    return res


def serve_section(args, torch, np, graphgen, bfsmi):
    """Open-loop Poisson queries over a pool of resident graphs.  Each result
    is delivered as int32 levels into a device buffer of the client (one
    per graph); the client learns of finished queries from the server's
    completion queue."""
    rng = np.random.default_rng(3000)
    scales = rng.integers(14, 23, size=24)
    graphs = [graphgen.rmat(int(sc), seed=3000 + i) for i, sc in enumerate(scales)]
    graphs += [graphgen.grid(256 * k) for k in range(1, 9)]
    kinds = ["rmat"] * 24 + ["grid"] * 8
    handles = [bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER) for g in graphs]
    nonzero = [np.nonzero(np.diff(g.off) > 0)[0] for g in graphs]
    dst = [torch.empty(g.V, dtype=torch.int32, device="cuda") for g in graphs]
    arena = torch.empty(args.serve_arena_gb << 30, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = bfsmi.bfs_server_create(arena, max_lanes=64, max_inflight=len(graphs))
    ids = [bfsmi.bfs_server_add_graph(s, h.handle) for h in handles]
    log("serve: %d graphs resident, %d GiB arena" % (len(graphs), args.serve_arena_gb))
    rate, warm, dur = args.serve_rate, 1.0, args.serve_seconds
    arr = np.random.default_rng(4000)
    n = int(rate * (warm + dur) * 1.2) + 10
    gaps = arr.exponential(1.0 / rate, size=n)
    gsel = arr.integers(0, len(graphs), size=n)
    rsel = arr.random(size=n)
    pending = {}
    rec = []  # (kind, arrive->done ms, arrive->admit ms, admit->done ms, lanes, levels)
    done_in_window = 0
    t_start = time.monotonic_ns()
    sched = t_start
    i = 0
    warm_ns = t_start + int(warm * 1e9)
    end_ns = t_start + int((warm + dur) * 1e9)
    st0 = None
    while True:
        now = time.monotonic_ns()
        if st0 is None and now >= warm_ns:
            st0 = bfsmi.bfs_server_get_stats(s)
        while i < n and sched <= now and sched < end_ns:
            gi = int(gsel[i])
            cand = nonzero[gi]
            root = int(cand[int(rsel[i] * len(cand))])
            t = bfsmi.bfs_submit(s, ids[gi], root)
            pending[t] = (sched, gi)
            sched += int(gaps[i] * 1e9)
            i += 1
        for t in bfsmi.bfs_server_completed(s):
            arrive, gi = pending.pop(t)
            code, tm = bfsmi.bfs_poll(s, t, dst[gi])
            if arrive >= warm_ns:
                rec.append((kinds[gi], (tm.done_ns - arrive) / 1e6, (tm.admit_ns - arrive) / 1e6,
                            (tm.done_ns - tm.admit_ns) / 1e6, tm.lanes_in_batch, tm.levels))
                if tm.done_ns <= end_ns:
                    done_in_window += 1
        if sched >= end_ns and not pending:
            break
        if time.monotonic_ns() > end_ns + int(30e9):
            break
        time.sleep(0.0001)
    st1 = bfsmi.bfs_server_get_stats(s)
    bfsmi.bfs_server_destroy(s)
    for h in handles:
        h.close()

    def pct(xs, q):
        return round(float(np.percentile(xs, q)), 3) if len(xs) else None

    lat = [r[1] for r in rec]
    res = {"graphs": len(graphs), "offered_qps": rate, "measured_s": dur,
           "completed": len(rec), "qps": round(done_in_window / dur, 1),
           "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
           "max_ms": round(max(lat), 3) if lat else None, "unfinished": len(pending),
           "delivery": "int32 levels into a client device buffer"}
    for kind in ("rmat", "grid"):
        sub = [r for r in rec if r[0] == kind]
        res[kind] = {"n": len(sub), "p50_ms": pct([r[1] for r in sub], 50),
                     "p99_ms": pct([r[1] for r in sub], 99),
                     "wait_p50_ms": pct([r[2] for r in sub], 50),
                     "run_p50_ms": pct([r[3] for r in sub], 50),
                     "lanes_mean": round(float(np.mean([r[4] for r in sub])), 2) if sub else None,
                     "levels_mean": round(float(np.mean([r[5] for r in sub])), 1) if sub else None}
    if st0 is not None:
        d = {f: getattr(st1, f) - getattr(st0, f) for f, _ in st1._fields_}
        res["server"] = {"rounds": int(d["rounds"]),
                         "persistent_rounds": int(d["persistent_rounds"]),
                         "wide_rounds": int(d["wide_rounds"]),
                         "levels": int(d["levels"]),
                         "lanes_per_level": round(d["lane_levels"] / max(d["levels"], 1), 2),
                         "batches": int(d["batches"]),
                         "device_ms_per_s": round(d["device_ms"] / max(
                             (time.monotonic_ns() - warm_ns) / 1e9, 1e-9), 1),
                         "arena_peak_gib": round(st1.arena_peak / 2**30, 2)}
    log("serve: %s" % res)
    return res


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
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-grid", action="store_true")
    ap.add_argument("--grid-side", type=int, default=4096)
    ap.add_argument("--grid-roots", type=int, default=16)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-scale", type=int, default=22)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-arena-gb", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
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
    if args.copy_calibration:
        n = 1 << 28  # int32 elements: 1 GiB read + 1 GiB written per copy
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": 3}))
        return
    def release():
        # each section starts from an empty device cache (the serving arena
        # in particular gets fresh, unfragmented memory)
        import gc
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    res, g = single_root(args, torch, np, graphgen, bfsmi)
    g_V, g_nnz = g.V, g.nnz
    del g
    release()
    grid = None if args.no_grid else grid_section(args, torch, np, graphgen, bfsmi)
    release()
    batch = None if args.no_batch else batch_section(args, torch, np, graphgen, bfsmi)
    release()
    serve = None if args.no_serve else serve_section(args, torch, np, graphgen, bfsmi)

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
                   "edgefactor": 16, "A": 0.57, "B": 0.19, "C": 0.19, "V": g_V, "nnz": g_nnz,
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
    if grid is not None:
        out["grid"] = grid
    if batch is not None:
        out["batch"] = batch
    if serve is not None:
        out["serve"] = serve
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
