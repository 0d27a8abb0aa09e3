#!/usr/bin/env python3
"""Benchmark of the single-GPU BFS path.

Headline: GTEPS of single-root searches on R-MAT scale 26 (edgefactor 16,
A/B/C = 0.57/0.19/0.19, relabelled, symmetrised, deduplicated), one search
per step from seeded roots of degree > 0, inputs resident in HBM.  TEPS
counts the undirected edges of the traversed component (half the directed
CSR entries scanned) over the search time; the value is the harmonic mean
over the timed steps, as the paper reports TEPS (Section 4).

The headline pass runs with no per-kernel events.  The JSON line also
carries:
  roofline      -- the expansion kernel k_expand from a second, profiled pass
                   over the same roots: the method's algorithmic bytes for its
                   launches (4 per frontier edge of those levels, row-skipped
                   ones included, + level and parent of each discovered
                   vertex) over their summed duration (HIP events around each
                   launch, on its stream), against the MI355X HBM peak of
                   8 TB/s; the bytes it actually streams are reported beside;
  plain_topdown -- the same searches without the row prefix skip (the plain
                   top-down expansion of Algorithm 3), GTEPS and roofline;
  direction_optimizing
                -- the same roots with dense levels searched bottom-up
                   (BFS_OPT_DIRECTION): GTEPS over the same component edges,
                   the edges the kernels actually read, parity of every root;
  cpu_baseline  -- the serial CPU oracle on every bench root of the same graph,
                   one search per host thread: all-cores GTEPS and roots/s,
                   the serial time per root, the CPU model and core count;
  parity        -- every bench root's levels against the oracle (exact) and
                   its parents through the oracle's validator;
  configs       -- plain single-root searches on R-MAT scales 16 (16 roots)
                   and 22 (64 roots), GTEPS and parity of every root;
  blocked       -- the same graph and roots on the in-GPU 2D processor grid
                   (bfs_grid2d_*, Section 2.2 / Algorithm 2) for each R x C
                   shape asked for: GTEPS, whole-search algorithmic GB/s, the
                   column and row exchange volumes with list / bitmap
                   messages against lists only, and every root's parity;
  grid          -- single-root searches on the 4096 x 4096 grid (GTEPS),
                   every root's levels against the Manhattan distance;
  batch         -- 64 roots in one multi-source batch on R-MAT scale 22:
                   roots/s, the speedup over 64 one-at-a-time searches, every
                   row against the oracle;
  serve         -- open-loop Poisson queries (2000/s) over 32 resident graphs
                   (24 R-MAT scales 14-22, 8 grids 256k x 256k): p50/p99
                   latency (completion - scheduled arrival), completed QPS,
                   and sampled results against the oracle.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--scale S]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import threading
import time

# The serving section drives one stream per resident graph; HIP maps a
# process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 by default), and
# with 4 a deep graph's rounds wait behind other graphs' kernels.  Set before
# anything starts HIP.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")

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
            text = fh.read()
        if f == "bfs_internal.h":
            # its constants and the control block, not the launcher declarations
            text = text.split(b"// ---- single-root kernels", 1)[0]
        h.update(text)
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


def timed_pass(bfsmi, G, roots, levels, parents, steps, log_steps=False):
    """steps searches over the roots in turn (host wall time of each
    synchronous bfs_run).  Returns (per-step seconds, stats, total seconds)."""
    stats, times = [], []
    t0 = time.perf_counter()
    for i in range(steps):
        r = int(roots[i % len(roots)])
        ts = time.perf_counter()
        st = bfsmi.bfs_run(G.handle, r, levels, parents)
        times.append(time.perf_counter() - ts)
        stats.append(st)
        if log_steps:
            log("step %d root %d: %.3f ms, levels %d (bitmap %d), reached %d, E_r %d, %.1f GTEPS"
                % (i, r, times[-1] * 1e3, st.levels, st.bitmap_levels, st.reached,
                   st.edges_scanned, st.edges_scanned / 2 / times[-1] / 1e9))
    return times, stats, time.perf_counter() - t0


def roofline_of(bfsmi, G, stats, V, kernel_hash):
    """Roofline of the expansion kernel from a profiled pass: the method's
    algorithmic bytes for its launches (4 per frontier edge of those levels,
    skipped ones included, + level and parent per discovered vertex) over
    their summed duration (HIP events on the launch stream)."""
    x_alg = sum(st.expand_alg_bytes for st in stats)
    x_str = sum(st.expand_bytes for st in stats)
    x_ms = sum(st.expand_ms for st in stats)
    x_launch = sum(st.expand_launches for st in stats)
    achieved = x_alg / (x_ms * 1e-3) / 1e9 if x_ms > 0 else 0.0
    streamed = x_str / (x_ms * 1e-3) / 1e9 if x_ms > 0 else 0.0
    ept = bfsmi.bfs_get_option(G.handle, bfsmi.BFS_OPT_EDGES_PER_THREAD)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(kernel_hash),
            "source_hash": kernel_hash,
            "kernel": "k_expand<%d>" % ept,
            "launches": x_launch,
            "avg_launch_ms": round(x_ms / max(x_launch, 1), 5),
            "alg_bytes_per_launch": x_alg // max(x_launch, 1),
            "streamed_bytes_per_launch": x_str // max(x_launch, 1),
            "streamed_gbs": round(streamed, 1),
            "streamed_frac": round(streamed / HBM_PEAK_GBS, 4)}


def search_summary(times, stats, V):
    teps = [st.edges_scanned / 2 / dt / 1e9 for st, dt in zip(stats, times)]
    # whole-search algorithmic bytes: init 8.125 V, 32 per reached vertex,
    # 4 per directed edge of the component
    b_alg = [8.125 * V + 32 * st.reached + 4 * st.edges_scanned for st in stats]
    gbs = sum(b_alg) / sum(times) / 1e9
    return {"gteps": round(harmonic_mean(teps), 3),
            "median_gteps": round(sorted(teps)[len(teps) // 2], 3),
            "ms_per_root": round(1e3 * sum(times) / len(times), 4),
            "bfs_alg_gbs": round(gbs, 1), "bfs_roofline_frac": round(gbs / HBM_PEAK_GBS, 4)}


def check_against_oracle(bfsmi, torch, g, G, roots, digest, parents=True, label=""):
    """Every root's GPU levels equal the oracle's and its parents pass the
    validator; results are checked on host threads in groups of 16."""
    from oracle import parallel
    levels = torch.empty(g.V, dtype=torch.int32, device="cuda")
    par = torch.empty(g.V, dtype=torch.int32, device="cuda") if parents else None
    ok, n = 0, 0
    for i in range(0, len(roots), 16):
        items = []
        for r in roots[i:i + 16]:
            bfsmi.bfs_run(G.handle, int(r), levels, par)
            torch.cuda.synchronize()
            items.append((int(r), levels.cpu().numpy(),
                          par.cpu().numpy() if parents else None))
        checks = parallel.check_roots(g.off, g.col, items, digest=digest)
        ok += sum(c.ok for c in checks)
        n += len(checks)
    log("%s: %d of %d roots equal the oracle (levels exact, parents valid)" % (label, ok, n))
    return {"roots_checked": n, "roots_ok": ok}


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

    # the CPU oracle on every bench root (the cpu_baseline figures; its
    # levels also gate the autotuner's candidates and check the GPU results)
    from oracle import parallel
    nthreads = parallel.default_workers(len(roots))
    digest = parallel.csr_digest(g.off, g.col, nthreads)
    ref_levels = []
    if not args.no_cpu_baseline:
        log("cpu baseline: serial oracle, %d roots on %d host threads ..." % (len(roots), nthreads))
        ref, wall, used = parallel.bfs_roots(g.off, g.col, [int(r) for r in roots],
                                             workers=nthreads, fresh=True, digest=digest)
        serial = [x.seconds for x in ref]
        edges = sum(x.edges_scanned for x in ref)
        cpu_baseline = {
            "value": round(edges / 2 / wall / 1e9, 5), "unit": "GTEPS", "cores": used,
            "kind": "oracle",
            "sample": "the %d bench roots of the same R-MAT scale %d graph, one serial oracle "
                      "search per host thread, %.1f s wall" % (len(roots), args.scale, wall),
            "roots_per_s_all_cores": round(len(roots) / wall, 4),
            "serial_s_per_root": round(sum(serial) / len(serial), 3),
            "serial_gteps": round(harmonic_mean([x.edges_scanned / 2 / x.seconds / 1e9
                                                 for x in ref]), 5),
            "cpu": cpu_model(), "nproc": os.cpu_count()}
        ref_levels = [x.level for x in ref[:args.tune_roots]]
        del ref

    # autotuned launch knobs, every candidate gated on the oracle's levels
    tuned = None
    if args.autotune and ref_levels:
        from paper_1408_1605_amd import autotune
        cls = "rmat_do" if not args.no_degree_order else "rmat"
        tuned = autotune.load_cached(cls, args.scale)
        troots = [int(r) for r in roots[:len(ref_levels)]]
        if tuned is None:
            t = time.time()
            best, table = autotune.tune_single(G, troots, ref_levels, log=log)
            dbest, dtable = autotune.tune_direction(G, troots, ref_levels, log=log)
            tuned = {"single": best, "direction": dbest,
                     "candidates": len(table) + len(dtable),
                     "failed_parity": sum(not x["parity"] for x in table + dtable),
                     "tuning_s": round(time.time() - t, 1)}
            autotune.save(cls, args.scale, tuned)
        autotune.apply(G, {k: v for k, v in (tuned.get("single") or {}).items()
                           if k in autotune.SINGLE_SPACE})
        log("autotuned configuration: %s" % tuned)
    del ref_levels
    if args.ept:
        G.set_option(bfsmi.BFS_OPT_EDGES_PER_THREAD, args.ept)
    G.set_option(bfsmi.BFS_OPT_PROFILE, 0)
    levels = torch.empty(g.V, dtype=torch.int32, device="cuda")
    parents = torch.empty(g.V, dtype=torch.int32, device="cuda")
    for i in range(args.warmup):
        bfsmi.bfs_run(G.handle, int(roots[i % len(roots)]), levels, parents)
    torch.cuda.synchronize()

    # headline: plain timing, no per-kernel events
    times, stats, total = timed_pass(bfsmi, G, roots, levels, parents, args.steps, log_steps=True)
    torch.cuda.synchronize()
    res = search_summary(times, stats, g.V)
    res["ms_per_step"] = total * 1e3 / args.steps
    # the bitmap levels' claim (0 atomic, 1 flags where they measured faster)
    # and the XCD-sliced early levels (1 automatic), as the headline ran them
    res["claim_mode"] = G.get_option(bfsmi.BFS_OPT_CLAIM_MODE) if flags else 0
    res["xcd_slices"] = G.get_option(bfsmi.BFS_OPT_XCD_SLICES) if flags else 0
    res["levels"] = stats[0].levels
    res["reached"] = stats[0].reached
    res["edges_scanned"] = stats[0].edges_scanned
    khash = kernel_source_hash()

    # roofline and breakdown: the same roots again with per-kernel HIP events
    G.set_option(bfsmi.BFS_OPT_PROFILE, 1)
    ptimes, pstats, _ = timed_pass(bfsmi, G, roots, levels, parents, len(roots))
    G.set_option(bfsmi.BFS_OPT_PROFILE, 0)
    res["roofline"] = roofline_of(bfsmi, G, pstats, g.V, khash)
    res["roofline"]["pass"] = ("profiled pass over the %d roots, %.3f ms per search "
                               "(headline pass %.3f ms)"
                               % (len(roots), 1e3 * sum(ptimes) / len(ptimes),
                                  res["ms_per_root"]))
    res["breakdown_ms_per_root"] = {
        k: round(sum(getattr(st, k) for st in pstats) / len(pstats), 4)
        for k in ("init_ms", "scan_ms", "expand_ms", "compact_ms", "device_ms")}

    # the plain top-down expansion of Algorithm 3 (no row prefix skip)
    plain = None
    if not args.no_degree_order and args.plain:
        G.set_option(bfsmi.BFS_OPT_ROW_SKIP, 0)
        bfsmi.bfs_run(G.handle, int(roots[0]), levels, parents)
        t2, s2, tot2 = timed_pass(bfsmi, G, roots, levels, parents, len(roots))
        plain = search_summary(t2, s2, g.V)
        G.set_option(bfsmi.BFS_OPT_PROFILE, 1)
        _, ps2, _ = timed_pass(bfsmi, G, roots, levels, parents, len(roots))
        G.set_option(bfsmi.BFS_OPT_PROFILE, 0)
        plain["roofline"] = roofline_of(bfsmi, G, ps2, g.V, khash)
        plain["config"] = {"row_skip": False, "degree_order": True}
        G.set_option(bfsmi.BFS_OPT_ROW_SKIP, 1)
        log("plain top-down (row skip off): %s" % plain)
    res["plain_topdown"] = plain

    # the direction-optimizing mode (dense levels bottom-up): the same roots;
    # TEPS keeps the traversed component's edges as numerator, the edges the
    # kernels actually read are reported beside it
    diropt = None
    if args.direction:
        if tuned and tuned.get("direction"):
            from paper_1408_1605_amd import autotune
            autotune.apply(G, {k: v for k, v in tuned["direction"].items()
                               if k in autotune.DIRECTION_SPACE})
        G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
        bfsmi.bfs_run(G.handle, int(roots[0]), levels, parents)
        t3, s3, _ = timed_pass(bfsmi, G, roots, levels, parents, len(roots))
        diropt = search_summary(t3, s3, g.V)
        diropt["bottom_up_levels_root0"] = s3[0].bottom_up_levels
        diropt["edges_examined_per_root"] = sum(x.edges_examined for x in s3) // len(s3)
        diropt["edges_in_component_per_root"] = sum(x.edges_scanned for x in s3) // len(s3)
        diropt["config"] = {"direction": "optimizing", "alpha": G.get_option(bfsmi.BFS_OPT_DO_ALPHA),
                            "beta": G.get_option(bfsmi.BFS_OPT_DO_BETA), "degree_order": flags != 0}
        G.set_option(bfsmi.BFS_OPT_DIRECTION, 0)
        log("direction-optimizing: %s" % diropt)
    res["direction_optimizing"] = diropt

    res["tuned"] = tuned
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline
        res["parity"] = check_against_oracle(bfsmi, torch, g, G, [int(r) for r in roots],
                                             digest, label="rmat%d default" % args.scale)
        if plain is not None:
            G.set_option(bfsmi.BFS_OPT_ROW_SKIP, 0)
            res["parity_plain_topdown"] = check_against_oracle(
                bfsmi, torch, g, G, [int(r) for r in roots], digest,
                label="rmat%d row skip off" % args.scale)
            G.set_option(bfsmi.BFS_OPT_ROW_SKIP, 1)
        if diropt is not None:
            G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
            diropt["parity"] = check_against_oracle(
                bfsmi, torch, g, G, [int(r) for r in roots], digest,
                label="rmat%d direction-optimizing" % args.scale)
            G.set_option(bfsmi.BFS_OPT_DIRECTION, 0)
    G.close()
    return res, g


def blocked_section(args, torch, g, roots, bfsmi):
    """The in-GPU 2D blocked search on the headline graph and roots, one
    R x C shape at a time: GTEPS (auto message form), the exchange volumes,
    a lists-only pass for comparison, and every root against the oracle."""
    from oracle import parallel
    digest = parallel.csr_digest(g.off, g.col)
    out = {}
    for shape in args.blocked.split(","):
        R, C = (int(x) for x in shape.lower().split("x"))
        t = time.time()
        G = bfsmi.Grid2D.from_csr(g.off, g.col, R, C)
        log("blocked %dx%d: partitioned in %.1fs" % (R, C, time.time() - t))
        lv = torch.empty(g.V, dtype=torch.int32, device="cuda")
        pa = torch.empty(g.V, dtype=torch.int32, device="cuda")
        res = {"R": R, "C": C}
        for mode, name in ((bfsmi.BFS_2D_MSG_AUTO, "auto"), (bfsmi.BFS_2D_MSG_LIST, "lists_only")):
            bfsmi.bfs_grid2d_run(G.handle, int(roots[0]), lv, pa, mode)
            torch.cuda.synchronize()
            times, stats = [], []
            for r in roots:
                t0 = time.perf_counter()
                st = bfsmi.bfs_grid2d_run(G.handle, int(r), lv, pa, mode)
                times.append(time.perf_counter() - t0)
                stats.append(st)
            summ = search_summary(times, stats, g.V)
            n = len(stats)
            summ.update({
                "expand_msgs_list": sum(x.expand_list_msgs for x in stats) // n,
                "expand_msgs_bitmap": sum(x.expand_bitmap_msgs for x in stats) // n,
                "expand_mb": round(sum(x.expand_bytes for x in stats) / n / 1e6, 2),
                "expand_mb_lists_only": round(sum(x.expand_list_only_bytes for x in stats) / n / 1e6, 2),
                "fold_msgs_list": sum(x.fold_list_msgs for x in stats) // n,
                "fold_msgs_bitmap": sum(x.fold_bitmap_msgs for x in stats) // n,
                "fold_mb": round(sum(x.fold_bytes for x in stats) / n / 1e6, 2),
                "fold_mb_lists_only": round(sum(x.fold_list_only_bytes for x in stats) / n / 1e6, 2),
                "updated_per_root": sum(x.updated for x in stats) // n})
            res[name] = summ
            log("blocked %dx%d %s: %s" % (R, C, name, summ))
        ok, nchk = 0, 0
        for i in range(0, len(roots), 16):
            items = []
            for r in roots[i:i + 16]:
                bfsmi.bfs_grid2d_run(G.handle, int(r), lv, pa, bfsmi.BFS_2D_MSG_AUTO)
                torch.cuda.synchronize()
                items.append((int(r), lv.cpu().numpy(), pa.cpu().numpy()))
            checks = parallel.check_roots(g.off, g.col, items, digest=digest)
            ok += sum(c.ok for c in checks)
            nchk += len(checks)
        res["parity"] = {"roots_checked": nchk, "roots_ok": ok}
        G.close()
        del G, lv, pa
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        out["%dx%d" % (R, C)] = res
    return out


def small_config(scale, nroots, args, torch, np, graphgen, bfsmi):
    """Plain single-root searches (levels and parents) on a smaller R-MAT
    graph, every root timed and checked against the oracle."""
    from oracle import parallel
    g = graphgen.rmat(scale)
    roots = [int(r) for r in graphgen.pick_roots(g, nroots, graphgen.root_seed(scale))]
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    levels = torch.empty(g.V, dtype=torch.int32, device="cuda")
    parents = torch.empty(g.V, dtype=torch.int32, device="cuda")
    for r in roots[:2]:
        bfsmi.bfs_run(G.handle, r, levels, parents)
    torch.cuda.synchronize()
    times, stats, _ = timed_pass(bfsmi, G, roots, levels, parents, len(roots))
    res = {"graph": "rmat%d" % scale, "V": g.V, "nnz": g.nnz, "roots": len(roots),
           "parents": True}
    res.update(search_summary(times, stats, g.V))
    res["levels_max"] = max(st.levels for st in stats)
    digest = parallel.csr_digest(g.off, g.col)
    res["parity"] = check_against_oracle(bfsmi, torch, g, G, roots, digest,
                                         label="rmat%d" % scale)
    G.close()
    log("rmat%d single roots: %s" % (scale, res))
    return res


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
    teps, levels, times = [], [], []
    for r in roots:
        t0 = time.perf_counter()
        st = bfsmi.bfs_run(G.handle, r, lv, pa)
        dt = time.perf_counter() - t0
        times.append(dt)
        teps.append(st.edges_scanned / 2 / dt / 1e9)
        levels.append(st.levels)
    # every root: levels equal the Manhattan distance (closed form), parents
    # pass the oracle's validator
    from oracle import validate
    rr, cc = np.divmod(np.arange(g.V, dtype=np.int64), w)
    ok = 0
    for r in roots:
        bfsmi.bfs_run(G.handle, r, lv, pa)
        torch.cuda.synchronize()
        r0, c0 = divmod(r, w)
        a = lv.cpu().numpy()
        ok += bool(np.array_equal(a, np.abs(rr - r0) + np.abs(cc - c0))) and \
            validate(g.off, g.col, r, a, pa.cpu().numpy())[0] == 0
    G.close()
    res = {"graph": "grid%dx%d" % (w, w), "roots": len(roots), "gteps": round(harmonic_mean(teps), 4),
           "ms_per_root": round(1e3 * sum(times) / len(times), 2),
           "levels_min": int(min(levels)), "levels_max": int(max(levels)),
           "parity": {"roots_checked": len(roots), "roots_ok": int(ok),
                      "check": "levels = Manhattan distance, parents validated"}}
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
    # the oracle's rows (the scale-22 single-root section has usually cached
    # these roots already): they gate the tile autotuner and check the result
    from oracle import parallel
    ref, _, _ = parallel.bfs_roots(g.off, g.col, roots)
    rows_ref = np.stack([x.level.astype(np.int8) for x in ref])
    del ref
    tuned = None
    if args.autotune:
        from paper_1408_1605_amd import autotune
        tuned = autotune.load_cached("rmat_batch", scale)
        if tuned is None:
            best, table = autotune.tune_batch(G, roots, rows_ref, log=log)
            tuned = {"batch": best, "candidates": len(table),
                     "failed_parity": sum(not x["parity"] for x in table)}
            autotune.save("rmat_batch", scale, tuned)
        autotune.apply(G, tuned.get("batch") or {})
        log("batch tile: %d" % G.get_option(bfsmi.BFS_OPT_BATCH_TILE))
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
    # every row against the oracle
    rows = out.cpu().numpy()
    ok = sum(bool(np.array_equal(rows[i], rows_ref[i])) for i in range(len(roots)))
    tile = G.get_option(bfsmi.BFS_OPT_BATCH_TILE)
    G.close()
    res = {"graph": "rmat%d" % scale, "n_roots": 64, "batch_ms": round(t_batch * 1e3, 3),
           "roots_per_s": round(64 / t_batch, 1), "sequential_roots_per_s": round(64 / t_seq, 1),
           "speedup_vs_sequential": round(t_seq / t_batch, 2), "union_levels": st.levels,
           "union_edges_scanned": st.edges_scanned, "batch_tile": tile,
           "tuned": tuned,
           "parity": {"rows_checked": len(roots), "rows_ok": int(ok)}}
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
    samples = []
    rec = []  # (kind, arrive->done ms, arrive->admit ms, admit->done ms, lanes, levels)
    done_in_window = 0
    t_start = time.monotonic_ns()
    sched = t_start
    i = 0
    warm_ns = t_start + int(warm * 1e9)
    end_ns = t_start + int((warm + dur) * 1e9)
    st0 = None
    # Each query's latency runs from its scheduled arrival.  By default this
    # thread submits the due arrivals between collecting results (a device
    # delivery is synchronous, so a slow one delays the next submissions and
    # that delay counts as latency); --serve-submit-thread gives submission a
    # thread of its own that keeps to the schedule.
    lock = threading.Lock()
    submitter = None
    if args.serve_submit_thread:
        def submit_loop():
            at = t_start
            for k in range(n):
                if at >= end_ns:
                    break
                while True:
                    left = at - time.monotonic_ns()
                    if left <= 0:
                        break
                    time.sleep(min(left / 1e9, 0.0002))
                gk = int(gsel[k])
                ck = nonzero[gk]
                rk = int(ck[int(rsel[k] * len(ck))])
                with lock:
                    tk = bfsmi.bfs_submit(s, ids[gk], rk)
                    pending[tk] = (at, gk, rk)
                at += int(gaps[k] * 1e9)
        submitter = threading.Thread(target=submit_loop, daemon=True)
        submitter.start()
        i = n  # the loop below only collects
    while True:
        now = time.monotonic_ns()
        if st0 is None and now >= warm_ns:
            st0 = bfsmi.bfs_server_get_stats(s)
        while i < n and sched <= now and sched < end_ns:
            gi = int(gsel[i])
            cand = nonzero[gi]
            root = int(cand[int(rsel[i] * len(cand))])
            t = bfsmi.bfs_submit(s, ids[gi], root)
            pending[t] = (sched, gi, root)
            sched += int(gaps[i] * 1e9)
            i += 1
        for t in bfsmi.bfs_server_completed(s):
            with lock:
                arrive, gi, root = pending.pop(t)
            code, tm = bfsmi.bfs_poll(s, t, dst[gi])
            if arrive >= warm_ns and len(rec) % 97 == 0 and len(samples) < 64:
                # kept for the check against the oracle after the window (a
                # device-side copy on the stream the delivery was ordered on)
                samples.append((gi, root, dst[gi].clone()))
            if arrive >= warm_ns:
                rec.append((kinds[gi], (tm.done_ns - arrive) / 1e6, (tm.admit_ns - arrive) / 1e6,
                            (tm.done_ns - tm.admit_ns) / 1e6, tm.lanes_in_batch, tm.levels))
                if tm.done_ns <= end_ns:
                    done_in_window += 1
        if submitter is not None:
            if not submitter.is_alive():
                with lock:
                    if not pending:
                        break
        elif sched >= end_ns and not pending:
            break
        if time.monotonic_ns() > end_ns + int(30e9):
            break
        time.sleep(0.0001)
    if submitter is not None:
        submitter.join(timeout=5.0)
    st1 = bfsmi.bfs_server_get_stats(s)
    bfsmi.bfs_server_destroy(s)
    for h in handles:
        h.close()
    # sampled results against the oracle (levels, tolerance 0)
    from oracle import parallel
    torch.cuda.synchronize()
    by_graph = {}
    for gi, root, buf in samples:
        by_graph.setdefault(gi, []).append((root, buf.cpu().numpy(), None))
    s_ok, s_n = 0, 0
    for gi, items in by_graph.items():
        checks = parallel.check_roots(graphs[gi].off, graphs[gi].col, items, cache=False)
        s_ok += sum(c.levels_equal for c in checks)
        s_n += len(checks)
    del samples

    def pct(xs, q):
        return round(float(np.percentile(xs, q)), 3) if len(xs) else None

    lat = [r[1] for r in rec]
    res = {"graphs": len(graphs), "offered_qps": rate, "measured_s": dur,
           "completed": len(rec), "qps": round(done_in_window / dur, 1),
           "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
           "max_ms": round(max(lat), 3) if lat else None, "unfinished": len(pending),
           "delivery": "int32 levels into a client device buffer",
           "submission": ("own thread, on schedule" if args.serve_submit_thread
                          else "between deliveries, late arrivals count as latency"),
           "parity": {"sampled_tickets": s_n, "tickets_ok": int(s_ok),
                      "kinds": sorted({kinds[gi] for gi in by_graph})}}
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
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default launch knobs (no oracle-gated tuning)")
    ap.add_argument("--tune-roots", type=int, default=4,
                    help="bench roots whose oracle levels gate the tuning candidates")
    ap.add_argument("--no-plain", dest="plain", action="store_false",
                    help="skip the plain top-down twin of the headline")
    ap.add_argument("--no-direction", dest="direction", action="store_false",
                    help="skip the direction-optimizing twin of the headline")
    ap.add_argument("--blocked", default="8x1,2x4",
                    help="R x C shapes of the 2D blocked search on the headline graph "
                         "(comma-separated; empty to skip)")
    ap.add_argument("--blocked-only", action="store_true",
                    help="generate the headline graph and run only the blocked section")
    ap.add_argument("--no-grid", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the scale-16 and scale-22 single-root configurations")
    ap.add_argument("--grid-side", type=int, default=4096)
    ap.add_argument("--grid-roots", type=int, default=16)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-scale", type=int, default=22)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving section")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-submit-thread", action="store_true",
                    help="submit serving queries from a thread of their own, on schedule")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-arena-gb", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the search runs on one GPU only (it has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
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

    if args.serve_only:
        print(json.dumps({"serve": serve_section(args, torch, np, graphgen, bfsmi)}), flush=True)
        return
    if args.blocked_only:
        g = graphgen.rmat(args.scale)
        roots = graphgen.pick_roots(g, args.roots, graphgen.root_seed(args.scale))
        print(json.dumps({"blocked": blocked_section(args, torch, g, roots, bfsmi)}), flush=True)
        return
    res, g = single_root(args, torch, np, graphgen, bfsmi)
    g_V, g_nnz = g.V, g.nnz
    release()
    blocked = None
    if args.blocked:
        roots = graphgen.pick_roots(g, args.roots, graphgen.root_seed(args.scale))
        blocked = blocked_section(args, torch, g, roots, bfsmi)
    del g
    release()
    small = {}
    if not args.no_small:
        small["rmat16"] = small_config(16, 16, args, torch, np, graphgen, bfsmi)
        release()
        small["rmat22"] = small_config(22, 64, args, torch, np, graphgen, bfsmi)
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
                   "row_skip": not args.no_degree_order, "parents": True,
                   "claim_mode": res.get("claim_mode"), "xcd_slices": res.get("xcd_slices"),
                   "edgefactor": 16, "A": 0.57, "B": 0.19, "C": 0.19, "V": g_V, "nnz": g_nnz,
                   "roots": args.roots, "levels_root0": res["levels"],
                   "reached_root0": res["reached"], "edges_scanned_root0": res["edges_scanned"]},
        "roofline": res["roofline"],
        "tuned": res.get("tuned"),
        "median_gteps": res["median_gteps"],
        "bfs_alg_gbs": res["bfs_alg_gbs"],
        "bfs_roofline_frac": res["bfs_roofline_frac"],
        "breakdown_ms_per_root": res["breakdown_ms_per_root"],
        "context": {"paper_1xK20X_scale21_gteps": 1.13, "paper_4096xK20X_gteps": 830},
    }
    if res.get("plain_topdown"):
        out["plain_topdown"] = res["plain_topdown"]
    if res.get("direction_optimizing"):
        out["direction_optimizing"] = res["direction_optimizing"]
    if "cpu_baseline" in res:
        out["cpu_baseline"] = res["cpu_baseline"]
        out["parity"] = res["parity"]
        if "parity_plain_topdown" in res:
            out["parity_plain_topdown"] = res["parity_plain_topdown"]
    if blocked is not None:
        out["blocked"] = blocked
    if small:
        out["configs"] = small
    if grid is not None:
        out["grid"] = grid
    if batch is not None:
        out["batch"] = batch
    if serve is not None:
        out["serve"] = serve
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
