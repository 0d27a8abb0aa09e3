"""Parity at the workloads' full sizes, with the roots and the launch
configuration that bench.py times (degree-ordered graphs, default options).

  R-MAT scale 26 (V = 2^26, ~2.1e9 directed entries): all 16 bench roots,
    with and without the row prefix skip;
  4096 x 4096 grid: all 16 bench roots (levels = Manhattan distance, parents
    validated);
  R-MAT scale 22: all 64 bench roots as single-root searches, and the
    64-root batch;
  R-MAT scale 16: all 16 bench roots;
  the direction-optimizing mode on all 16 scale-26 and all 64 scale-22
  roots;
  the in-GPU 2D blocked search (bfs_grid2d_*) on the scale-26 graph with
  the bench's 8 x 1 and 2 x 4 processor grids (all 16 roots) and on the
  scale-22 graph with 1 x 8 and 4 x 4 (all 64 roots).
Levels are compared with the serial oracle element by element, parents are
checked by the tree validator, and each search's level / reached / edge
counts must equal the oracle's.  The oracle runs on a pool of host threads
(one serial search per thread) with its results cached by (graph, root).
"""
import os
import time

import numpy as np
import pytest

import graphgen
import oracle
from oracle import parallel
from parity_util import assert_parity, gpu_results, manhattan, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("BFSMI_BIG", "1") == "0",
                                 reason="full-size graphs disabled (BFSMI_BIG=0)")]
torch = pytest.importorskip("torch")


def blocked_results(G2, roots):
    out = []
    for r in roots:
        lv, pa, st = G2.run(int(r))
        torch.cuda.synchronize()
        out.append((int(r), lv.cpu().numpy(), pa.cpu().numpy(), st))
    return out


@pytest.fixture(scope="module")
def bfsmi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_1605_amd as p
    p.load()
    return p


def test_rmat26_all_bench_roots(bfsmi):
    t = time.time()
    g = graphgen.rmat(26)
    say("rmat26 generated in %.1fs, nnz=%d" % (time.time() - t, g.nnz))
    roots = [int(r) for r in graphgen.pick_roots(g, 16, graphgen.root_seed(26))]
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    digest = parallel.csr_digest(g.off, g.col)
    items = gpu_results(torch, G, roots)
    say("rmat26: 16 GPU searches done")
    assert_parity(g, items, digest=digest, label="rmat26 default")
    del items
    # the plain top-down expansion (no row prefix skip), as the bench's
    # second headline runs it
    G.set_option(bfsmi.BFS_OPT_ROW_SKIP, 0)
    items = gpu_results(torch, G, roots)
    assert_parity(g, items, digest=digest, label="rmat26 row skip off")
    del items
    G.close()
    del G
    torch.cuda.empty_cache()
    # direction-optimizing searches (bottom-up dense levels) of the same roots
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
    items = gpu_results(torch, G, roots)
    assert all(st.bottom_up_levels > 0 for _, _, _, st in items)
    assert_parity(g, items, digest=digest, label="rmat26 direction-optimizing")
    del items
    G.close()
    del G
    torch.cuda.empty_cache()
    for R, C in ((8, 1), (2, 4)):
        G2 = bfsmi.Grid2D.from_csr(g.off, g.col, R, C)
        items = blocked_results(G2, roots)
        assert_parity(g, items, digest=digest, label="rmat26 blocked %dx%d" % (R, C))
        del items
        G2.close()
        del G2
        torch.cuda.empty_cache()


def test_grid4096_all_bench_roots(bfsmi):
    w = 4096
    g = graphgen.grid(w)
    rng = np.random.default_rng(2000 + w)
    roots = [int(x) for x in rng.choice(g.V, size=16, replace=False)]
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    items = []
    for r in roots:
        t = time.time()
        lv, pa, st = G.run(r)
        torch.cuda.synchronize()
        lv = lv.cpu().numpy()
        # the closed form pins the levels independently of the oracle
        assert np.array_equal(lv, manhattan(w, w, r)), r
        items.append((r, lv, pa.cpu().numpy(), st))
        say("grid4096 root %d: %d levels in %.2fs" % (r, st.levels, time.time() - t))
    assert_parity(g, items, label="grid4096")
    G.close()


def test_rmat22_all_single_roots_and_batch(bfsmi):
    g = graphgen.rmat(22)
    roots = [int(r) for r in graphgen.pick_roots(g, 64, graphgen.root_seed(22))]
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER | bfsmi.BFS_WS_BATCH)
    digest = parallel.csr_digest(g.off, g.col)
    comp = oracle.components(g.off, g.col)
    items = gpu_results(torch, G, roots)
    assert_parity(g, items, digest=digest, comp=comp, label="rmat22 single roots")
    del items
    G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
    assert_parity(g, gpu_results(torch, G, roots), digest=digest, comp=comp,
                  label="rmat22 direction-optimizing")
    G.set_option(bfsmi.BFS_OPT_DIRECTION, 0)
    out, st = G.run_batch(roots)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    res, _, _ = parallel.bfs_roots(g.off, g.col, roots, digest=digest)
    for i, x in enumerate(res):
        assert np.array_equal(got[i].astype(np.int32), x.level), (i, roots[i])
    G.close()
    del G
    torch.cuda.empty_cache()
    for R, C in ((1, 8), (4, 4)):
        G2 = bfsmi.Grid2D.from_csr(g.off, g.col, R, C)
        assert_parity(g, blocked_results(G2, roots), digest=digest, comp=comp,
                      label="rmat22 blocked %dx%d" % (R, C))
        G2.close()


def test_rmat16_all_bench_roots(bfsmi):
    g = graphgen.rmat(16)
    roots = [int(r) for r in graphgen.pick_roots(g, 16, graphgen.root_seed(16))]
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    comp = oracle.components(g.off, g.col)
    assert_parity(g, gpu_results(torch, G, roots), comp=comp, label="rmat16")
    G.close()
