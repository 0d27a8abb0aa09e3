"""Parity at the workloads' full sizes, in the launch configuration that
bench.py times (degree-ordered graph, default options).

R-MAT scale 26 (V = 2^26, ~2.1e9 directed entries): one root, levels
compared with the serial oracle element by element, parents checked by the
tree validator.  4096 x 4096 grid: levels equal the Manhattan distance for
two roots.  R-MAT scale 22: four single roots and a 64-root batch against
the oracle.
"""
import os
import sys
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("BFSMI_BIG", "1") == "0",
                                 reason="full-size graphs disabled (BFSMI_BIG=0)")]
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bfsmi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_1605_amd as p
    p.load()
    return p


def test_rmat26_root_matches_oracle(bfsmi):
    t = time.time()
    g = graphgen.rmat(26)
    _say("rmat26 generated in %.1fs, nnz=%d" % (time.time() - t, g.nnz))
    root = int(graphgen.pick_roots(g, 1, graphgen.root_seed(26))[0])
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    lv, pa, st = G.run(root)
    torch.cuda.synchronize()
    lv, pa = lv.cpu().numpy(), pa.cpu().numpy()
    # the same search without the row prefix skip
    G.set_option(bfsmi.BFS_OPT_ROW_SKIP, 0)
    lv2, _, st2 = G.run(root, want_parents=False)
    torch.cuda.synchronize()
    lv2 = lv2.cpu().numpy()
    G.close()
    _say("gpu done: levels %d reached %d" % (st.levels, st.reached))
    ref = oracle.bfs(g.off, g.col, root)
    assert np.array_equal(lv, ref.level)
    assert st.reached == ref.reached and st.edges_scanned == ref.edges_scanned
    assert np.array_equal(lv2, ref.level) and st2.edges_scanned == ref.edges_scanned
    code, bad = oracle.validate(g.off, g.col, root, lv, pa)
    assert code == 0, (oracle.INVARIANTS[code], bad)


def test_grid4096_manhattan(bfsmi):
    w = 4096
    g = graphgen.grid(w)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    r_, c_ = np.divmod(np.arange(g.V, dtype=np.int64), w)
    for root in (0, (w // 2) * w + 123):
        t = time.time()
        lv, pa, st = G.run(root)
        torch.cuda.synchronize()
        _say("grid4096 root %d: %d levels in %.2fs" % (root, st.levels, time.time() - t))
        r0, c0 = divmod(root, w)
        assert np.array_equal(lv.cpu().numpy(), np.abs(r_ - r0) + np.abs(c_ - c0))
        code, bad = oracle.validate(g.off, g.col, root, lv.cpu().numpy(), pa.cpu().numpy())
        assert code == 0, (oracle.INVARIANTS[code], bad)
    G.close()


def test_rmat22_roots_and_batch(bfsmi):
    g = graphgen.rmat(22)
    roots = graphgen.pick_roots(g, 64, graphgen.root_seed(22))
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER | bfsmi.BFS_WS_BATCH)
    for r in roots[:4]:
        lv, pa, st = G.run(int(r))
        torch.cuda.synchronize()
        ref = oracle.bfs(g.off, g.col, int(r))
        assert np.array_equal(lv.cpu().numpy(), ref.level)
        code, bad = oracle.validate(g.off, g.col, int(r), lv.cpu().numpy(), pa.cpu().numpy())
        assert code == 0, (oracle.INVARIANTS[code], bad)
    out, st = G.run_batch([int(r) for r in roots])
    torch.cuda.synchronize()
    exp = oracle.batch_levels_int8(g.off, g.col, roots)
    assert np.array_equal(out.cpu().numpy(), exp)
    G.close()
