"""Serving at the shape of the benchmark's pool: graphs taken from the same
seeded pool (R-MAT scales 14-21 with the pool's seeds, grids of side 256,
1024 and 2048) plus the scale-22 R-MAT graph, open-loop Poisson arrivals at
2000 queries/s, results delivered into client device buffers through the
completion queue, as bench.py does.  Every ticket's levels must equal the
single-root oracle for that query alone (tolerance 0)."""
import os
import time

import numpy as np
import pytest

import graphgen
from oracle import parallel
from parity_util import say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("BFSMI_BIG", "1") == "0",
                                 reason="full-size graphs disabled (BFSMI_BIG=0)")]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bfsmi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_1605_amd as p
    p.load()
    return p


def pool_graphs():
    # the benchmark pool draws 24 R-MAT scales from seed 3000; indices 8, 0,
    # 16 and 4 are its scales 21, 20, 18 and 14 (graph seed 3000 + index)
    scales = np.random.default_rng(3000).integers(14, 23, size=24)
    picks = [8, 0, 16, 4]
    graphs = [graphgen.rmat(int(scales[i]), seed=3000 + i) for i in picks]
    assert [g.V for g in graphs] == [1 << 21, 1 << 20, 1 << 18, 1 << 14]
    graphs.append(graphgen.rmat(22))
    graphs += [graphgen.grid(2048), graphgen.grid(1024), graphgen.grid(256)]
    return graphs


def test_serve_bench_pool_shape_matches_oracle(bfsmi):
    graphs = pool_graphs()
    handles = [bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER) for g in graphs]
    nonzero = [np.nonzero(np.diff(g.off) > 0)[0] for g in graphs]
    dst = [torch.empty(g.V, dtype=torch.int32, device="cuda") for g in graphs]
    arena = torch.empty(8 << 30, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = bfsmi.bfs_server_create(arena, max_lanes=64, max_inflight=len(graphs))
    ids = [bfsmi.bfs_server_add_graph(s, h.handle) for h in handles]
    rng = np.random.default_rng(4000)
    n = 240
    gaps = rng.exponential(1.0 / 2000.0, size=n)
    gsel = rng.integers(0, len(graphs), size=n)
    rsel = rng.random(size=n)
    meta, got = {}, {}
    t0 = time.monotonic()
    sched = t0
    i = 0
    while i < n or len(got) < n:
        now = time.monotonic()
        while i < n and sched <= now:
            gi = int(gsel[i])
            root = int(nonzero[gi][int(rsel[i] * len(nonzero[gi]))])
            meta[bfsmi.bfs_submit(s, ids[gi], root)] = (gi, root)
            sched += float(gaps[i])
            i += 1
        for t in bfsmi.bfs_server_completed(s):
            gi, root = meta[t]
            code, tm = bfsmi.bfs_poll(s, t, dst[gi])
            assert code == bfsmi.BFS_OK
            got[t] = dst[gi].cpu().numpy()
        assert time.monotonic() - t0 < 120, "queries did not finish"
        time.sleep(0.0002)
    say("serve pool: %d queries in %.2f s" % (n, time.monotonic() - t0))
    st = bfsmi.bfs_server_get_stats(s)
    assert st.completed == n and st.failed == 0
    bfsmi.bfs_server_destroy(s)
    for h in handles:
        h.close()
    del arena
    by_graph = {}
    for t, (gi, root) in meta.items():
        by_graph.setdefault(gi, []).append((root, got[t], None))
    for gi, items in sorted(by_graph.items()):
        g = graphs[gi]
        checks = parallel.check_roots(g.off, g.col, items)
        bad = [(c.root, c.first_diff) for c in checks if not c.levels_equal]
        say("serve pool graph %d (V=%d): %d tickets, %d differ" % (gi, g.V, len(items), len(bad)))
        assert not bad, bad[:4]
    assert len(by_graph) == len(graphs)
