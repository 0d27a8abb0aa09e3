"""GPU parity of the multi-source batch (bfs_run_batch) against the oracle.

Every row of the int8 output must equal the single-root oracle levels of its
root (-1 for unreached) bit-exactly: lanes never interact, so a root's row is
the same alone and with 63 others.
"""
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu
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


def run_batch(p, G, roots):
    lv, st = G.run_batch([int(r) for r in roots])
    torch.cuda.synchronize()
    return lv.cpu().numpy(), st


def check_batch(p, g, G, roots, tag=""):
    _say("batch", g.name, tag, "V=%d n_roots=%d" % (g.V, len(roots)))
    got, st = run_batch(p, G, roots)
    exp = oracle.batch_levels_int8(g.off, g.col, roots)
    assert got.shape == exp.shape
    bad = np.nonzero((got != exp).any(axis=1))[0]
    assert bad.size == 0, "rows differ: %s" % bad[:8]
    return st


@pytest.fixture(scope="module", params=["plain", "degree_order"])
def rmat16(bfsmi, request):
    g = graphgen.rmat(16)
    flags = bfsmi.BFS_WS_BATCH
    if request.param == "degree_order":
        flags |= bfsmi.BFS_DEGREE_ORDER
    return g, bfsmi.Graph.from_csr(g.off, g.col, flags=flags)


def test_batch_64_roots(bfsmi, rmat16):
    g, G = rmat16
    roots = graphgen.pick_roots(g, 64, graphgen.root_seed(16))
    st = check_batch(bfsmi, g, G, roots, "64")
    assert st.levels >= 2 and st.edges_scanned > 0


@pytest.mark.parametrize("n", [1, 2, 7, 33])
def test_batch_sizes(bfsmi, rmat16, n):
    g, G = rmat16
    roots = graphgen.pick_roots(g, n, 100 + n)
    check_batch(bfsmi, g, G, roots, "n=%d" % n)


def test_batch_duplicates_and_isolated(bfsmi, rmat16):
    g, G = rmat16
    roots = list(graphgen.pick_roots(g, 5, 7))
    iso = int(np.nonzero(np.diff(g.off) == 0)[0][0])
    roots = roots + [roots[0], iso, roots[2], iso]
    check_batch(bfsmi, g, G, roots, "dups")


def test_lane_independence(bfsmi, rmat16):
    g, G = rmat16
    roots = graphgen.pick_roots(g, 64, 5)
    full, _ = run_batch(bfsmi, G, roots)
    alone, _ = run_batch(bfsmi, G, roots[17:18])
    assert np.array_equal(full[17], alone[0])


@pytest.mark.parametrize("tile", [256, 512, 1024, 2048])
@pytest.mark.parametrize("driver", [1, 2])
def test_batch_tiles_and_drivers(bfsmi, tile, driver):
    g = graphgen.rmat(14)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_WS_BATCH)
    G.set_option(bfsmi.BFS_OPT_BATCH_TILE, tile)
    G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, driver)
    roots = graphgen.pick_roots(g, 40, 9)
    check_batch(bfsmi, g, G, roots, "tile=%d driver=%d" % (tile, driver))
    # a second call reuses the captured levels with a new output buffer
    check_batch(bfsmi, g, G, roots[::-1], "again")


def test_batch_grid_depth(bfsmi):
    # 64 x 64 grid: eccentricities up to 126 levels still fit int8
    g = graphgen.grid(64, 64)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_WS_BATCH)
    roots = [0, 63, 64 * 64 - 1, 64 * 32 + 31, 5, 2000]
    check_batch(bfsmi, g, G, roots, "grid64")


def test_batch_depth_overflow(bfsmi):
    n = 300
    g = graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n))
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_WS_BATCH)
    with pytest.raises(bfsmi.BFSError) as e:
        G.run_batch([0, 150])
    assert e.value.code == bfsmi.BFS_ERR_DEPTH
    # a 128-vertex path from one end: the deepest level is exactly 127
    m = 128
    p = graphgen.from_edges(m, np.arange(m - 1), np.arange(1, m))
    P = bfsmi.Graph.from_csr(p.off, p.col, flags=bfsmi.BFS_WS_BATCH)
    check_batch(bfsmi, p, P, [0, m - 1, 64], "path128")


def test_batch_needs_workspace_flag(bfsmi):
    g = graphgen.rmat(10)
    G = bfsmi.Graph.from_csr(g.off, g.col)
    with pytest.raises(bfsmi.BFSError) as e:
        G.run_batch([1, 2])
    assert e.value.code == bfsmi.BFS_ERR_INVALID


def test_batch_bad_arguments(bfsmi, rmat16):
    g, G = rmat16
    out = torch.empty((65, g.V), dtype=torch.int8, device="cuda")
    with pytest.raises(bfsmi.BFSError):
        bfsmi.bfs_run_batch(G.handle, list(range(65)), out)
    with pytest.raises(bfsmi.BFSError):
        bfsmi.bfs_run_batch(G.handle, [g.V], out)
    with pytest.raises(bfsmi.BFSError):
        bfsmi.bfs_run_batch(G.handle, [], out)


def test_batch_directed(bfsmi):
    rng = np.random.default_rng(5)
    n = 3000
    src = rng.integers(0, n, 12000)
    dst = rng.integers(0, n, 12000)
    g = graphgen.from_edges(n, src, dst, symmetric=False)
    for flags in (bfsmi.BFS_WS_BATCH, bfsmi.BFS_WS_BATCH | bfsmi.BFS_DEGREE_ORDER):
        G = bfsmi.Graph.from_csr(g.off, g.col, flags=flags)
        check_batch(bfsmi, g, G, rng.choice(n, 64, replace=False), "directed")


def test_batch_row_skip_matches(bfsmi):
    # the batch's row prefix skip (edges into the id prefix every searching
    # lane has seen are dropped by the scan) changes neither the rows nor the
    # union's edge count; roots include vertices of small components, whose
    # lanes stop early and must not hold the prefix back
    g = graphgen.rmat(18, seed=12)
    deg = np.diff(g.off)
    comp = oracle.components(g.off, g.col)
    sizes = np.bincount(comp)
    small = [int(v) for v in np.nonzero((deg > 0) & (sizes[comp] < 50))[0][:4]]
    assert small, "the graph has no small component"
    roots = [int(r) for r in graphgen.pick_roots(g, 60, 77)] + small
    ref = {r: oracle.bfs(g.off, g.col, r) for r in roots}
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER | bfsmi.BFS_WS_BATCH)
    outs = {}
    for skip in (1, 0):
        G.set_option(bfsmi.BFS_OPT_ROW_SKIP, skip)
        lv, st = G.run_batch(roots)
        torch.cuda.synchronize()
        outs[skip] = (lv.cpu().numpy(), st)
    for k, r in enumerate(roots):
        want = ref[r].level.astype(np.int8)
        assert np.array_equal(outs[1][0][k], want), ("skip", k, r)
        assert np.array_equal(outs[0][0][k], want), ("no skip", k, r)
    assert outs[1][1].edges_scanned == outs[0][1].edges_scanned
    G.close()
