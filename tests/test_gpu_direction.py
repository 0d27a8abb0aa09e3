"""The direction-optimizing mode (BFS_OPT_DIRECTION: dense levels searched
bottom-up, Beamer et al.'s switches) against the serial oracle.

Levels must equal the oracle's element by element, parents must pass the
tree validator, and the level / reached / edges_scanned counts must equal
the oracle's: searching a level bottom-up changes which edges are examined,
never the result.  Covered: degree-ordered and plain CSRs, several R-MAT
scales, extreme switch thresholds, a deep grid, a disconnected graph, and
the refusal on a directed CSR."""
import numpy as np
import pytest

import graphgen
import oracle
from parity_util import assert_parity, manhattan

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bfsmi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_1605_amd as p
    p.load()
    return p


def runs(G, roots):
    out = []
    for r in roots:
        lv, pa, st = G.run(int(r))
        torch.cuda.synchronize()
        out.append((int(r), lv.cpu().numpy(), pa.cpu().numpy(), st))
    return out


@pytest.mark.parametrize("scale", [14, 16, 18])
@pytest.mark.parametrize("degree_order", [True, False])
def test_direction_optimizing_rmat(bfsmi, scale, degree_order):
    g = graphgen.rmat(scale)
    roots = graphgen.pick_roots(g, 6, graphgen.root_seed(scale))
    flags = bfsmi.BFS_DEGREE_ORDER if degree_order else 0
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=flags)
    try:
        G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
        items = runs(G, roots)
        assert_parity(g, items, label="rmat%d direction-optimizing" % scale)
        if scale >= 16:
            assert all(st.bottom_up_levels > 0 for _, _, _, st in items)
            assert all(st.edges_examined < st.edges_scanned for _, _, _, st in items)
        # top-down again on the same handle: the same levels
        G.set_option(bfsmi.BFS_OPT_DIRECTION, 0)
        td = runs(G, roots[:2])
        for (r, lv, _, st), (r2, lv2, _, st2) in zip(items, td):
            assert np.array_equal(lv, lv2)
            assert st2.bottom_up_levels == 0
    finally:
        G.close()


@pytest.mark.parametrize("alpha,beta", [(1, 1), (1, 1000), (1000, 1), (1000, 1000), (4, 100)])
def test_direction_thresholds(bfsmi, alpha, beta):
    """Any switch points give the same result (alpha = 1000 goes bottom-up
    at the first heavy level, beta = 1 returns to top-down at once)."""
    g = graphgen.rmat(15)
    roots = graphgen.pick_roots(g, 4, graphgen.root_seed(15))
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    try:
        G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
        G.set_option(bfsmi.BFS_OPT_DO_ALPHA, alpha)
        G.set_option(bfsmi.BFS_OPT_DO_BETA, beta)
        assert_parity(g, runs(G, roots), label="rmat15 alpha %d beta %d" % (alpha, beta))
    finally:
        G.close()


def test_direction_grid_and_loop_driver(bfsmi):
    """A 200 x 200 grid (hundreds of levels, the persistent loop between
    heavy levels) with an eager switch; levels = Manhattan distance."""
    w = 200
    g = graphgen.grid(w)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    try:
        G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
        G.set_option(bfsmi.BFS_OPT_DO_ALPHA, 1000)
        for driver in (0, 1):
            G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, driver)
            items = runs(G, [0, w * w // 2 + 3])
            for r, lv, _, _ in items:
                assert np.array_equal(lv, manhattan(w, w, r)), (driver, r)
            assert_parity(g, items, label="grid200 direction-optimizing driver %d" % driver)
    finally:
        G.close()


def test_direction_disconnected(bfsmi):
    """Unreachable vertices are probed by every bottom-up step and never
    found; a root in the small component ends with the rest at -1."""
    r = graphgen.rmat(13)
    n = 50
    cs = np.arange(n)
    rs = np.repeat(np.arange(r.V), np.diff(r.off)) + n
    g = graphgen.from_edges(n + r.V, np.concatenate([cs, rs]),
                            np.concatenate([(cs + 1) % n, r.col.astype(np.int64) + n]))
    g.name = "cycle50+rmat13"
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    try:
        G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
        big = n + int(graphgen.pick_roots(r, 1, 9)[0])
        items = runs(G, [7, big])
        assert_parity(g, items, label="disconnected direction-optimizing")
        assert (items[0][1][n:] == -1).all()
        assert (items[1][1][:n] == -1).all()
    finally:
        G.close()


def test_direction_refused_on_directed_csr(bfsmi):
    rng = np.random.default_rng(3)
    g = graphgen.from_edges(500, rng.integers(0, 500, 3000), rng.integers(0, 500, 3000),
                            symmetric=False)
    G = bfsmi.Graph.from_csr(g.off, g.col)
    try:
        with pytest.raises(bfsmi.BFSError) as e:
            G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
        assert e.value.code == bfsmi.BFS_ERR_INVALID
        assert "symmetric" in str(e.value)
    finally:
        G.close()
    # the symmetric closure of the same edges is accepted
    s = graphgen.from_edges(500, rng.integers(0, 500, 3000), rng.integers(0, 500, 3000))
    G = bfsmi.Graph.from_csr(s.off, s.col)
    try:
        G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
        assert_parity(s, runs(G, [int(s.col[0])]), label="symmetric closure")
    finally:
        G.close()
