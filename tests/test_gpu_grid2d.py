"""The in-GPU 2D blocked search (bfs_grid2d_*: the R x C processor grid of
Section 2.2 with Algorithm 2's expand / fold exchanges, Algorithm 3's
tgtj grouping, the frontier update of Section 3.5 and the list / bitmap
messages of Section 5) against the serial oracle.

Levels must equal the oracle's element by element, parents must pass the
tree validator, and the search's level / reached / edge counts must equal
the oracle's, for every grid shape the library accepts, every message mode,
ragged block sizes, directed and disconnected inputs, and a deep graph."""
import numpy as np
import pytest

import graphgen
import oracle
from parity_util import assert_parity, manhattan

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(1, 1), (1, 2), (2, 1), (2, 2), (1, 4), (4, 1), (2, 4), (4, 2), (8, 1), (1, 8),
          (4, 4), (2, 8), (8, 8), (16, 4)]


@pytest.fixture(scope="module")
def bfsmi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_1605_amd as p
    p.load()
    return p


@pytest.fixture(scope="module")
def rmat14():
    return graphgen.rmat(14)


def run_roots(bfsmi, G, roots, mode):
    items = []
    for r in roots:
        lv, pa, st = G.run(int(r), msg_mode=mode)
        torch.cuda.synchronize()
        items.append((int(r), lv.cpu().numpy(), pa.cpu().numpy(), st))
    return items


@pytest.mark.parametrize("R,C", SHAPES)
def test_grid2d_rmat14_every_shape(bfsmi, rmat14, R, C):
    g = rmat14
    roots = graphgen.pick_roots(g, 3, graphgen.root_seed(14))
    G = bfsmi.Grid2D.from_csr(g.off, g.col, R, C)
    try:
        for mode in (bfsmi.BFS_2D_MSG_AUTO, bfsmi.BFS_2D_MSG_LIST, bfsmi.BFS_2D_MSG_BITMAP):
            items = run_roots(bfsmi, G, roots, mode)
            assert_parity(g, items, label="rmat14 %dx%d mode %d" % (R, C, mode))
            for _, _, _, st in items:
                if mode == bfsmi.BFS_2D_MSG_LIST:
                    assert st.fold_bitmap_msgs == 0 and st.expand_bitmap_msgs == 0
                if mode == bfsmi.BFS_2D_MSG_BITMAP:
                    assert st.fold_list_msgs == 0 and st.list_levels == 0
                if C == 1:
                    assert st.fold_list_msgs == 0 and st.fold_bitmap_msgs == 0
                    assert st.updated == 0
                if R == 1:
                    assert st.expand_list_msgs == 0 and st.expand_bitmap_msgs == 0
                assert st.fold_bytes >= 0 and st.fold_list_only_bytes >= 0
    finally:
        G.close()


def test_grid2d_rmat16_auto_switches_message_form(bfsmi):
    """At scale 16 the dense levels send bitmaps and the sparse ones lists,
    in both exchanges; as lists only, the same searches move more bytes."""
    g = graphgen.rmat(16)
    roots = graphgen.pick_roots(g, 4, graphgen.root_seed(16))
    G = bfsmi.Grid2D.from_csr(g.off, g.col, 2, 4)
    try:
        items = run_roots(bfsmi, G, roots, bfsmi.BFS_2D_MSG_AUTO)
        assert_parity(g, items, label="rmat16 2x4 auto")
        st = items[0][3]
        assert st.fold_bitmap_msgs > 0 and st.fold_list_msgs > 0
        assert st.expand_bitmap_msgs > 0 and st.expand_list_msgs > 0
        assert st.fold_bytes < st.fold_list_only_bytes
        assert st.expand_bytes < st.expand_list_only_bytes
        assert st.updated > 0
    finally:
        G.close()


@pytest.mark.parametrize("R,C", [(1, 8), (8, 1), (4, 2)])
def test_grid2d_directed_zero_outdegree(bfsmi, R, C):
    """Directed input: many vertices without out-edges, sources that are
    never reached; levels follow out-edges only."""
    rng = np.random.default_rng(71)
    V = 3000
    src = rng.integers(0, V // 3, size=9000)
    dst = rng.integers(0, V, size=9000)
    g = graphgen.from_edges(V, src, dst, symmetric=False)
    g.name = "directed3000"
    roots = [int(x) for x in src[:3]]
    G = bfsmi.Grid2D.from_csr(g.off, g.col, R, C)
    try:
        for mode in (0, 1, 2):
            assert_parity(g, run_roots(bfsmi, G, roots, mode), directed=True,
                          label="directed %dx%d mode %d" % (R, C, mode))
    finally:
        G.close()


@pytest.mark.parametrize("R,C", [(8, 8), (4, 1), (1, 2)])
def test_grid2d_tiny_and_disconnected(bfsmi, R, C):
    """Five vertices over up to 64 processors (most own no vertex), and a
    root in a small component of a disconnected graph."""
    path = graphgen.from_edges(5, np.arange(4), np.arange(1, 5))
    path.name = "path5"
    G = bfsmi.Grid2D.from_csr(path.off, path.col, R, C)
    try:
        for mode in (0, 1, 2):
            assert_parity(path, run_roots(bfsmi, G, [0, 2, 4], mode), label="path5")
    finally:
        G.close()
    # two components: a 40-cycle and an R-MAT scale-10 graph shifted past it
    r = graphgen.rmat(10)
    n = 40
    cyc_s = np.arange(n)
    cyc_d = (cyc_s + 1) % n
    rs = np.repeat(np.arange(r.V), np.diff(r.off)) + n
    rd = r.col.astype(np.int64) + n
    g = graphgen.from_edges(n + r.V, np.concatenate([cyc_s, rs]), np.concatenate([cyc_d, rd]))
    g.name = "cycle+rmat10"
    G = bfsmi.Grid2D.from_csr(g.off, g.col, R, C)
    try:
        items = run_roots(bfsmi, G, [3, n + int(graphgen.pick_roots(r, 1, 5)[0])], 0)
        assert_parity(g, items, label="disconnected")
        lv = items[0][1]
        assert (lv[n:] == -1).all() and lv[:n].max() == n // 2
    finally:
        G.close()


def test_grid2d_deep_grid(bfsmi):
    """A 96 x 96 grid: ~190 levels of small fronts, levels = Manhattan
    distance."""
    w = 96
    g = graphgen.grid(w)
    G = bfsmi.Grid2D.from_csr(g.off, g.col, 2, 4)
    try:
        for root in (0, w * w // 2 + 7):
            items = run_roots(bfsmi, G, [root], 0)
            assert np.array_equal(items[0][1], manhattan(w, w, root))
            assert_parity(g, items, label="grid96 2x4")
    finally:
        G.close()


def test_grid2d_argument_checks(bfsmi):
    with pytest.raises(bfsmi.BFSError) as e:
        bfsmi.bfs_grid2d_workspace_bytes(100, 10, 3, 3)
    assert e.value.code == bfsmi.BFS_ERR_INVALID
    g = graphgen.rmat(8)
    G = bfsmi.Grid2D.from_csr(g.off, g.col, 2, 2)
    try:
        with pytest.raises(bfsmi.BFSError):
            G.run(g.V)
        with pytest.raises(bfsmi.BFSError):
            G.run(0, msg_mode=3)
    finally:
        G.close()
