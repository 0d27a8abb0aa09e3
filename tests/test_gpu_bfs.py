"""GPU parity of the single-root search against the CPU oracle.

Levels must match the oracle bit-exactly; parents (not unique under atomic
races) must pass the oracle's tree validator; per-level frontier sizes must
equal the oracle's (each vertex claimed exactly once).  Everything goes
through the C ABI (libbfsmi.so) via the ctypes binding.
"""
import os
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


def check(p, g, G, root, mode=0, ept=4, want_parents=True, directed=False):
    _say("case", g.name, "V=%d nnz=%d root=%d mode=%d ept=%d" % (g.V, g.nnz, root, mode, ept))
    G.set_option(p.BFS_OPT_FRONTIER_MODE, mode)
    G.set_option(p.BFS_OPT_EDGES_PER_THREAD, ept)
    lv, pa, st = G.run(root, want_parents=want_parents)
    torch.cuda.synchronize()
    lv = lv.cpu().numpy()
    ref = oracle.bfs(g.off, g.col, root)
    assert np.array_equal(lv, ref.level), "levels differ at %s" % np.nonzero(lv != ref.level)[0][:10]
    assert st.levels == ref.nlevels
    assert st.reached == ref.reached
    assert st.edges_scanned == ref.edges_scanned
    if want_parents:
        pa = pa.cpu().numpy()
        code, bad = oracle.validate(g.off, g.col, root, lv, pa, directed=directed)
        assert code == 0, (oracle.INVARIANTS[code], bad)
    return st


def test_duplicates_and_self_loops(bfsmi):
    g = graphgen.from_edges(6, [0, 0, 0, 1, 1, 2, 3, 4], [1, 1, 0, 1, 2, 3, 4, 5])
    for flags in _flag_variants(bfsmi):
        G = bfsmi.Graph.from_csr(g.off, g.col, flags=flags)
        for r in range(6):
            check(bfsmi, g, G, r)


def test_path_and_disconnected(bfsmi):
    n = 2000
    src = np.concatenate([np.arange(999), np.arange(1000, 1999)])
    g = graphgen.from_edges(n, src, src + 1)
    for flags in _flag_variants(bfsmi):
        G = bfsmi.Graph.from_csr(g.off, g.col, flags=flags)
        for root in (0, 500, 1500, 1999):
            check(bfsmi, g, G, root)


@pytest.fixture(scope="module", params=["plain", "degree_order"])
def rmat16(bfsmi, request):
    g = graphgen.rmat(16)
    flags = bfsmi.BFS_VALIDATE_CSR
    if request.param == "degree_order":
        flags |= bfsmi.BFS_DEGREE_ORDER
    return g, bfsmi.Graph.from_csr(g.off, g.col, flags=flags)


def _flag_variants(p):
    return [0, p.BFS_DEGREE_ORDER]


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("ept", [1, 2, 4, 8])
def test_rmat16_modes_ept(bfsmi, rmat16, mode, ept):
    g, G = rmat16
    roots = graphgen.pick_roots(g, 4, graphgen.root_seed(16))
    for r in roots:
        check(bfsmi, g, G, int(r), mode=mode, ept=ept)


@pytest.mark.parametrize("driver", [1, 0])
def test_rmat16_sixteen_roots_auto(bfsmi, rmat16, driver):
    g, G = rmat16
    G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, driver)
    roots = graphgen.pick_roots(g, 16, graphgen.root_seed(16))
    nb = 0
    for r in roots:
        st = check(bfsmi, g, G, int(r))
        nb += st.bitmap_levels
    G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, 0)
    if driver == 1:
        assert nb > 0  # R-MAT frontiers cross T = V/32 at their peak


def test_isolated_root(bfsmi, rmat16):
    g, G = rmat16
    iso = int(np.nonzero(np.diff(g.off) == 0)[0][0])
    st = check(bfsmi, g, G, iso)
    assert st.levels == 1 and st.reached == 1


def test_no_parents(bfsmi, rmat16):
    g, G = rmat16
    r = int(graphgen.pick_roots(g, 1, 5)[0])
    check(bfsmi, g, G, r, want_parents=False)


def test_repeatable(bfsmi, rmat16):
    g, G = rmat16
    r = int(graphgen.pick_roots(g, 1, 9)[0])
    outs = [G.run(r)[0].cpu().numpy() for _ in range(5)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("w,h", [(1, 1), (1, 300), (37, 23), (128, 128)])
@pytest.mark.parametrize("dord", [0, 1])
def test_grids_manhattan(bfsmi, w, h, dord):
    g = graphgen.grid(w, h)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER if dord else 0)
    r_, c_ = np.divmod(np.arange(g.V), w)
    for root in sorted({0, g.V - 1, (h // 2) * w + w // 2}):
        check(bfsmi, g, G, root)
        lv = G.run(root)[0].cpu().numpy()
        r0, c0 = divmod(root, w)
        assert np.array_equal(lv, np.abs(r_ - r0) + np.abs(c_ - c0))


def test_hub_star(bfsmi):
    # one vertex of degree 200k: a single frontier entry spans many tiles
    n = 200_001
    g = graphgen.from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n))
    for flags in _flag_variants(bfsmi):
        G = bfsmi.Graph.from_csr(g.off, g.col, flags=flags)
        for ept in (1, 8):
            check(bfsmi, g, G, 0, ept=ept)
            check(bfsmi, g, G, 77, ept=ept)


def test_directed_zero_outdegree(bfsmi):
    """Directed graph where most frontier vertices have no out-edges: the
    tile's entry range exceeds the tile, exercising the global search."""
    rng = np.random.default_rng(3)
    n = 50_000
    # vertex 0 points to every other vertex; only 1% of them point onwards
    src = [np.zeros(n - 1, np.int64)]
    dst = [np.arange(1, n)]
    movers = rng.choice(np.arange(1, n), size=500, replace=False)
    src.append(movers)
    dst.append(rng.integers(1, n, size=500))
    g = graphgen.from_edges(n, np.concatenate(src), np.concatenate(dst), symmetric=False)
    for flags in _flag_variants(bfsmi):
        G = bfsmi.Graph.from_csr(g.off, g.col, flags=flags)
        for mode in (0, 1, 2):
            check(bfsmi, g, G, 0, mode=mode, directed=True)
            check(bfsmi, g, G, int(movers[0]), mode=mode, directed=True)


def test_bad_arguments_on_gpu(bfsmi, rmat16):
    g, G = rmat16
    lv = torch.empty(g.V, dtype=torch.int32, device="cuda")
    with pytest.raises(bfsmi.BFSError) as e:
        bfsmi.bfs_run(G.handle, g.V, lv)
    assert e.value.code == bfsmi.BFS_ERR_INVALID
    with pytest.raises(bfsmi.BFSError) as e:
        bfsmi.bfs_run(G.handle, -1, lv)
    assert e.value.code == bfsmi.BFS_ERR_INVALID
    # workspace too small
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(bfsmi.BFSError) as e:
        bfsmi.bfs_graph_create(g.V, g.nnz, G.off, G.col, ws, 1024)
    assert e.value.code == bfsmi.BFS_ERR_WORKSPACE
    # an out-of-range column id is rejected at creation
    bad = g.col.copy()
    bad[17] = g.V + 5
    with pytest.raises(bfsmi.BFSError) as e:
        bfsmi.Graph.from_csr(g.off, bad)
    assert e.value.code == bfsmi.BFS_ERR_INVALID
    # non-monotone offsets
    off = g.off.copy()
    off[10] = off[11] + 1
    with pytest.raises(bfsmi.BFSError) as e:
        bfsmi.Graph.from_csr(off, g.col)
    assert e.value.code == bfsmi.BFS_ERR_INVALID


@pytest.mark.parametrize("summary", [0, 1, 2])
@pytest.mark.parametrize("dord", [0, 1])
def test_visited_summary(bfsmi, summary, dord):
    g = graphgen.rmat(15)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER if dord else 0)
    G.set_option(bfsmi.BFS_OPT_VISITED_SUMMARY, summary)
    for r in graphgen.pick_roots(g, 3, 21):
        for mode in (0, 1, 2):
            check(bfsmi, g, G, int(r), mode=mode)


def test_visited_summary_odd_sizes(bfsmi):
    # V not a multiple of 32 or of the summary block: tail bits must not
    # count as open vertices, and a fully visited graph must still end
    for n in (33, 1000, 1025, 4097):
        src = np.arange(n - 1)
        g = graphgen.from_edges(n, np.zeros(n - 1, np.int64), src + 1)   # star
        G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
        for summary in (1, 2):
            G.set_option(bfsmi.BFS_OPT_VISITED_SUMMARY, summary)
            for r in (0, n - 1):
                for mode in (0, 2):
                    check(bfsmi, g, G, r, mode=mode)


@pytest.mark.skipif(os.environ.get("BFSMI_BIG", "1") == "0", reason="large graphs disabled")
@pytest.mark.parametrize("dord", [0, 1])
def test_rmat20_parity(bfsmi, dord):
    g = graphgen.rmat(20)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER if dord else 0)
    for r in graphgen.pick_roots(g, 3, graphgen.root_seed(20)):
        check(bfsmi, g, G, int(r))


@pytest.mark.parametrize("driver", [0, 1])
def test_loop_driver_equivalence(bfsmi, driver):
    # the persistent loop runs small levels back to back and hands heavy
    # levels back to the host; both drivers must give the oracle's levels,
    # sizes and a valid tree
    cases = [graphgen.grid(300, 300), graphgen.grid(1000, 3), graphgen.rmat(18)]
    for g in cases:
        G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
        G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, driver)
        roots = [0, g.V - 1] if g.name.startswith("grid") else \
            [int(r) for r in graphgen.pick_roots(g, 2, 33)]
        for r in roots:
            st = check(bfsmi, g, G, r)
            if driver == 1:
                assert st.device_loop_levels == 0
            elif g.name.startswith("grid"):
                assert st.device_loop_levels >= st.levels - 2
        G.close()


def test_device_loop_hands_back_heavy_level(bfsmi):
    # scale 20: the hub levels exceed the persistent loop's degree and edge
    # limits, so the search moves loop -> host -> loop
    g = graphgen.rmat(20)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    for r in graphgen.pick_roots(g, 3, 44):
        st = check(bfsmi, g, G, int(r))
        assert 0 < st.device_loop_levels < st.levels
    G.close()


def test_row_skip_matches_full_rows(bfsmi):
    # The row prefix skip drops a frontier row's leading edges into the fully
    # visited id prefix before the expansion: levels, frontier sizes, the edge
    # count and tree validity must not change, and on R-MAT the expansion
    # must stream fewer column bytes.
    g = graphgen.rmat(20)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    assert G.get_option(bfsmi.BFS_OPT_ROW_SKIP) == 1
    fewer = 0
    for r in graphgen.pick_roots(g, 3, 55):
        G.set_option(bfsmi.BFS_OPT_ROW_SKIP, 0)
        full = check(bfsmi, g, G, int(r))
        G.set_option(bfsmi.BFS_OPT_ROW_SKIP, 1)
        for mode in (0, 1, 2):
            st = check(bfsmi, g, G, int(r), mode=mode)
            assert st.edges_scanned == full.edges_scanned
        fewer += st.expand_bytes < full.expand_bytes
    assert fewer >= 1
    G.close()


@pytest.mark.parametrize("n", [70_000, 300_000, 1_100_000])
def test_row_skip_whole_rows(bfsmi, n):
    # star with a leaf as root: the last level's frontier is every other leaf
    # and each leaf row is one edge back to the visited centre (internal id 0),
    # so the skip drops whole rows (the level has no edges left to expand);
    # n spans the thresholds 2^16, 2^18 and 2^20
    leaves = np.arange(1, n, dtype=np.int64)
    g = graphgen.from_edges(n, np.zeros(n - 1, np.int64), leaves)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    for r in (1, n - 1, 0):
        for mode in (0, 1):
            check(bfsmi, g, G, r, mode=mode)
    G.close()


def _fan_tree(fans):
    """Rooted tree, vertex 0 the root; every vertex of depth d has fans[d]
    children (ids in breadth-first order)."""
    src, dst, level_start, width = [], [], 0, 1
    nxt = 1
    for f in fans:
        parents = np.arange(level_start, level_start + width, dtype=np.int64)
        kids = np.arange(nxt, nxt + width * f, dtype=np.int64)
        src.append(np.repeat(parents, f))
        dst.append(kids)
        level_start, width, nxt = nxt, width * f, nxt + width * f
    g = graphgen.from_edges(nxt, np.concatenate(src), np.concatenate(dst))
    g.name = "fan" + "x".join(str(f) for f in fans)
    return g


@pytest.mark.parametrize("fans", [(256, 256), (257, 256), (256, 256, 1), (16, 4096, 1)])
@pytest.mark.parametrize("dord", [0, 1])
def test_device_loop_frontier_at_capacity(bfsmi, fans, dord):
    # The persistent loop keeps each frontier entry's row start, degree and
    # caller id for at most 65536 entries and hands a larger frontier back to
    # the host.  (256, 256): a frontier of exactly 65536 leaves continues in
    # the loop; (257, 256): 65792 leaves go back to the host; the third level
    # of (256, 256, 1) and (16, 4096, 1) expands a full-capacity frontier
    # from the carried row data.
    g = _fan_tree(fans)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER if dord else 0)
    st = check(bfsmi, g, G, 0)
    # every expansion runs in the loop, except the one after a frontier
    # over capacity
    width = int(np.prod(fans[:2]))
    assert st.device_loop_levels == (st.levels if width <= 65536 else st.levels - 1)
    check(bfsmi, g, G, g.V - 1)
    G.close()


# ---------------------------------------------------------------------------
# Claim modes of the bitmap levels (BFS_OPT_CLAIM_MODE): the atomicOr claim
# of Algorithm 3 (0), byte flags (2) and the size-based choice (1) give the
# same levels and valid parents.

@pytest.mark.parametrize("claim", [0, 1, 2])
@pytest.mark.parametrize("scale", [12, 16, 18])
def test_claim_modes_rmat(bfsmi, claim, scale):
    g = graphgen.rmat(scale)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_CLAIM_MODE, claim)
    assert G.get_option(bfsmi.BFS_OPT_CLAIM_MODE) == claim
    if scale < 16:
        # small graphs run every level in the persistent loop by default
        G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, 1)
    roots = graphgen.pick_roots(g, 6, graphgen.root_seed(scale))
    nbitmap = 0
    for r in roots:
        st = check(bfsmi, g, G, int(r))
        nbitmap += st.bitmap_levels
    assert nbitmap > 0  # the bitmap levels (where the modes differ) ran


@pytest.mark.parametrize("claim", [0, 2])
@pytest.mark.parametrize("fmode", [1, 2])
def test_claim_modes_frontier_forms(bfsmi, claim, fmode):
    # list-only levels never use flags; bitmap-whenever-possible levels
    # flag every level the host drives
    g = graphgen.rmat(14)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_CLAIM_MODE, claim)
    G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, 1)  # every level from the host
    for r in graphgen.pick_roots(g, 4, graphgen.root_seed(14)):
        check(bfsmi, g, G, int(r), mode=fmode)


def test_claim_flags_cleared_between_searches(bfsmi):
    # flags set by one search must not leak into the next: alternate roots
    # in different components and sizes on one handle, with and without
    # parents
    a = graphgen.rmat(13)
    n = a.V
    # two copies of the graph side by side: roots in either half
    src = np.repeat(np.arange(2 * n), np.diff(np.concatenate([a.off, a.off[1:] + a.nnz])))
    dst = np.concatenate([a.col, a.col + n])
    g = graphgen.from_edges(2 * n, src, dst)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_CLAIM_MODE, 2)
    roots = graphgen.pick_roots(g, 8, 77)
    for i, r in enumerate(roots):
        check(bfsmi, g, G, int(r), want_parents=(i % 2 == 0))


@pytest.mark.parametrize("claim", [0, 2])
def test_claim_modes_direction_optimizing(bfsmi, claim):
    g = graphgen.rmat(16)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_CLAIM_MODE, claim)
    G.set_option(bfsmi.BFS_OPT_DIRECTION, 1)
    for r in graphgen.pick_roots(g, 4, graphgen.root_seed(16)):
        check(bfsmi, g, G, int(r))


@pytest.mark.parametrize("w,h", [(37, 23), (300, 200)])
def test_claim_flags_grids(bfsmi, w, h):
    g = graphgen.grid(w, h)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_CLAIM_MODE, 2)
    G.set_option(bfsmi.BFS_OPT_FRONTIER_MODE, 2)
    G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, 1)
    for root in (0, w * h - 1, (h // 2) * w + w // 3):
        lv, pa, st = G.run(root)
        torch.cuda.synchronize()
        r0, c0 = divmod(root, w)
        rr, cc = np.divmod(np.arange(w * h), w)
        assert np.array_equal(lv.cpu().numpy(), np.abs(rr - r0) + np.abs(cc - c0))
        code, bad = oracle.validate(g.off, g.col, root, lv.cpu().numpy(), pa.cpu().numpy())
        assert code == 0, (oracle.INVARIANTS[code], bad)


def test_claim_mode_rejects_bad_values(bfsmi):
    g = graphgen.rmat(10)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    for bad in (-1, 3):
        with pytest.raises(bfsmi.BFSError):
            G.set_option(bfsmi.BFS_OPT_CLAIM_MODE, bad)
    assert G.get_option(bfsmi.BFS_OPT_CLAIM_MODE) == 1


# ---------------------------------------------------------------------------
# XCD-sliced levels (BFS_OPT_XCD_SLICES): rows grouped by the slice of their
# targets, workgroup b of the expansion taking slice b mod 8 only.

@pytest.mark.parametrize("xs", [0, 1, 2])
@pytest.mark.parametrize("claim", [0, 1, 2])
@pytest.mark.parametrize("scale", [13, 17])
def test_xcd_slices_rmat(bfsmi, xs, claim, scale):
    g = graphgen.rmat(scale)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_XCD_SLICES, xs)
    G.set_option(bfsmi.BFS_OPT_CLAIM_MODE, claim)
    assert G.get_option(bfsmi.BFS_OPT_XCD_SLICES) == xs
    G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, 1)  # every level through the host path
    for r in graphgen.pick_roots(g, 5, graphgen.root_seed(scale)):
        check(bfsmi, g, G, int(r))


@pytest.mark.parametrize("fmode", [0, 1, 2])
@pytest.mark.parametrize("ept", [1, 4, 8])
def test_xcd_slices_forms_and_ept(bfsmi, fmode, ept):
    g = graphgen.rmat(15)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_XCD_SLICES, 2)
    G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, 1)
    for r in graphgen.pick_roots(g, 3, graphgen.root_seed(15)):
        check(bfsmi, g, G, int(r), mode=fmode, ept=ept)


def test_xcd_slices_odd_sizes_and_hubs(bfsmi):
    # V not a multiple of 1024 or 32, a hub touching every slice, ids on
    # both sides of the hot-id limit (8192), a disconnected part
    rng = np.random.default_rng(5)
    n = 20_011
    src = np.concatenate([np.zeros(n - 1, np.int64), rng.integers(0, n - 500, 60_000)])
    dst = np.concatenate([np.arange(1, n), rng.integers(0, n - 500, 60_000)])
    keep = (src < n - 500) & (dst < n - 500)
    src, dst = src[keep], dst[keep]
    tail = np.arange(n - 500, n - 1)
    g = graphgen.from_edges(n, np.concatenate([src, tail]), np.concatenate([dst, tail + 1]))
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_XCD_SLICES, 2)
    G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, 1)
    for r in (0, 1, 9000, n - 500, n - 1):
        check(bfsmi, g, G, r)


def test_xcd_slices_directed(bfsmi):
    # a directed CSR (rows are out-edges only): sliced levels follow them
    rng = np.random.default_rng(11)
    n = 50_000
    src = rng.integers(0, n, 400_000)
    dst = (src * 7 + rng.integers(0, 3000, 400_000) ** 2) % n
    g = graphgen.from_edges(n, src, dst, symmetric=False)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    G.set_option(bfsmi.BFS_OPT_XCD_SLICES, 2)
    G.set_option(bfsmi.BFS_OPT_LOOP_DRIVER, 1)
    for r in (0, 17, 4242):
        check(bfsmi, g, G, r, directed=True)


def test_xcd_slices_option_values(bfsmi):
    g = graphgen.rmat(10)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    assert G.get_option(bfsmi.BFS_OPT_XCD_SLICES) == 1
    for bad in (-1, 3):
        with pytest.raises(bfsmi.BFSError):
            G.set_option(bfsmi.BFS_OPT_XCD_SLICES, bad)
