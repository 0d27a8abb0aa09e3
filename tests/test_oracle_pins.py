"""Pins for the CPU oracle: closed forms, brute force on tiny graphs, an
independent library routine, and negative tests of the validator.

Nothing here re-types the oracle's loop: every expected value comes from a
different algorithm (Floyd-Warshall, boolean matrix powers, scipy's shortest
paths, union-find vs scipy components) or from a closed form of the graph.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphgen
import oracle


# ----------------------------------------------------------------------------
# helpers that do not share code with the oracle


def floyd_warshall_hops(adj: np.ndarray) -> np.ndarray:
    """All-pairs hop distances by Floyd-Warshall; -1 = unreachable."""
    n = adj.shape[0]
    INF = 10**9
    d = np.where(adj, 1, INF).astype(np.int64)
    np.fill_diagonal(d, 0)
    for k in range(n):
        d = np.minimum(d, d[:, [k]] + d[[k], :])
    return np.where(d >= INF, -1, d)


def matrix_power_levels(adj: np.ndarray, root: int) -> np.ndarray:
    """Hop distance from root via boolean powers: the set reached in exactly
    <= k steps is R_k = R_{k-1} | (R_{k-1} @ A)."""
    n = adj.shape[0]
    A = adj.astype(np.int64)
    lv = np.full(n, -1, dtype=np.int64)
    reach = np.zeros(n, dtype=bool)
    reach[root] = True
    lv[root] = 0
    k = 0
    while True:
        k += 1
        nxt = reach | ((reach.astype(np.int64) @ A) > 0)
        new = nxt & ~reach
        if not new.any():
            break
        lv[new] = k
        reach = nxt
    return lv


def check_result(g, root, res, directed=False):
    code, bad = oracle.validate(g.off, g.col, root, res.level, res.parent, directed=directed,
                                rows_sorted=True)
    assert code == 0, (oracle.INVARIANTS[code], bad)
    # frontier sizes are the level histogram; edges scanned = reached degrees
    assert np.array_equal(res.frontier_sizes, oracle.levels_hist(res.level))
    deg = np.diff(g.off)
    assert res.edges_scanned == int(deg[res.level >= 0].sum())


# ----------------------------------------------------------------------------
# closed forms


def path_graph(n):
    return graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n))


def cycle_graph(n):
    return graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)


@pytest.mark.parametrize("n", [1, 2, 7, 100])
def test_path_closed_form(n):
    g = path_graph(n) if n > 1 else graphgen.CSR(np.zeros(2, np.int64), np.zeros(0, np.int32))
    for r in {0, n // 2, n - 1}:
        res = oracle.bfs(g.off, g.col, r)
        assert np.array_equal(res.level, np.abs(np.arange(n) - r))
        check_result(g, r, res)


@pytest.mark.parametrize("n", [3, 8, 11])
def test_cycle_closed_form(n):
    g = cycle_graph(n)
    for r in range(n):
        res = oracle.bfs(g.off, g.col, r)
        d = np.abs(np.arange(n) - r)
        assert np.array_equal(res.level, np.minimum(d, n - d))
        check_result(g, r, res)


def test_star_and_complete():
    n = 9
    star = graphgen.from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n))
    res = oracle.bfs(star.off, star.col, 0)
    assert res.level.tolist() == [0] + [1] * (n - 1)
    assert res.parent.tolist() == [0] * n
    res = oracle.bfs(star.off, star.col, 3)
    assert res.level.tolist() == [1, 2, 2, 0, 2, 2, 2, 2, 2]
    check_result(star, 3, res)
    iu = np.triu_indices(n, 1)
    comp = graphgen.from_edges(n, iu[0], iu[1])
    for r in range(n):
        res = oracle.bfs(comp.off, comp.col, r)
        exp = np.ones(n, np.int64)
        exp[r] = 0
        assert np.array_equal(res.level, exp)
        assert np.all(res.parent == r)


def test_complete_binary_tree():
    n = 2**7 - 1
    child = np.arange(1, n)
    g = graphgen.from_edges(n, (child - 1) // 2, child)
    res = oracle.bfs(g.off, g.col, 0)
    assert np.array_equal(res.level, np.floor(np.log2(np.arange(n) + 1)).astype(int))
    # in a tree the parent is forced
    assert np.array_equal(res.parent[1:], (child - 1) // 2)
    check_result(g, 0, res)


@pytest.mark.parametrize("w,h", [(1, 1), (1, 9), (7, 5), (64, 64)])
def test_grid_manhattan(w, h):
    g = graphgen.grid(w, h)
    V = w * h
    r_, c_ = np.divmod(np.arange(V), w)
    for root in {0, V - 1, (h // 2) * w + w // 3}:
        res = oracle.bfs(g.off, g.col, root)
        r0, c0 = divmod(root, w)
        assert np.array_equal(res.level, np.abs(r_ - r0) + np.abs(c_ - c0))
        check_result(g, root, res)
        assert res.nlevels == int((np.abs(r_ - r0) + np.abs(c_ - c0)).max()) + 1


def test_disjoint_union_unreached():
    a = path_graph(5)
    # two paths 0-4 and 5-9 plus isolated vertex 10
    src = np.concatenate([np.arange(4), np.arange(5, 9)])
    dst = src + 1
    g = graphgen.from_edges(11, src, dst)
    res = oracle.bfs(g.off, g.col, 2)
    assert res.level.tolist() == [2, 1, 0, 1, 2] + [-1] * 6
    assert res.parent[5:].tolist() == [-1] * 6
    check_result(g, 2, res)
    res = oracle.bfs(g.off, g.col, 10)
    assert res.level.tolist() == [-1] * 10 + [0]
    assert res.nlevels == 1 and res.edges_scanned == 0
    check_result(g, 10, res)
    del a


def test_hypercube_hamming():
    d = 6
    n = 1 << d
    src, dst = [], []
    for v in range(n):
        for b in range(d):
            w = v ^ (1 << b)
            if v < w:
                src.append(v)
                dst.append(w)
    g = graphgen.from_edges(n, src, dst)
    for r in (0, 5, 63):
        res = oracle.bfs(g.off, g.col, r)
        ham = np.array([bin(v ^ r).count("1") for v in range(n)])
        assert np.array_equal(res.level, ham)
        check_result(g, r, res)


def test_self_loops_and_duplicates_are_legal():
    # path 0-1-2 with a self-loop on 1 and the edge 0-1 three times
    g = graphgen.from_edges(3, [0, 1, 0, 0, 1], [1, 1, 1, 1, 2])
    res = oracle.bfs(g.off, g.col, 0)
    assert res.level.tolist() == [0, 1, 2]
    assert res.parent.tolist() == [0, 0, 1]
    code, _ = oracle.validate(g.off, g.col, 0, res.level, res.parent)
    assert code == 0


# ----------------------------------------------------------------------------
# brute force


def all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        adj = np.zeros((n, n), dtype=bool)
        for i, (a, b) in enumerate(pairs):
            if mask >> i & 1:
                adj[a, b] = adj[b, a] = True
        yield adj


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_small_undirected(n):
    for adj in all_graphs(n):
        g = graphgen.from_dense(adj)
        fw = floyd_warshall_hops(adj)
        for r in range(n):
            res = oracle.bfs(g.off, g.col, r)
            assert np.array_equal(res.level, fw[r]), (adj.astype(int), r)
            check_result(g, r, res)


def test_random_directed_matrix_powers():
    rng = np.random.default_rng(7)
    for trial in range(60):
        n = int(rng.integers(1, 65))
        p = float(rng.choice([0.02, 0.05, 0.1, 0.3]))
        adj = rng.random((n, n)) < p
        np.fill_diagonal(adj, False)
        g = graphgen.from_dense(adj)
        for r in rng.choice(n, size=min(n, 4), replace=False):
            res = oracle.bfs(g.off, g.col, int(r))
            assert np.array_equal(res.level, matrix_power_levels(adj, int(r)))
            check_result(g, int(r), res, directed=True)


def test_random_undirected_matrix_powers():
    rng = np.random.default_rng(11)
    for trial in range(60):
        n = int(rng.integers(2, 65))
        adj = rng.random((n, n)) < rng.choice([0.03, 0.08, 0.2])
        adj = np.triu(adj, 1)
        adj = adj | adj.T
        g = graphgen.from_dense(adj)
        for r in rng.choice(n, size=min(n, 3), replace=False):
            res = oracle.bfs(g.off, g.col, int(r))
            assert np.array_equal(res.level, matrix_power_levels(adj, int(r)))
            check_result(g, int(r), res)


# ----------------------------------------------------------------------------
# independent library routine on R-MAT graphs


@pytest.mark.parametrize("scale", [10, 12, 14])
def test_rmat_vs_scipy(scale):
    g = graphgen.rmat(scale)
    A = sp.csr_matrix((np.ones(g.nnz, np.int8), g.col, g.off), shape=(g.V, g.V))
    roots = graphgen.pick_roots(g, 4, graphgen.root_seed(scale))
    dist = csgraph.shortest_path(A, unweighted=True, indices=roots)
    for i, r in enumerate(roots):
        res = oracle.bfs(g.off, g.col, int(r))
        exp = np.where(np.isinf(dist[i]), -1, dist[i]).astype(np.int64)
        assert np.array_equal(res.level, exp)
        check_result(g, int(r), res)


def test_components_vs_scipy():
    g = graphgen.rmat(12, edgefactor=2)
    A = sp.csr_matrix((np.ones(g.nnz, np.int8), g.col, g.off), shape=(g.V, g.V))
    ncomp, lab = csgraph.connected_components(A, directed=False)
    comp = oracle.components(g.off, g.col)
    # same partition: map scipy labels to our min-member labels
    assert len(np.unique(comp)) == ncomp
    for l in range(ncomp):
        members = np.nonzero(lab == l)[0]
        assert np.all(comp[members] == members.min())


# ----------------------------------------------------------------------------
# validator negative tests: every invariant must be able to fail


@pytest.fixture(scope="module")
def g12():
    g = graphgen.rmat(12)
    r = int(graphgen.pick_roots(g, 1, 99)[0])
    return g, r, oracle.bfs(g.off, g.col, r)


def _val(g, r, lv, pa, directed=False):
    return oracle.validate(g.off, g.col, r, lv, pa, directed=directed)[0]


def test_validator_accepts(g12):
    g, r, res = g12
    assert _val(g, r, res.level, res.parent) == 0


def test_validator_root(g12):
    g, r, res = g12
    lv, pa = res.level.copy(), res.parent.copy()
    pa[r] = -5 if r else 1
    assert _val(g, r, lv, pa) in (1,)
    lv, pa = res.level.copy(), res.parent.copy()
    lv[r] = 1
    assert _val(g, r, lv, pa) == 1


def test_validator_parent_not_neighbour(g12):
    g, r, res = g12
    lv, pa = res.level.copy(), res.parent.copy()
    # a vertex at level 2 gets a level-1 parent that is not its neighbour
    v = int(np.nonzero(lv == 2)[0][0])
    nbrs = set(g.col[g.off[v]:g.off[v + 1]].tolist())
    cand = [u for u in np.nonzero(lv == 1)[0] if int(u) not in nbrs]
    pa[v] = int(cand[0])
    assert _val(g, r, lv, pa) == 2


def test_validator_parent_wrong_level(g12):
    g, r, res = g12
    lv, pa = res.level.copy(), res.parent.copy()
    # choose v at level 2 with a neighbour at level 2 and use it as parent
    for v in np.nonzero(lv == 2)[0]:
        nb = g.col[g.off[v]:g.off[v + 1]]
        same = nb[lv[nb] == 2]
        if same.size:
            pa[v] = int(same[0])
            break
    assert _val(g, r, lv, pa) == 3


def test_validator_level_off_by_one(g12):
    g, r, res = g12
    lv, pa = res.level.copy(), res.parent.copy()
    leaves = np.nonzero(lv == lv.max())[0]
    lv[leaves[0]] += 1  # parent level now off by two
    assert _val(g, r, lv, pa) in (3, 4)
    lv2 = res.level.copy()
    lv2[lv2 > 0] += 0
    lv2[lv2 == lv2.max()] += 1  # every deepest vertex shifted; parents off
    assert _val(g, r, lv2, pa) in (3, 4)


def test_validator_missing_reach(g12):
    g, r, res = g12
    lv, pa = res.level.copy(), res.parent.copy()
    v = int(np.nonzero(lv == lv.max())[0][0])
    lv[v] = -1
    pa[v] = -1
    assert _val(g, r, lv, pa) == 4


def test_validator_reach_outside_component(g12):
    g, r, res = g12
    lv, pa = res.level.copy(), res.parent.copy()
    iso = np.nonzero(np.diff(g.off) == 0)[0]
    assert iso.size
    v = int(iso[0])
    # isolated vertex claimed reached with itself as parent: V2 catches it
    lv[v], pa[v] = 1, r
    assert _val(g, r, lv, pa) == 2


def test_validator_component_cross_check():
    # V2 + V3 tie every reached vertex to the root and V4 closes the reached
    # set under adjacency, so on a consistent result the reached set already
    # is the root's component and V5 cannot be the first check to fail.  V5
    # is a cross-check against labels from an independent algorithm: it
    # accepts union-find labels of the same graph and rejects labels that
    # disagree with the reached set.
    g = graphgen.from_edges(6, [0, 1, 3], [1, 2, 4])  # {0,1,2} {3,4} {5}
    comp = oracle.components(g.off, g.col)
    assert comp.tolist() == [0, 0, 0, 3, 3, 5]
    res = oracle.bfs(g.off, g.col, 1)
    assert oracle.validate(g.off, g.col, 1, res.level, res.parent, comp=comp)[0] == 0
    wrong = comp.copy()
    wrong[3] = 0  # labels claiming 3 shares the root's component
    assert oracle.validate(g.off, g.col, 1, res.level, res.parent, comp=wrong) == (5, 3)
    wrong = comp.copy()
    wrong[2] = 5  # labels claiming 2 is elsewhere
    assert oracle.validate(g.off, g.col, 1, res.level, res.parent, comp=wrong) == (5, 2)


def test_reached_set_is_the_component_rmat():
    g = graphgen.rmat(12, edgefactor=4)
    comp = oracle.components(g.off, g.col)
    for r in graphgen.pick_roots(g, 6, 17):
        res = oracle.bfs(g.off, g.col, int(r))
        assert np.array_equal(res.level >= 0, comp == comp[int(r)])
        assert oracle.validate(g.off, g.col, int(r), res.level, res.parent, comp=comp)[0] == 0


def test_validator_unreached_with_parent(g12):
    g, r, res = g12
    lv, pa = res.level.copy(), res.parent.copy()
    v = int(np.nonzero(lv == -1)[0][0])
    pa[v] = r
    assert _val(g, r, lv, pa) == 6


def test_validator_directed():
    # 0 -> 1 -> 2, 2 -> 0
    g = graphgen.from_edges(3, [0, 1, 2], [1, 2, 0], symmetric=False)
    res = oracle.bfs(g.off, g.col, 0)
    assert res.level.tolist() == [0, 1, 2]
    assert _val(g, 0, res.level, res.parent, directed=True) == 0
    assert _val(g, 0, np.array([0, 2, 1]), np.array([0, 2, 1]), directed=True) in (2, 3, 4)
    res = oracle.bfs(g.off, g.col, 1)
    assert res.level.tolist() == [2, 0, 1]


def test_oracle_rejects_bad_root():
    g = path_graph(4)
    with pytest.raises(ValueError):
        oracle.bfs(g.off, g.col, 4)
    with pytest.raises(ValueError):
        oracle.bfs(g.off, g.col, -1)


def test_batch_levels_int8():
    g = graphgen.rmat(10)
    roots = graphgen.pick_roots(g, 5, 3)
    b = oracle.batch_levels_int8(g.off, g.col, roots)
    assert b.dtype == np.int8 and b.shape == (5, g.V)
    for i, r in enumerate(roots):
        assert np.array_equal(b[i].astype(np.int32), oracle.bfs(g.off, g.col, int(r)).level)
    with pytest.raises(OverflowError):
        p = path_graph(200)
        oracle.batch_levels_int8(p.off, p.col, [0])
