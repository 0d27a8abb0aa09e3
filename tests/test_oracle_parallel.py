"""The oracle's many-roots runner (oracle/parallel.py): same results as the
serial calls, a cache keyed by (CSR digest, root) that returns what it
stored, and a checker that reports level mismatches and invalid parents."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import parallel


@pytest.fixture(scope="module")
def g12():
    g = graphgen.rmat(12)
    return g, [int(r) for r in graphgen.pick_roots(g, 8, 77)]


def test_pool_equals_serial(g12, tmp_path, monkeypatch):
    monkeypatch.setenv("BFSMI_ORACLE_CACHE", str(tmp_path))
    g, roots = g12
    res, wall, n = parallel.bfs_roots(g.off, g.col, roots, workers=4, cache=False)
    assert n == 4 and wall > 0
    for r, x in zip(roots, res):
        ref = oracle.bfs(g.off, g.col, r)
        assert x.root == r and not x.cached
        assert np.array_equal(x.level, ref.level)
        assert np.array_equal(x.frontier_sizes, ref.frontier_sizes)
        assert x.edges_scanned == ref.edges_scanned


def test_cache_round_trip(g12, tmp_path, monkeypatch):
    monkeypatch.setenv("BFSMI_ORACLE_CACHE", str(tmp_path))
    g, roots = g12
    first, _, _ = parallel.bfs_roots(g.off, g.col, roots[:3], workers=3)
    second, _, _ = parallel.bfs_roots(g.off, g.col, roots[:3], workers=3)
    assert not any(x.cached for x in first) and all(x.cached for x in second)
    for a, b in zip(first, second):
        assert np.array_equal(a.level, b.level) and a.level.dtype == b.level.dtype == np.int32
        assert np.array_equal(a.frontier_sizes, b.frontier_sizes)
        assert a.edges_scanned == b.edges_scanned


def test_digest_tracks_content(g12):
    g, _ = g12
    d0 = parallel.csr_digest(g.off, g.col)
    assert d0 == parallel.csr_digest(g.off.copy(), g.col.copy())
    col = g.col.copy()
    col[12345] = (col[12345] + 1) % g.V
    assert parallel.csr_digest(g.off, col) != d0
    off = g.off.copy()
    assert parallel.csr_digest(off[:-1], g.col[:off[-2]]) != d0


def test_check_roots_reports(g12, tmp_path, monkeypatch):
    monkeypatch.setenv("BFSMI_ORACLE_CACHE", str(tmp_path))
    g, roots = g12
    items = []
    for r in roots[:4]:
        ref = oracle.bfs(g.off, g.col, r)
        items.append((r, ref.level.copy(), ref.parent.copy()))
    # root 1: one level off; root 2: a parent that is not a neighbour
    lv = items[1][1]
    v = int(np.nonzero(lv == lv.max())[0][0])
    lv[v] += 1
    r2, lv2, pa2 = items[2]
    v2 = int(np.nonzero(lv2 == 2)[0][0])
    nb = set(g.col[g.off[v2]:g.off[v2 + 1]].tolist())
    pa2[v2] = int([u for u in np.nonzero(lv2 == 1)[0] if int(u) not in nb][0])
    out = parallel.check_roots(g.off, g.col, items, workers=4)
    assert [c.root for c in out] == roots[:4]
    assert out[0].ok and out[3].ok
    assert not out[1].levels_equal and v in out[1].first_diff
    assert out[2].levels_equal and out[2].validate_code == 2 and out[2].bad_vertex == v2
    comp = oracle.components(g.off, g.col)
    assert all(c.ok for c in parallel.check_roots(g.off, g.col, [items[0], items[3]], comp=comp))
