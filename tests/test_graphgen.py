"""The seeded input generators: determinism, structure, and the R-MAT
quadrant probabilities the workload is defined by."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def csr_digest(g):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g.off).tobytes())
    h.update(np.ascontiguousarray(g.col).tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("scale", [8, 11, 14])
def test_rmat_structure(scale):
    g = graphgen.rmat(scale)
    assert g.V == 1 << scale
    assert g.off[0] == 0 and np.all(np.diff(g.off) >= 0)
    assert g.col.min() >= 0 and g.col.max() < g.V
    rows = np.repeat(np.arange(g.V), np.diff(g.off))
    # no self-loops
    assert not np.any(rows == g.col)
    # rows strictly ascending (sorted, no duplicates)
    same_row = rows[1:] == rows[:-1]
    assert np.all(g.col[1:][same_row] > g.col[:-1][same_row])
    # symmetric: the set of (r, c) equals the set of (c, r)
    a = rows.astype(np.int64) * g.V + g.col
    b = g.col.astype(np.int64) * g.V + rows
    assert np.array_equal(np.sort(a), np.sort(b))
    # merged undirected edges never exceed the generated count
    assert g.nnz <= 2 * 16 * g.V


def test_rmat_deterministic_and_seeded():
    a, b = graphgen.rmat(12), graphgen.rmat(12)
    assert csr_digest(a) == csr_digest(b)
    c = graphgen.rmat(12, seed=5)
    assert csr_digest(a) != csr_digest(c)


def test_rmat_golden_digest():
    """Pins the generator across builds and machines (digest written by
    tests/golden/make_golden.py)."""
    with open(os.path.join(GOLDEN, "graphgen_digests.json")) as f:
        gold = json.load(f)
    for key, digest in gold["rmat"].items():
        scale = int(key)
        assert csr_digest(graphgen.rmat(scale)) == digest, key
    assert csr_digest(graphgen.grid(33, 17)) == gold["grid33x17"]


def test_rmat_thread_count_independent():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r); import graphgen, hashlib; "
            "g = graphgen.rmat(13); h = hashlib.sha256(); h.update(g.off.tobytes()); "
            "h.update(g.col.tobytes()); print(h.hexdigest())") % root
    outs = []
    for nt in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env).strip())
    assert outs[0] == outs[1] == outs[2]


def test_rmat_quadrant_frequencies():
    """Without relabelling, bit l of (src, dst) is the quadrant chosen at
    level l: (0,0) w.p. A, (0,1) B, (1,0) C, (1,1) D."""
    A, B, C = 0.57, 0.19, 0.19
    n = 200_000
    scale = 10
    src, dst = graphgen.rmat_edges(scale, n, A, B, C, seed=3, relabel=False)
    for l in (0, 4, 9):
        bi = (src >> (scale - 1 - l)) & 1
        bj = (dst >> (scale - 1 - l)) & 1
        q = np.bincount(bi * 2 + bj, minlength=4) / n
        for got, p in zip(q, (A, B, C, 1 - A - B - C)):
            sigma = np.sqrt(p * (1 - p) / n)
            assert abs(got - p) < 5 * sigma, (l, q)


def test_rmat_relabel_is_permutation_of_plain():
    s0, d0 = graphgen.rmat_edges(9, 5000, seed=4, relabel=False)
    s1, d1 = graphgen.rmat_edges(9, 5000, seed=4, relabel=True)
    # the same permutation maps plain ids to relabelled ids
    mapping = {}
    for a, b in zip(np.concatenate([s0, d0]), np.concatenate([s1, d1])):
        assert mapping.setdefault(int(a), int(b)) == int(b)
    assert len(set(mapping.values())) == len(mapping)


@pytest.mark.parametrize("scale", [1, 2, 5, 8, 11])
def test_permutation_is_bijection(scale):
    key = 12345
    img = [graphgen.permute(v, scale, key) for v in range(1 << scale)]
    assert sorted(img) == list(range(1 << scale))


@pytest.mark.parametrize("w,h", [(1, 1), (2, 1), (5, 3), (64, 64)])
def test_grid_structure(w, h):
    g = graphgen.grid(w, h)
    V = w * h
    assert g.nnz == 2 * (2 * V - w - h)
    deg = np.diff(g.off)
    r, c = np.divmod(np.arange(V), w)
    exp = (r > 0).astype(int) + (c > 0) + (c < w - 1) + (r < h - 1)
    assert np.array_equal(deg, exp)
    rows = np.repeat(np.arange(V), deg)
    d = np.abs(rows - g.col)
    assert np.all((d == 1) | (d == w))


def test_grid_4096_size():
    g = graphgen.grid(512)
    assert g.nnz == 2 * (2 * 512 * 512 - 1024)


def test_pick_roots():
    g = graphgen.rmat(12)
    r = graphgen.pick_roots(g, 64, 77)
    assert len(r) == 64 and len(set(r.tolist())) == 64
    assert np.all(np.diff(g.off)[r] > 0)
    assert np.array_equal(r, graphgen.pick_roots(g, 64, 77))
    assert not np.array_equal(r, graphgen.pick_roots(g, 64, 78))
    # fewer vertices with degree > 0 than asked for
    g2 = graphgen.from_edges(5, [0], [1])
    assert sorted(graphgen.pick_roots(g2, 4, 1).tolist()) == [0, 1]


def test_from_edges_and_dense():
    g = graphgen.from_edges(4, [0, 2], [1, 3])
    assert g.off.tolist() == [0, 1, 2, 3, 4]
    assert g.col.tolist() == [1, 0, 3, 2]
    adj = np.array([[0, 1, 1], [0, 0, 1], [0, 0, 0]], bool)
    d = graphgen.from_dense(adj)
    assert d.off.tolist() == [0, 2, 3, 3] and d.col.tolist() == [1, 2, 2]
