"""Plants plausible mistakes in a copy of the CPU oracle (on the CPU) and
checks that the pins catch each one: a dropped edge, an off-by-one level, a
wrong index, a missing visited test, a wrong parent, a stack instead of a
queue, a wrong per-level count, a weakened validator.
"""
import multiprocessing
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.sparse import csgraph
import scipy.sparse as sp

import graphgen
import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "bfs_oracle.c")

BFS_MUTANTS = {
    "distance_not_incremented": ("level[y] = dx + 1;", "level[y] = dx;"),
    "distance_fixed_at_one": ("level[y] = dx + 1;", "level[y] = 1;"),
    "drops_last_edge": ("for (int64_t e = a; e < b; ++e) {", "for (int64_t e = a; e < b - 1; ++e) {"),
    "wrong_neighbour_index": ("const int32_t y = col[e];", "const int32_t y = col[e > a ? e - 1 : e];"),
    "no_visited_test": ("if (level[y] < 0) {", "if (level[y] <= 0) {"),
    "parent_is_self": ("parent[y] = x;", "parent[y] = y;"),
    "root_not_marked": ("    level[root] = 0;\n", "\n"),
    "root_parent_unset": ("    parent[root] = root;\n", "\n"),
    "lifo_not_fifo": ("const int32_t x = fifo[head++];", "const int32_t x = fifo[--tail];"),
    "wrong_level_count": ("frontier_sizes[level[fifo[i]]]++;", "frontier_sizes[level[fifo[i]] / 2]++;"),
}

VALIDATOR_MUTANTS = {
    "no_span_check": ("if (lu >= 0 && (lu - lv > 1 || lv - lu > 1)) {", "if (0) {"),
    "no_parent_level": ("if (level[u] != level[v] - 1) {", "if (level[u] > level[v]) {"),
    "no_neighbour_check": ("        if (!ok) {\n            *bad_vertex = v;\n            return 2;",
                           "        if (0) {\n            *bad_vertex = v;\n            return 2;"),
    "no_unreached_check": ("if (level[v] < -1 || ((level[v] == -1) != (parent[v] == -1))) {",
                           "if (level[v] < -1) {"),
}


def build_mutant(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, name
    path = tmp_path / (name + ".c")
    path.write_text(text.replace(old, new))
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=gnu11", "-o", str(so),
                           str(path)])
    return str(so)


_GRAPHS = []


def _graphs():
    """Test graphs, built in the parent before any fork (the generator uses
    OpenMP, which must not be first entered in a forked child)."""
    if not _GRAPHS:
        child = np.arange(1, 15)
        _GRAPHS.extend([
            graphgen.from_edges(6, np.arange(5), np.arange(1, 6)),    # path
            graphgen.grid(5, 4),
            graphgen.from_edges(15, (child - 1) // 2, child),         # tree
            graphgen.rmat(10),
        ])
    return _GRAPHS


def pins_pass(lib):
    """The oracle pin battery (closed forms, brute force, scipy), run
    against the given library. Returns False at the first failure."""
    saved = oracle._lib
    oracle._lib = lib
    try:
        for g in _graphs():
            A = sp.csr_matrix((np.ones(g.nnz, np.int8), g.col, g.off), shape=(g.V, g.V))
            roots = [0, g.V - 1, g.V // 2]
            dist = csgraph.shortest_path(A, unweighted=True, indices=roots)
            for i, r in enumerate(roots):
                res = oracle.bfs(g.off, g.col, r)
                exp = np.where(np.isinf(dist[i]), -1, dist[i])
                if not np.array_equal(res.level, exp):
                    return False
                code, _ = oracle.validate(g.off, g.col, r, res.level, res.parent)
                if code != 0:
                    return False
                if not np.array_equal(res.frontier_sizes, oracle.levels_hist(res.level)):
                    return False
        return True
    finally:
        oracle._lib = saved


def validator_negatives_all_fail(lib):
    """True when the library's validator rejects every corrupted result."""
    saved = oracle._lib
    oracle._lib = lib
    try:
        g = _graphs()[-1]
        r = int(graphgen.pick_roots(g, 1, 5)[0])
        res = oracle.bfs(g.off, g.col, r)
        cases = []
        lv, pa = res.level.copy(), res.parent.copy()
        v = int(np.nonzero(lv == lv.max())[0][0])
        lv[v] += 1
        cases.append((lv, pa))
        lv, pa = res.level.copy(), res.parent.copy()
        # a parent one level up that is not a neighbour
        for v2 in np.nonzero(lv >= 2)[0]:
            nb = set(g.col[g.off[v2]:g.off[v2 + 1]].tolist())
            cand = [u for u in np.nonzero(lv == lv[v2] - 1)[0] if int(u) not in nb]
            if cand:
                pa[int(v2)] = int(cand[0])
                break
        else:
            raise AssertionError("no candidate")
        cases.append((lv, pa))
        lv, pa = res.level.copy(), res.parent.copy()
        # a same-level neighbour as parent
        for v3 in np.nonzero(lv >= 1)[0]:
            nb = g.col[g.off[v3]:g.off[v3 + 1]]
            same = nb[lv[nb] == lv[v3]]
            if same.size:
                pa[int(v3)] = int(same[0])
                break
        else:
            raise AssertionError("no same-level neighbour")
        cases.append((lv, pa))
        lv, pa = res.level.copy(), res.parent.copy()
        # a consistent but too deep tree: a childless v hangs below a
        # same-level neighbour (V2, V3 hold; only the edge span catches it)
        is_parent = np.zeros(g.V, bool)
        is_parent[pa[pa >= 0]] = True
        for v4 in np.nonzero((lv >= 1) & ~is_parent)[0]:
            nb = g.col[g.off[v4]:g.off[v4 + 1]]
            same = nb[lv[nb] == lv[v4]]
            if same.size:
                pa[int(v4)] = int(same[0])
                lv[int(v4)] += 1
                break
        else:
            raise AssertionError("no childless vertex with a same-level neighbour")
        cases.append((lv, pa))
        lv, pa = res.level.copy(), res.parent.copy()
        pa[int(np.nonzero(lv == -1)[0][0])] = r
        cases.append((lv, pa))
        lv, pa = res.level.copy(), res.parent.copy()
        # every vertex at the deepest level moved one deeper (parents off by 2,
        # edges to same-level neighbours now span... within 1)
        deep = lv == lv.max()
        lv[deep] = lv.max() + 5
        cases.append((lv, pa))
        return all(oracle.validate(g.off, g.col, r, a, b)[0] != 0 for a, b in cases)
    finally:
        oracle._lib = saved


def _in_child(fn, so_path):
    """Run fn(lib) in a forked child so a mutant that corrupts memory cannot
    take the test process down. Returns True/False, or None if it crashed."""
    def target(q):
        import faulthandler
        faulthandler.disable()  # a crashing mutant is an expected outcome
        q.put(bool(fn(oracle._bind(so_path))))
    _graphs()
    ctx = multiprocessing.get_context("fork")
    q = ctx.Queue()
    p = ctx.Process(target=target, args=(q,))
    p.start()
    p.join(120)
    if p.is_alive():
        p.kill()
        p.join()
        return None
    return q.get() if p.exitcode == 0 else None


def test_unmutated_passes(tmp_path):
    shutil.copy(SRC, tmp_path / "orig.c")
    build_mutant(tmp_path, "orig", "level[y] = dx + 1;", "level[y] = dx + 1;")
    so = str(tmp_path / "orig.so")
    assert _in_child(pins_pass, so) is True
    assert _in_child(validator_negatives_all_fail, so) is True


@pytest.mark.parametrize("name", sorted(BFS_MUTANTS))
def test_bfs_mutant_caught(tmp_path, name):
    old, new = BFS_MUTANTS[name]
    build_mutant(tmp_path, name, old, new)
    # False (a pin failed) or None (the mutant crashed) both count as caught
    assert _in_child(pins_pass, str(tmp_path / (name + ".so"))) is not True, name


@pytest.mark.parametrize("name", sorted(VALIDATOR_MUTANTS))
def test_validator_mutant_caught(tmp_path, name):
    old, new = VALIDATOR_MUTANTS[name]
    build_mutant(tmp_path, name, old, new)
    assert _in_child(validator_negatives_all_fail, str(tmp_path / (name + ".so"))) is not True
