"""CPU model of the serving loop's level scheme (host logic only, no GPU).

The persistent serving kernel finalizes one level's candidates and expands
the vertices that got new lanes in the same phase.  The next masks and the
candidate lists come in two parities, and the expansion's filter may read
seen masks (and the other parity's marks) that other workgroups are changing
in the same phase.  This model runs the same scheme with the filter reading
seen masks as they were at the start of the phase and the finalized parity's
marks already cleared (the worst a reader can see: spurious candidates then
reach the next phase, whose finalize must drop them),
ends rounds with a finalize-only phase that leaves the frontier and its lane
masks as the level kernels take them, joins new lanes between rounds, and
checks every lane's depths against the oracle's search from its root.
"""
import numpy as np
import pytest

import graphgen
import oracle


class Model:
    def __init__(self, g):
        self.g = g
        V = g.V
        self.seen = np.zeros(V, dtype=np.uint64)
        self.marks = [np.zeros(V, dtype=np.uint64), np.zeros(V, dtype=np.uint64)]
        self.front = self.marks[1]  # parity 1 doubles as the frontier masks
        self.queue = []             # frontier between rounds
        self.level = 1
        self.start = {}             # lane -> level at which it joined, minus one
        self.depth = {}             # lane -> int array of depths (-1: unreached)

    def join(self, lane, root):
        bit = np.uint64(1) << np.uint64(lane)
        self.start[lane] = self.level - 1
        self.depth[lane] = np.full(self.g.V, -1, dtype=np.int64)
        self.depth[lane][root] = 0
        self.seen[root] |= bit
        if self.front[root] == 0:
            self.queue.append(root)
        self.front[root] |= bit

    def _expand(self, items, tp, snap_seen, snap_other, out):
        """items: (vertex, lane mask) pairs; ORs new lanes into marks[tp],
        listing each target the first time its marks become non-zero."""
        off, col = self.g.off, self.g.col
        target = self.marks[tp]
        for u, f in items:
            for e in range(off[u], off[u + 1]):
                x = int(col[e])
                have = snap_seen[x] | target[x] | snap_other[x]
                nb = f & ~have
                if nb:
                    old = target[x]
                    target[x] = old | nb
                    if old == 0:
                        out.append(x)

    def round(self, max_levels):
        """One persistent launch: phase 0 expands the queue (masks in front,
        which it clears) into parity 0; phase j finalizes parity (j-1)&1 and,
        unless it is the last, expands the new frontier into parity j&1."""
        items = [(u, self.front[u]) for u in self.queue]
        for u in self.queue:
            self.front[u] = 0
        snap_seen, snap_other = self.seen.copy(), self.marks[1].copy()
        lists = [[], []]
        self._expand(items, 0, snap_seen, snap_other, lists[0])
        steps = 0
        for j in range(1, max_levels + 1):
            sp = (j - 1) & 1
            last = j == max_levels
            dl = self.level + j - 1
            snap_seen = self.seen.copy()
            cand, lists[sp] = lists[sp], []
            new = []
            for v in cand:
                nw = self.marks[sp][v] & ~self.seen[v]
                self.seen[v] |= nw
                self.marks[sp][v] = 0
                if last:
                    self.front[v] = nw
                if nw:
                    new.append((v, nw))
                    b = int(nw)
                    while b:
                        k = (b & -b).bit_length() - 1
                        self.depth[k][v] = dl - self.start[k]
                        b &= b - 1
            steps = j
            if last or not new:
                self.queue = [v for v, _ in new]
                break
            # the worst a reader can see: the finalized marks already cleared,
            # the seen masks they went to not yet updated
            self._expand(new, j & 1, snap_seen, self.marks[sp], lists[j & 1])
        self.level += steps
        assert not self.marks[0].any()  # every candidate's marks were cleared
        return len(self.queue)


def _tri_grid(side):
    i = np.arange(side * side, dtype=np.int64).reshape(side, side)
    src = np.concatenate([i[:, :-1].ravel(), i[:-1, :].ravel(), i[:-1, :-1].ravel()])
    dst = np.concatenate([i[:, 1:].ravel(), i[1:, :].ravel(), i[1:, 1:].ravel()])
    return graphgen.from_edges(side * side, src, dst)


def _random_graph(V, E, seed):
    rng = np.random.default_rng(seed)
    return graphgen.from_edges(V, rng.integers(0, V, E), rng.integers(0, V, E))


@pytest.mark.parametrize("name,g", [("grid", graphgen.grid(12, 9)),
                                    ("triangles", _tri_grid(11)),
                                    ("rmat9", graphgen.rmat(9)),
                                    ("random", _random_graph(300, 700, 3))])
@pytest.mark.parametrize("round_levels", [1, 2, 5])
def test_fused_levels_match_oracle(name, g, round_levels):
    rng = np.random.default_rng(len(name) * 10 + round_levels)
    m = Model(g)
    roots = {}
    lane = 0
    for r in range(40):
        # a few lanes join at every round boundary (continuous batching)
        for _ in range(int(rng.integers(0, 3))):
            if lane < 64:
                root = int(rng.integers(0, g.V))
                m.join(lane, root)
                roots[lane] = root
                lane += 1
        if m.queue:
            m.round(round_levels)
    # then the rounds run until every lane has ended
    for _ in range(g.V + 1):
        if not m.queue:
            break
        m.round(round_levels)
    assert not m.queue and roots
    for k, root in roots.items():
        assert np.array_equal(m.depth[k], oracle.bfs(g.off, g.col, root).level), (name, k, root)
