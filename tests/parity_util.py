"""Helpers for the GPU parity tests: run roots through the C ABI, then check
every result against the CPU oracle on a pool of host threads (levels
element by element, parents with the tree validator, and the search's own
counts against the oracle's)."""
import sys

import numpy as np

from oracle import parallel


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_results(torch, G, roots, want_parents=True):
    """(root, levels, parents or None, stats) for each root, on the host."""
    out = []
    for r in roots:
        lv, pa, st = G.run(int(r), want_parents=want_parents)
        torch.cuda.synchronize()
        out.append((int(r), lv.cpu().numpy(), pa.cpu().numpy() if want_parents else None, st))
    return out


def assert_parity(g, items, digest=None, comp=None, directed=False, check_stats=True,
                  label=""):
    """Every item's levels equal the oracle's; parents (when given) pass the
    validator; the search's level, reached and edge counts equal the
    oracle's."""
    checks = parallel.check_roots(g.off, g.col, [(r, lv, pa) for r, lv, pa, _ in items],
                                  comp=comp, directed=directed, digest=digest)
    bad = [(c.root, c.first_diff, c.validate_code, c.bad_vertex) for c in checks if not c.ok]
    say("%s: %d roots checked, %d failed" % (label or g.name, len(checks), len(bad)))
    assert not bad, bad[:4]
    if check_stats:
        for (r, _, _, st), c in zip(items, checks):
            assert (st.levels, st.reached, st.edges_scanned) == (c.nlevels, c.reached,
                                                                  c.edges_scanned), r
    return checks


def manhattan(w, h, root):
    r_, c_ = np.divmod(np.arange(w * h, dtype=np.int64), w)
    r0, c0 = divmod(int(root), w)
    return np.abs(r_ - r0) + np.abs(c_ - c0)
