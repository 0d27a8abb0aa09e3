"""Writes the stored values under tests/golden/.

graphgen_digests.json: SHA-256 of generated CSR arrays (pins the input
generator across builds).  oracle_rmat_s12.json: per-level frontier sizes of
the oracle on R-MAT scale 12 for its seeded roots (calls only ``oracle``).

Run from the repository root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402


def digest(g):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g.off).tobytes())
    h.update(np.ascontiguousarray(g.col).tobytes())
    return h.hexdigest()


def main():
    gold = {"rmat": {str(s): digest(graphgen.rmat(s)) for s in (8, 12)},
            "grid33x17": digest(graphgen.grid(33, 17))}
    with open(os.path.join(HERE, "graphgen_digests.json"), "w") as f:
        json.dump(gold, f, indent=1, sort_keys=True)
        f.write("\n")
    g = graphgen.rmat(12)
    roots = graphgen.pick_roots(g, 8, graphgen.root_seed(12))
    out = {"graph": "rmat scale 12 edgefactor 16 seed 1012",
           "roots": [int(r) for r in roots],
           "frontier_sizes": [], "edges_scanned": []}
    for r in roots:
        res = oracle.bfs(g.off, g.col, int(r))
        out["frontier_sizes"].append([int(x) for x in res.frontier_sizes])
        out["edges_scanned"].append(int(res.edges_scanned))
    with open(os.path.join(HERE, "oracle_rmat_s12.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
