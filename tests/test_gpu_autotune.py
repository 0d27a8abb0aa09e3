"""The autotuner gates every configuration on parity before timing it, and
its choice reproduces the oracle."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bfsmi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_1605_amd as p
    p.load()
    return p


def test_tune_single_and_batch(bfsmi, tmp_path, monkeypatch):
    from paper_1408_1605_amd import autotune
    monkeypatch.setattr(autotune, "CACHE_DIR", str(tmp_path))
    g = graphgen.rmat(14)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER | bfsmi.BFS_WS_BATCH)
    roots = [int(r) for r in graphgen.pick_roots(g, 4, 3)]
    best, table = autotune.tune_single(G, roots, reps=1)
    assert len(table) == 24 and all(t["parity"] for t in table)
    assert best is not None and best["ms"] > 0
    bbest, btable = autotune.tune_batch(G, roots * 8, reps=1)
    assert all(t["parity"] for t in btable) and bbest is not None
    path = autotune.save("rmat", 14, {"single": best, "batch": bbest})
    assert autotune.load_cached("rmat", 14)["single"] == best
    autotune.apply(G, dict(best, batch_tile=bbest["batch_tile"]))
    for r in roots:
        lv, pa, st = G.run(r)
        torch.cuda.synchronize()
        assert np.array_equal(lv.cpu().numpy(), oracle.bfs(g.off, g.col, r).level)
    del path
