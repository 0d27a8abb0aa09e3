"""The autotuner gates every candidate on the oracle's levels before timing
it: with the true levels every candidate passes and the choice reproduces
the oracle; with a planted mistake in the expected levels (on the CPU side)
every candidate fails and nothing is chosen."""
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


@pytest.fixture(scope="module")
def setup(bfsmi):
    g = graphgen.rmat(14)
    G = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER | bfsmi.BFS_WS_BATCH)
    roots = [int(r) for r in graphgen.pick_roots(g, 4, 3)]
    expected = [oracle.bfs(g.off, g.col, r).level for r in roots]
    yield g, G, roots, expected
    G.close()


def test_tune_single_direction_batch(bfsmi, setup, tmp_path, monkeypatch):
    from paper_1408_1605_amd import autotune
    monkeypatch.setattr(autotune, "CACHE_DIR", str(tmp_path))
    g, G, roots, expected = setup
    best, table = autotune.tune_single(G, roots, expected, reps=1)
    assert len(table) == 48 and all(t["parity"] for t in table)
    assert best is not None and best["ms"] > 0
    dbest, dtable = autotune.tune_direction(G, roots, expected, reps=1)
    assert len(dtable) == 15 and all(t["parity"] for t in dtable) and dbest is not None
    assert G.get_option(bfsmi.BFS_OPT_DIRECTION) == 0  # restored
    rows = oracle.batch_levels_int8(g.off, g.col, roots * 8)
    bbest, btable = autotune.tune_batch(G, roots * 8, rows, reps=1)
    assert all(t["parity"] for t in btable) and bbest is not None
    autotune.save("rmat", 14, {"single": best, "direction": dbest, "batch": bbest})
    assert autotune.load_cached("rmat", 14)["single"] == best
    autotune.apply(G, dict(best, batch_tile=bbest["batch_tile"]))
    for r, exp in zip(roots, expected):
        lv, pa, st = G.run(r)
        torch.cuda.synchronize()
        assert np.array_equal(lv.cpu().numpy(), exp)
    out, _ = G.run_batch(roots * 8)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), rows)


def test_tuner_rejects_wrong_expected_levels(bfsmi, setup):
    from paper_1408_1605_amd import autotune
    g, G, roots, expected = setup
    bad = [x.copy() for x in expected]
    v = int(np.nonzero(bad[1] > 0)[0][0])
    bad[1][v] += 1  # one vertex one level too deep
    best, table = autotune.tune_single(G, roots, bad, reps=1,
                                       space={"ept": (2, 4), "summary": (1,), "grid_wgs": (8,),
                                              "loop_limit": (65536,)})
    assert best is None and not any(t["parity"] for t in table)
    assert all(t["ms"] is None for t in table)
