"""The allocation-free entry point bfs_run_noalloc against bfs_run (the
entry point it is a variant of) and against the oracle, called through the
C ABI: two calls in a row, the second on a smaller graph, so the second
search runs over the first one's leftovers in the static scratch array.

Levels must equal bfs_run's and the oracle's element by element; parents
(which depend on which atomic wins) must pass the tree validator; the
search counts must equal bfs_run's."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_1605_amd import binding
    binding.load()
    return binding


def _noalloc(lib, g, d_off, d_col, root):
    lv = torch.full((g.V,), -7, dtype=torch.int32, device="cuda")
    pa = torch.full((g.V,), -7, dtype=torch.int32, device="cuda")
    so = lib.load()
    st = so.bfs_run_noalloc.argtypes[-1]._type_()  # the struct type the binding declared
    code = so.bfs_run_noalloc(g.V, g.nnz, d_off.data_ptr(), d_col.data_ptr(), int(root),
                              lv.data_ptr(), pa.data_ptr(),
                              torch.cuda.current_stream().cuda_stream, ctypes.byref(st))
    assert code == lib.BFS_OK, (code, lib.bfs_last_error())
    torch.cuda.synchronize()
    return lv.cpu().numpy(), pa.cpu().numpy(), st


def _check_pair(lib, g, roots):
    d_off = torch.from_numpy(np.ascontiguousarray(g.off, np.int64)).cuda()
    d_col = torch.from_numpy(np.ascontiguousarray(g.col, np.int32)).cuda()
    G = lib.Graph.from_csr(g.off, g.col)
    try:
        for r in roots:
            lv, pa, st = _noalloc(lib, g, d_off, d_col, r)
            elv, epa, est = G.run(int(r))
            torch.cuda.synchronize()
            elv = elv.cpu().numpy()
            assert np.array_equal(lv, elv), (g.name, r)
            ref = oracle.bfs(g.off, g.col, int(r))
            assert np.array_equal(lv, ref.level), (g.name, r)
            code, bad = oracle.validate(g.off, g.col, int(r), lv, pa)
            assert code == 0, (g.name, r, oracle.INVARIANTS[code], bad)
            assert (st.levels, st.reached, st.edges_scanned) == \
                (est.levels, est.reached, est.edges_scanned), (g.name, r)
    finally:
        G.close()


def test_noalloc_matches_bfs_run_two_calls_shrinking(lib):
    big = graphgen.rmat(16)      # several tiles, bitmap levels, persistent loop
    small = graphgen.rmat(11)    # second call: smaller input on a used array
    _check_pair(lib, big, graphgen.pick_roots(big, 2, graphgen.root_seed(16)))
    _check_pair(lib, small, graphgen.pick_roots(small, 2, graphgen.root_seed(11)))


def test_noalloc_deep_grid_then_tiny_path(lib):
    g = graphgen.grid(300)       # ~600 levels in the persistent loop
    _check_pair(lib, g, [0])
    p = graphgen.from_edges(5, np.arange(4), np.arange(1, 5))  # a 5-vertex path
    p.name = "path5"
    _check_pair(lib, p, [2])


def test_noalloc_rejects_oversize_before_device_work(lib):
    so = lib.load()
    dummy = torch.zeros(8, dtype=torch.int64, device="cuda")
    code = so.bfs_run_noalloc(1 << 22, 1 << 26, dummy.data_ptr(), dummy.data_ptr(), 0,
                              dummy.data_ptr(), None, None, None)
    assert code == lib.BFS_ERR_WORKSPACE
    assert "static array" in lib.bfs_last_error()
