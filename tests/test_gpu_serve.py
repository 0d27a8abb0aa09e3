"""Serving (bfs_server_*): every ticket's levels must equal the single-root
oracle for that query alone (tolerance 0), whatever else was in flight.
"""
import sys
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bfsmi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_1605_amd as p
    p.load()
    return p


def wait_all(p, s, tickets, V_of, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            buf = np.empty(V_of[t], dtype=np.int32)
            code, tm = p.bfs_poll(s, t, buf)
            if code == p.BFS_OK:
                out[t] = (buf, tm)
        assert time.time() - t0 < timeout, "queries did not finish"
        time.sleep(0.001)
    return out


@pytest.fixture(scope="module")
def pool(bfsmi):
    graphs = [graphgen.rmat(12), graphgen.rmat(14, seed=77), graphgen.grid(40, 30),
              graphgen.rmat(13, seed=5)]
    handles = [bfsmi.Graph.from_csr(graphs[0].off, graphs[0].col),
               bfsmi.Graph.from_csr(graphs[1].off, graphs[1].col, flags=bfsmi.BFS_DEGREE_ORDER),
               bfsmi.Graph.from_csr(graphs[2].off, graphs[2].col),
               bfsmi.Graph.from_csr(graphs[3].off, graphs[3].col)]
    return graphs, handles


def make_server(p, handles, arena_mb=512, lanes=64, inflight=8, arena_bytes=None):
    nbytes = arena_bytes if arena_bytes is not None else arena_mb << 20
    arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = p.bfs_server_create(arena, max_lanes=lanes, max_inflight=inflight)
    ids = [p.bfs_server_add_graph(s, h.handle) for h in handles]
    return s, ids, arena


def test_serve_mix_matches_oracle(bfsmi, pool):
    graphs, handles = pool
    s, ids, arena = make_server(bfsmi, handles)
    rng = np.random.default_rng(1)
    tickets, meta = [], {}
    for i in range(300):
        gi = int(rng.integers(0, len(graphs)))
        g = graphs[gi]
        r = int(rng.integers(0, g.V))
        t = bfsmi.bfs_submit(s, ids[gi], r)
        tickets.append(t)
        meta[t] = (gi, r)
        if i % 50 == 0:
            time.sleep(0.002)  # let some run before others arrive
    _say("submitted", len(tickets))
    res = wait_all(bfsmi, s, tickets, {t: graphs[meta[t][0]].V for t in tickets})
    for t in tickets:
        gi, r = meta[t]
        exp = oracle.bfs(graphs[gi].off, graphs[gi].col, r).level
        got, tm = res[t]
        assert np.array_equal(got, exp), (gi, r)
        assert tm.levels == int(exp.max()) + 1
        assert tm.done_ns >= tm.admit_ns >= tm.submit_ns > 0
    bfsmi.bfs_server_drain(s)
    bfsmi.bfs_server_destroy(s)
    del arena


def test_serve_alone_equals_mix(bfsmi, pool):
    graphs, handles = pool
    g, h = graphs[1], handles[1]
    root = int(graphgen.pick_roots(g, 1, 3)[0])
    s, ids, arena = make_server(bfsmi, [h])
    t_alone = bfsmi.bfs_submit(s, ids[0], root)
    alone = wait_all(bfsmi, s, [t_alone], {t_alone: g.V})[t_alone][0]
    others = [bfsmi.bfs_submit(s, ids[0], int(x)) for x in graphgen.pick_roots(g, 63, 11)]
    t_mix = bfsmi.bfs_submit(s, ids[0], root)
    res = wait_all(bfsmi, s, others + [t_mix], {t: g.V for t in others + [t_mix]})
    assert np.array_equal(res[t_mix][0], alone)
    bfsmi.bfs_server_destroy(s)
    del arena


def test_serve_budget_queues(bfsmi, pool):
    graphs, handles = pool
    g, h = graphs[0], handles[0]
    # room for one batch state and three result buffers at a time, so most
    # queries wait in the queue for memory
    def al(x):
        return (x + 255) // 256 * 256
    V = g.V
    state = (4 * al(8 * V) + al((V + 31) // 32 * 4) + 4 * al(4 * V) + al(8 * (V + 1)) + al(8 * ((V + 2047) // 2048 + 1))
             + al(4 * ((g.nnz + 255) // 256 + 2)) + al(128) + al(512) + al(256) + al(512))
    s, ids, arena = make_server(bfsmi, [h], arena_bytes=state + 3 * al(2 * V) + 256)
    roots = graphgen.pick_roots(g, 40, 5)
    ts = [bfsmi.bfs_submit(s, ids[0], int(r)) for r in roots]
    res = wait_all(bfsmi, s, ts, {t: g.V for t in ts})
    for t, r in zip(ts, roots):
        assert np.array_equal(res[t][0], oracle.bfs(g.off, g.col, int(r)).level)
    bfsmi.bfs_server_destroy(s)
    del arena


def test_serve_never_fits(bfsmi, pool):
    graphs, handles = pool
    # the scale-14 graph needs ~1 MB of batch state; give it 256 KB
    arena = torch.empty(256 << 10, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = bfsmi.bfs_server_create(arena)
    with pytest.raises(bfsmi.BFSError) as e:
        bfsmi.bfs_server_add_graph(s, handles[1].handle)
    assert e.value.code == bfsmi.BFS_ERR_BUDGET
    bfsmi.bfs_server_destroy(s)


def test_serve_bad_tickets_and_roots(bfsmi, pool):
    graphs, handles = pool
    s, ids, arena = make_server(bfsmi, handles[:1], arena_mb=64)
    with pytest.raises(bfsmi.BFSError) as e:
        bfsmi.bfs_poll(s, 12345)
    assert e.value.code == bfsmi.BFS_ERR_TICKET
    with pytest.raises(bfsmi.BFSError):
        bfsmi.bfs_submit(s, ids[0], graphs[0].V)
    with pytest.raises(bfsmi.BFSError):
        bfsmi.bfs_submit(s, 99, 0)
    t = bfsmi.bfs_submit(s, ids[0], 0)
    wait_all(bfsmi, s, [t], {t: graphs[0].V})
    with pytest.raises(bfsmi.BFSError) as e:  # retired
        bfsmi.bfs_poll(s, t)
    assert e.value.code == bfsmi.BFS_ERR_TICKET
    bfsmi.bfs_server_destroy(s)


def test_serve_deep_grid(bfsmi):
    # a 300-long path needs more levels than a lane round of 1 or 4
    g = graphgen.grid(300, 2)
    h = bfsmi.Graph.from_csr(g.off, g.col)
    s, ids, arena = make_server(bfsmi, [h], arena_mb=64)
    ts = [bfsmi.bfs_submit(s, ids[0], r) for r in (0, 299, 150, 599)]
    res = wait_all(bfsmi, s, ts, {t: g.V for t in ts})
    for t, r in zip(ts, (0, 299, 150, 599)):
        assert np.array_equal(res[t][0], oracle.bfs(g.off, g.col, r).level)
    bfsmi.bfs_server_destroy(s)


def drain_completed(p, s, tickets, timeout=60.0):
    """Collect tickets from the completion queue until all have been
    reported; every ticket must be reported exactly once."""
    seen = []
    t0 = time.time()
    while len(seen) < len(tickets):
        seen += p.bfs_server_completed(s)
        assert time.time() - t0 < timeout, "queries did not finish"
        time.sleep(0.0005)
    assert sorted(seen) == sorted(tickets)
    assert p.bfs_server_completed(s) == []
    return seen


def test_serve_completion_queue_and_device_delivery(bfsmi, pool):
    graphs, handles = pool
    s, ids, arena = make_server(bfsmi, handles)
    rng = np.random.default_rng(21)
    qs = []
    for k in range(40):
        gi = int(rng.integers(0, len(graphs)))
        qs.append((gi, int(rng.integers(0, graphs[gi].V))))
    ts = [bfsmi.bfs_submit(s, ids[gi], r) for gi, r in qs]
    drain_completed(bfsmi, s, ts)
    for k, (t, (gi, r)) in enumerate(zip(ts, qs)):
        g = graphs[gi]
        if k % 2:
            dst = torch.full((g.V,), 7, dtype=torch.int32, device="cuda")
            code, tm = bfsmi.bfs_poll(s, t, dst)
            got = dst.cpu().numpy()
        else:
            got = np.full(g.V, 7, dtype=np.int32)
            code, tm = bfsmi.bfs_poll(s, t, got)
        assert code == bfsmi.BFS_OK
        ref = oracle.bfs(g.off, g.col, r)
        assert np.array_equal(got, ref.level), (k, gi, r)
        assert tm.levels == int(ref.level.max()) + 1
        assert tm.submit_ns <= tm.admit_ns <= tm.done_ns
    st = bfsmi.bfs_server_get_stats(s)
    assert st.submitted == 40 and st.completed == 40 and st.failed == 0
    assert st.joins == 40 and st.levels >= st.rounds > 0
    assert st.lane_levels >= st.levels and st.device_ms > 0
    assert 0 < st.arena_peak <= arena.numel()
    bfsmi.bfs_server_destroy(s)


def test_serve_staggered_arrivals_shallow_and_deep(bfsmi):
    # graphs above the small-graph size: R-MAT (waves) and a 300 x 300 grid
    # (continuous joins once its lane lifetime is known); queries arrive
    # while earlier ones are on the device
    graphs = [graphgen.rmat(17, seed=9), graphgen.grid(300, 300)]
    handles = [bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER) for g in graphs]
    s, ids, arena = make_server(bfsmi, handles, arena_mb=1024)
    rng = np.random.default_rng(5)
    qs, ts = [], []
    for wave in range(6):
        for _ in range(12):
            gi = int(rng.integers(0, 2))
            r = int(graphgen.pick_roots(graphs[gi], 1, int(rng.integers(1 << 30)))[0])
            qs.append((gi, r))
            ts.append(bfsmi.bfs_submit(s, ids[gi], r))
        time.sleep(0.003)
    drain_completed(bfsmi, s, ts, timeout=120.0)
    for t, (gi, r) in zip(ts, qs):
        g = graphs[gi]
        got = np.empty(g.V, dtype=np.int32)
        code, tm = bfsmi.bfs_poll(s, t, got)
        assert code == bfsmi.BFS_OK
        assert np.array_equal(got, oracle.bfs(g.off, g.col, r).level), (gi, r)
    st = bfsmi.bfs_server_get_stats(s)
    _say("staggered: rounds %d levels %d lanes/level %.2f batches %d"
         % (st.rounds, st.levels, st.lane_levels / max(st.levels, 1), st.batches))
    assert st.completed == len(ts) and st.failed == 0
    bfsmi.bfs_server_destroy(s)
    for h in handles:
        h.close()


@pytest.mark.parametrize("flags", [0, 1])
def test_serve_persistent_rounds_match_oracle(bfsmi, flags):
    # deep graphs (lanes living hundreds of levels) run their rounds in the
    # persistent level kernel unless BFS_SRV_NO_PERSISTENT; an R-MAT graph
    # beside them keeps the captured rounds.  Queries arrive in waves so
    # lanes join running batches.
    graphs = [graphgen.grid(200, 200), graphgen.grid(1000, 3), graphgen.rmat(15, seed=4),
              graphgen.grid(2, 2), graphgen.grid(400, 400)]
    handles = [bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER) for g in graphs]
    nbytes = 512 << 20
    arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = bfsmi.bfs_server_create(arena, max_lanes=64, max_inflight=8, flags=flags)
    ids = [bfsmi.bfs_server_add_graph(s, h.handle) for h in handles]
    rng = np.random.default_rng(11 + flags)
    qs, ts = [], []
    for wave in range(8):
        # the 400 x 400 grid gets many lanes at once (wide union frontiers
        # are covered by test_serve_wide_deep_rounds)
        for k in range(16):
            gi = int(rng.integers(0, len(graphs))) if k < 10 else len(graphs) - 1
            r = int(rng.integers(0, graphs[gi].V))
            qs.append((gi, r))
            ts.append(bfsmi.bfs_submit(s, ids[gi], r))
        time.sleep(0.004)
    _say("persistent flags=%d: %d queries submitted" % (flags, len(ts)))
    drain_completed(bfsmi, s, ts, timeout=120.0)
    for t, (gi, r) in zip(ts, qs):
        g = graphs[gi]
        got = np.empty(g.V, dtype=np.int32)
        code, tm = bfsmi.bfs_poll(s, t, got)
        assert code == bfsmi.BFS_OK
        ref = oracle.bfs(g.off, g.col, r)
        assert np.array_equal(got, ref.level), (gi, r)
        assert tm.levels == int(ref.level.max()) + 1
    st = bfsmi.bfs_server_get_stats(s)
    _say("persistent flags=%d: rounds %d persistent %d levels %d"
         % (flags, st.rounds, st.persistent_rounds, st.levels))
    assert st.completed == len(ts) and st.failed == 0
    if flags:
        assert st.persistent_rounds == 0
    else:
        assert st.persistent_rounds > 0
    bfsmi.bfs_server_destroy(s)
    for h in handles:
        h.close()


def test_serve_wide_deep_rounds(bfsmi):
    # 48 lanes at once on a 1400 x 1400 grid: the union frontier grows past
    # what the persistent level kernel takes, so the batch's rounds move to
    # the captured level kernels and back; every result must still be the
    # oracle's
    g = graphgen.grid(1400, 1400)
    h = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    arena = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = bfsmi.bfs_server_create(arena, max_lanes=64, max_inflight=4, flags=0)
    gid = bfsmi.bfs_server_add_graph(s, h.handle)
    rng = np.random.default_rng(21)
    # the first two queries teach the server that the graph is deep
    first = [bfsmi.bfs_submit(s, gid, int(r)) for r in rng.integers(0, g.V, size=2)]
    drain_completed(bfsmi, s, first, timeout=120.0)
    roots = [int(r) for r in rng.integers(0, g.V, size=48)]
    ts = [bfsmi.bfs_submit(s, gid, r) for r in roots]
    _say("wide deep rounds: %d queries submitted" % len(ts))
    drain_completed(bfsmi, s, ts, timeout=120.0)
    for t, r in zip(ts, roots):
        got = np.empty(g.V, dtype=np.int32)
        code, tm = bfsmi.bfs_poll(s, t, got)
        assert code == bfsmi.BFS_OK
        assert np.array_equal(got, oracle.bfs(g.off, g.col, r).level), r
    st = bfsmi.bfs_server_get_stats(s)
    _say("wide deep rounds: rounds %d persistent %d wide %d"
         % (st.rounds, st.persistent_rounds, st.wide_rounds))
    assert st.failed == 0
    assert st.persistent_rounds > 0 and st.wide_rounds > 0
    bfsmi.bfs_server_destroy(s)
    h.close()


def _triangulated_grid(side):
    # a side x side lattice with one diagonal per cell: deep (about 2 * side
    # levels from a corner) and full of triangles, so vertices at one depth
    # are adjacent and a search finds some of them twice in one level
    i = np.arange(side * side, dtype=np.int64).reshape(side, side)
    src = np.concatenate([i[:, :-1].ravel(), i[:-1, :].ravel(), i[:-1, :-1].ravel()])
    dst = np.concatenate([i[:, 1:].ravel(), i[1:, :].ravel(), i[1:, 1:].ravel()])
    return graphgen.from_edges(side * side, src, dst)


def test_serve_deep_graph_with_same_level_edges(bfsmi):
    # the persistent rounds finalize one level and expand the next in the
    # same phase, reading other vertices' seen masks while they change; on a
    # graph with edges inside a level that admits spurious candidates, which
    # their own finalize must drop: every result must be the oracle's
    g = _triangulated_grid(300)
    h = bfsmi.Graph.from_csr(g.off, g.col, flags=bfsmi.BFS_DEGREE_ORDER)
    arena = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = bfsmi.bfs_server_create(arena, max_lanes=64, max_inflight=4, flags=0)
    gid = bfsmi.bfs_server_add_graph(s, h.handle)
    rng = np.random.default_rng(33)
    # the first two queries teach the server that the graph is deep
    first = [bfsmi.bfs_submit(s, gid, int(r)) for r in rng.integers(0, g.V, size=2)]
    drain_completed(bfsmi, s, first, timeout=120.0)
    roots = [int(r) for r in rng.integers(0, g.V, size=40)]
    ts = []
    for k, r in enumerate(roots):
        ts.append(bfsmi.bfs_submit(s, gid, r))
        if k % 8 == 7:
            time.sleep(0.003)  # later queries join batches already running
    _say("same-level edges: %d queries submitted" % len(ts))
    drain_completed(bfsmi, s, ts, timeout=120.0)
    for t, r in zip(ts, roots):
        got = np.empty(g.V, dtype=np.int32)
        code, tm = bfsmi.bfs_poll(s, t, got)
        assert code == bfsmi.BFS_OK
        assert np.array_equal(got, oracle.bfs(g.off, g.col, r).level), r
    st = bfsmi.bfs_server_get_stats(s)
    _say("same-level edges: rounds %d persistent %d" % (st.rounds, st.persistent_rounds))
    assert st.failed == 0
    assert st.persistent_rounds > 0
    bfsmi.bfs_server_destroy(s)
    h.close()


def test_serve_drain_reports_uncollected_results(bfsmi, pool):
    # room for one batch state and three results: after three queries finish
    # without being polled, nothing else can be admitted, so drain must
    # report BFS_ERR_BUDGET instead of blocking; polling frees the room and
    # the rest then completes, every result equal to the oracle's
    graphs, handles = pool
    g, h = graphs[0], handles[0]

    def al(x):
        return (x + 255) // 256 * 256
    V = g.V
    state = (4 * al(8 * V) + al((V + 31) // 32 * 4) + 4 * al(4 * V) + al(8 * (V + 1)) + al(8 * ((V + 2047) // 2048 + 1))
             + al(4 * ((g.nnz + 255) // 256 + 2)) + al(128) + al(512) + al(256) + al(512))
    s, ids, arena = make_server(bfsmi, [h], arena_bytes=state + 3 * al(2 * V) + 256)
    roots = [int(r) for r in graphgen.pick_roots(g, 40, 5)]
    ts = [bfsmi.bfs_submit(s, ids[0], r) for r in roots]
    t0 = time.time()
    with pytest.raises(bfsmi.BFSError) as e:
        bfsmi.bfs_server_drain(s)
    assert e.value.code == bfsmi.BFS_ERR_BUDGET
    _say("drain reported the stall after %.3f s" % (time.time() - t0))
    assert time.time() - t0 < 30
    done = {}
    while len(done) < len(ts):
        for t in bfsmi.bfs_server_completed(s):
            buf = np.empty(V, dtype=np.int32)
            code, _ = bfsmi.bfs_poll(s, t, buf)
            assert code == bfsmi.BFS_OK
            done[t] = buf
        assert time.time() - t0 < 60, "queries did not finish"
        time.sleep(0.001)
    bfsmi.bfs_server_drain(s)  # nothing outstanding: returns at once
    for t, r in zip(ts, roots):
        assert np.array_equal(done[t], oracle.bfs(g.off, g.col, r).level), r
    bfsmi.bfs_server_destroy(s)
    del arena
