"""Host-side arithmetic of the benchmark line (no GPU): the roofline of the
expansion kernel, the whole-search summary and the counter-traffic lookup."""
import importlib.util
import os
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _stats(**kw):
    return types.SimpleNamespace(**kw)


def test_harmonic_mean(bench):
    assert bench.harmonic_mean([1.0, 2.0, 4.0]) == pytest.approx(3 / (1 + 0.5 + 0.25))
    assert bench.harmonic_mean([2.0, 0.0, -1.0]) == pytest.approx(2.0)  # non-positive dropped
    assert bench.harmonic_mean([]) == 0.0


def test_roofline_fraction_and_per_launch_figures(bench):
    fake = types.SimpleNamespace(bfs_get_option=lambda h, k: 4, BFS_OPT_EDGES_PER_THREAD=1)
    G = types.SimpleNamespace(handle=None)
    stats = [_stats(expand_alg_bytes=4_000_000_000, expand_bytes=1_000_000_000, expand_ms=2.0,
                    expand_launches=2),
             _stats(expand_alg_bytes=2_000_000_000, expand_bytes=1_000_000_000, expand_ms=1.0,
                    expand_launches=1)]
    r = bench.roofline_of(fake, G, stats, 1 << 20, "no-such-hash")
    # 6 GB in 3 ms = 2000 GB/s, a quarter of the 8 TB/s peak
    assert r["achieved"] == pytest.approx(2000.0)
    assert r["frac"] == pytest.approx(0.25)
    assert r["peak"] == bench.HBM_PEAK_GBS == 8000.0
    assert r["launches"] == 3
    assert r["avg_launch_ms"] == pytest.approx(1.0)
    assert r["alg_bytes_per_launch"] == 2_000_000_000
    assert r["streamed_gbs"] == pytest.approx(2e9 / 3e-3 / 1e9, rel=1e-3)
    assert r["traffic"] is None  # counters only count for the sources they were taken on
    assert r["kernel"] == "k_expand<4>"


def test_search_summary(bench):
    V = 1000
    stats = [_stats(edges_scanned=2_000_000, reached=500), _stats(edges_scanned=4_000_000, reached=900)]
    times = [0.001, 0.004]
    s = bench.search_summary(times, stats, V)
    # TEPS counts each undirected edge once: 1e9 and 0.5e9 edges/s
    assert s["gteps"] == pytest.approx(2 / (1 / 1.0 + 1 / 0.5), rel=1e-3)
    assert s["ms_per_root"] == pytest.approx(2.5)
    b = (8.125 * V + 32 * 500 + 4 * 2e6) + (8.125 * V + 32 * 900 + 4 * 4e6)
    assert s["bfs_alg_gbs"] == pytest.approx(round(b / 0.005 / 1e9, 1))


def test_recorded_traffic_follows_the_source_hash(bench):
    h = bench.kernel_source_hash()
    assert len(h) == 16
    path = os.path.join(ROOT, "profiles", "k_expand_rmat26_traffic.txt")
    recorded = None
    with open(path) as f:
        for line in f:
            if line.startswith("source_hash"):
                recorded = line.split("=", 1)[1].strip()
    assert recorded is not None
    t = bench.recorded_traffic(recorded)
    assert isinstance(t, int) and t > 0
    assert bench.recorded_traffic("0" * 16) is None
    # the bench asks with the hash of the sources it runs: the recorded bytes,
    # or nothing once the expansion sources have changed since the counters
    assert bench.recorded_traffic(h) in (t, None)
    assert (bench.recorded_traffic(h) == t) == (h == recorded)
