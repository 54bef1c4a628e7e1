"""Host-side helpers of the measurement and tuning code (no device): the tuning cache, the
algorithmic byte counts, and how the benchmark reads committed traffic counts."""
import importlib
import json
import os
import sys

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_tune_cache_roundtrip(tmp_path, monkeypatch):
    from paper_2012_06646_amd import tune, workloads as wl
    monkeypatch.setenv("IB_TUNE_CACHE", str(tmp_path / "sub" / "t.json"))
    g = wl.grid(3, 64, 1.0)
    assert tune.cached(g, torch.float32, 100000) is None
    k = tune.key(g, torch.float32, 100000)
    assert k == tune.key(g, torch.float32, 120000)          # same power-of-two bucket
    assert k != tune.key(g, torch.float64, 100000)
    assert k != tune.key(wl.grid(3, 32, 1.0), torch.float32, 100000)
    tune._store(k, {"tuning": {"spread_tile": 2, "split_points": 0, "radix_bits": 8}, "ms": 1.0})
    assert tune.cached(g, torch.float32, 100000) == {"spread_tile": 2, "split_points": 0, "radix_bits": 8}
    data = json.load(open(tmp_path / "sub" / "t.json"))
    assert list(data) == [k]


def test_batch_tune_key_is_the_job_mix(tmp_path, monkeypatch):
    """The batch tuning cache key depends on the jobs' grids, operators and point-count
    buckets, not on their order; a stored choice is found for the same mix."""
    from paper_2012_06646_amd import tune, workloads as wl
    monkeypatch.setenv("IB_TUNE_CACHE", str(tmp_path / "t.json"))
    g32, g64 = wl.grid(3, 32, 1.0), wl.grid(3, 64, 1.0)

    def job(g, n, F=True, u=True):
        j = {"grid": g, "X": torch.empty(n, 3)}
        if F:
            j["F"] = torch.empty(n, 3)
        if u:
            j["u"] = torch.empty(3, *g["n"][::-1])
        return j
    mix = [job(g32, 1000), job(g64, 50000), job(g64, 3000, u=False)]
    k = tune.batch_key(mix, torch.float32)
    assert k == tune.batch_key(mix[::-1], torch.float32)
    assert k == tune.batch_key([job(g32, 1100), job(g64, 50000), job(g64, 3000, u=False)], torch.float32)
    assert k != tune.batch_key(mix, torch.float64)
    assert k != tune.batch_key([job(g32, 1000), job(g64, 50000), job(g64, 3000)], torch.float32)
    assert k != tune.batch_key([job(g32, 1000), job(g32, 50000), job(g64, 3000, u=False)], torch.float32)
    assert k != tune.batch_key([job(g32, 1000), job(g64, 200000), job(g64, 3000, u=False)], torch.float32)
    assert k != tune.batch_key(mix[:2], torch.float32)
    assert tune.cached_batch(mix, torch.float32) is None
    tune._store(k, {"tuning": {"spread_tile": 1, "split_points": 0, "radix_bits": 0}, "ms": 1.0})
    assert tune.cached_batch(mix[::-1], torch.float32) == {"spread_tile": 1, "split_points": 0,
                                                          "radix_bits": 0}


def test_algorithmic_bytes_of_the_benchmark_workload():
    bench = importlib.import_module("bench")
    a = bench.algorithmic_bytes(10 ** 6, 3, 3, 128 ** 3, 8)
    # plan: X + sorted keys and permutation; spread: plan + X + F + f; interp: perm + X + u + U
    assert a["plan"] == 24_000_000 + 24_000_000
    assert a["spread"] == 24_000_000 + 24_000_000 + 24_000_000 + 3 * 8 * 128 ** 3
    assert a["interp"] == 12_000_000 + 24_000_000 + 3 * 8 * 128 ** 3 + 24_000_000


def test_traffic_is_read_only_for_matching_kernel_sources(tmp_path, monkeypatch):
    bench = importlib.import_module("bench")
    f = tmp_path / "traffic.md"
    f.write_text(f"kernel sources sha256: {bench.kernel_source_hash()}\n"
                 "traffic f64 spread: 123456 bytes\ntraffic f32 interp: 789 bytes\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("spread", "f64") == 123456
    assert bench.measured_traffic("interp", "f32") == 789
    assert bench.measured_traffic("interp", "f64") is None
    f.write_text("kernel sources sha256: 0000000000000000\ntraffic f64 spread: 123456 bytes\n")
    assert bench.measured_traffic("spread", "f64") is None


def test_threaded_cpu_baseline_runs_the_oracle_on_chunks():
    import bench
    from paper_2012_06646_amd import workloads as wl
    g = wl.grid(3, 16, 1.0)
    X, F, u = wl.uniform_case(g, 3000, 77)
    r = bench.cpu_baseline_threads(g, X, F, u, 3000, 3)
    assert r["cores"] == 3 and r["kind"] == "oracle" and r["value"] > 0
