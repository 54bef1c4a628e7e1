"""Batched jobs (ib_batch_run) against the same jobs run one by one through the plan API
(bit for bit: the same kernels on the same data) and against the CPU oracle."""
import json

import numpy as np
import pytest
import torch

from paper_2012_06646_amd import workloads as wl
from tests.gpu_util import TOL, normwise, oracle_errors, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_06646_amd import ibops
    return ibops


def make_jobs(specs, dtype, seed):
    """specs: (grid, npts, spread?, interp?) -> job dicts on the device, plus host copies."""
    jobs, host = [], []
    for i, (g, n, sp, it) in enumerate(specs):
        X, F, u = wl.uniform_case(g, n, seed + i)
        job = {"grid": g, "X": to_dev(X, dtype)}
        if sp:
            job["F"] = to_dev(F, dtype)
        if it:
            job["u"] = to_dev(u, dtype)
        jobs.append(job)
        host.append((X, F, u))
    return jobs, host


def one_by_one(ib, job, dtype):
    p = ib.Plan(job["grid"], job["X"].shape[0], dtype).update(job["X"])
    f = p.spread(job["F"]) if "F" in job else None
    U = p.interpolate(job["u"]) if "u" in job else None
    return f, U


MIXED_3D = [
    (wl.grid(3, 32, 1.0), 1000, True, True),
    (wl.grid(3, 64, 1.0), 40000, True, True),
    (wl.grid(3, 96, 1.0), 150000, True, False),
    (wl.grid(3, [20, 24, 28], [1.0, 1.2, 1.4]), 5000, False, True),
    (wl.grid(3, 128, 1.0), 300000, True, True),
    (wl.grid(3, 32, 1.0), 0, True, True),
    (wl.grid(3, 16, 2.0), 1, True, True),
    (wl.grid(3, 48, 1.0), 4097, True, True),
    (wl.grid(3, 32, 1.0), 150000, True, True),   # dense: split spreading tiles
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_matches_one_by_one_bitwise(ib, dtype):
    jobs, _ = make_jobs(MIXED_3D, dtype, 4100)
    say(f"batch of {len(jobs)} mixed 3-D jobs dtype={dtype}")
    b = ib.Batch(jobs, dtype).run()
    assert b.status() == [0] * len(jobs)
    for j, ((f, U), job) in enumerate(zip(b.results(), jobs)):
        f1, U1 = one_by_one(ib, job, dtype)
        if f1 is not None:
            assert torch.equal(f, f1), f"job {j}: spread differs"
        else:
            assert f is None
        if U1 is not None:
            assert torch.equal(U, U1), f"job {j}: interpolation differs"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_crowded_job_rotated_adds_match_batch_bitwise(ib, dtype):
    """Most points in cells of five or more points (2000 cells of 8, 20000 scattered), far
    above the 1/12 share from which a plan's spreading rotates each lane's order of adds;
    batches keep the plain order.  The fixed-point sums make the two bitwise equal."""
    g = wl.grid(3, 48, 1.0)
    r = wl.rng(4242)
    h = 1.0 / 48
    cells = r.integers(0, 48, (2000, 3)) * h
    X = np.concatenate([np.repeat(cells, 8, axis=0) + r.random((16000, 3)) * h,
                        r.random((20000, 3))]) % 1.0
    X = X[r.permutation(X.shape[0])]
    F = r.standard_normal(X.shape)
    job = {"grid": g, "X": to_dev(X, dtype), "F": to_dev(F, dtype)}
    say(f"crowded 48^3 job dtype={dtype}")
    b = ib.Batch([job], dtype).run()
    assert b.status() == [0]
    f_batch = b.results()[0][0]
    f_plan, _ = one_by_one(ib, job, dtype)
    assert torch.equal(f_plan, f_batch)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_against_oracle(ib, orc, dtype):
    """Small jobs, a dense job whose spreading tiles are split over several blocks, and a
    job dense enough to interpolate through LDS tiles, against the oracle."""
    specs = [(wl.grid(3, 24, 1.0), 3000, True, True), (wl.grid(3, [16, 20, 12], 1.0), 2500, True, True),
             (wl.grid(3, 32, 2.0), 6000, True, True),
             (wl.grid(3, 32, 1.0), 150000, True, True),    # split spreading tiles
             (wl.grid(3, 96, 1.0), 150000, True, True)]    # LDS-tiled interpolation
    jobs, host = make_jobs(specs, dtype, 4200)
    say(f"batch against the oracle, dtype={dtype}")
    b = ib.Batch(jobs, dtype).run()
    nd = np.float32 if dtype == torch.float32 else np.float64
    for i, ((g, n, _, _), (f, U), (X, F, u)) in enumerate(zip(specs, b.results(), host)):
        X, F, u = (a.astype(nd) for a in (X, F, u))
        ef, eU = oracle_errors(orc, g, X, F, u, f, U, 4250 + i)
        say(f"   grid {g['n']} n={n}: spread err {ef:.2e} interp err {eU:.2e}")
        assert ef <= TOL[dtype] and eU <= TOL[dtype]


def test_batch_2d_and_reuse(ib, orc):
    dtype = torch.float64
    specs = [(wl.grid(2, 32, 1.0, stagger=[[0.5, 0.5], [0.5, 0.5]]), 1000, True, True),
             (wl.grid(2, [64, 40], 1.0), 7000, True, True)]
    jobs, host = make_jobs(specs, dtype, 4300)
    b = ib.Batch(jobs, dtype)
    b.run()
    first = [(f.clone(), U.clone()) for f, U in b.results()]
    b.run()  # the same batch again: identical results
    for (f0, U0), (f, U) in zip(first, b.results()):
        assert torch.equal(f0, f) and torch.equal(U0, U)
    for (g, n, _, _), (f, U), (X, F, u) in zip(specs, b.results(), host):
        assert normwise(to_host(f), orc.spread(g, X, F, tier=0)) <= TOL[dtype]
        assert normwise(to_host(U), orc.interp(g, X, u, tier=0)) <= TOL[dtype]


def test_batch_flags_bad_points_per_job(ib):
    dtype = torch.float64
    g = wl.grid(3, 16, 1.0)
    X0, F0, _ = wl.uniform_case(g, 100, 4400)
    Xbad = X0.copy()
    Xbad[7, 1] = np.nan
    jobs = [{"grid": g, "X": to_dev(X0, dtype), "F": to_dev(F0, dtype)},
            {"grid": g, "X": to_dev(Xbad, dtype), "F": to_dev(F0, dtype)}]
    b = ib.Batch(jobs, dtype).run()
    assert b.status() == [0, -6]


def test_max_jobs_batch(ib):
    dtype = torch.float32
    specs = [(wl.grid(3, 16 + 4 * (i % 5), 1.0), 200 + 37 * i, True, True) for i in range(128)]
    jobs, _ = make_jobs(specs, dtype, 5000)
    b = ib.Batch(jobs, dtype).run()
    res = b.results()
    for j in (0, 1, 63, 127):
        f1, U1 = one_by_one(ib, jobs[j], dtype)
        assert torch.equal(res[j][0], f1) and torch.equal(res[j][1], U1)


BATCH_TUNINGS = [{"spread_tile": 1}, {"spread_tile": 2}, {"split_points": 256}, {"split_points": -1},
                 {"radix_bits": 10}, {"spread_tile": 1, "split_points": 2048, "radix_bits": 6}]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_tuned_batch_matches_tuned_plans_bitwise(ib, dtype):
    """A batch run with one tuning for all its jobs gives each job the results of a plan
    created with the same tuning, bit for bit (every spreading tile shape, shared and
    unshared tiles, other bucket widths)."""
    jobs, _ = make_jobs(MIXED_3D, dtype, 4300)
    for t in BATCH_TUNINGS:
        say(f"tuned batch {t} of {len(jobs)} mixed 3-D jobs dtype={dtype}")
        b = ib.Batch(jobs, dtype, tuning=t).run()
        assert b.status() == [0] * len(jobs)
        for j, ((f, U), job) in enumerate(zip(b.results(), jobs)):
            p = ib.Plan(job["grid"], job["X"].shape[0], dtype, tuning=t).update(job["X"])
            if "F" in job:
                assert torch.equal(f, p.spread(job["F"])), f"tuning {t}, job {j}: spread differs"
            if "u" in job:
                assert torch.equal(U, p.interpolate(job["u"])), f"tuning {t}, job {j}: interp differs"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_tuned_2d_batch_matches_tuned_plans_and_oracle(ib, orc, dtype):
    """2-D batches with tunings that share spreading tiles or change the bucket width: each
    job equals a plan with the same tuning bit for bit, and the oracle within tolerance."""
    specs = [(wl.grid(2, 32, 1.0, stagger=[[0.5, 0.5], [0.5, 0.5]]), 1000, True, True),
             (wl.grid(2, [64, 40], 1.0), 7000, True, True),
             (wl.grid(2, 48, 1.0), 30000, True, False)]
    jobs, host = make_jobs(specs, dtype, 4500)
    for t in ({"split_points": 32}, {"split_points": -1}, {"radix_bits": 6}):
        say(f"tuned 2-D batch {t} dtype={dtype}")
        b = ib.Batch(jobs, dtype, tuning=t).run()
        assert b.status() == [0] * len(jobs)
        for j, ((f, U), job, (g, n, sp, it), (X, F, u)) in enumerate(zip(b.results(), jobs, specs, host)):
            p = ib.Plan(g, n, dtype, tuning=t).update(job["X"])
            assert torch.equal(f, p.spread(job["F"])), f"tuning {t}, job {j}: spread differs"
            nd = np.float64 if dtype == torch.float64 else np.float32
            Xc = X.astype(nd).astype(np.float64)
            assert normwise(to_host(f), orc.spread(g, Xc, F.astype(nd).astype(np.float64), tier=0)) <= TOL[dtype]
            if it:
                assert torch.equal(U, p.interpolate(job["u"])), f"tuning {t}, job {j}: interp differs"


def test_autotune_batch_caches_and_batch_finds_it(ib, tmp_path, monkeypatch):
    """The batch tuner times distinct layouts only, caches its choice under the job mix (in
    any job order), and Batch(..., tuning="auto") runs with it."""
    from paper_2012_06646_amd import tune
    monkeypatch.setenv("IB_TUNE_CACHE", str(tmp_path / "tune.json"))
    dtype = torch.float32
    jobs, _ = make_jobs(MIXED_3D[:5], dtype, 4400)
    say(f"autotune a batch of {len(jobs)} jobs")
    best, timings = tune.autotune_batch(jobs, dtype, reps=3)
    say(f"batch tuning {best} over {len(timings)} candidates")
    assert len(timings) >= 3 and "(0, 0, 0)" in timings
    entry = json.load(open(tmp_path / "tune.json"))[tune.batch_key(jobs, dtype)]
    assert entry["tuning"] == best
    assert tune.batch_key(list(reversed(jobs)), dtype) == tune.batch_key(jobs, dtype)
    b = ib.Batch(jobs, dtype, tuning="auto")
    assert b.tuning == best
    b.run()
    b2 = ib.Batch(jobs, dtype, tuning=best).run()
    for (f, U), (f2, U2) in zip(b.results(), b2.results()):
        assert (f is None and f2 is None) or torch.equal(f, f2)
        assert (U is None and U2 is None) or torch.equal(U, U2)
