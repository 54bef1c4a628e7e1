"""ib_batch_run_static (no workspace argument: the library's fixed device array) against
ib_batch_run on the same jobs, bit for bit, on two calls in a row (the second smaller, so
it runs over what the first left in the array), plus the per-job flags and the size limit."""
import numpy as np
import pytest
import torch

from paper_2012_06646_amd import workloads as wl
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_06646_amd import ibops
    return ibops


def make_jobs(spec, dtype, seed):
    jobs = []
    for i, (N, n) in enumerate(spec):
        g = wl.grid(3, N, 1.0)
        X, F, u = wl.uniform_case(g, n, seed + i)
        jobs.append({"grid": g, "X": to_dev(X, dtype), "F": to_dev(F, dtype), "u": to_dev(u, dtype)})
    return jobs


def results(b):
    return [(f.clone(), U.clone()) for f, U in b.results()]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_static_batch_matches_workspace_batch(ib, dtype):
    calls = [[(48, 40000), (32, 20000), (64, 50000), (32, 500)],   # first call
             [(16, 300), (24, 2000)]]                               # second, smaller
    for k, spec in enumerate(calls):
        jobs = make_jobs(spec, dtype, 7100 + 10 * k)
        b = ib.Batch(jobs, dtype)
        assert b.workspace_bytes <= ib.STATIC_SCRATCH_BYTES
        say(f"no-alloc batch call {k}: {spec} {dtype}")
        b.run()
        torch.cuda.synchronize()
        ref = results(b)
        for f, U in b.results():  # stale outputs must be overwritten
            f.fill_(7.0)
            U.fill_(7.0)
        flags = torch.full((len(jobs),), -1, dtype=torch.int32, device="cuda")
        b.run_static(flags=flags)
        torch.cuda.synchronize()
        assert flags.cpu().tolist() == [0] * len(jobs)
        for j, ((f0, U0), (f1, U1)) in enumerate(zip(ref, b.results())):
            assert torch.equal(f0, f1) and torch.equal(U0, U1), f"call {k} job {j}"


def test_static_batch_flags_and_limit(ib):
    dtype = torch.float64
    jobs = make_jobs([(16, 400), (16, 300), (16, 200)], dtype, 7300)
    Xh = jobs[1]["X"].cpu()
    Xh[5, 2] = float("nan")
    jobs[1]["X"] = Xh.to("cuda")
    b = ib.Batch(jobs, dtype)
    say("no-alloc batch with a flagged job")
    b.run()
    expect = b.status()
    flags = torch.zeros(3, dtype=torch.int32, device="cuda")
    b.run_static(flags=flags)
    torch.cuda.synchronize()
    got = flags.cpu().tolist()
    assert [s != 0 for s in expect] == [v != 0 for v in got] == [False, True, False]
    # without flags, and the jobs' results as with a workspace (the flagged job's NaNs too)
    ref = results(b)
    b.run_static()
    torch.cuda.synchronize()
    for (f0, U0), (f1, U1) in zip(ref, b.results()):
        for a0, a1 in ((f0, f1), (U0, U1)):
            assert torch.equal(a0.isnan(), a1.isnan())
            assert torch.equal(a0.nan_to_num(0.0), a1.nan_to_num(0.0))
    # a batch larger than the array is refused before any device work
    big = [{"grid": wl.grid(3, 128, 1.0), "X": torch.zeros((3_000_000, 3), dtype=dtype, device="cuda")}]
    nb = ib.Batch(big, dtype, workspace=False)
    assert nb.workspace_bytes > ib.STATIC_SCRATCH_BYTES
    with pytest.raises(ib.IBError):
        nb.run_static()
