"""The serving loop: jobs submitted one by one come back with the same results as the
same jobs run alone (bit for bit), under batching, arena pressure and bad inputs."""
import numpy as np
import pytest
import torch

from paper_2012_06646_amd import workloads as wl
from tests.gpu_util import TOL, oracle_errors, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_06646_amd import ibops
    return ibops


def serving_jobs(k, dtype, seed, sizes=(16, 24, 32, 48), nmax=20000):
    r = wl.rng(seed)
    jobs = []
    for i in range(k):
        g = wl.grid(3, int(r.choice(sizes)), 1.0)
        n = int(round(np.exp(r.uniform(np.log(10), np.log(nmax)))))
        X, F, u = wl.uniform_case(g, n, seed + 1 + i)
        shape = wl.grid_shape(g)
        jobs.append({"grid": g, "X": to_dev(X, dtype), "F": to_dev(F, dtype), "u": to_dev(u, dtype),
                     "f": torch.empty(shape, dtype=dtype, device="cuda"),
                     "U": torch.empty((n, 3), dtype=dtype, device="cuda")})
    return jobs


def alone(ib, job, dtype):
    p = ib.Plan(job["grid"], job["X"].shape[0], dtype).update(job["X"])
    return p.spread(job["F"]), p.interpolate(job["u"])


def run_all(srv, jobs):
    tickets = [srv.submit(j) for j in jobs]
    srv.drain()
    out = [srv.poll(t) for t in tickets]
    return out


@pytest.mark.parametrize("max_batch,graph", [(1, False), (5, False), (128, False), (1, True),
                                             (5, True), (128, True), (128, 3)])
def test_server_results_match_jobs_run_alone(ib, max_batch, graph):
    """Every batch (with graphs: every replay of the slot's graph, with other work and
    synchronisations between replays; graph = 3: graphs for batches of at most 3 jobs, direct
    launches for larger ones) against the same jobs run alone, bit for bit."""
    dtype = torch.float32
    jobs = serving_jobs(40, dtype, 6000)
    say(f"server max_batch={max_batch} graph={graph}: 40 jobs")
    srv = ib.Server(dtype, arena_bytes=256 << 20, max_jobs_per_batch=max_batch, use_graph=graph)
    out = run_all(srv, jobs)
    st = srv.stats()
    srv.close()
    assert all(s == 0 for s, _ in out), out
    assert all(lat > 0 for _, lat in out)
    assert st["jobs_done"] == 40 and st["batches"] >= (40 + max_batch - 1) // max_batch
    for j in range(40):
        f1, U1 = alone(ib, jobs[j], dtype)
        assert torch.equal(jobs[j]["f"], f1) and torch.equal(jobs[j]["U"], U1), f"job {j}"


@pytest.mark.parametrize("graph", [False, True])
def test_server_small_arena_wraps(ib, graph):
    """An arena that holds only a few jobs at a time: batches stay small, the ring wraps."""
    dtype = torch.float64
    jobs = serving_jobs(30, dtype, 6100, sizes=(32,), nmax=30000)
    sizes = [ib.workspace_bytes(j["grid"], dtype, j["X"].shape[0]) for j in jobs]
    arena = 3 * max(sizes) + (4 << 20)
    srv = ib.Server(dtype, arena_bytes=arena, max_jobs_per_batch=128, use_graph=graph)
    out = run_all(srv, jobs)
    st = srv.stats()
    srv.close()
    assert all(s == 0 for s, _ in out)
    assert st["batches"] >= -(-sum(sizes) // arena)  # no batch outgrows the arena
    for j in range(30):
        f1, U1 = alone(ib, jobs[j], dtype)
        assert torch.equal(jobs[j]["f"], f1) and torch.equal(jobs[j]["U"], U1)


@pytest.mark.parametrize("graph", [False, True])
def test_server_dense_jobs_tiled(ib, graph):
    """Dense jobs interpolate through LDS tiles inside batches (also in the slot graphs),
    mixed with sparse jobs that gather: bit for bit against the jobs run alone."""
    dtype = torch.float32
    jobs = []
    for i, (N, n) in enumerate([(96, 120000), (32, 2000), (96, 100000), (48, 5000), (96, 150000)]):
        g = wl.grid(3, N, 1.0)
        X, F, u = wl.uniform_case(g, n, 6400 + i)
        jobs.append({"grid": g, "X": to_dev(X, dtype), "F": to_dev(F, dtype), "u": to_dev(u, dtype),
                     "f": torch.empty(wl.grid_shape(g), dtype=dtype, device="cuda"),
                     "U": torch.empty((n, 3), dtype=dtype, device="cuda")})
    say(f"server dense jobs graph={graph}")
    srv = ib.Server(dtype, arena_bytes=512 << 20, max_jobs_per_batch=8, use_graph=graph)
    out = run_all(srv, jobs)
    srv.close()
    assert all(s == 0 for s, _ in out)
    for j, job in enumerate(jobs):
        f1, U1 = alone(ib, job, dtype)
        assert torch.equal(job["f"], f1) and torch.equal(job["U"], U1), f"job {j}"


def test_server_rejects_and_flags(ib):
    dtype = torch.float32
    jobs = serving_jobs(3, dtype, 6200, sizes=(16,), nmax=500)
    bad = serving_jobs(1, dtype, 6300, sizes=(16,), nmax=500)[0]
    Xh = bad["X"].cpu()
    Xh[0, 0] = float("inf")
    bad["X"] = Xh.to("cuda")
    srv = ib.Server(dtype, arena_bytes=64 << 20)
    big = {"grid": wl.grid(3, 128, 1.0), "X": torch.zeros((4_000_000, 3), dtype=dtype, device="cuda")}
    with pytest.raises(ib.IBError):
        srv.submit(big)  # larger than the whole arena
    t = [srv.submit(j) for j in jobs[:2]] + [srv.submit(bad)] + [srv.submit(jobs[2])]
    srv.drain()
    st = [srv.poll(x)[0] for x in t]
    assert st == [0, 0, -6, 0]
    assert srv.poll(t[0])[0] == -1  # reported once
    srv.close()


def test_server_sees_inputs_written_just_before_submit(ib):
    """Inputs produced by torch kernels on the caller's stream right before submit: the
    server (its own stream) sees them whole and gives the same results as the job run alone."""
    dtype = torch.float64
    jobs = serving_jobs(6, dtype, 6500, sizes=(32, 48), nmax=60000)
    say("server: inputs written on the caller's stream before each submit")
    srv = ib.Server(dtype, arena_bytes=512 << 20, max_jobs_per_batch=8)
    final = []
    tickets = []
    for j in jobs:
        X0, F0, u0 = j["X"].clone(), j["F"].clone(), j["u"].clone()
        final.append((X0, F0, u0))
        # stale contents first, then the real inputs written by a chain of kernels
        j["X"].fill_(0.5)
        j["F"].zero_()
        j["u"].zero_()
        for _ in range(20):
            j["F"].mul_(1.0)
        j["X"].copy_(X0)
        j["F"].copy_(F0)
        j["u"].copy_(u0)
        tickets.append(srv.submit(j))
    srv.drain()
    out = [srv.poll(t)[0] for t in tickets]
    srv.close()
    assert out == [0] * len(jobs)
    for j, (X0, F0, u0) in zip(jobs, final):
        ref = {"grid": j["grid"], "X": X0, "F": F0, "u": u0}
        f1, U1 = alone(ib, ref, dtype)
        assert torch.equal(j["f"], f1) and torch.equal(j["U"], U1)


@pytest.mark.parametrize("graph", [False, True])
def test_served_mix_against_oracle(ib, orc, graph):
    """A serving mix in FP32 (grids 32^3..128^3, 10^3..2*10^5 points, log-uniform) run by
    the server, every job against the oracle (the larger ones on sampled grid values and
    points)."""
    dtype = torch.float32
    r = wl.rng(6600)
    jobs, host = [], []
    for i in range(10):
        N = int(r.choice([32, 64, 96, 128]))
        n = int(round(np.exp(r.uniform(np.log(1e3), np.log(2e5)))))
        g = wl.grid(3, N, 1.0)
        X, F, u = (a.astype(np.float32) for a in wl.uniform_case(g, n, 6600 + 1 + i))
        host.append((g, X, F, u))
        jobs.append({"grid": g, "X": to_dev(X, dtype), "F": to_dev(F, dtype), "u": to_dev(u, dtype),
                     "f": torch.empty(wl.grid_shape(g), dtype=dtype, device="cuda"),
                     "U": torch.empty((n, 3), dtype=dtype, device="cuda")})
    say(f"served FP32 mix against the oracle, graph={graph}: {[j['X'].shape[0] for j in jobs]}")
    srv = ib.Server(dtype, arena_bytes=1 << 30, max_jobs_per_batch=4, use_graph=graph)
    out = run_all(srv, jobs)
    srv.close()
    assert all(st == 0 for st, _ in out)
    for i, (job, (g, X, F, u)) in enumerate(zip(jobs, host)):
        ef, eU = oracle_errors(orc, g, X, F, u, job["f"], job["U"], 6700 + i)
        say(f"   job {i} grid {g['n'][0]} n={X.shape[0]}: spread {ef:.2e} interp {eU:.2e}")
        assert ef <= TOL[dtype] and eU <= TOL[dtype], i
