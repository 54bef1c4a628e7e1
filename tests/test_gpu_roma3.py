"""GPU parity of the odd-support 3-point kernel (Roma, Peskin & Berger 1999; the s = 3 case
of Fig. 1(b)) through the C ABI: spreading and interpolation against the oracle on periodic
and walled grids, the dense split-tile path, batches and the serving loop (one graph per
kernel) against plans run alone, bit for bit."""
import numpy as np
import pytest
import torch

from paper_2012_06646_amd import workloads as wl
from tests.gpu_util import TOL, normwise, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_06646_amd import ibops
    return ibops


def check(ib, orc, g, X, F, u, dtype, label):
    nd = np.float32 if dtype == torch.float32 else np.float64
    Xc, Fc, uc = (np.asarray(a, dtype=nd) for a in (X, F, u))
    say(f"roma3 {label} n={X.shape[0]} grid={g['n']} walls={g.get('walls', 0)} dtype={dtype}")
    p = ib.Plan(g, X.shape[0], dtype).update(to_dev(Xc, dtype))
    f = to_host(p.spread(to_dev(Fc, dtype)))
    U = to_host(p.interpolate(to_dev(uc, dtype)))
    assert p.status() == 0
    f_ref = orc.spread(g, Xc.astype(np.float64), Fc.astype(np.float64))
    U_ref = orc.interp(g, Xc.astype(np.float64), uc.astype(np.float64))
    ef, eU = normwise(f, f_ref), normwise(U, U_ref)
    say(f"   spread err {ef:.3e}  interp err {eU:.3e}")
    assert ef <= TOL[dtype], f"spread {label}: {ef}"
    assert eU <= TOL[dtype], f"interp {label}: {eU}"


CASES = [("mac 3-D ragged", wl.grid(3, [20, 16, 12], 1.0, kernel="roma3"), 8000),
         ("mac 2-D", wl.grid(2, [40, 36], [1.0, 0.9], kernel="roma3"), 5000),
         ("collocated 2-D", wl.grid(2, 32, 1.0, stagger=[[0.5, 0.5]] * 2, kernel="roma3"), 1000),
         ("dense 32^3 (split tiles)", wl.grid(3, 32, 1.0, kernel="roma3"), 150000),
         ("128^3 (LDS-tiled interpolation)", wl.grid(3, 128, 1.0, kernel="roma3"), 250000)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_roma3_ops_match_oracle(ib, orc, ci, dtype):
    label, g, n = CASES[ci]
    X, F, u = wl.uniform_case(g, n, 500 + ci)
    check(ib, orc, g, X, F, u, dtype, label)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_roma3_midpoints_and_nodes(ib, orc, dtype):
    """Points on nodes (weights 1/6, 2/3, 1/6) and half-way between nodes (1/2, 1/2 and a
    zero at distance 3/2: the switch between the two window halves)."""
    g = wl.grid(3, 16, 1.0, kernel="roma3")
    r = wl.rng(510)
    idx = r.integers(0, 16, (3000, 3)).astype(np.float64)
    half = r.integers(0, 2, (3000, 3)) * 0.5
    X = (idx + half) / 16.0
    F = r.standard_normal((3000, 3))
    u = r.standard_normal(wl.grid_shape(g))
    check(ib, orc, g, X, F, u, dtype, "nodes and midpoints")


def test_roma3_walls(ib, orc):
    g = dict(wl.grid(3, [32, 24, 20], [1.0, 0.75, 0.625], kernel="roma3"), walls=5)
    r = wl.rng(520)
    L = np.array(g["length"])
    h = L / np.array(g["n"])
    lo = np.array([-2 * h[0], 0.0, -2 * h[2]])
    X = np.minimum(lo + r.random((20000, 3)) * (L - 2 * lo), L - lo - 1e-9)
    F = r.standard_normal((20000, 3))
    u = r.standard_normal(wl.grid_shape(g))
    for dtype in (torch.float64, torch.float32):
        check(ib, orc, g, X, F, u, dtype, "walls x and z")


def test_roma3_batch_and_server_match_plans(ib):
    dtype = torch.float32
    specs = [(wl.grid(3, 32, 1.0, kernel="roma3"), 150000), (wl.grid(3, 48, 1.0, kernel="roma3"), 4097),
             (wl.grid(3, 64, 1.0, kernel="roma3"), 40000), (wl.grid(3, 16, 1.0, kernel="roma3"), 1)]
    jobs = []
    for i, (g, n) in enumerate(specs):
        X, F, u = wl.uniform_case(g, n, 530 + i)
        jobs.append({"grid": g, "X": to_dev(X, dtype), "F": to_dev(F, dtype), "u": to_dev(u, dtype)})
    say(f"roma3 batch of {len(jobs)} jobs")
    b = ib.Batch(jobs, dtype).run()
    assert b.status() == [0] * len(jobs)
    alone = []
    for job in jobs:
        p = ib.Plan(job["grid"], job["X"].shape[0], dtype).update(job["X"])
        alone.append((p.spread(job["F"]), p.interpolate(job["u"])))
    for j, ((f, U), (f1, U1)) in enumerate(zip(b.results(), alone)):
        assert torch.equal(f, f1), f"job {j}: spread differs"
        assert torch.equal(U, U1), f"job {j}: interpolation differs"
    say("roma3 server with graphs")
    srv = ib.Server(dtype, arena_bytes=256 << 20, max_jobs_per_batch=8, use_graph=True)
    for job in jobs:
        job["f"] = torch.empty(wl.grid_shape(job["grid"]), dtype=dtype, device="cuda")
        job["U"] = torch.empty((job["X"].shape[0], 3), dtype=dtype, device="cuda")
    for rep in range(2):
        tickets = [srv.submit(j) for j in jobs]
        srv.drain()
        assert all(srv.poll(t)[0] == 0 for t in tickets)
        for j, (job, (f1, U1)) in enumerate(zip(jobs, alone)):
            assert torch.equal(job["f"], f1), f"server rep {rep} job {j}: spread differs"
            assert torch.equal(job["U"], U1), f"server rep {rep} job {j}: interpolation differs"
    srv.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("walls", [0, 0b010])
def test_roma3_keys_are_the_odd_support_cells(ib, orc, dtype, walls):
    """Plans of the 3-point kernel key each point by its nearest node (the de facto cell of
    Fig. 1(b)), for every staggering: keys, sorted keys, permutation, run offsets and q equal
    the oracle's bit for bit.  Walled plans key on the padded grid."""
    from tests.test_gpu_parity import check_plan
    g = wl.grid(3, [20, 16, 12], [1.0, 0.8, 1.2], kernel="roma3")
    X, _, _ = wl.uniform_case(g, 20000, 7300)
    if not walls:
        check_plan(ib, orc, g, X, dtype, "roma3 odd-support keys")
        return
    # h = 1 along every axis keeps n / L exact on both grids, so keys compare bit for bit
    g = dict(wl.grid(3, [16, 12, 10], [16.0, 12.0, 10.0], kernel="roma3"), walls=walls)
    gp = wl.grid(3, [16, 16, 10], [16.0, 16.0, 10.0], kernel="roma3")
    X = wl.rng(7301).random((5000, 3)) * np.array([16.0, 12.0, 10.0])
    nd = np.float32 if dtype == torch.float32 else np.float64
    Xc = X.astype(nd)
    say(f"roma3 walled keys dtype={dtype}")
    p = ib.Plan(g, X.shape[0], dtype).update(to_dev(Xc, dtype))
    got = p.export(0)
    # the padded grid continues the caller's indices periodically (ghosts at n .. n + 3)
    k_ref, bad = orc.keys(gp, Xc.astype(np.float64), g["stagger"][p.stagger_of(0)],
                          "f32" if dtype == torch.float32 else "f64")
    assert bad == 0
    assert np.array_equal(to_host(got["keys"]), k_ref)
