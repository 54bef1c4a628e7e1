"""GPU parity of walled (non-periodic) dimensions (Sec. 3.1) through the C ABI: plans whose
grid has walls, against the oracle with the same walls, for points inside the box and up to
two cells outside it; the keys of a walled plan on its padded grid; batches refuse walls."""
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


def walled(g, walls):
    g = dict(g)
    g["walls"] = walls
    return g


def points_near_box(g, n, seed):
    """Uniform in the box widened by two cells along walled dimensions (the range where
    the non-periodic semantics hold), uniform in the box along periodic ones."""
    r = wl.rng(seed)
    L = np.array(g["length"], dtype=np.float64)
    h = L / np.array(g["n"])
    lo = np.where([(g["walls"] >> k) & 1 for k in range(g["dim"])], -2 * h, 0.0)
    X = lo + r.random((n, g["dim"])) * (L - 2 * lo)
    return np.minimum(X, L - lo - 1e-9 * L)


CASES = [(wl.grid(3, [32, 24, 20], [1.0, 0.75, 0.625]), 4, 20000),
         (wl.grid(3, 24, 1.0), 7, 30000),
         (wl.grid(3, [40, 16, 16], [2.5, 1.0, 1.0]), 1, 15000),
         (wl.grid(2, [48, 40], [1.2, 1.0]), 2, 8000),
         (wl.grid(3, 64, 1.0), 4, 120000),
         (wl.grid(3, 128, 1.0), 4, 250000),  # dense enough for LDS-tiled interpolation
         (wl.grid(3, 128, 1.0), 3, 270000)]  # tiled, with ghost columns and rows (x, y walls)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_walled_ops_match_oracle(ib, orc, ci, dtype):
    g0, walls, n = CASES[ci]
    g = walled(g0, walls)
    say(f"walls={walls} grid={g['n']} n={n} dtype={dtype}")
    nd = np.float32 if dtype == torch.float32 else np.float64
    X = points_near_box(g, n, 80 + ci).astype(nd)
    r = wl.rng(90 + ci)
    F = r.standard_normal((n, len(g["stagger"]))).astype(nd)
    u = r.standard_normal(wl.grid_shape(g)).astype(nd)
    Xh, Fh, uh = (a.astype(np.float64) for a in (X, F, u))
    p = ib.Plan(g, n, dtype).update(to_dev(X, dtype))
    f = p.spread(to_dev(F, dtype))
    U = p.interpolate(to_dev(u, dtype))
    assert p.status() == 0
    f_ref, U_ref = orc.spread(g, Xh, Fh), orc.interp(g, Xh, uh)
    assert normwise(to_host(f), f_ref) <= TOL[dtype]
    assert normwise(to_host(U), U_ref) <= TOL[dtype]
    # accumulate adds the spread values into the caller's field
    f2 = p.spread(to_dev(F, dtype), f.clone(), accumulate=True)
    assert normwise(to_host(f2), 2 * f_ref) <= TOL[dtype]
    # the position gradient of interpolation
    W = r.standard_normal((n, len(g["stagger"]))).astype(nd)
    dX = p.interpolate_grad(to_dev(u, dtype), to_dev(W, dtype))
    assert normwise(to_host(dX), orc.interp_grad(g, Xh, uh, W.astype(np.float64))) <= 10 * TOL[dtype]
    if g["dim"] == len(g["stagger"]):
        # interpolation with the position update: no wrap along walls
        dt = 0.37 * min(g["length"][k] / g["n"][k] for k in range(g["dim"]))
        Xd = to_dev(X, dtype)
        U2 = p.interpolate_advect(to_dev(u, dtype), Xd, dt)
        assert torch.equal(U2, U)
        Xa = orc.advect(g, Xh, to_host(U).astype(np.float64), dt)
        tol = 0.0 if dtype == torch.float64 else 4e-7 * max(g["length"])
        assert np.abs(to_host(Xd) - Xa).max() <= tol
        # the standalone update gives the same positions
        Xd2 = to_dev(X, dtype)
        ib.advect(g, Xd2, U, dt)
        assert torch.equal(Xd2, Xd)


@pytest.mark.parametrize("tuning", [{"spread_tile": 1}, {"spread_tile": 2, "split_points": -1},
                                    {"split_points": 64, "radix_bits": 6}])
def test_walled_tunings_match_oracle(ib, orc, tuning):
    """Walled plans with other spreading tiles, unshared or more widely shared tiles and
    another bucket width still write and read only the caller's unpadded field."""
    dtype = torch.float64
    g = walled(wl.grid(3, 24, 1.0), 7)
    n = 30000
    say(f"walls=7 grid={g['n']} n={n} tuning={tuning}")
    X = points_near_box(g, n, 97)
    r = wl.rng(98)
    F = r.standard_normal((n, 3))
    u = r.standard_normal(wl.grid_shape(g))
    p = ib.Plan(g, n, dtype, tuning=tuning).update(to_dev(X, dtype))
    f = p.spread(to_dev(F, dtype))
    U = p.interpolate(to_dev(u, dtype))
    assert p.status() == 0
    assert normwise(to_host(f), orc.spread(g, X, F)) <= TOL[dtype]
    assert normwise(to_host(U), orc.interp(g, X, u)) <= TOL[dtype]


def test_walled_keys_on_the_padded_grid(ib, orc):
    # h = 1 makes n / L exact on both grids, so the keys can be compared bit for bit
    g = walled(wl.grid(3, [16, 12, 10], [16.0, 12.0, 10.0]), 5)
    gp = wl.grid(3, [20, 12, 14], [20.0, 12.0, 14.0])
    X = points_near_box(g, 5000, 95)
    p = ib.Plan(g, 5000, torch.float64).update(to_dev(X, torch.float64))
    got = p.export(0)
    k_ref, bad = orc.keys(gp, X, g["stagger"][p.stagger_of(0)])
    assert bad == 0
    sk, perm, seg, q = orc.plan(k_ref)
    assert np.array_equal(to_host(got["keys"]), k_ref)
    assert np.array_equal(to_host(got["perm"]), perm)
    assert got["q"] == q


def test_batches_refuse_walls(ib):
    g = walled(wl.grid(3, 16, 1.0), 1)
    X = torch.rand((100, 3), dtype=torch.float64, device="cuda")
    F = torch.rand((100, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(ib.IBError):
        ib.Batch([{"grid": g, "X": X, "F": F}], torch.float64)


def test_bad_walls_rejected(ib):
    with pytest.raises(ib.IBError):
        ib.Plan(walled(wl.grid(2, 16, 1.0), 4), 10, torch.float64)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_walled_plan_without_points(ib, dtype):
    g = walled(wl.grid(3, 16, 1.0), 3)
    p = ib.Plan(g, 0, dtype).update(torch.empty((0, 3), dtype=dtype, device="cuda"))
    f = torch.full(p.grid_shape, 7.0, dtype=dtype, device="cuda")
    p.spread(torch.empty((0, 3), dtype=dtype, device="cuda"), f)
    assert p.status() == 0
    assert torch.count_nonzero(f).item() == 0  # overwritten with the empty sum
    U = p.interpolate(torch.ones(p.grid_shape, dtype=dtype, device="cuda"))
    assert U.shape == (0, 3)
