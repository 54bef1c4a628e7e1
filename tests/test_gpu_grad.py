"""GPU gradients (position gradient kernel and the autograd wrappers) against the CPU
oracle's gradient and against central finite differences of the GPU's own operators."""
import numpy as np
import pytest
import torch

from paper_2012_06646_amd import workloads as wl
from tests.gpu_util import TOL, normwise, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_06646_amd import autograd, ibops
    return ibops, autograd


def oracle_loss_grads(orc, g, X, F, u, gfield):
    """Gradients of L = 1/2 |J(X)u|^2 + <S(X)F, g>_h from the oracle's operators."""
    hd = float(np.prod(np.array(g["length"]) / np.array(g["n"])))
    U = orc.interp(g, X, u)
    dF = orc.interp(g, X, gfield)                 # J g
    du = orc.spread(g, X, U) * hd                 # J^T U = h^d S U
    dX = orc.interp_grad(g, X, u, U) + orc.interp_grad(g, X, gfield, F)
    return dX, dF, du


def gpu_loss_grads(ag, g, X, F, u, gfield, dtype):
    hd = float(np.prod(np.array(g["length"]) / np.array(g["n"])))
    Xd = to_dev(X, dtype).requires_grad_(True)
    Fd = to_dev(F, dtype).requires_grad_(True)
    ud = to_dev(u, dtype).requires_grad_(True)
    gd = to_dev(gfield, dtype)
    U = ag.interpolate(Xd, ud, g)
    f = ag.spread(Xd, Fd, g)
    L = 0.5 * (U * U).sum() + hd * (f * gd).sum()
    L.backward()
    return to_host(Xd.grad), to_host(Fd.grad), to_host(ud.grad)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kernel", ["peskin4", "cosine4", "roma3"])
def test_loss_gradients_match_oracle(mods, orc, dtype, kernel):
    ib, ag = mods
    g = wl.grid(3, [24, 20, 16], [1.2, 1.0, 0.8], kernel=kernel)
    X, F, u = wl.uniform_case(g, 6000, 41)
    gfield = wl.rng(42).standard_normal(wl.grid_shape(g))
    nd = np.float32 if dtype == torch.float32 else np.float64
    X, F, u, gfield = (a.astype(nd) for a in (X, F, u, gfield))
    say(f"grad small {kernel} {dtype}")
    dX, dF, du = gpu_loss_grads(ag, g, X, F, u, gfield, dtype)
    rX, rF, ru = oracle_loss_grads(orc, g, X, F, u, gfield)
    tol = TOL[dtype]
    for name, a, b in (("dX", dX, rX), ("dF", dF, rF), ("du", du, ru)):
        e = normwise(a, b)
        say(f"   {name} err {e:.3e}")
        assert e <= tol, (name, e)


def test_position_gradient_matches_central_differences(mods):
    """Per-point losses l_j = 1/2 |U_j|^2 + F_j . (J g)_j depend on X_j only, so a central
    difference on one point's coordinate isolates its gradient (eps = 1e-6 length units)."""
    ib, ag = mods
    g = wl.grid(3, [16, 16, 16], 1.0)
    X, F, u = wl.uniform_case(g, 2000, 43)
    gfield = wl.rng(44).standard_normal(wl.grid_shape(g))
    dt = torch.float64
    dX, _, _ = gpu_loss_grads(ag, g, X, F, u, gfield, dt)
    Fd, ud, gd = to_dev(F, dt), to_dev(u, dt), to_dev(gfield, dt)

    def per_point(Xh):
        p = ib.Plan(g, Xh.shape[0], dt).update(to_dev(Xh, dt))
        U = to_host(p.interpolate(ud))
        Jg = to_host(p.interpolate(gd))
        return 0.5 * (U * U).sum(1) + (F * Jg).sum(1)

    eps = 1e-6
    r = wl.rng(45)
    for k in range(3):
        Xp, Xm = X.copy(), X.copy()
        Xp[:, k] += eps
        Xm[:, k] -= eps
        fd = (per_point(Xp) - per_point(Xm)) / (2 * eps)
        # skip coordinates within eps of a kernel breakpoint (phi'' jumps at |r| = 1, 2)
        t = X[:, k] * 16 - (0.0 if k == 0 else 0.5)
        ok = np.abs(t - np.round(t)) > 1e-3
        err = np.abs(fd - dX[:, k])[ok].max() / np.abs(dX[:, k]).max()
        say(f"fd axis {k}: {err:.2e}")
        assert err < 1e-7


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rbc128_gradients(mods, orc, dtype):
    """128^3 MAC grid, 78 RBCs (about 2 x 10^5 surface points), loss of the
    differentiation workload; GPU gradients against the oracle's."""
    ib, ag = mods
    nd = np.float32 if dtype == torch.float32 else np.float64
    g, X, F, u, gfield, _ = wl.rbc128(nd)
    say(f"grad rbc128 {dtype} n={X.shape[0]}")
    dX, dF, du = gpu_loss_grads(ag, g, X, F, u, gfield, dtype)
    rX, rF, ru = oracle_loss_grads(orc, g, X, F, u, gfield)
    tol = TOL[dtype]
    for name, a, b in (("dX", dX, rX), ("dF", dF, rF), ("du", du, ru)):
        e = normwise(a, b)
        say(f"   {name} err {e:.3e}")
        assert e <= tol, (name, e)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("walls", [0, 0b100])
def test_scaled_entry_points(mods, orc, dtype, walls):
    """The scaled calls against the oracle's operators times the scale, and scale 1 against
    the unscaled calls bit for bit.  Interpolation and its gradient round the product once
    after the sum: bitwise the unscaled result times the scale in the plan's precision."""
    ib, _ = mods
    g = dict(wl.grid(3, [24, 20, 16], [1.2, 1.0, 0.8]), walls=walls)
    X, F, u = wl.uniform_case(g, 5000, 77)
    W = wl.rng(78).standard_normal(F.shape)
    nd = np.float32 if dtype == torch.float32 else np.float64
    X, F, u, W = (a.astype(nd) for a in (X, F, u, W))
    say(f"scaled entry points {dtype} walls={walls}")
    p = ib.Plan(g, X.shape[0], dtype).update(to_dev(X, dtype))
    Fd, ud, Wd = to_dev(F, dtype), to_dev(u, dtype), to_dev(W, dtype)
    tol = TOL[dtype]
    for s in (1.0, 0.37, -2.5e3):
        f = p.spread(Fd, scale=s)
        U = p.interpolate(ud, scale=s)
        dX = p.interpolate_grad(ud, Wd, scale=s)
        assert normwise(to_host(f), s * orc.spread(g, X, F)) <= tol
        assert normwise(to_host(U), s * orc.interp(g, X, u)) <= tol
        assert normwise(to_host(dX), s * orc.interp_grad(g, X, u, W)) <= tol
        assert torch.equal(U, p.interpolate(ud) * s)
        assert torch.equal(dX, p.interpolate_grad(ud, Wd) * s)
        if s == 1.0:
            assert torch.equal(f, p.spread(Fd))
        # accumulation adds the scaled result
        acc = p.interpolate_grad(ud, Wd)
        p.interpolate_grad(ud, Wd, dX=acc, accumulate=True, scale=s)
        assert torch.equal(acc, p.interpolate_grad(ud, Wd) + dX)
        facc = p.spread(Fd)
        p.spread(Fd, f=facc, accumulate=True, scale=s)
        assert torch.equal(facc, p.spread(Fd) + f)
    with pytest.raises(ib.IBError):
        p.interpolate(ud, scale=float("inf"))
