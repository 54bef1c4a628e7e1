"""Pins of the oracle's pieces of the unstructured-point test (Sec. 4.1): the position
update, the tether force, the shear-flow field and one step of the test, against exact
dyadic cases and closed forms (the 4-point kernel reproduces linear fields, the two
interpolations of a step give the same velocity, spreading conserves the total force)."""
import numpy as np
import pytest

from paper_2012_06646_amd import workloads as wl

BOX = {"dim": 3, "n": [16, 16, 16], "length": [16.0, 16.0, 16.0],
       "stagger": wl.mac_stagger(3), "kernel": "peskin4"}


def test_advect_dyadic_cases_and_wrap(orc):
    X = np.array([[15.5, 0.25, 3.0], [0.0, 15.75, 8.0]])
    U = np.array([[8.0, -4.0, 1.0], [-0.5, 2.0, 0.0]])
    got = orc.advect(BOX, X, U, 0.125)
    # 15.5 + 1 = 16.5 -> 0.5; 0.25 - 0.5 -> 15.75; 3 + 0.125; 0 - 1/16 -> 16 - 1/16;
    # 15.75 + 0.25 = 16 -> 0 (a value equal to L wraps to 0); 8 unchanged
    assert got.tolist() == [[0.5, 15.75, 3.125], [16.0 - 0.0625, 0.0, 8.0]]


def test_advect_rounds_once(orc):
    # dt U = 2^-53 (1 + 2^-52)(1 - 2^-53) lies just above half an ulp of 1: the exact sum
    # 1 + dt U rounds up, while rounding dt U first gives exactly half an ulp, a tie that
    # rounds to even (1.0).
    g = {"dim": 1, "n": [4], "length": [4.0], "stagger": [[0.5]], "kernel": "peskin4"}
    dt = 1.0 + 2.0 ** -52
    u = 2.0 ** -53 * (1.0 - 2.0 ** -53)
    assert 1.0 + dt * u == 1.0
    got = orc.advect(g, np.array([[1.0]]), np.array([[u]]), dt)
    assert got[0, 0] == 1.0 + 2.0 ** -52


def test_tether_force_nearest_image(orc):
    X0 = np.array([[0.25, 15.75, 8.0], [8.0, 4.0, 12.0]])
    X = np.array([[15.75, 0.25, 0.0], [8.5, 3.0, 4.0]])
    got = orc.tether_force(BOX, X0, X, 2.0)
    # d = X0 - X: -15.5 -> 0.5; 15.5 -> -0.5; 8 = L/2 -> -8 (half-open); -0.5; 1; 8 -> -8
    assert got.tolist() == [[1.0, -1.0, -16.0], [-1.0, 2.0, -16.0]]
    # the force pulls a displaced point back towards its anchor
    assert orc.tether_force(BOX, np.array([[4.0, 4.0, 4.0]]), np.array([[4.5, 3.5, 4.0]]),
                            1.0).tolist() == [[-0.5, 0.5, 0.0]]


def test_shear_field_is_interpolated_exactly_away_from_the_jump(orc):
    g, X0, u = wl.unstructured_case(16, 2000, seed=6101)
    h = 1.0
    U = orc.interp(g, X0, u)
    y = X0[:, 1]
    inner = (y >= 2 * h) & (y <= 16.0 - 3 * h)
    assert inner.sum() > 1000
    assert np.all(U[:, :2] == 0.0)
    expect = wl.UNSTRUCTURED_SHEAR * (y[inner] - 8.0)
    assert np.abs(U[inner, 2] - expect).max() <= 1e-13 * wl.UNSTRUCTURED_SHEAR * 8.0
    # next to the jump at y = 0 the stencil mixes both ends of the sawtooth
    edge = y < 1.0
    assert np.abs(U[edge, 2] - wl.UNSTRUCTURED_SHEAR * (y[edge] - 8.0)).max() > 1e-4


@pytest.mark.parametrize("N", [16, 32])
def test_one_step_closed_form(orc, N):
    g, X0, u = wl.unstructured_case(N, 3000, seed=6102)
    k, dt, rate = wl.UNSTRUCTURED_TETHER, wl.UNSTRUCTURED_DT, wl.UNSTRUCTURED_SHEAR
    Xn, Xs, F, f, U = orc.unstructured_step(g, X0, X0, u, k, dt)
    h = 16.0 / N
    y = X0[:, 1]
    inner = (y >= 2 * h) & (y <= 16.0 - 3 * h)
    vz = rate * (y - 8.0)
    # the points move along z only, by dt times the shear velocity (wrapped)
    assert np.array_equal(Xs[:, :2], X0[:, :2])
    dz = (Xs[:, 2] - X0[:, 2] + 8.0) % 16.0 - 8.0
    assert np.abs(dz[inner] - dt * vz[inner]).max() <= 1e-14
    # both interpolations see the same velocity, so the corrected step lands on X*
    assert np.array_equal(Xn, Xs)
    # the springs pull back by k times the displacement
    assert np.all(F[:, :2] == 0.0)
    assert np.abs(F[inner, 2] + k * dt * vz[inner]).max() <= k * 1e-14
    # spreading conserves the total force: sum_i f_i h^3 = sum_j F_j
    tot = f.reshape(3, -1).sum(axis=1) * h ** 3
    assert np.abs(tot - F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()
