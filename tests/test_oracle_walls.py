"""Pins of the oracle with walled (non-periodic) dimensions (Sec. 3.1: grid indices outside
0..n_k-1 of a walled dimension are no grid points).  Checked against the independent dense
matrix, the periodic oracle away from the walls, closed forms for a point on the first
grid node (the 4-point kernels keep 3/4 of their weight there), the adjoint identity and
the unwrapped position update."""
import numpy as np
import pytest

from oracle import allpairs
from paper_2012_06646_amd import workloads as wl


def walled(g, walls):
    g = dict(g)
    g["walls"] = walls
    return g


CASES = [(wl.grid(2, [6, 5], [1.5, 1.0]), 1), (wl.grid(2, [6, 5], [1.5, 1.0]), 3),
         (wl.grid(3, [4, 5, 6], [1.0, 1.0, 1.2]), 4), (wl.grid(3, [5, 4, 4], [1.0, 0.8, 0.8]), 7),
         (wl.grid(3, [6, 4, 5], [1.5, 1.0, 1.0], stagger=[[0.25, 0.75, 0.0]]), 2)]


@pytest.mark.parametrize("ci", range(len(CASES)))
@pytest.mark.parametrize("kernel", ["peskin4", "cosine4"])
def test_tiers_and_dense_matrix_agree_with_walls(orc, ci, kernel):
    g0, walls = CASES[ci]
    g = walled(dict(g0, kernel=kernel), walls)
    r = wl.rng(60 + ci)
    L = np.array(g["length"])
    h = L / np.array(g["n"])
    X = r.uniform(-2.0, 1.0, (31, g["dim"])) * L + r.uniform(0.0, 1.0, (31, g["dim"])) * L
    X = np.clip(X, -2 * h, L + 2 * h - 1e-9)  # within two cells of the box
    F = r.standard_normal((31, len(g["stagger"])))
    u = r.standard_normal(wl.grid_shape(g))
    fd = allpairs.spread(g, X, F)
    Ud = allpairs.interp(g, X, u)
    for tier in (0, 1):
        assert np.abs(orc.spread(g, X, F, tier=tier) - fd).max() <= 1e-14 * np.abs(fd).max()
        assert np.abs(orc.interp(g, X, u, tier=tier) - Ud).max() <= 1e-14 * np.abs(Ud).max()
    # a mistake in the wall handling of either side shows: the periodic result differs
    assert np.abs(orc.spread(walled(g, 0), X, F) - fd).max() > 1e-3 * np.abs(fd).max()


def test_interior_points_do_not_see_the_walls(orc):
    g = wl.grid(3, [8, 9, 10], [1.0, 1.0, 1.0])
    r = wl.rng(70)
    h = np.array([1 / 8, 1 / 9, 1 / 10])
    X = 3 * h + r.random((200, 3)) * (1.0 - 6 * h)  # three cells from every wall
    F = r.standard_normal((200, 3))
    u = r.standard_normal(wl.grid_shape(g))
    for walls in (1, 5, 7):
        gw = walled(g, walls)
        assert np.array_equal(orc.spread(gw, X, F), orc.spread(g, X, F))
        assert np.array_equal(orc.interp(gw, X, u), orc.interp(g, X, u))


@pytest.mark.parametrize("kernel", ["peskin4", "cosine4"])
def test_point_on_the_first_node_keeps_three_quarters(orc, kernel):
    # phi(0) = 1/2, phi(+-1) = 1/4, phi(+-2) = 0 for both kernels: with index -1 gone, the
    # node's own dimension keeps 1/2 + 1/4 of the weight, the periodic ones all of it
    g = wl.grid(3, [8, 8, 8], [1.0, 1.0, 1.0], stagger=[[0.5, 0.5, 0.5]], kernel=kernel)
    gw = walled(g, 2)
    h = 1 / 8
    X = np.array([[0.3, 0.5 * h, 0.6]])  # on the first node along y (xi = 1/2)
    f = orc.spread(gw, X, np.array([[1.0]]))
    assert f.sum() * h ** 3 == pytest.approx(0.75, abs=1e-15)
    U = orc.interp(gw, X, np.full(wl.grid_shape(gw), 2.0))
    assert U[0, 0] == pytest.approx(1.5, abs=1e-15)
    # on the last node the same holds (index n is gone)
    X = np.array([[0.3, (8 - 0.5) * h, 0.6]])
    assert orc.spread(gw, X, np.array([[1.0]])).sum() * h ** 3 == pytest.approx(0.75, abs=1e-15)


def test_adjoint_identity_with_walls(orc):
    g = walled(wl.grid(3, [6, 7, 8], [1.2, 1.0, 0.9]), 6)
    r = wl.rng(71)
    L = np.array(g["length"])
    X = r.random((150, 3)) * L
    F = r.standard_normal((150, 3))
    u = r.standard_normal(wl.grid_shape(g))
    hd = np.prod(L / np.array(g["n"]))
    lhs = hd * np.sum(orc.spread(g, X, F) * u)
    rhs = np.sum(F * orc.interp(g, X, u))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_advect_and_tether_along_walls(orc):
    g = walled(wl.grid(3, 16, 16.0), 2)
    X = np.array([[15.75, 15.75, 0.25]])
    U = np.array([[4.0, 4.0, -4.0]])
    # x and z wrap; y (walled) does not
    assert orc.advect(g, X, U, 0.125).tolist() == [[0.25, 16.25, 15.75]]
    F = orc.tether_force(g, np.array([[0.25, 0.25, 0.25]]), np.array([[15.75, 15.75, 15.75]]), 1.0)
    assert F.tolist() == [[0.5, -15.5, 0.5]]
