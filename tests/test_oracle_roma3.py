"""Pins of the oracle's odd-support kernel: the 3-point kernel of Roma, Peskin & Berger
(J. Comput. Phys. 153, 1999), the s = 3 case of Fig. 1(b).

That kernel is defined by its support (|r| < 3/2) and three sums over the integer
offsets: partition of unity, a vanishing first moment and a sum of squares of 1/2.  The
tests check those conditions, finite differences of the derivative, the two oracle tiers
against the independent dense matrix, exactness on constant and linear fields,
conservation, and an exact dyadic case (points half-way between nodes, where the two
nonzero weights are 1/2 each).
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import allpairs
from paper_2012_06646_amd import workloads as wl


def sums(phi_fn, r):
    j = np.arange(-2, 4)[None, :]
    d = r[:, None] - j
    w = phi_fn(d)
    return dict(total=w.sum(1), first=(d * w).sum(1), square=(w * w).sum(1),
                nonzero=(w != 0).sum(1))


def test_roma3_defining_sums(orc):
    r = wl.rng(40).random(20000)
    m = sums(lambda d: orc.phi(d, "roma3"), r)
    assert np.abs(m["total"] - 1.0).max() < 1e-15
    assert np.abs(m["first"]).max() < 1e-15
    assert np.abs(m["square"] - 0.5).max() < 1e-15
    assert m["nonzero"].max() == 3  # s = 3: three support points per dimension


def test_roma3_support_and_symmetry(orc):
    r = wl.rng(41).uniform(1.5, 4.0, 1000)
    assert np.all(orc.phi(r, "roma3") == 0.0) and np.all(orc.phi(-r, "roma3") == 0.0)
    r = wl.rng(42).uniform(0.0, 1.5, 1000)
    assert np.array_equal(orc.phi(r, "roma3"), orc.phi(-r, "roma3"))
    assert np.all(orc.phi(r[r < 1.49], "roma3") > 0.0)


@pytest.mark.parametrize("mutant", ["sign", "drop_sqrt", "coefficient"])
def test_roma3_sums_reject_planted_mistakes(mutant):
    """A slip in the formula (sign of a root, a dropped root, a wrong coefficient) breaks
    at least one defining sum."""
    def bad(d):
        a = np.abs(d)
        s_in = np.sqrt(np.clip(1 - 3 * a * a, 0, None))
        s_out = np.sqrt(np.clip(1 - 3 * (1 - a) ** 2, 0, None))
        k = 3.0
        if mutant == "sign":
            s_out = -s_out
        if mutant == "drop_sqrt":
            s_in = 1.0
        if mutant == "coefficient":
            k = 2.0
        return np.where(a <= 0.5, (1 + s_in) / 3, np.where(a <= 1.5, (5 - k * a - s_out) / 6, 0))
    m = sums(bad, wl.rng(43).random(2000))
    worst = max(np.abs(m["total"] - 1).max(), np.abs(m["first"]).max(),
                np.abs(m["square"] - 0.5).max())
    assert worst > 1e-6


def test_roma3_dphi_matches_central_differences(orc):
    r = wl.rng(44).uniform(-1.8, 1.8, 4000)
    a = np.abs(r)
    r = r[(np.abs(a - 0.5) > 1e-3) & (np.abs(a - 1.5) > 1e-3) & (a > 1e-3)]
    e = 1e-6
    fd = (orc.phi(r + e, "roma3") - orc.phi(r - e, "roma3")) / (2 * e)
    assert np.abs(fd - orc.dphi(r, "roma3")).max() < 1e-8


def tiny_cases():
    return [wl.grid(2, [4, 6], [1.0, 1.5], kernel="roma3"),
            wl.grid(3, [4, 5, 6], [1.0, 1.0, 1.2], kernel="roma3"),
            wl.grid(3, [6, 4, 4], [1.5, 1.0, 1.0], stagger=[[0.25, 0.75, 0.0]], kernel="roma3")]


@pytest.mark.parametrize("gi", range(3))
def test_roma3_tiers_and_dense_matrix_agree(orc, gi):
    g = tiny_cases()[gi]
    r = wl.rng(45 + gi)
    L = np.array(g["length"])
    X = r.uniform(-1.0, 2.0, (23, g["dim"])) * L
    F = r.standard_normal((23, len(g["stagger"])))
    u = r.standard_normal(wl.grid_shape(g))
    fd = allpairs.spread(g, X, F)
    sc = np.abs(fd).max()
    for tier in (0, 1):
        assert np.abs(orc.spread(g, X, F, tier=tier) - fd).max() <= 1e-14 * sc
    Ud = allpairs.interp(g, X, u)
    sc = np.abs(Ud).max()
    for tier in (0, 1):
        assert np.abs(orc.interp(g, X, u, tier=tier) - Ud).max() <= 1e-14 * sc


@pytest.mark.parametrize("dim", [2, 3])
def test_roma3_reproduces_constant_and_linear_fields(orc, dim):
    n = [16, 20, 12][:dim]
    L = [1.0, 1.25, 0.75][:dim]
    g = wl.grid(dim, n, L, kernel="roma3")
    h = np.array(L) / np.array(n)
    r = wl.rng(48)
    X = (3 * h + r.random((400, dim)) * (np.array(L) - 6 * h))
    U = orc.interp(g, X, np.full(wl.grid_shape(g), -1.5))
    assert np.abs(U + 1.5).max() < 1e-14
    a = r.standard_normal((dim, dim))
    b = r.standard_normal(dim)
    u = np.zeros(wl.grid_shape(g))
    for c in range(dim):
        u[c] = (allpairs.grid_points(g, c) @ a[c] + b[c]).reshape(u.shape[1:])
    assert np.abs(orc.interp(g, X, u) - (X @ a.T + b)).max() < 1e-13


def test_roma3_spread_conserves_total_force(orc):
    g = wl.grid(3, [8, 6, 10], [1.0, 0.75, 1.25], kernel="roma3")
    r = wl.rng(49)
    X = r.uniform(-2, 3, (300, 3))
    F = r.standard_normal((300, 3))
    f = orc.spread(g, X, F)
    hd = np.prod(np.array(g["length"]) / np.array(g["n"]))
    assert np.abs(f.reshape(3, -1).sum(1) * hd - F.sum(0)).max() < 1e-12 * np.abs(F).sum()


def test_roma3_midpoints_are_exact(orc):
    """A point half-way between two nodes in every dimension has weights 1/2, 1/2 there and
    0 at the third node (phi(3/2) = 0), so every spread value is an exact dyadic rational."""
    g = wl.grid(3, [8, 8, 8], 1.0, stagger=[[0.5, 0.5, 0.5]], kernel="roma3")
    r = wl.rng(50)
    idx = r.integers(0, 8, (40, 3))
    X = idx / 8.0  # nodes of this grid sit at (i + 1/2) h: X lies half-way between i-1 and i
    F = r.integers(-8, 9, (40, 1)).astype(np.float64)
    f = orc.spread(g, X, F)[0]
    acc = np.zeros((8, 8, 8), dtype=object)
    for j in range(40):
        for sz in (-1, 0):
            for sy in (-1, 0):
                for sx in (-1, 0):
                    z, y, x = (idx[j, 2] + sz) % 8, (idx[j, 1] + sy) % 8, (idx[j, 0] + sx) % 8
                    acc[z, y, x] += Fraction(1, 8) * int(F[j, 0]) * 512
    assert np.array_equal(f, acc.astype(np.float64))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("N,L,xi", [(32, 1.0, 0.5), (20, 1.3, 0.0), (96, 1.0, 0.0), (100, 0.9, 0.5)])
def test_odd_support_keys_are_the_fig1b_cells(orc, prec, N, L, xi):
    """Keys of the 3-point kernel name the de facto cells of Fig. 1(b): the region of points
    that share one set of support points, identified by the grid point inside it.  So the
    nodes key - 1, key, key + 1 carry every nonzero weight of the point (the oracle's own
    phi decides which are nonzero), and the key's node lies within half a cell of the point.
    The even rule (the node at or below the point) fails both for points past the half."""
    g = wl.grid(1, N, L, stagger=[[xi]], kernel="roma3")
    g = dict(g, dim=1)
    X = wl.rng(70 + N).random(5000) * L
    k, bad = orc.keys(g, X[:, None], [xi], prec)
    assert bad == 0
    ft = np.float32 if prec == "f32" else np.float64
    inv_h = ft(ft(N) / ft(L))
    y = np.array([float(Fraction(float(ft(ft(x) * inv_h))) - Fraction(xi)) for x in X])  # exact t - xi
    # the node of the key, unwrapped next to y
    node = k + N * np.round((y - k) / N)
    for off in range(-3, 4):
        w = orc.phi(y - (node + off), "roma3")
        if abs(off) <= 1:
            continue
        assert np.all(w == 0.0), off
    w3 = sum(orc.phi(y - (node + off), "roma3") for off in (-1, 0, 1))
    assert np.abs(w3 - 1.0).max() < 1e-14
    assert np.all(np.abs(y - node) <= 0.5)


def test_odd_support_keys_ties_and_even_rule(orc):
    """A point exactly half-way between two nodes belongs to the upper node's cell; the
    4-point kernels keep the node at or below the point."""
    N = 16
    h = 1.0 / N
    X = np.array([[2.5 * h], [3.0 * h], [3.25 * h], [3.75 * h], [15.5 * h]])  # dyadic: exact
    g3 = dict(wl.grid(1, N, 1.0, stagger=[[0.0]], kernel="roma3"), dim=1)
    g4 = dict(wl.grid(1, N, 1.0, stagger=[[0.0]], kernel="peskin4"), dim=1)
    k3, _ = orc.keys(g3, X, [0.0])
    k4, _ = orc.keys(g4, X, [0.0])
    assert list(k3) == [3, 3, 3, 4, 0]   # 15.5 goes up to 16, wrapped to 0
    assert list(k4) == [2, 3, 3, 3, 15]
