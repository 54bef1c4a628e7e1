"""Second, independent oracle in NumPy: the dense matrix S of Sec. 2 (test infrastructure).

Builds the spreading matrix S = (delta_h(x_i - X_j)) explicitly for tiny problems (grid
point i in rows, IB point j in columns; eq. (matrix-spread) and its transpose J for
interpolation), with phi written independently of the C oracle, so that the two can be
compared on small cases.  Only for G * n up to a few million entries.
"""
import numpy as np


def phi_peskin4(r):
    a = np.abs(np.asarray(r, dtype=np.float64))
    inner = (3.0 - 2.0 * a + np.sqrt(np.clip(1.0 + 4.0 * a - 4.0 * a * a, 0.0, None))) / 8.0
    outer = (5.0 - 2.0 * a - np.sqrt(np.clip(-7.0 + 12.0 * a - 4.0 * a * a, 0.0, None))) / 8.0
    return np.where(a <= 1.0, inner, np.where(a <= 2.0, outer, 0.0))


def phi_cosine4(r):
    a = np.abs(np.asarray(r, dtype=np.float64))
    return np.where(a <= 2.0, 0.25 * (1.0 + np.cos(np.pi * a / 2.0)), 0.0)


def phi_roma3(r):
    """3-point kernel (Roma, Peskin & Berger 1999), support |r| < 3/2."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    inner = (1.0 + np.sqrt(np.clip(1.0 - 3.0 * a * a, 0.0, None))) / 3.0
    b = 1.0 - a
    outer = (5.0 - 3.0 * a - np.sqrt(np.clip(1.0 - 3.0 * b * b, 0.0, None))) / 6.0
    return np.where(a <= 0.5, inner, np.where(a <= 1.5, outer, 0.0))


PHI = {"peskin4": phi_peskin4, "cosine4": phi_cosine4, "roma3": phi_roma3}


def grid_points(grid, c):
    """Coordinates of all grid points of component c, x = h (i + xi), x-fastest order."""
    dim = grid["dim"]
    n = list(grid["n"])
    h = [grid["length"][k] / n[k] for k in range(dim)]
    axes = [h[k] * (np.arange(n[k]) + grid["stagger"][c][k]) for k in range(dim)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")  # slowest dimension first
    return np.stack([m.ravel() for m in mesh[::-1]], axis=1)  # (G, dim), x fastest


def matrix(grid, X, c):
    """Dense S for component c: S[i, j] = prod_k h_k^-1 phi((x_ik - X_jk)/h_k), the
    difference taken to its minimum image along periodic dimensions; along a walled
    dimension (bit k of grid["walls"]) only the grid points 0..n_k-1 exist, unfolded."""
    dim = grid["dim"]
    kern = PHI[grid.get("kernel", "peskin4")]
    X = np.asarray(X, dtype=np.float64).reshape(-1, dim)
    xg = grid_points(grid, c)
    S = np.ones((xg.shape[0], X.shape[0]))
    for k in range(dim):
        L = grid["length"][k]
        h = L / grid["n"][k]
        d = xg[:, k][:, None] - X[:, k][None, :]
        if not (int(grid.get("walls", 0)) >> k) & 1:
            d = d - L * np.round(d / L)
        S *= kern(d / h) / h
    return S


def spread(grid, X, F):
    dim = grid["dim"]
    ncomp = len(grid["stagger"])
    F = np.asarray(F, dtype=np.float64).reshape(-1, ncomp)
    shape = [int(v) for v in grid["n"]][::-1]
    return np.stack([(matrix(grid, X, c) @ F[:, c]).reshape(shape) for c in range(ncomp)])


def interp(grid, X, u):
    dim = grid["dim"]
    ncomp = len(grid["stagger"])
    hd = float(np.prod([grid["length"][k] / grid["n"][k] for k in range(dim)]))
    u = np.asarray(u, dtype=np.float64).reshape(ncomp, -1)
    return np.stack([matrix(grid, X, c).T @ (u[c] * hd) for c in range(ncomp)], axis=1)
