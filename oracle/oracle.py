"""ctypes front end of the C oracle in ``ib_oracle.c`` (test infrastructure only).

Every function takes plain numpy arrays.  Floating-point inputs are converted to float64
(an exact upcast for float32 data); the job precision only matters for the cell keys,
which follow the rounding rule of the key step (one rounded multiply in the job precision).

Grid description used throughout (a plain dict, independent of the product's structs):
    dim      2 or 3
    n        cells per dimension (list of dim ints)
    length   periodic box edge per dimension (list of dim floats); h_k = length_k / n_k
    stagger  list of ncomp staggerings xi_c (each a list of dim floats in [0, 1))
    kernel   "peskin4", "cosine4" or "roma3" (the 3-point kernel of Roma, Peskin & Berger)
    walls    optional bit mask of non-periodic dimensions (bit k: dimension k has walls)
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

KERNELS = {"peskin4": 0, "cosine4": 1, "roma3": 2}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_phi.restype = ctypes.c_double
        L.or_phi.argtypes = [ctypes.c_int, ctypes.c_double]
        L.or_dphi.restype = ctypes.c_double
        L.or_dphi.argtypes = [ctypes.c_int, ctypes.c_double]
        L.or_keys.restype = ctypes.c_long
        L.or_keys.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_long, _dp,
                              _i32p]
        L.or_plan.restype = ctypes.c_long
        L.or_plan.argtypes = [ctypes.c_long, _i32p, _i32p, _i32p, _i32p]
        common = [ctypes.c_int, _ip, _dp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int]
        L.or_spread.restype = ctypes.c_int
        L.or_spread.argtypes = common + [ctypes.c_int, ctypes.c_long, _dp, _dp, _dp]
        L.or_interp.restype = ctypes.c_int
        L.or_interp.argtypes = common + [ctypes.c_int, ctypes.c_long, _dp, _dp, _dp]
        L.or_spread_at.restype = ctypes.c_int
        L.or_spread_at.argtypes = common + [ctypes.c_long, _dp, _dp, ctypes.c_long, _i32p,
                                            _i64p, _dp]
        L.or_interp_grad.restype = ctypes.c_int
        L.or_interp_grad.argtypes = common + [ctypes.c_long, _dp, _dp, _dp, _dp]
        L.or_advect.restype = None
        L.or_advect.argtypes = [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_long, _dp, _dp,
                                ctypes.c_double, _dp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _grid_args(grid):
    dim = int(grid["dim"])
    n = np.array(list(grid["n"]) + [1] * (3 - dim), dtype=np.intc)
    length = np.array(list(grid["length"]) + [1.0] * (3 - dim), dtype=np.float64)
    st = np.zeros((len(grid["stagger"]), 3), dtype=np.float64)
    for c, xi in enumerate(grid["stagger"]):
        st[c, :dim] = xi
    ncomp = st.shape[0]
    kernel = KERNELS[grid.get("kernel", "peskin4")]
    return dim, n, length, ncomp, st, kernel, int(grid.get("walls", 0))


def phi(r, kernel="peskin4"):
    L = lib()
    k = KERNELS[kernel]
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda x: L.or_phi(k, float(x)), otypes=[np.float64])(r)


def dphi(r, kernel="peskin4"):
    L = lib()
    k = KERNELS[kernel]
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda x: L.or_dphi(k, float(x)), otypes=[np.float64])(r)


def keys(grid, X, xi, prec="f64"):
    """Cell keys of the points X (np x dim) on the staggering xi; -1 marks invalid points.
    The cell rule follows the kernel's support size: the nearest node for the 3-point kernel
    (odd support, Fig. 1(b)), the node at or below the point otherwise."""
    dim, n, length, _, _, kernel, _ = _grid_args(grid)
    X = _f64(X).reshape(-1, dim)
    xi_a = np.zeros(3)
    xi_a[:dim] = xi
    out = np.empty(X.shape[0], dtype=np.int32)
    odd = 1 if kernel == KERNELS["roma3"] else 0
    bad = lib().or_keys(dim, _ptr(n, _ip), _ptr(length, _dp), _ptr(xi_a, _dp),
                        1 if prec == "f32" else 0, odd, X.shape[0], _ptr(X, _dp), _ptr(out, _i32p))
    return out, int(bad)


def plan(k):
    """Stable ascending sort of keys: (sorted_keys, perm, seg_off[0..q], q)."""
    k = np.ascontiguousarray(np.asarray(k, dtype=np.int32))
    npts = k.shape[0]
    sk = np.empty(npts, dtype=np.int32)
    perm = np.empty(npts, dtype=np.int32)
    seg = np.empty(npts + 1, dtype=np.int32)
    q = lib().or_plan(npts, _ptr(k, _i32p), _ptr(sk, _i32p), _ptr(perm, _i32p),
                      _ptr(seg, _i32p))
    return sk, perm, seg[: q + 1].copy(), int(q)


def spread(grid, X, F, tier=1):
    """f (ncomp x n_{d-1} x ... x n_0) from points X (np x dim) and forces F (np x ncomp)."""
    dim, n, length, ncomp, st, kernel, walls = _grid_args(grid)
    X = _f64(X).reshape(-1, dim)
    F = _f64(F).reshape(-1, ncomp)
    G = int(np.prod(n[:dim]))
    f = np.empty(ncomp * G, dtype=np.float64)
    rc = lib().or_spread(dim, _ptr(n, _ip), _ptr(length, _dp), ncomp, _ptr(st, _dp), kernel,
                         walls, tier, X.shape[0], _ptr(X, _dp), _ptr(F, _dp), _ptr(f, _dp))
    if rc != 0:
        raise MemoryError("oracle spread: allocation failed")
    return f.reshape([ncomp] + [int(v) for v in n[:dim][::-1]])


def interp(grid, X, u, tier=1):
    """U (np x ncomp) from grid values u (ncomp x ...)."""
    dim, n, length, ncomp, st, kernel, walls = _grid_args(grid)
    X = _f64(X).reshape(-1, dim)
    u = _f64(u).reshape(ncomp, -1)
    U = np.empty((X.shape[0], ncomp), dtype=np.float64)
    lib().or_interp(dim, _ptr(n, _ip), _ptr(length, _dp), ncomp, _ptr(st, _dp), kernel, walls,
                    tier,
                    X.shape[0], _ptr(X, _dp), _ptr(u, _dp), _ptr(U, _dp))
    return U


def spread_at(grid, X, F, comp, target):
    """Spread values at sampled (component, flat grid index) pairs, by plain loops."""
    dim, n, length, ncomp, st, kernel, walls = _grid_args(grid)
    X = _f64(X).reshape(-1, dim)
    F = _f64(F).reshape(-1, ncomp)
    comp = np.ascontiguousarray(np.asarray(comp, dtype=np.int32))
    target = np.ascontiguousarray(np.asarray(target, dtype=np.int64))
    out = np.empty(comp.shape[0], dtype=np.float64)
    lib().or_spread_at(dim, _ptr(n, _ip), _ptr(length, _dp), ncomp, _ptr(st, _dp), kernel,
                       walls, X.shape[0], _ptr(X, _dp), _ptr(F, _dp), comp.shape[0],
                       _ptr(comp, _i32p), _ptr(target, _i64p), _ptr(out, _dp))
    return out


def interp_grad(grid, X, u, W):
    """dX (np x dim): sum_c W_{j,c} dU_{j,c}/dX_j for U = J(X)u."""
    dim, n, length, ncomp, st, kernel, walls = _grid_args(grid)
    X = _f64(X).reshape(-1, dim)
    u = _f64(u).reshape(ncomp, -1)
    W = _f64(W).reshape(-1, ncomp)
    dX = np.empty_like(X)
    lib().or_interp_grad(dim, _ptr(n, _ip), _ptr(length, _dp), ncomp, _ptr(st, _dp), kernel,
                         walls, X.shape[0], _ptr(X, _dp), _ptr(u, _dp), _ptr(W, _dp), _ptr(dX, _dp))
    return dX


def mac_stagger(dim):
    """MAC staggering: component c sits at the cell centre shifted by -h e_c / 2 (Sec. 2)."""
    return [[0.0 if k == c else 0.5 for k in range(dim)] for c in range(dim)]


def advect(grid, X, U, dt):
    """Position update of the IB step (Sec. 2, steps (b) and (g)): X + dt U per coordinate,
    rounded once, wrapped into [0, L_k) (a result that rounds to L_k or below 0 is set to 0).
    U has dim columns."""
    dim = int(grid["dim"])
    L = np.array(grid["length"][:dim], dtype=np.float64)
    X = _f64(X).reshape(-1, dim)
    U = _f64(U).reshape(-1, dim)
    out = np.empty_like(X)
    lib().or_advect(dim, _ptr(L, _dp), int(grid.get("walls", 0)), X.shape[0], _ptr(X, _dp),
                    _ptr(U, _dp), float(dt), _ptr(out, _dp))
    return out


def tether_force(grid, X0, X, k):
    """Hookean tether of the unstructured-point test (Sec. 4.1): F = k (X0 - X), each
    coordinate difference of a periodic dimension taken to its nearest periodic image, in
    [-L_k / 2, L_k / 2); along walled dimensions the plain difference."""
    dim = int(grid["dim"])
    L = np.array(grid["length"][:dim], dtype=np.float64)
    periodic = np.array([not (int(grid.get("walls", 0)) >> k) & 1 for k in range(dim)])
    d = _f64(X0).reshape(-1, dim) - _f64(X).reshape(-1, dim)
    folded = np.where(d >= 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
    return float(k) * np.where(periodic, folded, d)


def unstructured_step(grid, X, X0, u, k, dt):
    """One step of the unstructured-point test (Sec. 4.1), in the paper's order: U = J(X)u
    and the predicted X* = X + dt U; F = k (X0 - X*) spread from X*; then the velocity at X
    again and X + dt U.  Returns (X_next, X_star, F, f, U)."""
    U = interp(grid, X, u)
    Xs = advect(grid, X, U, dt)
    F = tether_force(grid, X0, Xs, k)
    f = spread(grid, Xs, F)
    U2 = interp(grid, X, u)
    return advect(grid, X, U2, dt), Xs, F, f, U2
