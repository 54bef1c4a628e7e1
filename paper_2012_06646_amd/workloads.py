"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no spreading or interpolation arithmetic: it only draws positions,
forces and grid fields, and builds red-blood-cell surface point sets.  All draws use
``numpy.random.Generator(PCG64(seed))`` in the order documented per workload, so the GPU
path and the CPU oracle see identical bytes.

Grid descriptions are plain dicts:
    dim, n (cells per dim), length (box edge per dim), stagger (list of xi_c), kernel
"""
import math

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def mac_stagger(dim):
    """MAC staggering: component c at the cell centre minus h e_c / 2 (Sec. 2)."""
    return [[0.0 if k == c else 0.5 for k in range(dim)] for c in range(dim)]


def grid(dim, n, length, stagger=None, kernel="peskin4"):
    if isinstance(n, int):
        n = [n] * dim
    if isinstance(length, (int, float)):
        length = [float(length)] * dim
    if stagger is None:
        stagger = mac_stagger(dim)
    return {"dim": dim, "n": list(n), "length": [float(v) for v in length],
            "stagger": [list(map(float, s)) for s in stagger], "kernel": kernel}


def grid_shape(g):
    return [len(g["stagger"])] + [int(v) for v in g["n"]][::-1]


def uniform_case(g, npts, seed, dtype=np.float64):
    """Uniform points in the box, then N(0,1) forces (npts x ncomp), then N(0,1) grid field.

    Draw order: X, F, u (C order)."""
    r = rng(seed)
    dim = g["dim"]
    L = np.array(g["length"], dtype=np.float64)
    X = r.random((npts, dim)) * L
    F = r.standard_normal((npts, len(g["stagger"])))
    u = r.standard_normal(grid_shape(g))
    return X.astype(dtype), F.astype(dtype), u.astype(dtype)


# ---- the named workloads ----------------------------------------------------------

def square32_1k():
    """2-D periodic unit square, 32 x 32 collocated (cell-centred) grid with two components,
    1000 uniform points, FP64; seed 1001."""
    g = grid(2, 32, 1.0, stagger=[[0.5, 0.5], [0.5, 0.5]])
    X, F, u = uniform_case(g, 1000, 1001)
    return g, X, F, u


def cube128_1m(dtype=np.float64, npts=1_000_000):
    """3-D periodic unit cube, 128^3 MAC grid, 10^6 uniform points; seed 1002."""
    g = grid(3, 128, 1.0)
    X, F, u = uniform_case(g, npts, 1002, dtype)
    return g, X, F, u


# ---- red blood cells (Evans-Fung / Omori reference shape, Sec. 4.2) -----------------

RBC_R0 = 3.91  # micrometres


def rbc_p(r):
    return 0.105 + r * r - 0.56 * r ** 4


def icosphere(level):
    """Unit-sphere vertices of an icosahedron subdivided `level` times (midpoints,
    re-normalised).  Level 4 gives 2562 vertices."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
             (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9),
             (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2),
             (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
             (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts)


def rbc_surface(level=4):
    """Body-frame RBC vertices: each unit vector (a, b, c) maps to theta = atan2(b, a),
    phi = asin(c), then x = R0 cos(theta) cos(phi), y = R0 sin(theta) cos(phi),
    z = R0 p(cos(phi)) sin(phi)  (Sec. 4.2, reference configuration)."""
    v = icosphere(level)
    th = np.arctan2(v[:, 1], v[:, 0])
    ph = np.arcsin(np.clip(v[:, 2], -1.0, 1.0))
    x = RBC_R0 * np.cos(th) * np.cos(ph)
    y = RBC_R0 * np.sin(th) * np.cos(ph)
    z = RBC_R0 * rbc_p(np.cos(ph)) * np.sin(ph)
    return np.stack([x, y, z], axis=1)


def rbc_volume():
    """Enclosed volume of the reference RBC, 2 pi R0^3 (0.105*2/3 + 4/15 - 0.56*16/105)."""
    return 2.0 * math.pi * RBC_R0 ** 3 * (0.105 * 2.0 / 3.0 + 4.0 / 15.0 - 0.56 * 16.0 / 105.0)


def random_rotations(r, k):
    """k uniform random rotation matrices (Shoemake's quaternion method)."""
    u1, u2, u3 = r.random(k), r.random(k), r.random(k)
    q = np.stack([np.sqrt(1 - u1) * np.sin(2 * np.pi * u2), np.sqrt(1 - u1) * np.cos(2 * np.pi * u2),
                  np.sqrt(u1) * np.sin(2 * np.pi * u3), np.sqrt(u1) * np.cos(2 * np.pi * u3)], 1)
    x, y, z, w = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _inside_rbc(p, margin):
    """Body-frame points p (m x 3) strictly inside the RBC grown by `margin`."""
    rho = np.sqrt(p[:, 0] ** 2 + p[:, 1] ** 2)
    R = RBC_R0 + margin
    s = np.clip(rho / R, 0.0, 1.0)
    half = R * rbc_p(s) * np.sqrt(np.clip(1.0 - s * s, 0.0, None)) + margin
    return (rho < R) & (np.abs(p[:, 2]) < half)


def place_rbcs(box, count, seed_pos, seed_rot, max_trials=200_000, margin=0.05):
    """Random sequential addition of `count` RBCs in a periodic cube of edge `box`:
    uniform centres (seed_pos) and uniform rotations (seed_rot); a trial is rejected when a
    vertex of either cell lies inside the other (minimum periodic image, `margin` um).
    When trials run out, the remaining cells are placed at random positions (they may
    overlap).  Returns (centres, rotations, number placed without overlap)."""
    rp, rr = rng(seed_pos), rng(seed_rot)
    surf = rbc_surface(4)
    sub = surf[:: max(1, len(surf) // 162)]  # coarse vertex subset for the overlap test
    centres, rots = [], []
    trials = 0
    reach = 2.0 * (RBC_R0 + margin)
    while len(centres) < count and trials < max_trials:
        trials += 1
        c = rp.random(3) * box
        R = random_rotations(rr, 1)[0]
        ok = True
        if centres:
            C = np.array(centres)
            d = C - c
            d -= box * np.round(d / box)
            near = np.nonzero(np.einsum("ij,ij->i", d, d) < reach * reach)[0]
            mine = sub @ R.T
            for k in near:
                Rk = rots[k]
                # my vertices in k's body frame; k's vertices in my body frame
                pk = (mine - d[k]) @ Rk
                if _inside_rbc(pk, margin).any():
                    ok = False
                    break
                pm = (sub @ Rk.T + d[k]) @ R
                if _inside_rbc(pm, margin).any():
                    ok = False
                    break
        if ok:
            centres.append(c)
            rots.append(R)
    placed = len(centres)
    while len(centres) < count:
        centres.append(rp.random(3) * box)
        rots.append(random_rotations(rr, 1)[0])
    return np.array(centres), np.array(rots), placed


def rbc_points(box, count, seed_pos, seed_rot, max_trials=200_000):
    surf = rbc_surface(4)
    C, R, placed = place_rbcs(box, count, seed_pos, seed_rot, max_trials)
    pts = np.einsum("kij,vj->kvi", R, surf) + C[:, None, :]
    pts = np.mod(pts, box)
    return pts.reshape(-1, 3), placed


def smooth_force(X, box, seed, modes=16):
    """F_c(x) = sum_m a_cm cos(2 pi kappa_cm . x / L + psi_cm), a ~ N(0,1),
    kappa in {-4..4}^3, psi ~ U[0, 2 pi); each component rescaled to max |F_c| = 1."""
    r = rng(seed)
    F = np.zeros((X.shape[0], 3))
    for c in range(3):
        a = r.standard_normal(modes)
        kap = r.integers(-4, 5, size=(modes, 3))
        psi = r.random(modes) * 2 * np.pi
        arg = 2 * np.pi * (X @ kap.T) / box + psi
        F[:, c] = np.cos(arg) @ a
        m = np.abs(F[:, c]).max()
        if m > 0:
            F[:, c] /= m
    return F


def _cached(name, builder):
    """Deterministic generator output, cached under $IBOPS_CACHE (default /tmp/ibops_cache)."""
    import os
    d = os.environ.get("IBOPS_CACHE", "/tmp/ibops_cache")
    path = os.path.join(d, name + ".npz")
    try:
        with np.load(path) as z:
            return {k: z[k] for k in z.files}
    except (OSError, ValueError, KeyError):
        pass
    out = builder()
    try:
        os.makedirs(d, exist_ok=True)
        np.savez(path + ".tmp.npz", **out)
        os.replace(path + ".tmp.npz", path)
    except OSError:
        pass
    return out


def rbc_case(box, n, count, seeds, dtype, max_trials):
    """RBC surface points (count cells, 2562 vertices each) in a periodic cube of edge `box`
    on an n^3 MAC grid; seeds = (positions, rotations, forces, grid field)."""
    def build():
        X, placed = rbc_points(box, count, seeds[0], seeds[1], max_trials)
        F = smooth_force(X, box, seeds[2])
        u = rng(seeds[3]).standard_normal((3, n, n, n))
        return {"X": X, "F": F, "u": u, "placed": np.array(placed)}
    z = _cached(f"rbc_{box}_{n}_{count}_{'_'.join(map(str, seeds))}_{max_trials}", build)
    g = grid(3, n, box)
    return g, z["X"].astype(dtype), z["F"].astype(dtype), z["u"].astype(dtype), int(z["placed"])


def rbc256(dtype=np.float32):
    """256^3 MAC grid in a 64 um periodic box (h = 0.25 um), 1111 RBCs of 2562 vertices
    (40% volume fraction), seeds 3001-3004.  Random sequential addition jams below 40%; the
    cells that do not fit without overlap are placed at random (count returned)."""
    return rbc_case(64.0, 256, 1111, (3001, 3002, 3003, 3004), dtype, 40000)


def rbc128(dtype=np.float64):
    """128^3 MAC grid in a 32 um periodic box (h = 0.25 um), 78 RBCs (about 2 x 10^5 points),
    seeds 5001-5004; the loss's grid field g is drawn with seed 5005."""
    g, X, F, u, placed = rbc_case(32.0, 128, 78, (5001, 5002, 5003, 5004), dtype, 200000)
    gfield = rng(5005).standard_normal((3, 128, 128, 128)).astype(dtype)
    return g, X, F, u, gfield, placed


# ---- the serving mix: independent jobs of mixed grid and point counts -----------------

SERVE_GRIDS = (32, 64, 96, 128)


def serving_job_sizes(count, seed=4001):
    """Grid edge N_j uniform on {32, 64, 96, 128} and point count n_j = round(exp(U(ln 1e3,
    ln 1e6))) for jobs j = 0..count-1, drawn in that order per job from one stream."""
    r = rng(seed)
    out = []
    for _ in range(count):
        N = int(SERVE_GRIDS[int(r.integers(0, len(SERVE_GRIDS)))])
        n = int(round(math.exp(r.uniform(math.log(1e3), math.log(1e6)))))
        out.append((N, n))
    return out


def serving_job(N, n, j, dtype=np.float32):
    """Job j's points and forces on the unit-cube N^3 MAC grid: X ~ U[0,1)^3 then F ~ N(0,1),
    seed 4000 + j."""
    r = rng(4000 + j)
    X = r.random((n, 3))
    F = r.standard_normal((n, 3))
    return X.astype(dtype), F.astype(dtype)


def serving_field(N, dtype=np.float32):
    """The grid velocity interpolated by every job on an N^3 grid: u ~ N(0,1), seed 4000 + N
    (read-only, so jobs on one grid size share it)."""
    return rng(4000 + N).standard_normal((3, N, N, N)).astype(dtype)


def poisson_arrivals(count, rate_per_s, seed=4001):
    """Open-loop arrival times (seconds from the start) of a Poisson stream."""
    r = rng(seed + 7)
    return np.cumsum(r.exponential(1.0 / rate_per_s, count))


# ---- the paper's unstructured-point test (Sec. 4.1) ------------------------------------
# Units: micrometres and microseconds; forces in dyn.  The test runs in a 16 um triply
# periodic box with the shear-like flow u = (0, 0, rate (y - 8 um)), rate 1000 / s, and
# points tied to their initial positions by springs of 0.01 dyn/cm.  The paper states no
# time step for this test; 0.1 us, the step of its red-blood-cell tests, is used.

UNSTRUCTURED_BOX = 16.0           # um
UNSTRUCTURED_SHEAR = 1.0e-3       # 1000 / s in 1 / us
UNSTRUCTURED_TETHER = 1.0e-6      # 0.01 dyn/cm in dyn / um
UNSTRUCTURED_DT = 0.1             # us
UNSTRUCTURED_GRIDS = (16, 32, 64, 128)  # grid points per 16 um, at 2^16 points (Sec. 4.1.1)
# Weak scaling (Sec. 4.1.3): 2^16 .. 2^19 points on the 64^3 grid (h = 0.25 um).  The table's
# caption says h = 0.5 um, but the text's densities (one point per 4 cells at 2^16 points, 2
# per cell at 2^19) and the grid the paper keeps from Sec. 4.1.1 on are those of 64^3.
UNSTRUCTURED_WEAK_GRID = 64
UNSTRUCTURED_WEAK = (1 << 16, 1 << 17, 1 << 18, 1 << 19)


def shear_field(g, rate=UNSTRUCTURED_SHEAR):
    """The shear-like grid velocity on the MAC grid g: u_x = u_y = 0 and
    u_z = rate (y - L_y / 2) at the y-coordinate (j + xi_{z,y}) h_y of every u_z node (a
    jump at the periodic boundary y = 0)."""
    n = [int(v) for v in g["n"]]
    h = g["length"][1] / n[1]
    u = np.zeros(grid_shape(g))
    y = (np.arange(n[1]) + g["stagger"][2][1]) * h
    u[2] = (rate * (y - 0.5 * g["length"][1]))[None, :, None]
    return u


def unstructured_case(N, npts, seed=6001, dtype=np.float64):
    """npts points uniform in the 16 um box (seed 6001 unless given), the N^3 MAC grid and
    its shear field: the initial (tether) positions X0 and the grid velocity u."""
    g = grid(3, N, UNSTRUCTURED_BOX)
    X0 = rng(seed).random((npts, 3)) * UNSTRUCTURED_BOX
    return g, X0.astype(dtype), shear_field(g).astype(dtype)
