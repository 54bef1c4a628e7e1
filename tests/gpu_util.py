"""Helpers for the GPU parity tests (no spreading/interpolation arithmetic here)."""
import sys

import numpy as np
import torch


def say(msg):
    """Name the case before a GPU step, flushed, so a failing run shows where it was."""
    sys.stdout.write(f"[gpu] {msg}\n")
    sys.stdout.flush()


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def normwise(a, b):
    """||a - b||_inf / ||b||_inf (0 when both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    num = np.abs(a - b).max() if b.size else 0.0
    if den == 0.0:
        return float(num)
    return float(num / den)


TOL = {torch.float64: 1e-12, torch.float32: 2e-6}


def oracle_errors(orc, g, X, F, u, f, U, seed, full_below=20000, nsample=3000):
    """Normwise errors of a job's spread f and interpolation U (device tensors or None)
    against the oracle, on host inputs X, F, u in the precision the device used.  Jobs with
    fewer than full_below points are compared whole; larger ones on nsample grid values
    (half at random, half at the cells of random points, so most are nonzero) and nsample
    points, each computed by the oracle on its own."""
    n = X.shape[0]
    r = np.random.default_rng(seed)
    ef = eU = 0.0
    if f is not None:
        fh = to_host(f)
        if n < full_below:
            ef = normwise(fh, orc.spread(g, X, F))
        else:
            ncomp, shape = fh.shape[0], fh.shape[1:]
            comp = r.integers(0, ncomp, nsample).astype(np.int32)
            flat = r.integers(0, int(np.prod(shape)), nsample)
            # cells of random points (staggering ignored: any nearby value will do)
            h = np.array(g["length"], dtype=np.float64) / np.array(g["n"])
            pick = X[r.integers(0, n, nsample // 2)].astype(np.float64)
            cells = np.floor(pick / h).astype(np.int64) % np.array(g["n"])
            near = np.zeros(nsample // 2, dtype=np.int64)
            for k in reversed(range(g["dim"])):
                near = near * int(g["n"][k]) + cells[:, k]
            flat[: nsample // 2] = near
            got = fh.reshape(ncomp, -1)[comp, flat]
            ef = normwise(got, orc.spread_at(g, X, F, comp, flat))
    if U is not None:
        Uh = to_host(U)
        if n < full_below:
            eU = normwise(Uh, orc.interp(g, X, u))
        else:
            rows = r.choice(n, min(n, nsample), replace=False)
            eU = normwise(Uh[rows], orc.interp(g, X[rows], u))
    return ef, eU
