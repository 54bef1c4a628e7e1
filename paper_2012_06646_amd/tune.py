"""Autotuner for plan tunings (ib_tuning): the spreading tile shape, the number of points per
block before a spreading tile is shared, and the radix digit width of the key sort.

For a representative point set, each candidate tuning builds a plan and times the step the
plan serves -- plan update, spreading, interpolation -- with HIP events on the device; the
fastest wins.  The search is coordinate-wise (tile shape, then splitting, then digit width),
starting from the built-in choices, so a handful of candidates are timed; a candidate must
beat the current choice by 2% to replace it, which keeps timing noise from deciding.  Results are kept
in a JSON cache (``$IB_TUNE_CACHE``, default ``~/.cache/ibops_tune.json``) keyed by dtype,
grid and the point count rounded to a power of two, where ``Plan(..., tuning="auto")``
finds them.
"""
import json
import math
import os

import torch

from . import ibops

TILE_SHAPES = {1: "32x16x13", 2: "32x8x13", 3: "64x8x8"}  # 0: built-in (FP64 1, FP32 2)
SPLIT_CHOICES = (0, 256, 2048, -1)     # 0: built-in (~512 blocks, >= 128 points each); -1: never split
RADIX_CHOICES = (0, 8, 6)              # 0: built-in (even digits of at most 8 bits)
MARGIN = 0.02                          # a candidate must be this much faster to be taken


def cache_path():
    return os.environ.get("IB_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                          "ibops_tune.json"))


def key(grid, dtype, npts):
    dt = "f64" if dtype == torch.float64 else "f32"
    n = "x".join(str(int(v)) for v in grid["n"][: int(grid["dim"])])
    bucket = 0 if npts <= 0 else int(round(math.log2(npts)))
    return f"{dt}/{grid['dim']}d/{n}/{len(grid['stagger'])}c/{grid.get('kernel', 'peskin4')}/n2^{bucket}"


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def cached(grid, dtype, npts):
    """The cached tuning for this case, or None (built-in choices)."""
    hit = _load().get(key(grid, dtype, npts))
    return dict(hit["tuning"]) if hit else None


def _store(k, entry):
    data = _load()
    data[k] = entry
    path = cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_tuning(grid, X, F, u, tuning, reps=10):
    """Average ms of one plan update + spread + interpolate with this tuning."""
    dtype = X.dtype
    p = ibops.Plan(grid, X.shape[0], dtype, X.device, tuning=tuning)
    f = torch.empty(p.grid_shape, dtype=dtype, device=X.device)
    U = torch.empty((X.shape[0], p.ncomp), dtype=dtype, device=X.device)

    def once():
        p.update(X)
        p.spread(F, f)
        p.interpolate(u, U)
    once()
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    st = torch.cuda.current_stream()
    s0.record(st)
    for _ in range(reps):
        once()
    s1.record(st)
    torch.cuda.synchronize()
    return s0.elapsed_time(s1) / reps


def autotune(grid, X, F, u, reps=10, store=True, verbose=False):
    """Search the tunings for this point set and grid; return (best tuning, timings)."""
    best = {"spread_tile": 0, "split_points": 0, "radix_bits": 0}
    timings = {}

    def measure(t):
        k = (t["spread_tile"], t["split_points"], t["radix_bits"])
        if k not in timings:
            timings[k] = time_tuning(grid, X, F, u, t, reps)
            if verbose:
                print(f"  tuning {t}: {timings[k]:.4f} ms", flush=True)
        return timings[k]

    time_tuning(grid, X, F, u, best, reps)  # warm-up: first-use costs stay out of the timings
    cur = measure(best)
    axes = [("split_points", SPLIT_CHOICES), ("radix_bits", RADIX_CHOICES)]
    if int(grid["dim"]) == 3:
        builtin = 2 if X.dtype == torch.float32 else 1
        axes.insert(0, ("spread_tile", tuple(k for k in TILE_SHAPES if k != builtin)))
    for name, choices in axes:
        for c in choices:
            cand = dict(best, **{name: c})
            t = measure(cand)
            if t < cur * (1.0 - MARGIN):
                best, cur = cand, t
    if store:
        _store(key(grid, X.dtype, X.shape[0]),
               {"tuning": best, "ms": round(cur, 5),
                "default_ms": round(timings[(0, 0, 0)], 5), "candidates": len(timings)})
    return best, {str(k): round(v, 5) for k, v in timings.items()}
