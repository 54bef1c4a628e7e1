"""Autotuner for plan tunings (ib_tuning): the spreading tile shape, the number of points per
block before a spreading tile is shared, and the bucket bits of the key sort.

For a representative point set, each candidate tuning builds a plan and times the step the
plan serves -- plan update, spreading, interpolation -- with HIP events on the device.  The
search is coordinate-wise (tile shape, then splitting, then bucket bits), starting from the
built-in choices.  Candidates that resolve to the same plan layout (the same tile shape and
the same workspace size, which changes with the split count and the bucket bits) run the
same kernels and are timed once.  The candidates of one axis are timed interleaved, one step
each per round, and compared by their median step time, so drift of the device clock or of
other work affects them alike; a candidate must beat the current choice by 2%, and by more
than the spread of the current choice's own repeats, to replace it.  Results are kept in a JSON cache (``$IB_TUNE_CACHE``, default
``~/.cache/ibops_tune.json``) keyed by dtype, grid and the point count rounded to a power of
two, where ``Plan(..., tuning="auto")`` finds them.

Batches (``autotune_batch``) are tuned the same way, one tuning for all jobs of the batch
(``ib_batch_run_tuned``), timing whole ``Batch.run`` calls; their cache key is the job mix:
dtype, dimension, kernel, and each job's grid, components, operators and point count rounded
to a power of two.  ``Batch(..., tuning="auto")`` finds them.
"""
import hashlib
import json
import math
import os

import torch

from . import ibops

TILE_SHAPES = {1: "32x16x13", 2: "32x8x13", 3: "64x8x8"}  # 0: built-in (64x8x8)
BUILTIN_TILE = 3
SPLIT_CHOICES = (0, 256, 2048, -1)     # 0: built-in (~512 blocks, >= 128 points each); -1: never split
# bucket bits: 0 = built-in (about 2048 points and at most 8192 cells per bucket), or 10, the
# most buckets.  Fewer buckets than the built-in are not offered: their buckets start near
# the 4096 points one block sorts in LDS, and once moving points crowd some cells those
# buckets take the slower path through global memory.
RADIX_CHOICES = (0, 10)
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


def layout_key(grid, dtype, npts, tuning):
    """Tunings with equal keys build the same plan layout and run the same kernels."""
    tile = 0
    if int(grid["dim"]) == 3:
        tile = int(tuning.get("spread_tile", 0)) or BUILTIN_TILE
    desc = ibops.make_desc(grid)
    nbytes = ibops._lib.ib_plan_workspace_bytes_tuned(
        ibops.ctypes.byref(desc), ibops._dtype_code(dtype), int(npts),
        ibops.ctypes.byref(ibops.make_tuning(tuning)))
    return (tile, int(nbytes))


def _time_runs(runs, reps):
    """(median ms, interquartile range in ms) of each callable, timed interleaved on the
    current stream: round r times one call of every candidate in turn."""
    st = torch.cuda.current_stream()
    for once in runs:
        once()  # first-use costs stay out of the timings
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in runs] for _ in range(reps)]
    for r in range(reps):
        for i, once in enumerate(runs):
            ev[r][i][0].record(st)
            once()
            ev[r][i][1].record(st)
    torch.cuda.synchronize()
    out = []
    for i in range(len(runs)):
        ms = sorted(ev[r][i][0].elapsed_time(ev[r][i][1]) for r in range(reps))
        out.append((ms[len(ms) // 2], ms[(3 * len(ms)) // 4] - ms[len(ms) // 4]))
    return out


def time_tunings(grid, X, F, u, tunings, reps=10):
    """(median ms, interquartile range in ms) of one plan update + spread + interpolate for
    each tuning, timed interleaved."""
    dtype = X.dtype
    runs = []
    for t in tunings:
        p = ibops.Plan(grid, X.shape[0], dtype, X.device, tuning=t)
        f = torch.empty(p.grid_shape, dtype=dtype, device=X.device)
        U = torch.empty((X.shape[0], p.ncomp), dtype=dtype, device=X.device)

        def once(p=p, f=f, U=U):
            p.update(X)
            p.spread(F, f)
            p.interpolate(u, U)
        runs.append(once)
    return _time_runs(runs, reps)


def time_tuning(grid, X, F, u, tuning, reps=10):
    """Median ms of one plan update + spread + interpolate with this tuning."""
    return time_tunings(grid, X, F, u, [tuning], reps)[0][0]


def _tkey(t):
    return (t["spread_tile"], t["split_points"], t["radix_bits"])


def _search(time_fn, layout_fn, three_d, reps, verbose):
    """Coordinate-wise search from the built-in choices: time_fn(tunings, reps) -> [(median,
    iqr)], layout_fn(tuning) -> a key equal for tunings that run the same kernels.  Returns
    (best tuning, its median ms, {tuning key: median ms})."""
    best = {"spread_tile": 0, "split_points": 0, "radix_bits": 0}
    timings = {}  # tuning key -> median ms (candidates of distinct layouts only)
    seen = {}     # layout key -> tuning key timed for it
    cur = time_fn([best], reps)[0][0]
    timings[_tkey(best)] = cur
    seen[layout_fn(best)] = _tkey(best)
    axes = [("split_points", SPLIT_CHOICES), ("radix_bits", RADIX_CHOICES)]
    if three_d:
        axes.insert(0, ("spread_tile", tuple(k for k in TILE_SHAPES if k != BUILTIN_TILE)))
    for name, choices in axes:
        cands = []
        for c in choices:
            cand = dict(best, **{name: c})
            lk = layout_fn(cand)
            if lk in seen:
                continue  # the same kernels as a candidate already timed
            seen[lk] = _tkey(cand)
            cands.append(cand)
        if not cands:
            continue
        res = time_fn([best] + cands, reps)  # the incumbent again, alongside
        cur, cur_iqr = res[0]
        timings[_tkey(best)] = cur
        for cand, (t, _) in zip(cands, res[1:]):
            timings[_tkey(cand)] = t
            if verbose:
                print(f"  tuning {cand}: {t:.4f} ms (current {cur:.4f})", flush=True)
        i = min(range(len(cands)), key=lambda k: res[1 + k][0])
        # a candidate must win by the margin and by more than the incumbent's own spread
        # between repeats (its interquartile range)
        if res[1 + i][0] < cur - max(MARGIN * cur, cur_iqr):
            best, cur = cands[i], res[1 + i][0]
    return best, cur, timings


def autotune(grid, X, F, u, reps=10, store=True, verbose=False):
    """Search the tunings for this point set and grid; return (best tuning, timings)."""
    dtype, npts = X.dtype, X.shape[0]
    best, cur, timings = _search(lambda ts, r: time_tunings(grid, X, F, u, ts, r),
                                 lambda t: layout_key(grid, dtype, npts, t),
                                 int(grid["dim"]) == 3, reps, verbose)
    if store:
        _store(key(grid, X.dtype, X.shape[0]),
               {"tuning": best, "ms": round(cur, 5),
                "default_ms": round(timings[(0, 0, 0)], 5), "candidates": len(timings)})
    return best, {str(k): round(v, 5) for k, v in timings.items()}


# ---- batches ------------------------------------------------------------------------------

def batch_key(jobs, dtype):
    """Cache key of a job mix: dtype, dimension and kernel of the batch, its job count, and a
    digest of its jobs' grids, components, operators and point counts (rounded to a power of
    two), taken in sorted order so that the order of the jobs does not matter."""
    dt = "f64" if dtype == torch.float64 else "f32"
    g0 = jobs[0]["grid"]
    parts = []
    for job in jobs:
        g, n = job["grid"], int(job["X"].shape[0])
        ops = ("F" if job.get("F") is not None else "") + ("u" if job.get("u") is not None else "")
        b = 0 if n <= 0 else int(round(math.log2(n)))
        parts.append(f"{'x'.join(str(int(v)) for v in g['n'][: int(g['dim'])])}/{len(g['stagger'])}c/"
                     f"{ops}/n2^{b}")
    digest = hashlib.sha1(";".join(sorted(parts)).encode()).hexdigest()[:16]
    return f"batch/{dt}/{g0['dim']}d/{g0.get('kernel', 'peskin4')}/{len(jobs)}jobs/{digest}"


def cached_batch(jobs, dtype):
    """The cached tuning for this job mix, or None (built-in choices)."""
    hit = _load().get(batch_key(jobs, dtype))
    return dict(hit["tuning"]) if hit else None


def time_batch_tunings(jobs, dtype, tunings, reps=10, device="cuda"):
    """(median ms, interquartile range in ms) of one Batch.run of these jobs for each
    tuning, timed interleaved."""
    batches = [ibops.Batch(jobs, dtype, device, tuning=t) for t in tunings]
    return _time_runs([b.run for b in batches], reps)


def autotune_batch(jobs, dtype=torch.float32, reps=10, store=True, verbose=False, device="cuda"):
    """Search one tuning for all jobs of this batch; return (best tuning, timings)."""
    three_d = int(jobs[0]["grid"]["dim"]) == 3
    probe = ibops.Batch(jobs, dtype, device, workspace=False)  # its job table sizes the layouts

    def layout_fn(t):
        tile = (int(t.get("spread_tile", 0)) or BUILTIN_TILE) if three_d else 0
        nbytes = ibops._lib.ib_batch_workspace_bytes_tuned(
            probe._arr, len(jobs), probe.code, ibops.ctypes.byref(ibops.make_tuning(t)))
        return (tile, int(nbytes))

    best, cur, timings = _search(lambda ts, r: time_batch_tunings(jobs, dtype, ts, r, device),
                                 layout_fn, three_d, reps, verbose)
    if store:
        _store(batch_key(jobs, dtype),
               {"tuning": best, "ms": round(cur, 5),
                "default_ms": round(timings[(0, 0, 0)], 5), "candidates": len(timings)})
    return best, {str(k): round(v, 5) for k, v in timings.items()}
