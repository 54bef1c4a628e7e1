"""Benchmark: spread + interpolate Lagrangian points/s on the 128^3 MAC grid with 10^6 points.

One step of the workload (3-D periodic unit cube, 128^3 staggered MAC grid, 10^6 uniform
points, Peskin 4-point kernel):
    plan(X_k) -> f_k = S(X_k) F -> U_k = J(X_k) u -> X_{k+1} = wrap(X_k + 0.1 h U_k)
All four stages are kernels of libibops.so, launched on torch's current stream; inputs are
resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--dtype f64|f32]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spread+interp Lagrangian points/s at 128^3 (HBM GB/s %); batched p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(npts, dim, ncomp, G, b):
    """Compulsory off-chip bytes per launch: each array once per producer/consumer.
    plan:   read X (d b n) + write sorted keys and permutation (8 d n)
    spread: read sorted keys + permutation (8 d n) + X (d b n) + F (d b n) + write f (d b G)
    interp: read permutation (4 d n) + X (d b n) + u (d b G) + write U (d b n)"""
    n = npts
    return {
        "plan": dim * b * n + 8 * ncomp * n,
        "spread": 8 * ncomp * n + dim * b * n + ncomp * b * n + ncomp * b * G,
        "interp": 4 * ncomp * n + dim * b * n + ncomp * b * G + ncomp * b * n,
    }


def cpu_baseline(g, X, F, u, sample):
    """The CPU oracle as it stands (single thread) on the first `sample` points of the same
    workload: keys + stable sort for each staggering, spreading, interpolation."""
    from oracle import oracle as orc
    Xs, Fs = np.asarray(X[:sample], np.float64), np.asarray(F[:sample], np.float64)
    t0 = time.perf_counter()
    for c in range(len(g["stagger"])):
        k, _ = orc.keys(g, Xs, g["stagger"][c])
        orc.plan(k)
    orc.spread(g, Xs, Fs)
    orc.interp(g, Xs, np.asarray(u, np.float64))
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample} points of the same workload (one step: keys+sort per "
                      f"staggering, spread, interpolate), single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--npts", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample", type=int, default=250_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy 5 times (the reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        nbytes = 512 << 20
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE={world}); multi-GPU sharding is a design note, not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2012_06646_amd import ibops, workloads as wl

    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    b = 8 if args.dtype == "f64" else 4
    g, X0, F, u = wl.config2(np.float64, args.npts)
    npts, dim, ncomp = X0.shape[0], 3, 3
    G = 128 ** 3
    h = 1.0 / 128

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    X = torch.from_numpy(X0).to(dev, dtype)
    Fd = torch.from_numpy(F).to(dev, dtype)
    ud = torch.from_numpy(u).to(dev, dtype)
    f = torch.empty([3, 128, 128, 128], dtype=dtype, device=dev)
    U = torch.empty((npts, 3), dtype=dtype, device=dev)
    plan = ibops.Plan(g, npts, dtype, dev)
    stream = torch.cuda.current_stream()

    def step():
        plan.update(X)
        plan.spread(Fd, f)
        plan.interpolate(ud, U)
        ibops.advect(g, X, U, 0.1 * h)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_host0 = time.perf_counter()
    start.record(stream)
    for k in range(K):
        e = ev[k]
        e[0].record(stream)
        plan.update(X)
        e[1].record(stream)
        plan.spread(Fd, f)
        e[2].record(stream)
        plan.interpolate(ud, U)
        e[3].record(stream)
        ibops.advect(g, X, U, 0.1 * h)
        e[4].record(stream)
    end.record(stream)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host0
    if plan.status() != 0:
        print("bench.py: device flagged a data error", file=sys.stderr)
        sys.exit(1)

    ms_total = start.elapsed_time(end)
    ms_step = ms_total / K
    stage_ms = {name: float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)]))
                for i, name in enumerate(["plan", "spread", "interp", "advect"])}
    value = npts * K / (ms_total / 1e3)

    algo = algorithmic_bytes(npts, dim, ncomp, G, b)
    dom = max(("spread", "interp"), key=lambda s: stage_ms[s])
    achieved = algo[dom] / (stage_ms[dom] / 1e3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None,
                "algorithmic_bytes_per_launch": algo[dom]}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "128^3 periodic MAC grid (unit cube), 10^6 uniform random points, "
                               "N(0,1) forces and grid velocities, Peskin 4-point; step = plan + "
                               "spread + interpolate + advect (dt = 0.1 h)",
                   "grid": [128, 128, 128], "npts": npts, "seed": 1002},
        "stages_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "step_algorithmic_bytes": sum(algo.values()),
        "step_hbm_frac": round(sum(algo.values()) / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "host_wall_s": round(t_host, 4),
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, X0.astype(np.float32 if b == 4 else np.float64)
                                           .astype(np.float64), F, u, min(args.cpu_sample, npts))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
