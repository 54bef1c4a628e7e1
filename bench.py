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
    # (the fused position update adds reading and writing X: 2 d b n)


# Kernels behind each operator call (the roofline's unit is one operator call).
OP_KERNELS = {"spread": "ib_spread = spread_kernel (forces read through the permutation)",
              "interp_advect": "ib_interpolate_advect = interp_tile_kernel with the position update"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_128cube_1e6pts.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2012_06646_amd", "csrc", f)
                  for f in ("ops_kernels.hip", "device_common.h", "ib_internal.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(op, dtype):
    """HBM bytes per operator call from the committed FETCH_SIZE/WRITE_SIZE summary, scaled
    by the copy calibration; None when the summary is missing or the operator kernels'
    sources changed after the counters were taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    want = f"traffic {dtype} {op}:"
    src = None
    for line in text.splitlines():
        if line.startswith("kernel sources sha256:"):
            src = line.split(":", 1)[1].strip()
        if line.startswith(want) and src == kernel_source_hash():
            return int(line.split(":", 1)[1].split()[0])
    return None


def device_facts(torch):
    """What the runtime reports about the device (not assumed)."""
    p = torch.cuda.get_device_properties(0)
    facts = {"name": p.name, "compute_units": p.multi_processor_count,
             "memory_GiB": round(p.total_memory / 2 ** 30, 1)}
    for attr in ("gcnArchName", "L2_cache_size", "warp_size", "max_threads_per_multi_processor"):
        if hasattr(p, attr):
            facts[attr] = getattr(p, attr)
    return facts


def cpu_baseline_threads(g, X, F, u, sample, threads):
    """The same oracle calls on the host's cores: the points split into `threads` contiguous
    chunks, one thread each (the oracle's C functions release the GIL).  Keys and
    interpolation per chunk; one stable sort per staggering of all the keys; spreading per
    chunk into a grid of its own, the chunk grids then added in chunk order."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as orc
    orc.lib()
    Xs, Fs = np.asarray(X[:sample], np.float64), np.asarray(F[:sample], np.float64)
    uu = np.asarray(u, np.float64)
    cuts = np.linspace(0, sample, threads + 1).astype(np.int64)
    chunks = list(zip(cuts[:-1], cuts[1:]))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        for xi in g["stagger"]:
            parts = list(ex.map(lambda ab, xi=xi: orc.keys(g, Xs[ab[0]:ab[1]], xi)[0], chunks))
            orc.plan(np.concatenate(parts))
        grids = list(ex.map(lambda ab: orc.spread(g, Xs[ab[0]:ab[1]], Fs[ab[0]:ab[1]]), chunks))
        f = grids[0]
        for part in grids[1:]:
            f = f + part
        U = np.concatenate(list(ex.map(lambda ab: orc.interp(g, Xs[ab[0]:ab[1]], uu), chunks)))
    dt = time.perf_counter() - t0
    assert f.shape[0] == len(g["stagger"]) and U.shape[0] == sample
    return {"value": sample / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} points of the same workload (one step: keys+sort per "
                      f"staggering, spread, interpolate), points split over {threads} threads, "
                      f"{dt:.1f} s"}


def rbc_bench(torch, ibops, wl, K):
    """Red-blood-cell surfaces: 64 um periodic box on a 256^3 MAC grid (h = 0.25 um), 1111
    biconcave cells of 2562 vertices (2,846,382 points, FP32), smooth forces.  A step is plan
    update + spread + interpolate (the points do not move); K steps between two events."""
    dt = torch.float32
    dev = torch.device("cuda:0")
    g, X, F, u, placed = wl.rbc256(np.float32)
    n = X.shape[0]
    Xd, Fd, ud = (torch.from_numpy(a).to(dev) for a in (X, F, u))
    p = ibops.Plan(g, n, dt, dev)
    f = torch.empty(p.grid_shape, dtype=dt, device=dev)
    U = torch.empty((n, 3), dtype=dt, device=dev)
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    for _ in range(3):
        p.update(Xd)
        p.spread(Fd, f)
        p.interpolate(ud, U)
    torch.cuda.synchronize()
    for k in range(K):
        e = ev[k]
        e[0].record(stream)
        p.update(Xd)
        e[1].record(stream)
        p.spread(Fd, f)
        e[2].record(stream)
        p.interpolate(ud, U)
        e[3].record(stream)
    torch.cuda.synchronize()
    ms = ev[0][0].elapsed_time(ev[K - 1][3]) / K
    stage = {name: round(float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)])), 5)
             for i, name in enumerate(["plan", "spread", "interp"])}
    b = 4
    algo = algorithmic_bytes(n, 3, 3, 256 ** 3, b)
    spread_gbs = algo["spread"] / (stage["spread"] / 1e3) / 1e9
    return {"workload": "RBC surfaces, 256^3 MAC grid, 64 um box, 1111 cells x 2562 vertices "
                        f"({placed} placed without overlap), FP32, step = plan + spread + interpolate",
            "npts": n, "ms_per_step": round(ms, 5), "points_per_s": round(n / (ms / 1e3), 1),
            "stage_ms": stage, "spread_hbm_frac": round(spread_gbs / HBM_PEAK_GBS, 4)}


# The paper's own per-call GPU times for this test (one K80 die, FP64, 2^16 points, seconds),
# from the grid-refinement table of Sec. 4.1.1: interpolation (Alg. 3) and spreading by
# sort + segmented reduce (Alg. 4) and with pre-allocated buffers (Alg. 5, its fastest).
PAPER_K80_S = {16: (0.01253, 0.03930, 0.01715), 32: (0.01317, 0.04020, 0.02049),
               64: (0.01722, 0.04215, 0.02370), 128: (0.01816, 0.04755, 0.03656)}


def unstructured_bench(torch, ibops, wl, K):
    """The paper's unstructured-point test (Sec. 4.1), FP64: random points tethered to their
    initial positions in a 16 um periodic box with a shear-like flow; per step, the velocity
    is interpolated twice and the tether force spread once (two plan updates).  Times per
    call, from events around every call of K steps: the grid-refinement series at 2^16
    points and the weak-scaling series on the 64^3 grid."""
    from paper_2012_06646_amd.unstructured import TetheredPoints
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    cases = [(N, 1 << 16) for N in wl.UNSTRUCTURED_GRIDS]
    cases += [(wl.UNSTRUCTURED_WEAK_GRID, n) for n in wl.UNSTRUCTURED_WEAK if n != 1 << 16]
    out = []
    for N, n in cases:
        g, X0, u = wl.unstructured_case(N, n)
        t = TetheredPoints(g, torch.from_numpy(X0).to(dev), torch.from_numpy(u).to(dev), device=dev)
        for _ in range(5):
            t.step()
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(8)] for _ in range(K)]
        for k in range(K):
            e = ev[k]
            e[0].record(stream)
            t.plan.update(t.X)
            e[1].record(stream)
            t.Xstar.copy_(t.X)
            e[2].record(stream)
            t.plan.interpolate_advect(t.u, t.Xstar, t.dt, t.U)
            e[3].record(stream)
            ibops.tether_force(g, t.X0, t.Xstar, t.k, t.F)
            e[4].record(stream)
            t.plan_star.update(t.Xstar)
            e[5].record(stream)
            t.plan_star.spread(t.F, t.f)
            e[6].record(stream)
            t.correct()
            e[7].record(stream)
        torch.cuda.synchronize()

        def avg(i, j):
            return float(np.mean([ev[k][i].elapsed_time(ev[k][j]) for k in range(K)])) * 1e3

        row = {"grid": N, "npts": n, "h_um": 16.0 / N,
               "step_us": round(ev[0][0].elapsed_time(ev[K - 1][7]) / K * 1e3, 2),
               "plan_us": round(0.5 * (avg(0, 1) + avg(4, 5)), 2),
               "interp_us": round(0.5 * (avg(2, 3) + avg(6, 7)), 2),
               "spread_us": round(avg(5, 6), 2),
               "plan_and_spread_us": round(avg(4, 6), 2),
               "tether_us": round(avg(3, 4), 2),
               "copy_us": round(avg(1, 2), 2)}
        if n == 1 << 16 and N in PAPER_K80_S:
            ki, ks4, ks5 = PAPER_K80_S[N]
            row["paper_k80_us"] = {"interp_alg3": ki * 1e6, "spread_alg4": ks4 * 1e6,
                                   "spread_alg5": ks5 * 1e6}
        out.append(row)
        del t
    return {"workload": "unstructured-point test of Sec. 4.1: 16 um periodic box, MAC grid, "
                        "u = (0, 0, 1000/s (y - 8 um)), uniform random points tied by 0.01 dyn/cm "
                        "springs, dt = 0.1 us, FP64; per step 2 plan updates, 2 interpolations "
                        "(with the position update), 1 tether force, 1 spread",
            "steps": K, "cases": out}


def variant_bench(torch, ibops, wl, K, dtype, walls=0, kernel="peskin4"):
    """The 128^3 / 10^6 workload with walls (a bit mask of non-periodic dimensions) or with
    another one-dimensional kernel: plan update, spread and interpolation per call, from
    events around K calls each.  A walled plan runs on a grid padded by 4 ghost planes per
    walled dimension, with the caller's field copied in (zero ghost values) before
    interpolation and out (ghost values dropped) after spreading."""
    dev = torch.device("cuda:0")
    g, X, F, u = wl.cube128_1m(np.float64)
    g = dict(g, walls=walls, kernel=kernel)
    Xd, Fd, ud = (torch.from_numpy(a).to(dev, dtype) for a in (X, F, u))
    n = X.shape[0]
    p = ibops.Plan(g, n, dtype, dev)
    f = torch.empty(p.grid_shape, dtype=dtype, device=dev)
    U = torch.empty((n, 3), dtype=dtype, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        p.update(Xd)
        p.spread(Fd, f)
        p.interpolate(ud, U)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    for k in range(K):
        e = ev[k]
        e[0].record(stream)
        p.update(Xd)
        e[1].record(stream)
        p.spread(Fd, f)
        e[2].record(stream)
        p.interpolate(ud, U)
        e[3].record(stream)
    torch.cuda.synchronize()
    stage = {name: round(float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)])), 5)
             for i, name in enumerate(["plan", "spread", "interp"])}
    walled = "".join("xyz"[k] for k in range(3) if (walls >> k) & 1)
    return {"workload": f"128^3 MAC grid, unit box, {kernel} kernel, "
                        + (f"walled along {walled}" if walled else "periodic")
                        + ", 10^6 uniform points at their initial positions, N(0,1) forces "
                          "and grid velocities",
            "dtype": "f64" if dtype == torch.float64 else "f32", "stage_ms": stage}


def serving_bench(torch, ibops, wl, pool_size=256, warm=200, measured=2000,
                  rhos=(0.5, 0.8, 0.95, 1.2)):
    """The serving mix: independent FP32 jobs on {32,64,96,128}^3 MAC grids with
    log-uniform point counts in [1e3, 1e6] (spread + interpolate each).  mu1 is the
    closed-loop job rate of one job per launch sequence (plan update, spread, interpolate
    through the plan API, jobs back to back); the batched rate submits the same jobs to the
    server at once.  Then open-loop Poisson arrivals at rho * mu1 go to a server with
    batches of one job and to one with batches of up to 128, and the measured jobs' latency
    (scheduled arrival to observed completion) gives p50 / p99."""
    dt = torch.float32
    dev = torch.device("cuda:0")
    sizes = wl.serving_job_sizes(pool_size)
    fields = {N: torch.from_numpy(wl.serving_field(N)).to(dev) for N in sorted({N for N, _ in sizes})}
    pool = []
    for j, (N, n) in enumerate(sizes):
        X, F = wl.serving_job(N, n, j)
        pool.append({"grid": wl.grid(3, N, 1.0), "X": torch.from_numpy(X).to(dev),
                     "F": torch.from_numpy(F).to(dev), "u": fields[N],
                     "f": torch.empty((3, N, N, N), dtype=dt, device=dev),
                     "U": torch.empty((n, 3), dtype=dt, device=dev)})
    pool_pts = sum(n for _, n in sizes)
    stream = torch.cuda.current_stream()

    # closed loop, one job per launch sequence
    plans = [ibops.Plan(jb["grid"], jb["X"].shape[0], dt, dev) for jb in pool]

    def one_pass():
        for p, jb in zip(plans, pool):
            p.update(jb["X"])
            p.spread(jb["F"], jb["f"])
            p.interpolate(jb["u"], jb["U"])
    one_pass()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    one_pass()
    one_pass()
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = e0.elapsed_time(e1) / 1e3
    mu1 = 2 * pool_size / t1
    del plans

    def closed_batched(graph):
        srv = ibops.Server(dt, arena_bytes=16 << 30, max_jobs_per_batch=128, use_graph=graph)
        for jb in pool:
            srv.submit(jb, inputs_ready=True)
        srv.drain()
        c0 = srv.clock_us()
        for _ in range(2):
            for jb in pool:
                srv.submit(jb, inputs_ready=True)
        srv.drain()
        tb = (srv.clock_us() - c0) / 1e6
        st = srv.stats()
        srv.close()
        return 2 * pool_size / tb, st

    muB, stB = closed_batched(False)
    muG, _ = closed_batched(True)

    def closed_by_batch(k, graph):
        """Closed loop with batches of at most k jobs: the pool twice, after one warm pass."""
        srv = ibops.Server(dt, arena_bytes=16 << 30, max_jobs_per_batch=k, use_graph=graph)
        for jb in pool:
            srv.submit(jb, inputs_ready=True)
        srv.drain()
        c0 = srv.clock_us()
        for _ in range(2):
            for jb in pool:
                srv.submit(jb, inputs_ready=True)
        srv.drain()
        tb = (srv.clock_us() - c0) / 1e6
        srv.close()
        return round(2 * pool_size / tb, 1)

    by_batch = {}
    for k in (1, 2, 4, 8, 16, 32, 64, 128):
        by_batch[str(k)] = {"direct_jobs_per_s": closed_by_batch(k, False),
                            "graph_jobs_per_s": closed_by_batch(k, True)}

    def open_loop(max_batch, rate, graph):
        srv = ibops.Server(dt, arena_bytes=16 << 30, max_jobs_per_batch=max_batch, use_graph=graph)
        total = warm + measured
        arr = wl.poisson_arrivals(total, rate)
        start = srv.clock_us() + 2000.0
        tickets, targets = [], []
        for i in range(total):
            target = start + arr[i] * 1e6
            while True:
                now = srv.clock_us()
                if now >= target:
                    break
                if target - now > 400.0:
                    time.sleep((target - now - 300.0) / 1e6)
            tickets.append(srv.submit(pool[i % pool_size], arrival_us=target, inputs_ready=True))
            targets.append(target)
        srv.drain()
        res = [srv.poll(t) for t in tickets]
        st = srv.stats()
        srv.close()
        bad = sum(1 for s_, _ in res if s_ != 0)
        lat = np.array([l for _, l in res[warm:]])
        done = np.array(targets[warm:]) + lat
        span = (done.max() - targets[warm]) / 1e6
        pts = sum(pool[i % pool_size]["X"].shape[0] for i in range(warm, total))
        return {"p50_us": round(float(np.percentile(lat, 50)), 1),
                "p99_us": round(float(np.percentile(lat, 99)), 1),
                "jobs_per_s": round(measured / span, 1), "points_per_s": round(pts / span, 1),
                "mean_batch": round(st["jobs_done"] / max(st["batches"], 1), 2), "errors": bad}

    # one batch of the mix's first 64 jobs (ib_batch_run): the batch tuner's choice for it,
    # and Batch.run with the built-in and the tuned choice, timed interleaved
    from paper_2012_06646_amd import tune
    bjobs = pool[:64]
    best, cand = tune.autotune_batch(bjobs, dt, reps=5, store=False)
    (t_def, _), (t_tuned, _) = tune.time_batch_tunings(bjobs, dt, [None, best], reps=10)
    batch_tuning = {"jobs": len(bjobs), "points": int(sum(jb["X"].shape[0] for jb in bjobs)),
                    "tuning": best, "candidates_ms": cand, "builtin_ms": round(t_def, 4),
                    "tuned_ms": round(t_tuned, 4),
                    "builtin_jobs_per_s": round(len(bjobs) / (t_def / 1e3), 1),
                    "tuned_jobs_per_s": round(len(bjobs) / (t_tuned / 1e3), 1)}
    progress("batch tuning done")

    runs = {}
    for rho in rhos:
        rate = rho * mu1
        runs[str(rho)] = {"arrival_jobs_per_s": round(rate, 1),
                          "one_job_per_launch": open_loop(1, rate, False),
                          "batched": open_loop(128, rate, False),
                          "batched_graph": open_loop(128, rate, True),
                          "batched_default": open_loop(128, rate, None)}
    return {
        "workload": "independent FP32 jobs, N^3 MAC grid with N uniform on {32,64,96,128}, "
                    "n log-uniform in [1e3,1e6] uniform points, spread + interpolate each; "
                    f"pool of {pool_size} distinct jobs (seeds 4000+j) cycled; Poisson arrivals "
                    f"(seed 4008), {warm} warm-up + {measured} measured jobs per load",
        "one_job_per_launch_jobs_per_s": round(mu1, 1),
        "one_job_per_launch_points_per_s": round(mu1 * pool_pts / pool_size, 1),
        "batched_closed_loop_jobs_per_s": round(muB, 1),
        "batched_closed_loop_points_per_s": round(muB * pool_pts / pool_size, 1),
        "batched_closed_loop_mean_batch": round(stB["jobs_done"] / max(stB["batches"], 1), 2),
        "batched_graph_closed_loop_jobs_per_s": round(muG, 1),
        "closed_loop_by_max_batch": by_batch,
        "graph_max_jobs_default": ibops.GRAPH_MAX_JOBS,
        "batch_tuning": batch_tuning,
        "open_loop_by_load": runs,
    }


def progress(msg):
    """One line on stderr per finished part (the JSON line alone goes to stdout)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Achieved HBM bandwidth of a plain device-to-device copy of nbytes (torch's copy
    kernel): bytes read + written over the mean event time of reps copies.  The practical
    ceiling beside the nominal 8 TB/s."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, c
    return {"GB_per_s": round(2 * nbytes / sec / 1e9, 1), "bytes_per_copy": 2 * nbytes,
            "kernel": "torch copy_ of a 1 GiB uint8 buffer", "reps": reps}


def host_facts():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0))}


def c1_bench(torch, ibops, wl, K):
    """The small 2-D case: 32 x 32 collocated grid, two components, 1000 points, FP64.  A
    step is plan update + spread + interpolate; launch-bound at this size."""
    dev = torch.device("cuda:0")
    g, X, F, u = wl.square32_1k()
    Xd, Fd, ud = (torch.from_numpy(a).to(dev) for a in (X, F, u))
    n = X.shape[0]
    p = ibops.Plan(g, n, torch.float64, dev)
    f = torch.empty(p.grid_shape, dtype=torch.float64, device=dev)
    U = torch.empty((n, 2), dtype=torch.float64, device=dev)
    for _ in range(5):
        p.update(Xd)
        p.spread(Fd, f)
        p.interpolate(ud, U)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        p.update(Xd)
        p.spread(Fd, f)
        p.interpolate(ud, U)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    return {"workload": "2-D periodic unit square, 32^2 collocated grid, 2 components, 1000 "
                        "uniform points, FP64; step = plan update + spread + interpolate",
            "ms_per_step": round(ms, 5), "points_per_s": round(n / (ms / 1e3), 1)}


def c2_leg(torch, ibops, wl, dt_name, args, snap_steps):
    """The 128^3 / 10^6 step in one precision: K timed steps (per-stage events), the same
    steps with cold caches, optionally replayed from a HIP graph, and (snap_steps) an
    untimed pass that copies X_k and U_k = J(X_k) u to the host at the given steps."""
    dtype = torch.float64 if dt_name == "f64" else torch.float32
    b = 8 if dt_name == "f64" else 4
    g, X0, F, u = wl.cube128_1m(np.float64, args.npts)
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
    tuning, tune_info = None, None
    if args.tune == "auto":
        from paper_2012_06646_amd import tune
        tuning, tried = tune.autotune(g, X, Fd, ud, reps=5, store=False)
        tune_info = {"chosen": tuning, "candidates_ms": tried}
    plan = ibops.Plan(g, npts, dtype, dev, tuning=tuning)
    stream = torch.cuda.current_stream()

    fresh = [True]

    def replan():
        """The plan of the current positions: from X after a restart, else from the
        positions the last step's interpolate_advect produced (the same plan, with the
        sort reading its input in the previous sorted order)."""
        if fresh[0]:
            plan.update(X)
            fresh[0] = False
        else:
            plan.update_advected()

    def step():
        replan()
        plan.spread(Fd, f)
        plan.interpolate_advect(ud, X, 0.1 * h, U)

    X0d = X.clone()

    def restart():
        """Every timed region starts from the initial positions, so all of them follow the
        same trajectory (the points gather in crowded cells as they are advected)."""
        X.copy_(X0d)
        fresh[0] = True
        torch.cuda.synchronize()

    for _ in range(args.warmup):
        step()
    restart()

    # The timed region: K whole steps, no host synchronisation inside; HIP events between
    # the stages of every step give each stage's average duration over the same region.
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    t_host0 = time.perf_counter()
    for k in range(K):
        e = ev[k]
        e[0].record(stream)
        replan()
        e[1].record(stream)
        plan.spread(Fd, f)
        e[2].record(stream)
        plan.interpolate_advect(ud, X, 0.1 * h, U)
        e[3].record(stream)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host0
    if plan.status() != 0:
        print("bench.py: device flagged a data error", file=sys.stderr)
        sys.exit(1)
    ms_step = ev[0][0].elapsed_time(ev[K - 1][3]) / K
    stage_ms = {name: float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)]))
                for i, name in enumerate(["plan", "spread", "interp_advect"])}
    per_step = np.array([ev[k][0].elapsed_time(ev[k][3]) for k in range(K)])
    step_pct = {f"p{q}": round(float(np.percentile(per_step, q)), 5) for q in (10, 50, 90)}

    # Cold caches: the same steps with 1 GiB streamed through the memory system between them
    # (outside the timed events), so no step finds its data in L2 or the MALL.
    restart()
    flush_src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    flush_dst = torch.empty_like(flush_src)
    cold = []
    for k in range(K):
        flush_dst.copy_(flush_src)
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        step()
        c1.record(stream)
        cold.append((c0, c1))
    torch.cuda.synchronize()
    cold_ms = float(np.mean([a_.elapsed_time(b_) for a_, b_ in cold]))  # same K steps
    del flush_src, flush_dst

    graph_ms = None
    if args.graph:
        # The graph holds one step that re-plans from the positions the previous step
        # advanced (update_advected), so it is captured after one eager step from X_0; the
        # timed replays are steps 1 .. K of the same trajectory.
        restart()
        step()
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(stream)
        with torch.cuda.stream(cap):
            with torch.cuda.graph(gr, stream=cap):
                step()
        stream.wait_stream(cap)
        restart()
        step()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for _ in range(K):
            gr.replay()
        g1.record(stream)
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / K

    snap = None
    if snap_steps:
        restart()
        snap = {}
        for k in range(K):
            Xk = X.cpu().numpy() if k in snap_steps else None
            step()
            if Xk is not None:
                snap[k] = (Xk, U.cpu().numpy())
        torch.cuda.synchronize()

    algo = algorithmic_bytes(npts, dim, ncomp, G, b)
    dom = "spread" if stage_ms["spread"] >= stage_ms["interp_advect"] else "interp_advect"
    dom_bytes = algo["spread"] if dom == "spread" else algo["interp"] + 2 * dim * b * npts
    achieved = dom_bytes / (stage_ms[dom] / 1e3) / 1e9
    traffic = measured_traffic("spread" if dom == "spread" else "interp", dt_name)
    roofline = {"bound": "hbm", "kernel": OP_KERNELS[dom], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "algorithmic_bytes_per_launch": dom_bytes}
    leg = {"dtype": dt_name, "value": npts / (ms_step / 1e3), "ms_per_step": ms_step,
           "ms_per_step_graph": graph_ms, "step_ms_percentiles": step_pct,
           "cold_cache_ms_per_step": round(cold_ms, 5),
           "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()}, "tuning": tune_info,
           "step_algorithmic_bytes": sum(algo.values()),
           "step_hbm_frac": round(sum(algo.values()) / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
           "host_wall_s": round(t_host, 4), "roofline": roofline}
    del plan, X, Fd, ud, f, U, X0d
    torch.cuda.empty_cache()
    return leg, snap


def oracle_at_steps(g, F, u, snap, sample, nrows=2000):
    """The oracle at the positions the GPU produced at steps k (snap: k -> (X_k, U_k) on the
    host): single-thread timing of one step (keys + sort per staggering, spread, interpolate)
    on the first `sample` points of X_k, and the GPU's U_k against the oracle's at nrows
    sampled points (normwise)."""
    from oracle import oracle as orc
    rng = np.random.default_rng(5)
    total_pts, total_s, per = 0, 0.0, {}
    for k, (Xk, Uk) in sorted(snap.items()):
        Xh = Xk.astype(np.float64)
        m = min(sample, Xh.shape[0])
        Xs, Fs = Xh[:m], np.asarray(F[:m], np.float64)
        t0 = time.perf_counter()
        for c in range(len(g["stagger"])):
            kk, _ = orc.keys(g, Xs, g["stagger"][c])
            orc.plan(kk)
        orc.spread(g, Xs, Fs)
        orc.interp(g, Xs, np.asarray(u, np.float64))
        dt = time.perf_counter() - t0
        total_pts += m
        total_s += dt
        rows = rng.choice(Xh.shape[0], min(nrows, Xh.shape[0]), replace=False)
        ref = orc.interp(g, Xh[rows], np.asarray(u, np.float64).astype(Uk.dtype).astype(np.float64))
        err = float(np.abs(Uk[rows] - ref).max() / np.abs(ref).max())
        per[str(k)] = {"oracle_s": round(dt, 3), "points": m, "interp_normwise_err": err}
    return {"steps": per,
            "cpu_baseline": {"value": total_pts / total_s, "unit": "points/s", "cores": 1,
                             "kind": "oracle",
                             "sample": f"first {sample} points of X_k for steps {sorted(snap)} as "
                                       f"the GPU advanced them (one step each: keys + sort per "
                                       f"staggering, spread, interpolate), single thread, "
                                       f"{total_s:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--npts", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample", type=int, default=100_000,
                    help="points per sampled step for the single-thread oracle timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", choices=["auto", "none"], default="auto",
                    help="pick the plan tuning (spreading tile, tile sharing, radix digits) with "
                         "the autotuner on the initial positions, or use the built-in choices")
    ap.add_argument("--no-rbc", action="store_true",
                    help="skip the red-blood-cell workload (256^3, 2.8 million clustered points)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the batched-serving measurement (Poisson job stream)")
    ap.add_argument("--no-unstructured", action="store_true",
                    help="skip the paper's unstructured-point test (Sec. 4.1 grid and weak series)")
    ap.add_argument("--no-walls", action="store_true",
                    help="skip the walled-grid measurement (128^3 with walls along z)")
    ap.add_argument("--no-kernels", action="store_true",
                    help="skip the per-kernel measurements (4-point, cosine, 3-point; 128^3, periodic)")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="also time the step captured once in a HIP graph and replayed")
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
        print(f"bench.py: ibops runs on one GPU per run (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE={world}); multi-GPU sharding is a design note, not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2012_06646_amd import ibops, workloads as wl

    if args.serving_only:
        torch.cuda.set_device(0)
        print(json.dumps({"serving": serving_bench(torch, ibops, wl)}), flush=True)
        return

    dt_other = "f32" if args.dtype == "f64" else "f64"
    snaps = sorted({0, 1, args.steps - 1})
    leg, snap = c2_leg(torch, ibops, wl, args.dtype, args, snaps)
    progress(f"128^3 step {args.dtype}: {leg['ms_per_step']:.4f} ms")
    other, _ = c2_leg(torch, ibops, wl, dt_other, args, None)
    progress(f"128^3 step {dt_other}: {other['ms_per_step']:.4f} ms")
    g, X0, F, u = wl.cube128_1m(np.float64, args.npts)
    npts = X0.shape[0]

    out = {
        "metric": METRIC,
        "value": leg["value"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "128^3 periodic MAC grid (unit cube), 10^6 uniform random points, "
                               "N(0,1) forces and grid velocities, Peskin 4-point; step = plan + "
                               "spread + interpolate with the advection X += 0.1 h U fused in",
                   "grid": [128, 128, 128], "npts": npts, "seed": 1002},
        "roofline": leg["roofline"],
        "cpu_baseline": None,
    }
    out.update({k: v for k, v in leg.items() if k not in ("value", "ms_per_step", "roofline")})
    out["c2_" + dt_other] = other
    out["copy_bandwidth"] = copy_bandwidth(torch)
    out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / out["copy_bandwidth"]["GB_per_s"], 4)
    out["device"] = device_facts(torch)
    out["host"] = host_facts()
    out["c1_2d_32"] = c1_bench(torch, ibops, wl, args.steps)
    progress("copy bandwidth and 2-D 32^2 case done")
    out.update({"cpu_baseline_threads": None, "oracle_at_gpu_steps": None, "rbc_256": None,
                "paper_unstructured": None, "walls_128": None, "kernels_128": None, "serving": None})
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    if not args.no_rbc:
        out["rbc_256"] = rbc_bench(torch, ibops, wl, args.steps)
        progress("rbc 256^3 done")
    if not args.no_unstructured:
        out["paper_unstructured"] = unstructured_bench(torch, ibops, wl, args.steps)
        progress("unstructured test done")
    if not args.no_walls:
        out["walls_128"] = variant_bench(torch, ibops, wl, args.steps, dtype, walls=4)
        progress("walls done")
    if not args.no_kernels:
        out["kernels_128"] = {k: variant_bench(torch, ibops, wl, args.steps, dtype, kernel=k)
                              for k in ("peskin4", "cosine4", "roma3")}
    if not args.no_serving:
        out["serving"] = serving_bench(torch, ibops, wl)
        progress("serving done")
    if not args.no_cpu_baseline:
        out["oracle_at_gpu_steps"] = oracle_at_steps(g, F, u, snap, args.cpu_sample)
        out["cpu_baseline"] = out["oracle_at_gpu_steps"].pop("cpu_baseline")
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        Xh = snap[0][0].astype(np.float64)
        out["cpu_baseline_threads"] = cpu_baseline_threads(g, Xh, F, u, npts, threads)
        progress("oracle timings done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
