"""The C-ABI library: it loads, exports every function include/ib.h declares, and its host
logic (descriptor validation, workspace sizing) behaves as documented.  No device calls."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ib.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ib_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def ib():
    from paper_2012_06646_amd import ibops
    return ibops


def test_library_exports_every_declared_function(ib):
    names = declared_functions()
    assert "ib_spread" in names and "ib_plan_create" in names
    for name in names:
        assert hasattr(ib._lib, name), f"{name} declared in include/ib.h but not exported"
    assert set(ib.EXPORTED) <= set(names)
    # the binding declares every entry point's argument types, so ctypes converts each call
    assert set(ib.EXPORTED) == set(names)
    for name in names:
        assert getattr(ib._lib, name).argtypes is not None, f"{name}: no argtypes in the binding"


def test_status_strings(ib):
    for code in (0, -1, -2, -3, -4, -5, -6, 1):
        assert ib._lib.ib_status_string(code)


def test_workspace_bytes_and_validation(ib):
    from paper_2012_06646_amd import workloads as wl
    import torch
    g = wl.grid(3, 128, 1.0)
    nb = ib.workspace_bytes(g, torch.float64, 10**6)
    # keys, two key/value pairs, run offsets: at least 6 int32 per point per staggering
    assert nb >= 3 * 6 * 4 * 10**6
    assert ib.workspace_bytes(g, torch.float64, 0) > 0
    bad = wl.grid(3, [3, 8, 8], 1.0)  # fewer than 4 cells
    assert ib.workspace_bytes(bad, torch.float64, 10) == 0
    d = ib.make_desc(g)
    h = ctypes.c_void_p()
    # unaligned workspace pointer -> IB_ERR_ARG; too small -> IB_ERR_OOM (no device access)
    assert ib._lib.ib_plan_create(ctypes.byref(d), 0, 100, ctypes.c_void_p(4096 + 8), 1 << 30,
                                  ctypes.byref(h)) == -1
    assert ib._lib.ib_plan_create(ctypes.byref(d), 0, 100, ctypes.c_void_p(4096), 16,
                                  ctypes.byref(h)) == -2
    d.kernel = 7
    assert ib._lib.ib_plan_create(ctypes.byref(d), 0, 100, ctypes.c_void_p(4096), 1 << 30,
                                  ctypes.byref(h)) == -4
    d = ib.make_desc(g)
    d.stagger[0][0] = 1.0  # staggering must lie in [0, 1)
    assert ib._lib.ib_plan_create(ctypes.byref(d), 0, 100, ctypes.c_void_p(4096), 1 << 30,
                                  ctypes.byref(h)) == -1
    d = ib.make_desc(g)
    d.n[0], d.n[1], d.n[2] = 2048, 2048, 1024  # more than 2^31 - 1 cells
    assert ib._lib.ib_plan_create(ctypes.byref(d), 0, 100, ctypes.c_void_p(4096), 1 << 30,
                                  ctypes.byref(h)) == -4


def test_mac_grid_has_three_staggers_collocated_one(ib):
    from paper_2012_06646_amd import workloads as wl
    h = ctypes.c_void_p()
    for g, expect in ((wl.grid(3, 16, 1.0), 3), (wl.grid(2, 16, 1.0, stagger=[[.5, .5], [.5, .5]]), 1)):
        d = ib.make_desc(g)
        nb = ib._lib.ib_plan_workspace_bytes(ctypes.byref(d), 0, 1000)
        # creation touches no device memory, so a fake aligned address is fine here
        assert ib._lib.ib_plan_create(ctypes.byref(d), 0, 1000, ctypes.c_void_p(1 << 20), nb,
                                      ctypes.byref(h)) == 0
        assert ib._lib.ib_plan_num_staggers(h) == expect
        ib._lib.ib_plan_destroy(h)


def test_batch_workspace_sizing_and_validation(ib):
    from paper_2012_06646_amd import workloads as wl
    g3, g2 = ib.make_desc(wl.grid(3, 32, 1.0)), ib.make_desc(wl.grid(2, 32, 1.0))
    arr = (ib.JobDesc * 3)()
    for j in range(3):
        arr[j].grid = g3
        arr[j].npts = 1000 * (j + 1)
        arr[j].X = 4096
        arr[j].F = 4096
        arr[j].f = 4096
    one = ib._lib.ib_plan_workspace_bytes(ctypes.byref(g3), 0, 3000)
    total = ib._lib.ib_batch_workspace_bytes(arr, 3, 0)
    assert total > one  # three plans and the job table
    assert ib._lib.ib_batch_staging_bytes(3) > 0
    assert ib._lib.ib_batch_staging_bytes(0) == 0
    assert ib._lib.ib_batch_staging_bytes(ib.BATCH_MAX_JOBS + 1) == 0
    assert ib._lib.ib_batch_workspace_bytes(arr, 0, 0) == 0
    arr[1].grid = g2  # mixed dimensions are not batched together
    assert ib._lib.ib_batch_workspace_bytes(arr, 3, 0) == 0
    arr[1].grid = g3
    arr[2].F = None  # spreading requested without forces
    assert ib._lib.ib_batch_workspace_bytes(arr, 3, 0) == 0
    arr[2].F = 4096
    # argument errors are found before any device work
    assert ib._lib.ib_batch_run(arr, 3, 0, ctypes.c_void_p(4096 + 8), total, None, None) == -1
    assert ib._lib.ib_batch_run(arr, 3, 0, ctypes.c_void_p(4096), total - 1, None, None) == -2
    assert ib._lib.ib_batch_run(arr, 3, 7, ctypes.c_void_p(4096), total, None, None) == -4


def test_tuned_batch_workspace_and_validation(ib):
    """ib_batch_workspace_bytes_tuned / ib_batch_run_tuned: a NULL or all-default tuning sizes
    the batch like ib_batch_workspace_bytes, a tuning that splits spreading tiles needs more
    room, and a tuning outside its ranges is refused before any device work."""
    from paper_2012_06646_amd import workloads as wl
    g3 = ib.make_desc(wl.grid(3, 32, 1.0))
    arr = (ib.JobDesc * 3)()
    for j in range(3):
        arr[j].grid = g3
        arr[j].npts = 1000 * (j + 1)
        arr[j].X = arr[j].F = arr[j].f = 4096  # never dereferenced
    base = ib._lib.ib_batch_workspace_bytes(arr, 3, 0)
    assert base > 0
    assert ib._lib.ib_batch_workspace_bytes_tuned(arr, 3, 0, None) == base
    assert ib._lib.ib_batch_workspace_bytes_tuned(arr, 3, 0, ctypes.byref(ib.Tuning(0, 0, 0))) == base
    split = ib._lib.ib_batch_workspace_bytes_tuned(arr, 3, 0, ctypes.byref(ib.Tuning(0, 16, 0)))
    assert split > base  # partial integer tiles of the shared spreading tiles
    for bad in (ib.Tuning(9, 0, 0), ib.Tuning(0, 0, 3), ib.Tuning(0, 0, 11)):  # FP64 sorts use <= 10 bits
        assert ib._lib.ib_batch_workspace_bytes_tuned(arr, 3, 0, ctypes.byref(bad)) == 0
        assert ib._lib.ib_batch_run_tuned(arr, 3, 0, ctypes.byref(bad), ctypes.c_void_p(4096), base,
                                          None, None) == -1
    assert ib._lib.ib_batch_workspace_bytes_tuned(arr, 3, 1, ctypes.byref(ib.Tuning(0, 0, 11))) > 0
    assert ib._lib.ib_batch_run_tuned(arr, 3, 0, ctypes.byref(ib.Tuning(0, 16, 0)), ctypes.c_void_p(4096),
                                      split - 1, None, None) == -2


def test_tuned_workspace_and_validation(ib):
    from paper_2012_06646_amd import workloads as wl
    g = ib.make_desc(wl.grid(3, 32, 1.0))
    T = ib.Tuning
    base = ib._lib.ib_plan_workspace_bytes(ctypes.byref(g), 0, 10**6)
    assert ib._lib.ib_plan_workspace_bytes_tuned(ctypes.byref(g), 0, 10**6, None) == base
    assert ib._lib.ib_plan_workspace_bytes_tuned(ctypes.byref(g), 0, 10**6, ctypes.byref(T(0, 0, 0))) == base
    # a dense point set shares tiles between blocks (partial tiles); never sharing needs less
    assert ib._lib.ib_plan_workspace_bytes_tuned(ctypes.byref(g), 0, 10**6, ctypes.byref(T(0, -1, 0))) < base
    # tile 0 is the built-in shape, 64x8x8, in both precisions
    assert ib._lib.ib_plan_workspace_bytes_tuned(ctypes.byref(g), 0, 10**6, ctypes.byref(T(3, 0, 0))) == base
    base32 = ib._lib.ib_plan_workspace_bytes(ctypes.byref(g), 1, 10**6)
    assert ib._lib.ib_plan_workspace_bytes_tuned(ctypes.byref(g), 1, 10**6, ctypes.byref(T(3, 0, 0))) == base32
    for shape in (1, 2, 3):
        assert ib._lib.ib_plan_workspace_bytes_tuned(ctypes.byref(g), 0, 10**6, ctypes.byref(T(shape, 0, 0))) > 0
    # 2^11 buckets for FP32 plans only (FP64 sorts keep their positions in the scatter's LDS)
    assert ib._lib.ib_plan_workspace_bytes_tuned(ctypes.byref(g), 1, 10**6, ctypes.byref(T(0, 0, 11))) > 0
    assert ib._lib.ib_plan_workspace_bytes_tuned(ctypes.byref(g), 1, 10**6, ctypes.byref(T(0, 0, 12))) == 0
    for bad in (T(4, 0, 0), T(-1, 0, 0), T(0, 0, 3), T(0, 0, 11)):
        assert ib._lib.ib_plan_workspace_bytes_tuned(ctypes.byref(g), 0, 1000, ctypes.byref(bad)) == 0
        h = ctypes.c_void_p()
        assert ib._lib.ib_plan_create_tuned(ctypes.byref(g), 0, 1000, ctypes.byref(bad),
                                            ctypes.c_void_p(4096), 1 << 30, ctypes.byref(h)) == -1


def test_binding_rejects_bad_buffers_before_any_launch(ib):
    """Output and in-place buffers are checked (dtype, device, contiguity, exact shape)
    before the library is called; a host tensor or a wrong shape raises instead of reaching
    a kernel.  Runs on the CPU: the plan object is built without a device workspace."""
    import torch
    g = {"dim": 3, "n": [8, 8, 8], "length": [1.0, 1.0, 1.0],
         "stagger": [[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]]}
    p = object.__new__(ib.Plan)  # no workspace: only the argument checks run
    p.dtype, p.device, p.npts, p.dim, p.ncomp = torch.float64, torch.device("cuda", 0), 10, 3, 3
    p.grid_shape = [3, 8, 8, 8]
    ok_pts = torch.empty(10, 3, dtype=torch.float64)
    with pytest.raises(ValueError):  # host tensor
        p._pts(ok_pts, 3, "U", output=True)
    with pytest.raises(TypeError):  # dtype
        p._pts(ok_pts.float(), 3, "U", output=True)
    meta = torch.empty(10, 4, dtype=torch.float64, device="meta")
    with pytest.raises(ValueError):
        p._pts(meta, 3, "U", output=True)
    with pytest.raises(ValueError):  # grid shape
        p._grid(torch.empty(3, 8, 8, 7, dtype=torch.float64), "f", output=True)
    for bad in ({"X": ok_pts, "U": torch.empty(10, 2, dtype=torch.float64)},
                {"X": torch.empty(10, 2, dtype=torch.float64), "U": ok_pts}):
        with pytest.raises(ValueError):
            ib._point_arrays(g, **bad)


def test_batch_and_server_jobs_reject_host_tensors(ib):
    """Batch jobs and served jobs hand their tensors' pointers to kernels, so a host tensor
    (or any input on the wrong kind of device) raises before anything is allocated or
    launched.  Runs on the CPU."""
    import torch
    g = {"dim": 3, "n": [8, 8, 8], "length": [1.0, 1.0, 1.0],
         "stagger": [[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]]}
    X = torch.rand(10, 3, dtype=torch.float64)
    F = torch.rand(10, 3, dtype=torch.float64)
    u = torch.rand(3, 8, 8, 8, dtype=torch.float64)
    for job in ({"grid": g, "X": X, "F": F}, {"grid": g, "X": X, "u": u}):
        with pytest.raises(ValueError, match="job 0: X"):
            ib.Batch([job], dtype=torch.float64, device="cuda:0")
        with pytest.raises(ValueError, match="X must be a tensor on"):
            ib.job_desc(job, torch.float64)
    meta = torch.empty(10, 3, dtype=torch.float64, device="meta")
    with pytest.raises(ValueError, match="job 0: X"):
        ib.Batch([{"grid": g, "X": meta, "F": F}], dtype=torch.float64, device="cuda:0")
    with pytest.raises(TypeError):
        ib.job_desc({"grid": g, "X": X.numpy()}, torch.float64)


def test_static_batch_refuses_oversize_before_device_work(ib):
    """ib_batch_run_static checks the batch's workspace against IB_STATIC_SCRATCH_BYTES on the
    host and returns IB_ERR_OOM before touching a device (no GPU needed); the size limit in
    the header and the binding agree."""
    import re
    from paper_2012_06646_amd import workloads as wl
    hdr = open(os.path.join(ROOT, "include", "ib.h")).read()
    m = re.search(r"#define IB_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == ib.STATIC_SCRATCH_BYTES
    arr = (ib.JobDesc * 1)()
    arr[0].grid = ib.make_desc(wl.grid(3, 128, 1.0))
    arr[0].npts = 3_000_000
    arr[0].X = arr[0].F = arr[0].f = arr[0].u = arr[0].U = 4096  # never dereferenced
    assert ib._lib.ib_batch_workspace_bytes(arr, 1, 0) > ib.STATIC_SCRATCH_BYTES
    assert ib._lib.ib_batch_run_static(arr, 1, 0, None, None, None) == -2
    assert ib._lib.ib_batch_run_static(arr, 0, 0, None, None, None) == -1  # no jobs
