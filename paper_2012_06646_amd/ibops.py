"""Thin Python binding of libibops.so (the C ABI declared in include/ib.h).

Argument marshalling only: every step of spreading, interpolation and plan construction
runs in the library's HIP kernels.  PyTorch provides device memory and streams.  Importing
this module loads the library and raises ImportError if it has not been built
(``python -m paper_2012_06646_amd.build``); there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibops.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libibops.so not built ({LIB_PATH}); run python -m paper_2012_06646_amd.build")

_lib = ctypes.CDLL(LIB_PATH)

IB_F64, IB_F32 = 0, 1
KERNELS = {"peskin4": 0, "cosine4": 1, "roma3": 2}
STATUS = {0: "IB_OK", -1: "IB_ERR_ARG", -2: "IB_ERR_OOM", -3: "IB_ERR_HIP",
          -4: "IB_ERR_UNSUPPORTED", -5: "IB_ERR_BUSY", -6: "IB_ERR_DEVICE_FLAG", 1: "IB_PENDING"}


class GridDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("length", ctypes.c_double * 3),
                ("ncomp", ctypes.c_int32), ("stagger", (ctypes.c_double * 3) * 3),
                ("kernel", ctypes.c_int32), ("walls", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("spread_tile", ctypes.c_int32), ("split_points", ctypes.c_int32),
                ("radix_bits", ctypes.c_int32)]


def make_tuning(t):
    """ib_tuning from None (defaults) or a dict with any of spread_tile, split_points,
    radix_bits."""
    if t is None:
        return None
    return Tuning(int(t.get("spread_tile", 0)), int(t.get("split_points", 0)), int(t.get("radix_bits", 0)))


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_lib.ib_status_string.restype = ctypes.c_char_p
_lib.ib_status_string.argtypes = [_i32]
_lib.ib_plan_workspace_bytes.restype = ctypes.c_size_t
_lib.ib_plan_workspace_bytes.argtypes = [ctypes.POINTER(GridDesc), _i32, ctypes.c_int64]
_lib.ib_plan_create.restype = _i32
_lib.ib_plan_create.argtypes = [ctypes.POINTER(GridDesc), _i32, ctypes.c_int64, _vp, ctypes.c_size_t,
                                ctypes.POINTER(_vp)]
_lib.ib_plan_workspace_bytes_tuned.restype = ctypes.c_size_t
_lib.ib_plan_workspace_bytes_tuned.argtypes = [ctypes.POINTER(GridDesc), _i32, ctypes.c_int64, ctypes.POINTER(Tuning)]
_lib.ib_plan_create_tuned.restype = _i32
_lib.ib_plan_create_tuned.argtypes = [ctypes.POINTER(GridDesc), _i32, ctypes.c_int64, ctypes.POINTER(Tuning), _vp,
                                      ctypes.c_size_t, ctypes.POINTER(_vp)]
_lib.ib_plan_num_staggers.restype = _i32
_lib.ib_plan_num_staggers.argtypes = [_vp]
_lib.ib_plan_stagger_of.restype = _i32
_lib.ib_plan_stagger_of.argtypes = [_vp, _i32]
_lib.ib_plan_update.restype = _i32
_lib.ib_plan_update.argtypes = [_vp, _vp, _vp]
_lib.ib_plan_update_advected.restype = _i32
_lib.ib_plan_update_advected.argtypes = [_vp, _vp]
_lib.ib_plan_export.restype = _i32
_lib.ib_plan_export.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.ib_plan_status.restype = _i32
_lib.ib_plan_status.argtypes = [_vp]
_lib.ib_plan_destroy.restype = None
_lib.ib_plan_destroy.argtypes = [_vp]
_lib.ib_spread.restype = _i32
_lib.ib_spread.argtypes = [_vp, _vp, _vp, _i32, _vp]
_lib.ib_interpolate.restype = _i32
_lib.ib_interpolate.argtypes = [_vp, _vp, _vp, _vp]

_lib.ib_interpolate_advect.restype = _i32
_lib.ib_interpolate_advect.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double, _vp]
_lib.ib_interpolate_grad.restype = _i32
_lib.ib_interpolate_grad.argtypes = [_vp, _vp, _vp, _vp, _i32, _vp]
_lib.ib_spread_scaled.restype = _i32
_lib.ib_spread_scaled.argtypes = [_vp, _vp, _vp, ctypes.c_double, _i32, _vp]
_lib.ib_interpolate_scaled.restype = _i32
_lib.ib_interpolate_scaled.argtypes = [_vp, _vp, _vp, ctypes.c_double, _vp]
_lib.ib_interpolate_grad_scaled.restype = _i32
_lib.ib_interpolate_grad_scaled.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double, _i32, _vp]
class JobDesc(ctypes.Structure):
    _fields_ = [("grid", GridDesc), ("npts", ctypes.c_int64), ("X", ctypes.c_void_p),
                ("F", ctypes.c_void_p), ("f", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("U", ctypes.c_void_p)]


_lib.ib_batch_workspace_bytes.restype = ctypes.c_size_t
_lib.ib_batch_workspace_bytes.argtypes = [ctypes.POINTER(JobDesc), _i32, _i32]
_lib.ib_batch_staging_bytes.restype = ctypes.c_size_t
_lib.ib_batch_staging_bytes.argtypes = [_i32]
_lib.ib_batch_run.restype = _i32
_lib.ib_batch_run.argtypes = [ctypes.POINTER(JobDesc), _i32, _i32, _vp, ctypes.c_size_t, _vp, _vp]
_lib.ib_batch_workspace_bytes_tuned.restype = ctypes.c_size_t
_lib.ib_batch_workspace_bytes_tuned.argtypes = [ctypes.POINTER(JobDesc), _i32, _i32, ctypes.POINTER(Tuning)]
_lib.ib_batch_run_tuned.restype = _i32
_lib.ib_batch_run_tuned.argtypes = [ctypes.POINTER(JobDesc), _i32, _i32, ctypes.POINTER(Tuning), _vp,
                                    ctypes.c_size_t, _vp, _vp]
_lib.ib_batch_run_static.restype = _i32
_lib.ib_batch_run_static.argtypes = [ctypes.POINTER(JobDesc), _i32, _i32, _vp, _vp, _vp]
_lib.ib_batch_status.restype = _i32
_lib.ib_batch_status.argtypes = [ctypes.POINTER(JobDesc), _i32, _i32, _vp, ctypes.POINTER(_i32), _vp]
class ServerOpts(ctypes.Structure):
    _fields_ = [("dtype", _i32), ("max_jobs_per_batch", _i32), ("max_inflight", _i32),
                ("max_queue", _i32), ("use_graph", _i32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("jobs_done", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("points", ctypes.c_uint64)]


_lib.ib_server_create.restype = _i32
_lib.ib_server_create.argtypes = [ctypes.POINTER(ServerOpts), _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]
_lib.ib_server_clock_us.restype = ctypes.c_double
_lib.ib_server_clock_us.argtypes = [_vp]
_lib.ib_batch_submit.restype = _i32
_lib.ib_batch_submit.argtypes = [_vp, ctypes.POINTER(JobDesc), ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]
_lib.ib_batch_poll.restype = _i32
_lib.ib_batch_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
_lib.ib_server_drain.restype = _i32
_lib.ib_server_drain.argtypes = [_vp]
_lib.ib_server_get_stats.restype = _i32
_lib.ib_server_get_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
_lib.ib_server_destroy.restype = None
_lib.ib_server_destroy.argtypes = [_vp]
_lib.ib_advect.restype = _i32
_lib.ib_advect.argtypes = [ctypes.POINTER(GridDesc), _i32, ctypes.c_int64, _vp, _vp, ctypes.c_double, _vp]
_lib.ib_tether_force.restype = _i32
_lib.ib_tether_force.argtypes = [ctypes.POINTER(GridDesc), _i32, ctypes.c_int64, _vp, _vp, ctypes.c_double, _vp, _vp]

EXPORTED = ["ib_interpolate_advect", "ib_plan_workspace_bytes_tuned", "ib_plan_create_tuned", "ib_server_create", "ib_server_clock_us", "ib_batch_submit", "ib_batch_poll",
            "ib_server_drain", "ib_server_get_stats", "ib_server_destroy", "ib_batch_workspace_bytes", "ib_batch_staging_bytes", "ib_batch_run", "ib_batch_status",
            "ib_batch_workspace_bytes_tuned", "ib_batch_run_tuned",
            "ib_batch_run_static",
            "ib_advect", "ib_tether_force", "ib_interpolate_grad", "ib_status_string", "ib_plan_workspace_bytes", "ib_plan_create", "ib_plan_num_staggers",
            "ib_plan_stagger_of", "ib_plan_update", "ib_plan_update_advected", "ib_plan_export", "ib_plan_status",
            "ib_plan_destroy", "ib_spread", "ib_interpolate", "ib_spread_scaled", "ib_interpolate_scaled",
            "ib_interpolate_grad_scaled"]


class IBError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)} ({_lib.ib_status_string(code).decode()})")


def _check(code, what):
    if code < 0:
        raise IBError(code, what)
    return code


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def make_desc(grid):
    """ib_grid_desc from a grid dict (dim, n, length, stagger, kernel; optional walls: bit k
    set for a non-periodic dimension k)."""
    d = GridDesc()
    d.dim = int(grid["dim"])
    for k in range(3):
        d.n[k] = int(grid["n"][k]) if k < d.dim else 1
        d.length[k] = float(grid["length"][k]) if k < d.dim else 1.0
    d.ncomp = len(grid["stagger"])
    for c, xi in enumerate(grid["stagger"]):
        for k in range(3):
            d.stagger[c][k] = float(xi[k]) if k < d.dim else 0.0
    d.kernel = KERNELS[grid.get("kernel", "peskin4")]
    d.walls = int(grid.get("walls", 0))
    return d


def _dtype_code(dtype):
    if dtype == torch.float64:
        return IB_F64
    if dtype == torch.float32:
        return IB_F32
    raise TypeError(f"unsupported dtype {dtype}")


def workspace_bytes(grid, dtype, npts):
    return int(_lib.ib_plan_workspace_bytes(ctypes.byref(make_desc(grid)), _dtype_code(dtype), int(npts)))


class Plan:
    """Cell keys, stable sort and segments of a point set (Alg. 4 preparation), resident on
    the device.  `update(X)` recomputes them; spread/interpolate use the last update."""

    def __init__(self, grid, npts, dtype=torch.float64, device="cuda", tuning=None):
        """tuning: None (built-in choices), a dict of ib_tuning fields, or "auto" (the
        cached autotuner result for this grid, dtype and point count, if any)."""
        self.grid = grid
        self.desc = make_desc(grid)
        self.npts = int(npts)
        self.dtype = dtype
        self.device = torch.device(device)
        self.dim = self.desc.dim
        self.ncomp = self.desc.ncomp
        if tuning == "auto":
            from . import tune
            tuning = tune.cached(grid, dtype, self.npts)
        self.tuning = tuning
        tz = make_tuning(tuning)
        tp = ctypes.byref(tz) if tz is not None else None
        code = _dtype_code(dtype)
        nbytes = int(_lib.ib_plan_workspace_bytes_tuned(ctypes.byref(self.desc), code, self.npts, tp))
        if nbytes == 0:
            _check(-4, "ib_plan_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(_lib.ib_plan_create_tuned(ctypes.byref(self.desc), code, self.npts, tp,
                                         _ptr(self.workspace), nbytes, ctypes.byref(h)), "ib_plan_create")
        self._h = h
        self.X = None
        self.nstag = _lib.ib_plan_num_staggers(h)
        self.grid_shape = [self.ncomp] + [int(self.desc.n[k]) for k in range(self.dim)][::-1]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:  # the module may be gone at exit
            _lib.ib_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def stagger_of(self, c):
        return _lib.ib_plan_stagger_of(self._h, c)

    def update(self, X, stream=None):
        X = self._pts(X, self.dim, "X")
        _check(_lib.ib_plan_update(self._h, _ptr(X), _stream(stream)), "ib_plan_update")
        self.X = X  # the library references X; keep it alive
        return self

    def update_advected(self, stream=None):
        """Plan of the positions the last interpolate_advect wrote (into its X), sorted from
        the previous order: the same plan as update(X) of those positions."""
        _check(_lib.ib_plan_update_advected(self._h, _stream(stream)), "ib_plan_update_advected")
        return self

    def export(self, stagger_id=0, stream=None):
        n = self.npts
        dev = self.device
        out = dict(keys=torch.empty(n, dtype=torch.int32, device=dev),
                   sorted_keys=torch.empty(n, dtype=torch.int32, device=dev),
                   perm=torch.empty(n, dtype=torch.int32, device=dev),
                   seg_off=torch.empty(n + 1, dtype=torch.int32, device=dev),
                   q=torch.empty(1, dtype=torch.int32, device=dev))
        _check(_lib.ib_plan_export(self._h, stagger_id, _ptr(out["keys"]), _ptr(out["sorted_keys"]),
                                   _ptr(out["perm"]), _ptr(out["seg_off"]), _ptr(out["q"]),
                                   _stream(stream)), "ib_plan_export")
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        q = int(out["q"].item())
        out["q"] = q
        out["seg_off"] = out["seg_off"][: q + 1]
        return out

    def status(self):
        return _lib.ib_plan_status(self._h)

    def _check(self, t, shape, name, output):
        """An input (copied to contiguous memory if need be) or an output / in-place
        buffer (which must already be contiguous: the library writes through its pointer)
        of the plan's dtype, on the plan's device, with exactly this shape."""
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != self.dtype:
            raise TypeError(f"{name} must be {self.dtype}, got {t.dtype}")
        if t.device.type != "cuda" or (self.device.index is not None and t.device.index != self.device.index):
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if output:
            if not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous (it is written in place)")
            return t
        return t.contiguous()

    def _pts(self, t, cols, name, output=False):
        return self._check(t, (self.npts, cols), name, output)

    def _grid(self, t, name, output=False):
        return self._check(t, self.grid_shape, name, output)

    def spread(self, F, f=None, accumulate=False, stream=None, scale=None):
        """f (+)= S(X) F, or scale * S(X) F (ib_spread_scaled) when scale is given."""
        F = self._pts(F, self.ncomp, "F")
        if f is None:
            f = torch.empty(self.grid_shape, dtype=self.dtype, device=self.device)
            accumulate = False
        else:
            f = self._grid(f, "f", output=True)
        if scale is None:
            _check(_lib.ib_spread(self._h, _ptr(F), _ptr(f), int(bool(accumulate)), _stream(stream)),
                   "ib_spread")
        else:
            _check(_lib.ib_spread_scaled(self._h, _ptr(F), _ptr(f), float(scale), int(bool(accumulate)),
                                         _stream(stream)), "ib_spread_scaled")
        return f

    def interpolate_advect(self, u, X, dt, U=None, stream=None):
        """U = J(X) u, then X <- wrap(X + dt U) in place (one pass; same results as
        interpolate followed by advect)."""
        u = self._grid(u, "u")
        X = self._pts(X, self.dim, "X", output=True)
        if U is None:
            U = torch.empty((self.npts, self.ncomp), dtype=self.dtype, device=self.device)
        else:
            U = self._pts(U, self.ncomp, "U", output=True)
        _check(_lib.ib_interpolate_advect(self._h, _ptr(u), _ptr(U), _ptr(X), float(dt), _stream(stream)),
               "ib_interpolate_advect")
        return U

    def interpolate(self, u, U=None, stream=None, scale=None):
        """U = J(X) u, or scale * J(X) u (ib_interpolate_scaled) when scale is given."""
        u = self._grid(u, "u")
        if U is None:
            U = torch.empty((self.npts, self.ncomp), dtype=self.dtype, device=self.device)
        else:
            U = self._pts(U, self.ncomp, "U", output=True)
        if scale is None:
            _check(_lib.ib_interpolate(self._h, _ptr(u), _ptr(U), _stream(stream)), "ib_interpolate")
        else:
            _check(_lib.ib_interpolate_scaled(self._h, _ptr(u), _ptr(U), float(scale), _stream(stream)),
                   "ib_interpolate_scaled")
        return U


def _interp_grad(plan, u, W, dX=None, accumulate=False, stream=None, scale=None):
    """dX (+)= the position gradient of J(X) u against W (times scale when given)."""
    u = plan._grid(u, "u")
    W = plan._pts(W, plan.ncomp, "W")
    if dX is None:
        dX = torch.empty((plan.npts, plan.dim), dtype=plan.dtype, device=plan.device)
        accumulate = False
    else:
        dX = plan._pts(dX, plan.dim, "dX", output=True)
    if scale is None:
        _check(_lib.ib_interpolate_grad(plan._h, _ptr(u), _ptr(W), _ptr(dX), int(bool(accumulate)),
                                        _stream(stream)), "ib_interpolate_grad")
    else:
        _check(_lib.ib_interpolate_grad_scaled(plan._h, _ptr(u), _ptr(W), _ptr(dX), float(scale),
                                               int(bool(accumulate)), _stream(stream)),
               "ib_interpolate_grad_scaled")
    return dX


Plan.interpolate_grad = _interp_grad


def _point_arrays(grid, **arrays):
    """Point arrays of a grid-level call: same dtype (FP64 or FP32), all on one CUDA
    device, contiguous, shape (n, dim) with one n."""
    d = int(grid["dim"])
    n = None
    dev = None
    dtype = None
    for name, t in arrays.items():
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be a CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.dim() != 2 or t.shape[1] != d:
            raise ValueError(f"{name} must have shape (n, {d}), got {tuple(t.shape)}")
        n = t.shape[0] if n is None else n
        dev = t.device if dev is None else dev
        dtype = t.dtype if dtype is None else dtype
        if t.shape[0] != n or t.device != dev or t.dtype != dtype:
            raise ValueError("point arrays must agree in length, device and dtype")
    _dtype_code(dtype)
    return n


def advect(grid, X, U, dt, stream=None):
    """In place: X <- X + dt U, wrapped into the periodic box (IB step position update)."""
    _point_arrays(grid, X=X, U=U)
    _check(_lib.ib_advect(ctypes.byref(make_desc(grid)), _dtype_code(X.dtype), X.shape[0], _ptr(X),
                          _ptr(U), float(dt), _stream(stream)), "ib_advect")
    return X


def tether_force(grid, X0, X, k, F=None, stream=None):
    """F = k (X0 - X), per coordinate to the nearest periodic image: the Hookean tether of the
    unstructured-point test (Sec. 4.1)."""
    if F is None:
        _point_arrays(grid, X0=X0, X=X)
        F = torch.empty_like(X)
    _point_arrays(grid, X0=X0, X=X, F=F)
    _check(_lib.ib_tether_force(ctypes.byref(make_desc(grid)), _dtype_code(X.dtype), X.shape[0],
                                _ptr(X0), _ptr(X), float(k), _ptr(F), _stream(stream)),
           "ib_tether_force")
    return F


def spread(grid, X, F):
    """f = S(X) F on `grid` (convenience: builds a plan)."""
    p = Plan(grid, X.shape[0], X.dtype, X.device).update(X)
    return p.spread(F)


def interpolate(grid, X, u):
    """U = J(X) u on `grid` (convenience: builds a plan)."""
    p = Plan(grid, X.shape[0], X.dtype, X.device).update(X)
    return p.interpolate(u)


BATCH_MAX_JOBS = 128


def _on_device(t, name, device=None):
    """A job tensor must live on the GPU (on `device` when given): the library hands its
    pointer to kernels, so a host tensor would be read by the device."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda" or (device is not None and device.index is not None
                                   and t.device.index != device.index):
        raise ValueError(f"{name} must be a tensor on {device or 'a CUDA device'}, got {t.device}")
STATIC_SCRATCH_BYTES = 64 << 20  # IB_STATIC_SCRATCH_BYTES: largest workspace of run_static


class Batch:
    """Independent spread/interpolate jobs run together, one launch per stage for all jobs
    (ib_batch_run).  Each job is a dict with keys grid, X and optionally F (spread) and u
    (interpolate); all share a dtype, dimension and kernel.  Outputs (f and U per job) and
    the workspace are allocated once; `run()` may be called again after the inputs'
    contents change (same shapes).  workspace=False allocates no workspace: such a batch runs
    only through run_static (the library's fixed device array, ib_batch_run_static).
    tuning: None (built-in choices), a dict of ib_tuning fields applied to every job
    (ib_batch_run_tuned), or "auto" (the autotuner's cached choice for this job mix, if
    any); run_static always uses the built-in choices."""

    def __init__(self, jobs, dtype=torch.float64, device="cuda", workspace=True, tuning=None):
        if not 1 <= len(jobs) <= BATCH_MAX_JOBS:
            raise ValueError(f"a batch holds 1..{BATCH_MAX_JOBS} jobs")
        self.dtype = dtype
        self.device = torch.device(device)
        self.code = _dtype_code(dtype)
        self.jobs = []
        arr = (JobDesc * len(jobs))()
        for j, job in enumerate(jobs):
            g = job["grid"]
            d = make_desc(g)
            X = job["X"]
            for name in ("X", "F", "u"):
                if job.get(name) is not None:
                    _on_device(job[name], f"job {j}: {name}", self.device)
            if X.dtype != dtype or X.dim() != 2 or X.shape[1] != d.dim:
                raise ValueError(f"job {j}: X must be (n, {d.dim}) {dtype}")
            X = X.contiguous()
            n = X.shape[0]
            shape = [d.ncomp] + [int(d.n[k]) for k in range(d.dim)][::-1]
            F = job.get("F")
            u = job.get("u")
            rec = {"grid": g, "X": X, "npts": n, "F": None, "f": None, "u": None, "U": None}
            if F is not None:
                if F.dtype != dtype or tuple(F.shape) != (n, d.ncomp):
                    raise ValueError(f"job {j}: F must be ({n}, {d.ncomp}) {dtype}")
                rec["F"] = F.contiguous()
                rec["f"] = torch.empty(shape, dtype=dtype, device=self.device)
            if u is not None:
                if u.dtype != dtype or list(u.shape) != shape:
                    raise ValueError(f"job {j}: u must be {shape} {dtype}")
                rec["u"] = u.contiguous()
                rec["U"] = torch.empty((n, d.ncomp), dtype=dtype, device=self.device)
            arr[j].grid = d
            arr[j].npts = n
            arr[j].X = X.data_ptr() if n else None
            arr[j].F = rec["F"].data_ptr() if rec["F"] is not None and n else None
            arr[j].f = rec["f"].data_ptr() if rec["f"] is not None else None
            arr[j].u = rec["u"].data_ptr() if rec["u"] is not None else None
            arr[j].U = rec["U"].data_ptr() if rec["U"] is not None and n else None
            self.jobs.append(rec)
        self._arr = arr
        if tuning == "auto":
            from . import tune
            tuning = tune.cached_batch(jobs, dtype)
        self.tuning = tuning
        self._tuning = make_tuning(tuning)
        tp = ctypes.byref(self._tuning) if self._tuning is not None else None
        nbytes = int(_lib.ib_batch_workspace_bytes_tuned(arr, len(jobs), self.code, tp))
        if nbytes == 0:
            _check(-4, "ib_batch_workspace_bytes_tuned")
        self.workspace_bytes = nbytes
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device) if workspace else None
        nst = int(_lib.ib_batch_staging_bytes(len(jobs)))
        self.staging = torch.empty(nst, dtype=torch.uint8, pin_memory=True)

    def run(self, stream=None):
        if self.workspace is None:
            raise ValueError("this batch has no workspace: use run_static")
        tp = ctypes.byref(self._tuning) if self._tuning is not None else None
        _check(_lib.ib_batch_run_tuned(self._arr, len(self.jobs), self.code, tp, _ptr(self.workspace),
                                       self.workspace.numel(), ctypes.c_void_p(self.staging.data_ptr()),
                                       _stream(stream)), "ib_batch_run_tuned")
        return self

    def run_static(self, flags=None, stream=None):
        """Run without a workspace of its own (ib_batch_run_static); flags: None or a device
        int32/uint32 tensor of one word per job, receiving the jobs' device error flags."""
        on_dev = flags is not None and flags.device.type == "cuda" and (
            self.device.index is None or flags.device.index == self.device.index)
        if flags is not None and (not on_dev or flags.numel() < len(self.jobs)
                                  or flags.element_size() != 4 or not flags.is_contiguous()):
            raise ValueError(f"flags must be a contiguous device tensor of {len(self.jobs)} 32-bit words")
        _check(_lib.ib_batch_run_static(self._arr, len(self.jobs), self.code,
                                        ctypes.c_void_p(self.staging.data_ptr()),
                                        None if flags is None else _ptr(flags), _stream(stream)),
               "ib_batch_run_static")
        return self

    def status(self, stream=None):
        if self.workspace is None:
            raise ValueError("this batch has no workspace: read the flags of run_static")
        out = (_i32 * len(self.jobs))()
        r = _lib.ib_batch_status(self._arr, len(self.jobs), self.code, _ptr(self.workspace), out,
                                 _stream(stream))
        if r < 0 and r != -6:
            _check(r, "ib_batch_status")
        return [int(v) for v in out]

    def results(self):
        return [(rec["f"], rec["U"]) for rec in self.jobs]


IB_PENDING = 1


def job_desc(job, dtype):
    """ib_job for a dict with grid, X and optionally F + f (spread) and u + U (interpolate);
    f and U are caller-allocated outputs."""
    d = make_desc(job["grid"])
    X = job["X"]
    for name in ("X", "F", "f", "u", "U"):
        if job.get(name) is not None:
            _on_device(job[name], name)
    n = X.shape[0]
    if X.dtype != dtype or not X.is_contiguous() or X.shape[1] != d.dim:
        raise ValueError(f"X must be a contiguous (n, {d.dim}) {dtype} tensor")
    jd = JobDesc()
    jd.grid = d
    jd.npts = n
    jd.X = X.data_ptr() if n else None
    shape = [d.ncomp] + [int(d.n[k]) for k in range(d.dim)][::-1]
    for name, t, shp in (("F", job.get("F"), (n, d.ncomp)), ("f", job.get("f"), tuple(shape)),
                         ("u", job.get("u"), tuple(shape)), ("U", job.get("U"), (n, d.ncomp))):
        if t is None:
            continue
        if t.dtype != dtype or tuple(t.shape) != shp or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {shp} {dtype} tensor")
        setattr(jd, name, t.data_ptr() if t.numel() else None)
    return jd


# Batches of at most this many jobs replay a captured graph by default; larger ones launch
# their stages directly (graph replay against direct launches, measured per batch size on the
# serving mix of grids 32^3..128^3 with 10^3..10^6 points).
GRAPH_MAX_JOBS = 0


class Server:
    """The serving loop (ib_server_*): submit jobs one at a time, poll their tickets.  The
    device arena (the server's HBM budget) is allocated here with torch and handed over.
    use_graph: False (direct launches), True (every batch replays a captured graph), an int k
    (batches of at most k jobs replay it), or None (GRAPH_MAX_JOBS)."""

    def __init__(self, dtype=torch.float32, arena_bytes=16 << 30, max_jobs_per_batch=BATCH_MAX_JOBS,
                 max_inflight=2, max_queue=1 << 20, use_graph=None, device="cuda"):
        self.dtype = dtype
        self.device = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        if use_graph is None:
            use_graph = GRAPH_MAX_JOBS
        g = -1 if use_graph is True else 0 if use_graph is False else int(use_graph)
        o = ServerOpts(_dtype_code(dtype), int(max_jobs_per_batch), int(max_inflight), int(max_queue), g)
        h = ctypes.c_void_p()
        _check(_lib.ib_server_create(ctypes.byref(o), _ptr(self.arena), self.arena.numel(),
                                     ctypes.byref(h)), "ib_server_create")
        self._h = h
        self._live = {}

    def clock_us(self):
        return _lib.ib_server_clock_us(self._h)

    def submit(self, job, arrival_us=-1.0, inputs_ready=False):
        """Queue a job.  The server reads the job's inputs on its own stream, so they must
        be complete when the job is submitted: unless inputs_ready says they are, the
        caller's current stream is synchronised first (inputs produced by torch kernels
        just before the call are then seen whole)."""
        if not inputs_ready:
            torch.cuda.current_stream(self.device).synchronize()
        jd = job_desc(job, self.dtype)
        t = ctypes.c_uint64()
        _check(_lib.ib_batch_submit(self._h, ctypes.byref(jd), float(arrival_us), ctypes.byref(t)),
               "ib_batch_submit")
        self._live[t.value] = job  # keep the job's tensors alive until it is reported
        return t.value

    def poll(self, ticket):
        """(status, latency_us): status IB_PENDING (1) while unfinished."""
        lat = ctypes.c_double(0.0)
        r = _lib.ib_batch_poll(self._h, ticket, ctypes.byref(lat))
        if r != IB_PENDING:
            self._live.pop(ticket, None)
        return r, lat.value

    def drain(self):
        _check(_lib.ib_server_drain(self._h), "ib_server_drain")

    def stats(self):
        st = ServerStats()
        _check(_lib.ib_server_get_stats(self._h, ctypes.byref(st)), "ib_server_get_stats")
        return {"jobs_done": st.jobs_done, "batches": st.batches, "points": st.points}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:  # the module may be gone at exit
            _lib.ib_server_destroy(h)
            self._h = None
        self._live.clear()

    def __del__(self):
        self.close()
