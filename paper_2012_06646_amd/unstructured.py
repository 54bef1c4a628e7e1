"""The paper's unstructured-point test (Sec. 4.1) as a sequence of library calls.

Points lie at random in the periodic box and hang on Hookean springs from their initial
positions X0.  The fluid is not solved for; the grid velocity u stays fixed.  One time step
does what a fluid solver's step would ask of the two operators (two interpolations and one
spread):

1. interpolate u to the points at X^n and predict X* = X^n + dt U (wrapped);
2. compute the tether forces F = k (X0 - X*);
3. spread F from X* onto the grid (f is not fed back into u, so the points never settle);
4. interpolate u at X^n again and move the points: X^{n+1} = X^n + dt U.

Every arithmetic step runs in the HIP library (plan updates, ``ib_interpolate_advect``,
``ib_tether_force``, ``ib_spread``); this module only allocates and orders the calls.
"""
import torch

from . import ibops
from . import workloads as wl


class TetheredPoints:
    """State of the test: two plans (at X^n and at the predicted X*), the positions, and
    the per-step outputs U (velocity at X^n), F (tether force at X*) and f = S(X*) F."""

    def __init__(self, grid, X0, u, k=wl.UNSTRUCTURED_TETHER, dt=wl.UNSTRUCTURED_DT,
                 device="cuda", tuning=None):
        self.grid = grid
        self.X0 = torch.as_tensor(X0, device=device).contiguous()
        self.dtype = self.X0.dtype
        self.npts = self.X0.shape[0]
        self.u = torch.as_tensor(u, device=device, dtype=self.dtype).contiguous()
        self.k = float(k)
        self.dt = float(dt)
        self.plan = ibops.Plan(grid, self.npts, self.dtype, device, tuning)
        self.plan_star = ibops.Plan(grid, self.npts, self.dtype, device, tuning)
        self.X = self.X0.clone()
        self.Xstar = torch.empty_like(self.X0)
        self.U = torch.empty_like(self.X0)
        self.F = torch.empty_like(self.X0)
        self.f = torch.empty(wl.grid_shape(grid), dtype=self.dtype, device=device)

    def predict(self, stream=None):
        """Plan at X^n; U = J(X^n) u; X* = wrap(X^n + dt U); F = k (X0 - X*)."""
        self.plan.update(self.X, stream)
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            self.Xstar.copy_(self.X)  # the copy is ordered on the same stream as the calls
        self.plan.interpolate_advect(self.u, self.Xstar, self.dt, self.U, stream)
        ibops.tether_force(self.grid, self.X0, self.Xstar, self.k, self.F, stream)

    def spread(self, stream=None):
        """Plan at X*; f = S(X*) F."""
        self.plan_star.update(self.Xstar, stream)
        self.plan_star.spread(self.F, self.f, stream=stream)

    def correct(self, stream=None):
        """U = J(X^n) u again; X^{n+1} = wrap(X^n + dt U)."""
        self.plan.interpolate_advect(self.u, self.X, self.dt, self.U, stream)

    def step(self, stream=None):
        self.predict(stream)
        self.spread(stream)
        self.correct(stream)
