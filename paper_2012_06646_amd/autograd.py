"""Differentiable spreading and interpolation (torch.autograd.Function wrappers).

Gradients follow from the adjoint pair of Sec. 2 (S and J = S^T with the integration
weights of eqs. (disc-interp), (disc-spread)):

    U = J(X) u:   dL/du = J^T gU = h^d S(X) gU,    dL/dX_j = sum_c gU_{j,c} dU_{j,c}/dX_j
    f = S(X) F:   dL/dF = h^-d J(X) gf,             dL/dX_j = h^-d sum_c F_{j,c} d(J gf)_{j,c}/dX_j

where h^d = prod_k h_k and the position terms use the derivative of the delta kernel
(ib_interpolate_grad).  Every step, the h^(+-d) factors included (the scaled entry
points), runs in libibops kernels; torch only carries tensors.
For L = 1/2 |J(X)u|^2 + <S(X)F, g>_h with <a, b>_h = h^d sum a b, this gives dL/dF = J g and
dL/du = h^d S(J u), i.e. S v in the h-weighted grid inner product.
"""
import math

import torch

from . import ibops


def cell_volume(grid):
    return math.prod(float(grid["length"][k]) / int(grid["n"][k]) for k in range(int(grid["dim"])))


def _plan(grid, X):
    return ibops.Plan(grid, X.shape[0], X.dtype, X.device).update(X.detach().contiguous())


class Interpolate(torch.autograd.Function):
    """U = J(X) u (points x components) from grid values u (components x grid)."""

    @staticmethod
    def forward(ctx, X, u, grid):
        plan = _plan(grid, X)
        u = u.detach().contiguous()
        U = plan.interpolate(u)
        ctx.plan = plan
        ctx.hd = cell_volume(grid)
        ctx.save_for_backward(u)
        return U

    @staticmethod
    def backward(ctx, gU):
        (u,) = ctx.saved_tensors
        plan = ctx.plan
        gU = gU.contiguous()
        dX = du = None
        if ctx.needs_input_grad[1]:
            du = plan.spread(gU, scale=ctx.hd)
        if ctx.needs_input_grad[0]:
            dX = plan.interpolate_grad(u, gU)
        return dX, du, None


class Spread(torch.autograd.Function):
    """f = S(X) F (components x grid) from point forces F (points x components)."""

    @staticmethod
    def forward(ctx, X, F, grid):
        plan = _plan(grid, X)
        F = F.detach().contiguous()
        f = plan.spread(F)
        ctx.plan = plan
        ctx.hd = cell_volume(grid)
        ctx.save_for_backward(F)
        return f

    @staticmethod
    def backward(ctx, gf):
        (F,) = ctx.saved_tensors
        plan = ctx.plan
        gf = gf.contiguous()
        dX = dF = None
        if ctx.needs_input_grad[1]:
            dF = plan.interpolate(gf, scale=1.0 / ctx.hd)
        if ctx.needs_input_grad[0]:
            dX = plan.interpolate_grad(gf, F, scale=1.0 / ctx.hd)
        return dX, dF, None


def interpolate(X, u, grid):
    return Interpolate.apply(X, u, grid)


def spread(X, F, grid):
    return Spread.apply(X, F, grid)
