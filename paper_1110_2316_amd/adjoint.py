"""Differentiable solve u(theta) = X^{-1} b(theta) for the Legendre source
coefficients theta (sem_set_source_legendre), as a torch.autograd.Function.

Forward: source data, b = A^T M d(theta), PCG.  Backward: X is symmetric, so
the adjoint state is one more PCG solve, lambda = X^{-1} dL/du (on a graded
space the projected system, with dL/du projected first), and
dL/dtheta = sem_source_adjoint(lambda).  Every step runs in the library's
kernels; this module only allocates the device vectors and sequences calls.
"""
import torch

from .semlib import SemError


class SourceSolve(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta, ctx, rtol, maxit, precision):
        theta = theta.detach().contiguous()
        ctx.set_source_legendre(theta)
        b = torch.zeros(ctx.ndof, dtype=torch.float64, device=theta.device)
        ctx.rhs(b)
        u = torch.zeros_like(b)
        info = ctx.pcg_solve(b, u, rtol=rtol, maxit=maxit, precision=precision)
        fctx.sem = ctx
        fctx.opts = (rtol, maxit, precision)
        fctx.ntheta = theta.numel()
        fctx.forward_info = info
        return u

    @staticmethod
    def backward(fctx, grad_u):
        ctx = fctx.sem
        rtol, maxit, precision = fctx.opts
        # on a graded space (sem_set_degrees) the solve's right-hand side must
        # lie in it: lambda = (Q X Q)^+ Q dL/du (a no-op when ungraded)
        g = grad_u.detach().clone().contiguous()
        ctx.project(g)
        lam = torch.zeros_like(g)
        if torch.count_nonzero(g) > 0:
            ctx.pcg_solve(g, lam, rtol=rtol, maxit=maxit, precision=precision)
        grad = torch.zeros(fctx.ntheta, dtype=torch.float64, device=g.device)
        ctx.source_adjoint(lam, grad)
        return grad, None, None, None, None


def solve_source(theta, ctx, rtol=1e-12, maxit=100000, precision="fp64"):
    """u(theta), differentiable with respect to theta (float64 device tensor of deg^3)."""
    if theta.dtype != torch.float64 or not theta.is_cuda:
        raise SemError(-1, "theta must be a float64 device tensor")
    return SourceSolve.apply(theta, ctx, rtol, maxit, precision)
