"""Differentiable K(x) u = f solve (adjoint method).

For an objective J(u(x, f)): the adjoint lambda solves K(x) lambda = dJ/du (K is
symmetric), dJ/dx_e = -lambda_e' K_e u_e and dJ/df = lambda.  The backward pass
runs the same MG-PCG for the adjoint and the library's element-sensitivity
kernel; it keeps only x and u (or recomputes u), never Krylov vectors."""
import torch

from .solver import OP_K


class _SolveK(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, f, solver, rtol, maxit, save_u):
        solver.set_density(x.detach())
        u, info = solver.pcg(f.detach(), OP_K, rtol=rtol, maxit=maxit)
        ctx.solver, ctx.rtol, ctx.maxit, ctx.save_u = solver, rtol, maxit, save_u
        ctx.info = info
        if save_u:
            ctx.save_for_backward(x.detach(), f.detach(), u)
        else:
            ctx.save_for_backward(x.detach(), f.detach())
        return u

    @staticmethod
    def backward(ctx, gu):
        solver = ctx.solver
        if ctx.save_u:
            x, f, u = ctx.saved_tensors
            solver.set_density(x)
        else:
            x, f = ctx.saved_tensors
            solver.set_density(x)
            u, _ = solver.pcg(f, OP_K, rtol=ctx.rtol, maxit=ctx.maxit)
        lam, _ = solver.pcg(gu.contiguous(), OP_K, rtol=ctx.rtol, maxit=ctx.maxit)
        gx = solver.element_sens(lam, u, -1.0)
        return gx, lam, None, None, None, None


def solve_K(x, f, solver, rtol=1e-8, maxit=1000, save_u=True):
    """u = K(x)^-1 f, differentiable in x and f."""
    return _SolveK.apply(x, f, solver, rtol, maxit, save_u)
