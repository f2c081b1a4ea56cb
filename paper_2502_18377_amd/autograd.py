"""Differentiable solve: torch.autograd.Function around mpde_solve and
mpde_solve_adjoint (backward pass of Eq. 11).

Forward keeps only the native problem (which stores u*); backward recomputes
the derivative unknowns and duals pointwise from u* (V-cycle checkpointing:
no per-iteration state is kept)."""
import torch

from .api import Problem


class MPDESolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeff, rhs, bc_values, shapes, steps, bc, mset, opts):
        prob = Problem(coeff.detach().contiguous(), rhs.detach().contiguous(),
                       bc_values.detach().contiguous(), shapes, steps, bc, mset, **(opts or {}))
        z, info = prob.solve()
        ctx.prob = prob
        ctx.info = info
        return z

    @staticmethod
    def backward(ctx, g_z):
        gc, gf, gw, _ = ctx.prob.adjoint(g_z.contiguous())
        return gc, gf, gw, None, None, None, None, None


def solve(coeff, rhs, bc_values, shapes, steps, bc, mset, **opts):
    """Differentiable batched solve; returns the concatenated z."""
    return MPDESolve.apply(coeff, rhs, bc_values, shapes, steps, bc, mset, opts)
