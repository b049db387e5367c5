"""Differentiable FMG solve (torch.autograd.Function over the C interface).

Every step of FMG (Fig. 2 of the paper) and of its segmental-refinement form
(Figs. 5-6) is linear in the right-hand side for the linear operator L, so a
solve is a linear map M: f -> u that approximates L^{-1}.  L is self-adjoint,
so the gradient of u = L^{-1} f is grad_f = L^{-1} grad_u, which the backward
computes with the same solver: grad_f = M grad_u.  M itself is not symmetric
(the smoothing order and the transfers differ between the down and the up
leg), so this is the adjoint of the operator the solve approximates, not the
exact transpose of M; the two differ by the solver's algebraic error.

Level checkpoints: with keep_levels the forward also returns each level's
solution right after its FMG stage (the solver's per-level state), recorded
by the library during the same solve.
"""
import torch

from . import fmg


class FMGSolve(torch.autograd.Function):
    """u = FMG(f) with grad_f = FMG(grad_u); plan is an fmg.Plan of f's size."""

    @staticmethod
    def forward(ctx, f, plan, keep_levels):
        f = f.contiguous()
        levels = []
        if keep_levels:
            levels = [torch.empty((n, n, n), dtype=torch.float64, device=f.device)
                      for n in plan.level_edges()]
            plan.set_checkpoints(levels)
        try:
            u = plan.execute(f)
        finally:
            if keep_levels:
                plan.set_checkpoints(None)
        ctx.plan = plan
        ctx.mark_non_differentiable(*levels)
        return (u, *levels)

    @staticmethod
    def backward(ctx, grad_u, *grad_levels):
        grad_f = ctx.plan.execute(grad_u.contiguous())
        return grad_f, None, None


def solve(f, plan, keep_levels=False):
    """Differentiable u = FMG(f) on `plan`; with keep_levels, returns
    (u, [level solutions, coarsest first])."""
    out = FMGSolve.apply(f, plan, keep_levels)
    if keep_levels:
        return out[0], list(out[1:])
    return out[0]
