"""torch.autograd.Function over the cell-solve library.

forward: kappa = exp(log_kappa) per fine element -> every constrained cell
problem of the hierarchy (mch_solve_cells) -> effective tensors A_eff[P, M, M]
(mch_effective_coeffs). backward: the library's adjoint
(mch_effective_coeffs_backward) returns dLoss/dlog(kappa) per fine element.

The library keeps the local solutions of the most recent forward of a plan;
a backward issued after a newer forward on the same plan raises MCH_ESTALE.
"""
from __future__ import annotations

import torch

from . import mch


class HierHomog(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log_kappa: torch.Tensor, label: torch.Tensor, plan: "mch.Plan"):
        kappa = torch.exp(log_kappa.detach()).contiguous().view(-1)
        lab = label.contiguous().view(-1)
        plan.solve_cells(kappa, lab)
        A = torch.empty(plan.P * plan.M * plan.M, dtype=torch.float64, device=kappa.device)
        plan.effective_coeffs(kappa, A)
        ctx.plan = plan
        ctx.generation = plan.generation
        ctx.shape = log_kappa.shape
        # the adjoint kernels read the forward's kappa and labels: keep both
        # arrays alive (and at the addresses the forward used) until backward
        ctx.save_for_backward(kappa, lab)
        return A.view(plan.P, plan.M, plan.M)

    @staticmethod
    def backward(ctx, gA: torch.Tensor):
        kappa, _lab = ctx.saved_tensors
        plan = ctx.plan
        if plan.generation != ctx.generation:
            raise mch.MchError(mch.MCH_ESTALE, "backward after a newer forward on the same plan")
        g = torch.empty_like(kappa)
        plan.effective_coeffs_backward(kappa, gA.contiguous().view(-1), g)
        return g.view(ctx.shape), None, None


def effective_tensors(log_kappa: torch.Tensor, label: torch.Tensor, plan: "mch.Plan") -> torch.Tensor:
    """A_eff[P, M, M] as a differentiable function of per-element log kappa."""
    return HierHomog.apply(log_kappa, label, plan)
