"""torch.autograd bridge: G-SP2 density matrix as a differentiable function of
H's stored values.  Forward and backward both run in libgsp2.so; this module
only passes tensors through the C ABI."""
from __future__ import annotations

import torch

from .gsp2 import DeviceCSR, Plan, gsp2_backward, gsp2_density


class GSP2Density(torch.autograd.Function):
    """P_val = gsp2_density(plan, H(H_val), n_occ); dL/dH_val from gsp2_backward
    with the forward run's branch sequence.  H_val: float64 GPU tensor of H's
    stored values (CSR order of `pattern`)."""

    @staticmethod
    def forward(ctx, H_val: torch.Tensor, plan: Plan, pattern: DeviceCSR, n_occ: float, max_iter: int = 60):
        H = DeviceCSR(pattern.n, pattern.row_ptr, pattern.col, H_val.detach().contiguous())
        P_val = torch.empty(plan.nnz_P, dtype=torch.float32, device=H_val.device)
        run = gsp2_density(plan, H, n_occ, P_val, max_iter=max_iter)
        ctx.plan, ctx.H, ctx.alpha = plan, H, list(run["alpha"])
        ctx.run = run
        return P_val

    @staticmethod
    def backward(ctx, dP: torch.Tensor):
        dH, _ = gsp2_backward(ctx.plan, ctx.H, ctx.alpha, dP.detach().float().contiguous())
        return dH, None, None, None, None


def gsp2_density_autograd(H_val, plan, pattern, n_occ, max_iter=60):
    return GSP2Density.apply(H_val, plan, pattern, n_occ, max_iter)
