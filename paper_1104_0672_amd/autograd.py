"""torch.autograd binding of the convolution: d/dx through the transposed
ring pipeline (arkcos_convolve_adjoint) and d/d(knots) through the
per-ring-pair Fourier correlation (arkcos_kernel_grad).  Argument marshalling
only; every step runs in libarkcos.so."""
from __future__ import annotations

import torch

from .arkcos import Plan


class ArkcosConv(torch.autograd.Function):
    """y = C(knots) x for a spline-profile plan (or a fixed-profile plan when
    knots is None).

    keep_spectra=True keeps the forward workspace (which holds the extended
    spectra of x) alive until backward, so the knot gradient does not redo the
    ring transforms of x; False recomputes them and frees the memory at once.
    """

    @staticmethod
    def forward(ctx, x, knots, plan: Plan, keep_spectra: bool = True):
        if knots is not None:
            plan.set_knots(knots.detach().double().cpu().tolist())
        ws = torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8, device=x.device)
        y = plan.convolve(x.contiguous(), ws=ws)
        ctx.plan = plan
        ctx.has_knots = knots is not None
        ctx.keep = bool(keep_spectra)
        ctx.ws = ws if keep_spectra else None
        ctx.save_for_backward(x)
        return y

    @staticmethod
    def backward(ctx, gy):
        (x,) = ctx.saved_tensors
        plan = ctx.plan
        gy = gy.contiguous()
        ws = ctx.ws if ctx.ws is not None else torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8,
                                                           device=gy.device)
        gk = None
        if ctx.has_knots and ctx.needs_input_grad[1]:
            gk = plan.kernel_grad(x, gy, ws=ws, reuse_spectra=ctx.keep)
        gx = plan.adjoint(gy, ws=ws) if ctx.needs_input_grad[0] else None
        ctx.ws = None
        return gx, gk, None, None


def convolve(x: torch.Tensor, plan: Plan, knots: torch.Tensor | None = None, keep_spectra: bool = True):
    return ArkcosConv.apply(x, knots, plan, keep_spectra)
