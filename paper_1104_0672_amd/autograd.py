"""torch.autograd binding of the convolution: d/dx through the transposed
ring pipeline (arkcos_convolve_adjoint) and d/d(knots) through the
per-ring-pair Fourier correlation (arkcos_kernel_grad).  Argument marshalling
only; every step runs in libarkcos.so."""
from __future__ import annotations

import weakref

import torch

from .arkcos import Plan


def _apply_knots(plan: Plan, knots: torch.Tensor) -> torch.Tensor:
    """Make the plan hold these knot values; returns the device snapshot the
    plan now uses.  Skipped when the plan already holds the values of this
    very tensor at its current version (no comparison of values, so no host
    synchronisation); otherwise the values are copied on the current stream
    and applied there with arkcos_set_knots_async."""
    src = getattr(plan, "_knots_src", None)
    if src is not None and src[0]() is knots and src[1] == knots._version:
        return plan._knots_applied
    snap = knots.detach().to(device=plan.device, dtype=torch.float64).contiguous().clone()
    plan.set_knots_async(snap)
    plan._knots_applied = snap
    plan._knots_src = (weakref.ref(knots), knots._version)
    return snap


def _restore_knots(plan: Plan, snap: torch.Tensor):
    """Re-apply a forward call's knot snapshot if the plan has moved on."""
    if getattr(plan, "_knots_applied", None) is not snap:
        plan.set_knots_async(snap)
        plan._knots_applied = snap
        plan._knots_src = None


class ArkcosConv(torch.autograd.Function):
    """y = C(knots) x for a spline-profile plan (or a fixed-profile plan when
    knots is None).

    The knot values of each forward call are kept (a 64-double device copy)
    and re-applied in its backward if the plan was given other knots in
    between, so one plan may serve several knot tensors in one graph.

    keep_spectra=True keeps the forward workspace (which holds the extended
    spectra of x) alive until backward, so the knot gradient does not redo the
    ring transforms of x; False recomputes them and frees the memory at once.
    """

    @staticmethod
    def forward(ctx, x, knots, plan: Plan, keep_spectra: bool = True):
        ctx.knots = _apply_knots(plan, knots) if knots is not None else None
        ws = torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8, device=x.device)
        y = plan.convolve(x.contiguous(), ws=ws)
        ctx.plan = plan
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
        if ctx.knots is not None and ctx.needs_input_grad[1]:
            # the gradient is linear in the kernel: it does not read the knots
            gk = plan.kernel_grad(x, gy, ws=ws, reuse_spectra=ctx.keep)
        gx = None
        if ctx.needs_input_grad[0]:
            if ctx.knots is not None:
                _restore_knots(plan, ctx.knots)
            gx = plan.adjoint(gy, ws=ws)
        ctx.ws = None
        return gx, gk, None, None


def convolve(x: torch.Tensor, plan: Plan, knots: torch.Tensor | None = None, keep_spectra: bool = True):
    return ArkcosConv.apply(x, knots, plan, keep_spectra)
