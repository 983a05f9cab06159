"""torch.autograd.Function over the C ABI (argument marshalling only).
When a gradient is needed, the forward is sos_filt_for_backward, which
also fills the adjoint's workspace, and the backward sos_filt_backward_stored;
otherwise the forward is sos_filt."""
from __future__ import annotations

import numpy as np
import torch

from . import sosfilt as S


class SosFilt(torch.autograd.Function):
    """y = cascade(x) for a 1-D device tensor x and a [K, 6] tensor of rows
    (b0, b1, b2, a0, a1, a2); differentiable in both."""

    @staticmethod
    def forward(ctx, x, sos, N=32, solver="auto"):
        io = "f32" if x.dtype == torch.float32 else "f64"
        plan = S.Plan(sos.detach().to("cpu", torch.float64).numpy(), io_dtype=io, compute_dtype="f64",
                      solver=solver, N=N)
        xc = x.contiguous()
        ctx.plan = plan
        ctx.ws = None
        if any(ctx.needs_input_grad[:2]):
            y, ctx.ws = S.filt_for_backward(plan, xc)
        else:
            y = S.filt(plan, xc)
        ctx.save_for_backward(xc, sos)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, sos = ctx.saved_tensors
        if ctx.ws is not None:
            gx, gsos = S.filt_backward_stored(ctx.plan, x, gy.contiguous(), ctx.ws)
        else:
            gx, gsos = S.filt_backward(ctx.plan, x, gy.contiguous())
        gsos = gsos.to(device=sos.device, dtype=sos.dtype)
        return (gx if ctx.needs_input_grad[0] else None,
                gsos if ctx.needs_input_grad[1] else None, None, None)


def sosfilt(x, sos, N: int = 32, solver: str = "auto"):
    """Differentiable cascade: y = sosfilt(x, sos)."""
    if not isinstance(sos, torch.Tensor):
        sos = torch.as_tensor(np.asarray(sos, dtype=np.float64))
    return SosFilt.apply(x, sos, N, solver)
