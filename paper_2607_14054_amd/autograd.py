"""torch.autograd.Function over the C ABI: forward sos_filt, backward
sos_filt_backward (argument marshalling only)."""
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
        y = S.filt(plan, xc)
        ctx.plan = plan
        ctx.save_for_backward(xc, sos)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, sos = ctx.saved_tensors
        gx, gsos = S.filt_backward(ctx.plan, x, gy.contiguous())
        gsos = gsos.to(device=sos.device, dtype=sos.dtype)
        return (gx if ctx.needs_input_grad[0] else None,
                gsos if ctx.needs_input_grad[1] else None, None, None)


def sosfilt(x, sos, N: int = 32, solver: str = "auto"):
    """Differentiable cascade: y = sosfilt(x, sos)."""
    if not isinstance(sos, torch.Tensor):
        sos = torch.as_tensor(np.asarray(sos, dtype=np.float64))
    return SosFilt.apply(x, sos, N, solver)
