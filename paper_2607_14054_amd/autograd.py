"""torch.autograd.Function over the C ABI (argument marshalling only).
When a gradient is needed, the forward is sos_filt_for_backward, which
also fills the adjoint's workspace, and the backward sos_filt_backward_stored;
otherwise the forward is sos_filt."""
from __future__ import annotations

import threading
from collections import OrderedDict

import numpy as np
import torch

from . import sosfilt as S

# Plans by (coefficient bytes, I/O dtype, N, solver, device): building one
# computes the host tables and allocates its device tables, which a training
# loop with fixed coefficients should pay once, not every step.  Least
# recently used plans beyond the cap are released.
_PLAN_CACHE_CAP = 64
_plans: "OrderedDict[tuple, S.Plan]" = OrderedDict()
_plans_lock = threading.Lock()


def cached_plan(sos_rows: np.ndarray, io: str, N: int, solver: str, device: torch.device) -> S.Plan:
    """The plan for these rows (float64 [K, 6]) on `device`, built at most once
    while it stays among the _PLAN_CACHE_CAP most recently used."""
    rows = np.ascontiguousarray(sos_rows, dtype=np.float64)
    dev = device.index if device.index is not None else torch.cuda.current_device()
    key = (rows.shape, rows.tobytes(), io, int(N), solver, dev)
    with _plans_lock:
        plan = _plans.get(key)
        if plan is not None:
            _plans.move_to_end(key)
            return plan
    with torch.cuda.device(dev):
        plan = S.Plan(rows, io_dtype=io, compute_dtype="f64", solver=solver, N=N)
    with _plans_lock:
        _plans[key] = plan
        while len(_plans) > _PLAN_CACHE_CAP:
            _plans.popitem(last=False)   # released when no pending backward holds it
    return plan


class SosFilt(torch.autograd.Function):
    """y = cascade(x) for a 1-D device tensor x and a [K, 6] tensor of rows
    (b0, b1, b2, a0, a1, a2); differentiable in both."""

    @staticmethod
    def forward(ctx, x, sos, N=32, solver="auto"):
        io = "f32" if x.dtype == torch.float32 else "f64"
        plan = cached_plan(sos.detach().to("cpu", torch.float64).numpy(), io, N, solver, x.device)
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
