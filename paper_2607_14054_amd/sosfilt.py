"""Python binding of libsosfilt.so (include/sosfilt.h), argument marshalling only.

Every step of the filter runs in the HIP kernels behind the C ABI; this module
only turns numpy arrays and torch tensors into pointers, sizes and a stream.
There is no fallback: if the library is missing, importing the binding's
entry points raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsosfilt.so")

(SOS_OK, SOS_E_ARG, SOS_E_COEF, SOS_E_UNSTABLE, SOS_E_UNSUPPORTED, SOS_E_DEVICE, SOS_E_NOMEM,
 SOS_E_SCRATCH) = range(8)
SOS_STATIC_SCRATCH_BYTES = 16 << 20
SOS_F32, SOS_F64, SOS_F16, SOS_BF16 = 0, 1, 2, 3
SOS_AUTO, SOS_PH, SOS_CR, SOS_PH_DEFERRED, SOS_SCALAR, SOS_BLOCK = 0, 1, 2, 3, 4, 5
SOS_FLAG_HOST_ONLY = 0x1
SOS_FLAG_CARRY_SCAN = 0x2
SOS_FLAG_CARRY_RUNIN = 0x4
_CARRY = {"auto": 0, "scan": SOS_FLAG_CARRY_SCAN, "runin": SOS_FLAG_CARRY_RUNIN}
SOS_FLAG_ADJ_SAVE = 0x8
SOS_FLAG_ADJ_RECOMPUTE = 0x10


def SOS_FLAG_SLICES(s: int) -> int:
    return (int(s) & 7) << 8
_ADJOINT = {"auto": 0, "save": SOS_FLAG_ADJ_SAVE, "recompute": SOS_FLAG_ADJ_RECOMPUTE}
(SOS_TABLE_ROWS, SOS_TABLE_U1, SOS_TABLE_U2, SOS_TABLE_C, SOS_TABLE_PH_POWERS,
 SOS_TABLE_CR_LEVELS, SOS_TABLE_CR_TERMINAL, SOS_TABLE_CR_POWERS, SOS_TABLE_TRANSITION,
 SOS_TABLE_THETA, SOS_TABLE_COUPLING) = range(11)

EXPORTED = ["sos_plan", "sos_plan_destroy", "sos_plan_query", "sos_plan_table", "sos_plan_tile",
            "sos_workspace_size", "sos_filt", "sos_batch_plan", "sos_batch_destroy",
            "sos_batch_query", "sos_batch_replan", "sos_filt_batched", "sos_batch_tune", "sos_backward_workspace_size",
            "sos_filt_backward", "sos_batch_backward_workspace_size", "sos_batch_query_adjoint",
            "sos_filt_backward_batched", "sos_filt_for_backward", "sos_filt_backward_stored",
            "sos_filt_batched_for_backward", "sos_filt_backward_batched_stored", "sos_status_string",
            "sos_filt_static"]

_DTYPES = {"f32": SOS_F32, "f64": SOS_F64, "f16": SOS_F16, "bf16": SOS_BF16,
           np.float32: SOS_F32, np.float64: SOS_F64}
_DTYPE_NAMES = {SOS_F32: "f32", SOS_F64: "f64", SOS_F16: "f16", SOS_BF16: "bf16"}
_SOLVERS = {"auto": SOS_AUTO, "ph": SOS_PH, "cr": SOS_CR, "phd": SOS_PH_DEFERRED, "scalar": SOS_SCALAR,
            "block": SOS_BLOCK}


class SosError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s: %s (status %d)" % (what, status_string(code), code))


class _Opts(ctypes.Structure):
    _fields_ = [("io_dtype", ctypes.c_int32), ("compute_dtype", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("N", ctypes.c_int32), ("L", ctypes.c_int32),
                ("tile_groups", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class _Info(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("N", ctypes.c_int32), ("L", ctypes.c_int32),
                ("io_dtype", ctypes.c_int32), ("compute_dtype", ctypes.c_int32),
                ("b0_factored", ctypes.c_int32), ("warm_samples", ctypes.c_int64),
                ("gain", ctypes.c_double), ("transition_norm_W", ctypes.c_double),
                ("simds", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("block_slices", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("tile_groups", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("max_channels", ctypes.c_int32), ("max_sections", ctypes.c_int32),
                ("max_samples", ctypes.c_int64)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("L", ctypes.c_int32), ("tile_groups", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("seconds", ctypes.c_double)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsosfilt.so is not built (python -m paper_2607_14054_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.sos_plan.argtypes = [ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(_Opts), ctypes.POINTER(vp)]
        L.sos_plan_destroy.argtypes = [vp]
        L.sos_plan_query.argtypes = [vp, ctypes.POINTER(_Info), ctypes.POINTER(ctypes.c_int32)]
        L.sos_plan_table.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(ctypes.c_int32)]
        L.sos_plan_tile.argtypes = [vp, i64]
        L.sos_plan_tile.restype = ctypes.c_int64
        L.sos_workspace_size.argtypes = [vp, i64]
        L.sos_workspace_size.restype = ctypes.c_size_t
        L.sos_filt.argtypes = [vp, vp, vp, i64, vp, vp]
        L.sos_filt_static.argtypes = [vp, vp, vp, i64, vp]
        L.sos_status_string.argtypes = [ctypes.c_int]
        L.sos_status_string.restype = ctypes.c_char_p
        p64 = ctypes.POINTER(ctypes.c_int64)
        L.sos_batch_plan.argtypes = [ctypes.POINTER(vp), i32, p64, p64, ctypes.POINTER(_BatchOpts),
                                     ctypes.POINTER(vp)]
        L.sos_batch_destroy.argtypes = [vp]
        L.sos_batch_replan.argtypes = [vp, ctypes.POINTER(vp), i32, p64, p64, vp]
        L.sos_batch_query.argtypes = [vp, p64, p64, p64, p64, ctypes.POINTER(ctypes.c_int32)]
        L.sos_filt_batched.argtypes = [vp, vp, vp, vp, vp]
        pi32 = ctypes.POINTER(ctypes.c_int32)
        L.sos_batch_tune.argtypes = [ctypes.POINTER(ctypes.POINTER(ctypes.c_double)), pi32, i32, p64, p64,
                                     ctypes.POINTER(_Opts), pi32, i32, pi32, i32, pi32, i32, vp, vp, i32, vp,
                                     ctypes.POINTER(_TuneResult), ctypes.POINTER(_TuneResult)]
        L.sos_backward_workspace_size.argtypes = [vp, i64]
        L.sos_backward_workspace_size.restype = ctypes.c_size_t
        L.sos_filt_backward.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
        L.sos_batch_backward_workspace_size.argtypes = [vp]
        L.sos_batch_backward_workspace_size.restype = ctypes.c_size_t
        L.sos_batch_query_adjoint.argtypes = [vp, p64, p64]
        L.sos_filt_backward_batched.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.sos_filt_for_backward.argtypes = [vp, vp, vp, i64, vp, vp]
        L.sos_filt_backward_stored.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
        L.sos_filt_batched_for_backward.argtypes = [vp, vp, vp, vp, vp]
        L.sos_filt_backward_batched_stored.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        for f in ("sos_plan", "sos_plan_destroy", "sos_plan_query", "sos_plan_table", "sos_filt", "sos_filt_static",
                  "sos_batch_plan", "sos_batch_destroy", "sos_batch_query", "sos_batch_replan",
                  "sos_filt_batched",
                  "sos_batch_tune", "sos_filt_backward", "sos_batch_query_adjoint",
                  "sos_filt_backward_batched", "sos_filt_for_backward", "sos_filt_backward_stored",
                  "sos_filt_batched_for_backward", "sos_filt_backward_batched_stored"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().sos_status_string(int(code)).decode()


def _check(code: int, what: str):
    if code != SOS_OK:
        raise SosError(code, what)


@dataclass
class PlanInfo:
    K: int
    N: int
    L: int
    io_dtype: str
    compute_dtype: str
    b0_factored: bool
    warm_samples: int
    gain: float
    transition_norm_W: float
    solver: list
    simds: int
    waves_per_simd: int
    block_slices: int


class Plan:
    """Owns a sos_plan_t.  sos: [K, 6] rows (b0, b1, b2, a0, a1, a2).
    carry: "auto" (the library picks the run-in or the exact scan per call),
    "scan" or "runin".  adjoint: "auto", "save" (every section's output kept
    for the backward pass) or "recompute" (group checkpoints, section inputs
    recomputed)."""

    def __init__(self, sos, io_dtype="f32", compute_dtype="f64", solver="auto", N=0,
                 tile_groups=0, host_only=False, carry="auto", adjoint="auto", slices=0, L=16):
        s = np.ascontiguousarray(np.asarray(sos, dtype=np.float64))
        if s.ndim != 2 or s.shape[1] != 6:
            raise ValueError("sos must be [K, 6]")
        o = _Opts(_DTYPES[io_dtype], _DTYPES[compute_dtype], _SOLVERS[solver], int(N), int(L),
                  int(tile_groups),
                  (SOS_FLAG_HOST_ONLY if host_only else 0) | _CARRY[carry] | _ADJOINT[adjoint]
                  | SOS_FLAG_SLICES(slices))
        h = ctypes.c_void_p()
        _check(lib().sos_plan(s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), s.shape[0],
                              ctypes.byref(o), ctypes.byref(h)), "sos_plan")
        self._h = h
        self.K = s.shape[0]
        self.host_only = bool(host_only)
        self._sos = s
        self.io_dtype = io_dtype if isinstance(io_dtype, str) else ("f32" if io_dtype == np.float32 else "f64")

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sos_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> PlanInfo:
        inf = _Info()
        sol = (ctypes.c_int32 * self.K)()
        _check(lib().sos_plan_query(self._h, ctypes.byref(inf), sol), "sos_plan_query")
        names = {SOS_PH: "ph", SOS_CR: "cr", SOS_PH_DEFERRED: "phd", SOS_SCALAR: "scalar", SOS_BLOCK: "block"}
        return PlanInfo(inf.K, inf.N, inf.L, _DTYPE_NAMES[inf.io_dtype],
                        _DTYPE_NAMES[inf.compute_dtype], bool(inf.b0_factored),
                        int(inf.warm_samples), float(inf.gain), float(inf.transition_norm_W),
                        [names[int(v)] for v in sol], int(inf.simds), int(inf.waves_per_simd),
                        int(inf.block_slices))

    def table(self, which: int, section: int = 0) -> np.ndarray:
        size = ctypes.c_int32()
        _check(lib().sos_plan_table(self._h, which, section, None, 0, ctypes.byref(size)), "sos_plan_table")
        out = np.zeros(size.value, dtype=np.float64)
        _check(lib().sos_plan_table(self._h, which, section,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    size.value, None), "sos_plan_table")
        return out

    def tile(self, n: int) -> int:
        """Samples per tile sos_filt uses for n samples."""
        return int(lib().sos_plan_tile(self._h, int(n)))

    def workspace_size(self, n: int) -> int:
        return int(lib().sos_workspace_size(self._h, int(n)))

    def backward_workspace_size(self, n: int) -> int:
        return int(lib().sos_backward_workspace_size(self._h, int(n)))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on(stream):
    """Context in which the binding allocates what a launch on `stream`
    uses: the caching allocator then ties those blocks to that stream, so it
    does not hand them out again while the launch may still run."""
    import torch
    return torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream())


def filt(plan: Plan, x, y=None, stream=None):
    """y = cascade(x) for a 1-D CUDA (HIP) tensor x of the plan's io dtype."""
    import torch
    want = torch.float32 if plan.io_dtype == "f32" else torch.float64
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == want and x.dim() == 1):
        raise ValueError("x must be a 1-D device tensor of dtype %s" % want)
    x = x.contiguous()
    if y is None:
        with _on(stream):
            y = torch.empty_like(x)
    if not (y.is_cuda and y.dtype == want and y.shape == x.shape and y.is_contiguous()):
        raise ValueError("y must be a contiguous device tensor like x")
    n = x.numel()
    ws = plan.workspace_size(n)
    # the temporary workspace belongs to the launch stream: allocated there,
    # the caching allocator does not hand it out again before the kernels
    # enqueued on that stream have run
    with _on(stream):
        wsb = torch.empty(ws, dtype=torch.uint8, device=x.device) if ws else None
    _check(lib().sos_filt(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                          n, ctypes.c_void_p(wsb.data_ptr()) if wsb is not None else None,
                          _stream_ptr(stream)), "sos_filt")
    return y


def filt_static(plan: Plan, x, y, stream=None):
    """sos_filt_static: y = cascade(x) into the caller's y, with the exact
    carry's workspace in the library's static device buffer (nothing is
    allocated).  Raises SosError(SOS_E_SCRATCH) if the call needs more than
    SOS_STATIC_SCRATCH_BYTES."""
    import torch
    want = torch.float32 if plan.io_dtype == "f32" else torch.float64
    for t in (x, y):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == want and t.dim() == 1
                and t.is_contiguous()):
            raise ValueError("x and y must be contiguous 1-D device tensors of dtype %s" % want)
    if y.shape != x.shape:
        raise ValueError("y must have x's shape")
    _check(lib().sos_filt_static(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                 x.numel(), _stream_ptr(stream)), "sos_filt_static")
    return y


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


class Batch:
    """Owns a sos_batch_t: channel c (length lengths[c]) filtered with
    plans[c], at offsets[c] of the concatenated buffers (None: dense)."""

    def __init__(self, plans, lengths, offsets=None, tile_groups=0, host_only=False,
                 max_channels=0, max_samples=0, max_sections=0):
        plans, n, off = self._args(plans, lengths, offsets)
        C = len(plans)
        hs = (ctypes.c_void_p * C)(*[p.handle.value for p in plans])
        o = _BatchOpts(int(tile_groups), SOS_FLAG_HOST_ONLY if host_only else 0, int(max_channels),
                       int(max_sections), int(max_samples))
        h = ctypes.c_void_p()
        _check(lib().sos_batch_plan(hs, C, _i64p(n), _i64p(off) if off is not None else None,
                                    ctypes.byref(o), ctypes.byref(h)), "sos_batch_plan")
        self._h = h
        self._adopt(plans, n)

    @staticmethod
    def _args(plans, lengths, offsets):
        plans = list(plans)
        C = len(plans)
        n = np.ascontiguousarray(np.asarray(lengths, dtype=np.int64))
        if n.shape != (C,):
            raise ValueError("one length per plan")
        off = None
        if offsets is not None:
            off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
            if off.shape != (C,):
                raise ValueError("one offset per plan")
        return plans, n, off

    def _adopt(self, plans, n):
        self.plans = plans              # the batch refers to their device tables
        self.C = len(plans)
        self.lengths = n
        self.io_dtype = plans[0].io_dtype
        q = self.query()
        self.total = q["total"]
        self.offsets = q["offsets"]

    def replan(self, plans, lengths, offsets=None, stream=None):
        """sos_batch_replan: a new channel set in this batch's room; later
        launches must run on `stream` (default: the current stream)."""
        plans, n, off = self._args(plans, lengths, offsets)
        C = len(plans)
        hs = (ctypes.c_void_p * C)(*[p.handle.value for p in plans])
        sp = _stream_ptr(stream) if not self._host_only() else None
        _check(lib().sos_batch_replan(self._h, hs, C, _i64p(n), _i64p(off) if off is not None else None, sp),
               "sos_batch_replan")
        self._adopt(plans, n)

    def _host_only(self):
        return any(getattr(p, "host_only", False) for p in self.plans)

    @property
    def handle(self):
        return self._h

    def query(self) -> dict:
        total, items = ctypes.c_int64(), ctypes.c_int64()
        off = np.zeros(self.C, np.int64)
        tile = np.zeros(self.C, np.int64)
        order = np.zeros(self.C, np.int32)
        _check(lib().sos_batch_query(self._h, ctypes.byref(total), ctypes.byref(items), _i64p(off),
                                     _i64p(tile), order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
               "sos_batch_query")
        return {"total": int(total.value), "items": int(items.value), "offsets": off, "tile": tile,
                "order": order}

    def backward_workspace_size(self) -> int:
        return int(lib().sos_batch_backward_workspace_size(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sos_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def filt_batched(batch: Batch, x, y=None, stream=None):
    """Every channel of a concatenated 1-D device tensor x (batch.total
    samples) through its own cascade; returns y (same layout)."""
    import torch
    want = torch.float32 if batch.io_dtype == "f32" else torch.float64
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == want and x.dim() == 1
            and x.numel() >= batch.total and x.is_contiguous()):
        raise ValueError("x must be a contiguous 1-D device tensor of dtype %s with %d samples"
                         % (want, batch.total))
    if y is None:
        with _on(stream):
            y = torch.zeros_like(x)
    if not (y.is_cuda and y.dtype == want and y.numel() >= batch.total and y.is_contiguous()):
        raise ValueError("y must be a contiguous device tensor like x")
    _check(lib().sos_filt_batched(batch.handle, ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(y.data_ptr()), None, _stream_ptr(stream)),
           "sos_filt_batched")
    return y


def batch_tune(sos_list, lengths, x, y, offsets=None, io_dtype="f32", compute_dtype="f64",
               solver="ph", Ns=(16, 32, 64), Ls=(16,), tiles=(0, 8, 16, 32), reps=3, stream=None):
    """sos_batch_tune: the fastest (N, L, tile_groups) for this batch on the
    given device buffers.  Returns (best, rows) with rows one dict per
    candidate."""
    C = len(sos_list)
    arrs = [np.ascontiguousarray(np.asarray(s, dtype=np.float64)) for s in sos_list]
    ptrs = (ctypes.POINTER(ctypes.c_double) * C)(
        *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs])
    K = np.array([a.shape[0] for a in arrs], dtype=np.int32)
    n = np.ascontiguousarray(np.asarray(lengths, dtype=np.int64))
    off = None if offsets is None else np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    o = _Opts(_DTYPES[io_dtype], _DTYPES[compute_dtype], _SOLVERS[solver], 0, 16, 0, 0)
    Na = np.asarray(Ns, dtype=np.int32)
    La = np.asarray(Ls, dtype=np.int32)
    Ta = np.asarray(tiles, dtype=np.int32)
    res = (_TuneResult * (len(Na) * len(La) * len(Ta)))()
    best = _TuneResult()
    pi32 = ctypes.POINTER(ctypes.c_int32)
    _check(lib().sos_batch_tune(ptrs, K.ctypes.data_as(pi32), C, _i64p(n),
                                _i64p(off) if off is not None else None, ctypes.byref(o),
                                Na.ctypes.data_as(pi32), len(Na), La.ctypes.data_as(pi32), len(La),
                                Ta.ctypes.data_as(pi32), len(Ta),
                                ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), int(reps),
                                _stream_ptr(stream), res, ctypes.byref(best)), "sos_batch_tune")
    rows = [{"N": r.N, "L": r.L, "tile_groups": r.tile_groups, "seconds": r.seconds} for r in res]
    return {"N": best.N, "L": best.L, "tile_groups": best.tile_groups, "seconds": best.seconds}, rows


def filt_backward(plan: Plan, x, gy, gx=None, stream=None):
    """(gx, gsos) for y = cascade(x) and upstream gradient gy: 1-D device
    tensors of the plan's io dtype; gsos is a [K, 6] float64 device tensor
    with respect to the rows (b0, b1, b2, a0, a1, a2)."""
    import torch
    want = torch.float32 if plan.io_dtype == "f32" else torch.float64
    for name, t in (("x", x), ("gy", gy)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == want and t.dim() == 1
                and t.is_contiguous()):
            raise ValueError("%s must be a contiguous 1-D device tensor of dtype %s" % (name, want))
    if gy.shape != x.shape:
        raise ValueError("gy must have the shape of x")
    n = x.numel()
    ws = int(lib().sos_backward_workspace_size(plan.handle, n))
    with _on(stream):
        if gx is None:
            gx = torch.empty_like(x)
        gsos = torch.empty((plan.K, 6), dtype=torch.float64, device=x.device)
        wsb = torch.empty(max(ws, 16), dtype=torch.uint8, device=x.device)
    _check(lib().sos_filt_backward(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                   ctypes.c_void_p(gx.data_ptr()), ctypes.c_void_p(gsos.data_ptr()), n,
                                   ctypes.c_void_p(wsb.data_ptr()), _stream_ptr(stream)), "sos_filt_backward")
    return gx, gsos


def _workspace(given, nbytes, device):
    import torch
    if given is None:
        return torch.empty(max(nbytes, 16), dtype=torch.uint8, device=device)
    if not (given.is_cuda and given.dtype == torch.uint8 and given.is_contiguous() and given.numel() >= nbytes):
        raise ValueError("workspace must be a contiguous uint8 device tensor of at least %d bytes" % nbytes)
    return given


def filt_for_backward(plan: Plan, x, y=None, stream=None, workspace=None):
    """sos_filt_for_backward: (y, workspace) for a training step's forward
    pass; hand the workspace to filt_backward_stored.  workspace: a uint8
    device tensor to reuse (allocated when None)."""
    import torch
    want = torch.float32 if plan.io_dtype == "f32" else torch.float64
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == want and x.dim() == 1 and x.is_contiguous()):
        raise ValueError("x must be a contiguous 1-D device tensor of dtype %s" % want)
    n = x.numel()
    ws = int(lib().sos_backward_workspace_size(plan.handle, n))
    with _on(stream):
        if y is None:
            y = torch.empty_like(x)
        wsb = _workspace(workspace, ws, x.device)
    _check(lib().sos_filt_for_backward(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), n,
                                       ctypes.c_void_p(wsb.data_ptr()), _stream_ptr(stream)), "sos_filt_for_backward")
    return y, wsb


def filt_backward_stored(plan: Plan, x, gy, workspace, gx=None, stream=None):
    """sos_filt_backward_stored: (gx, gsos) from filt_for_backward's
    workspace (same plan and x)."""
    import torch
    want = torch.float32 if plan.io_dtype == "f32" else torch.float64
    for name, t in (("x", x), ("gy", gy)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == want and t.dim() == 1
                and t.is_contiguous()):
            raise ValueError("%s must be a contiguous 1-D device tensor of dtype %s" % (name, want))
    if gy.shape != x.shape:
        raise ValueError("gy must have the shape of x")
    n = x.numel()
    if workspace.numel() < int(lib().sos_backward_workspace_size(plan.handle, n)):
        raise ValueError("workspace is smaller than this plan needs for n samples")
    with _on(stream):
        if gx is None:
            gx = torch.empty_like(x)
        gsos = torch.empty((plan.K, 6), dtype=torch.float64, device=x.device)
    _check(lib().sos_filt_backward_stored(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                          ctypes.c_void_p(gx.data_ptr()), ctypes.c_void_p(gsos.data_ptr()), n,
                                          ctypes.c_void_p(workspace.data_ptr()), _stream_ptr(stream)),
           "sos_filt_backward_stored")
    return gx, gsos


def filt_batched_for_backward(batch: Batch, x, y=None, stream=None, workspace=None):
    """sos_filt_batched_for_backward: (y, workspace) in the batch's layout.
    workspace: a uint8 device tensor to reuse (allocated when None)."""
    import torch
    want = torch.float32 if batch.io_dtype == "f32" else torch.float64
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == want and x.dim() == 1
            and x.is_contiguous() and x.numel() >= batch.total):
        raise ValueError("x must be a contiguous 1-D device tensor of dtype %s with %d samples" % (want, batch.total))
    ws = int(lib().sos_batch_backward_workspace_size(batch.handle))
    with _on(stream):
        if y is None:
            y = torch.zeros_like(x)
        wsb = _workspace(workspace, ws, x.device)
    _check(lib().sos_filt_batched_for_backward(batch.handle, ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(wsb.data_ptr()),
                                               _stream_ptr(stream)), "sos_filt_batched_for_backward")
    return y, wsb


def filt_backward_batched_stored(batch: Batch, x, gy, workspace, gx=None, stream=None):
    """sos_filt_backward_batched_stored: (gx, gsos, first_row) from
    filt_batched_for_backward's workspace."""
    import torch
    want = torch.float32 if batch.io_dtype == "f32" else torch.float64
    for name, t in (("x", x), ("gy", gy)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == want and t.dim() == 1
                and t.is_contiguous() and t.numel() >= batch.total):
            raise ValueError("%s must be a contiguous 1-D device tensor of dtype %s with %d samples"
                             % (name, want, batch.total))
    if workspace.numel() < int(lib().sos_batch_backward_workspace_size(batch.handle)):
        raise ValueError("workspace is smaller than this batch needs")
    rows = ctypes.c_int64()
    first = np.zeros(batch.C, np.int64)
    _check(lib().sos_batch_query_adjoint(batch.handle, ctypes.byref(rows), _i64p(first)), "sos_batch_query_adjoint")
    with _on(stream):
        if gx is None:
            gx = torch.zeros_like(x)
        gsos = torch.empty((max(rows.value, 1), 6), dtype=torch.float64, device=x.device)
    _check(lib().sos_filt_backward_batched_stored(batch.handle, ctypes.c_void_p(x.data_ptr()),
                                                  ctypes.c_void_p(gy.data_ptr()), ctypes.c_void_p(gx.data_ptr()),
                                                  ctypes.c_void_p(gsos.data_ptr()),
                                                  ctypes.c_void_p(workspace.data_ptr()), _stream_ptr(stream)),
           "sos_filt_backward_batched_stored")
    return gx, gsos[:rows.value], first


def filt_backward_batched(batch: Batch, x, gy, gx=None, stream=None):
    """(gx, gsos, first_row) for every channel of a device batch: x, gy in
    the batch's concatenated layout; gsos is a [rows, 6] float64 device
    tensor whose rows first_row[c] .. first_row[c] + K_c - 1 belong to
    channel c."""
    import torch
    want = torch.float32 if batch.io_dtype == "f32" else torch.float64
    for name, t in (("x", x), ("gy", gy)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == want and t.dim() == 1
                and t.is_contiguous() and t.numel() >= batch.total):
            raise ValueError("%s must be a contiguous 1-D device tensor of dtype %s with %d samples"
                             % (name, want, batch.total))
    rows = ctypes.c_int64()
    first = np.zeros(batch.C, np.int64)
    _check(lib().sos_batch_query_adjoint(batch.handle, ctypes.byref(rows), _i64p(first)), "sos_batch_query_adjoint")
    ws = int(lib().sos_batch_backward_workspace_size(batch.handle))
    with _on(stream):
        if gx is None:
            gx = torch.zeros_like(x)
        gsos = torch.empty((max(rows.value, 1), 6), dtype=torch.float64, device=x.device)
        wsb = torch.empty(max(ws, 16), dtype=torch.uint8, device=x.device)
    _check(lib().sos_filt_backward_batched(batch.handle, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(gy.data_ptr()), ctypes.c_void_p(gx.data_ptr()),
                                           ctypes.c_void_p(gsos.data_ptr()), ctypes.c_void_p(wsb.data_ptr()),
                                           _stream_ptr(stream)), "sos_filt_backward_batched")
    return gx, gsos[:rows.value], first
