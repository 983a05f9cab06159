"""FP64 CPU oracle for cascaded-biquad filtering (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never does, and the two share no code.

``liboracle.so`` is compiled from ``sosfilt_oracle.c`` with gcc at
``-O2 -ffp-contract=off`` (every product and sum rounded separately).  It is
built on first use when missing or older than its source.

Functions (each follows Section II's definition of the cascade; see the C
source for the adjoint's derivation from Section III's matrix form):

* ``sosfilt(x, sos, zi=None)``   -> y (float64), optionally (y, zf)
* ``sosfilt_ld(x, sos)``         -> y evaluated in x87 long double
* ``sosfilt_f32arith(x, sos)``   -> y evaluated in plain float32
* ``sosfilt_backward(x, sos, g)``-> (dL/dx, dL/dsos) for L = sum(y * g)
* ``sosfilt_batch(xs, soss)``    -> list of y, channels on host threads

``oracle.method`` takes the method's own steps in FP64, and
``oracle.lowprec`` models block filtering with FP16 / BF16 products.

Pins: ``tests/test_oracle.py`` (the FP64 cascade and its adjoint: closed
forms, frequency response, dense solves, finite differences),
``tests/test_oracle_twins.py`` (``sosfilt_ld`` against the exact recurrence
and 50-digit closed forms where FP64 loses digits; ``sosfilt_f32arith``
bit-exact where FP32 arithmetic is exact, and at scipy's single-precision
error elsewhere; ``sosfilt_batch`` against closed forms per channel),
``tests/test_method_model.py`` and ``tests/test_oracle_lowprec.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sosfilt_oracle.c")
_IMPL = os.path.join(_HERE, "backward_impl.h")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
          "-shared", "-fPIC"]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc; returns its path."""
    stale = (not os.path.exists(_LIB)
             or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_IMPL)))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            fp = ctypes.POINTER(ctypes.c_float)
            i64, i32 = ctypes.c_int64, ctypes.c_int32
            lib.oracle_sosfilt_f64.argtypes = [dp, i64, dp, i32, dp, dp, dp]
            lib.oracle_sosfilt_f32in.argtypes = [fp, i64, dp, i32, dp]
            lib.oracle_sosfilt_ld.argtypes = [dp, i64, dp, i32, dp]
            lib.oracle_sosfilt_f32arith.argtypes = [fp, i64, dp, i32, fp]
            lib.oracle_sosfilt_backward_f64.argtypes = [dp, i64, dp, i32, dp, dp, dp]
            lib.oracle_sosfilt_backward_ld.argtypes = [dp, i64, dp, i32, dp, dp, dp]
            for f in (lib.oracle_sosfilt_f64, lib.oracle_sosfilt_f32in,
                      lib.oracle_sosfilt_ld, lib.oracle_sosfilt_f32arith,
                      lib.oracle_sosfilt_backward_f64, lib.oracle_sosfilt_backward_ld):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _sos(sos) -> np.ndarray:
    s = np.ascontiguousarray(np.asarray(sos, dtype=np.float64))
    if s.ndim != 2 or s.shape[1] != 6 or s.shape[0] < 1:
        raise ValueError("sos must be a [K, 6] array")
    return s


def _check(rc: int):
    if rc != 0:
        raise ValueError("oracle rejected its arguments (code %d)" % rc)


def sosfilt(x, sos, zi=None, return_zf: bool = False):
    """Cascade output in FP64 for FP32 or FP64 input (zero state unless zi)."""
    lib = _load()
    s = _sos(sos)
    K = s.shape[0]
    x = np.asarray(x)
    n = x.shape[0]
    y = np.empty(n, dtype=np.float64)
    if x.dtype == np.float32 and zi is None and not return_zf:
        xc = np.ascontiguousarray(x)
        _check(lib.oracle_sosfilt_f32in(_fptr(xc), n, _dptr(s), K, _dptr(y)))
        return y
    xd = np.ascontiguousarray(x, dtype=np.float64)
    zip_ = None
    if zi is not None:
        zi = np.ascontiguousarray(np.asarray(zi, dtype=np.float64).reshape(K, 4))
        zip_ = _dptr(zi)
    zf = np.empty((K, 4), dtype=np.float64) if return_zf else None
    _check(lib.oracle_sosfilt_f64(_dptr(xd), n, _dptr(s), K, zip_, _dptr(y),
                                  _dptr(zf) if zf is not None else None))
    return (y, zf) if return_zf else y


def sosfilt_ld(x, sos):
    lib = _load()
    s = _sos(sos)
    xd = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(xd)
    _check(lib.oracle_sosfilt_ld(_dptr(xd), xd.shape[0], _dptr(s), s.shape[0], _dptr(y)))
    return y


def sosfilt_f32arith(x, sos):
    lib = _load()
    s = _sos(sos)
    xf = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(xf)
    _check(lib.oracle_sosfilt_f32arith(_fptr(xf), xf.shape[0], _dptr(s), s.shape[0], _fptr(y)))
    return y


def sosfilt_backward(x, sos, gy):
    """(dL/dx, dL/dsos) in FP64 for L = sum(y * gy), zero initial state."""
    lib = _load()
    s = _sos(sos)
    xd = np.ascontiguousarray(x, dtype=np.float64)
    gd = np.ascontiguousarray(gy, dtype=np.float64)
    if gd.shape != xd.shape:
        raise ValueError("gy must have the shape of x")
    gx = np.empty_like(xd)
    gs = np.zeros_like(s)
    _check(lib.oracle_sosfilt_backward_f64(_dptr(xd), xd.shape[0], _dptr(s), s.shape[0],
                                           _dptr(gd), _dptr(gx), _dptr(gs)))
    return gx, gs


def sosfilt_backward_ld(x, sos, gy):
    """The adjoint of sosfilt_backward in x86 extended precision (long
    double), rounded to FP64: the arbiter for FP64 adjoints."""
    lib = _load()
    s = _sos(sos)
    xd = np.ascontiguousarray(x, dtype=np.float64)
    gd = np.ascontiguousarray(gy, dtype=np.float64)
    if gd.shape != xd.shape:
        raise ValueError("gy must have the shape of x")
    gx = np.empty_like(xd)
    gs = np.zeros_like(s)
    _check(lib.oracle_sosfilt_backward_ld(_dptr(xd), xd.shape[0], _dptr(s), s.shape[0],
                                          _dptr(gd), _dptr(gx), _dptr(gs)))
    return gx, gs


def sosfilt_batch(xs, soss, threads: int | None = None):
    """Filter independent channels (list of 1-D arrays, list of [K, 6] rows)
    with ``sosfilt``, one host thread per channel at a time (the C library
    releases the GIL); returns the FP64 outputs in channel order."""
    _load()
    threads = threads or os.cpu_count() or 1
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda a: sosfilt(a[0], a[1]), zip(xs, soss)))


def rel_rms(y, y_ref) -> float:
    """||y - y_ref||_2 / ||y_ref||_2 (both promoted to float64)."""
    y = np.asarray(y, dtype=np.float64)
    r = np.asarray(y_ref, dtype=np.float64)
    den = float(np.sqrt(np.sum(r * r)))
    num = float(np.sqrt(np.sum((y - r) ** 2)))
    return num / den if den > 0 else num


def max_rel(y, y_ref) -> float:
    """max|y - y_ref| / rms(y_ref)."""
    y = np.asarray(y, dtype=np.float64)
    r = np.asarray(y_ref, dtype=np.float64)
    rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
    m = float(np.max(np.abs(y - r))) if r.size else 0.0
    return m / rms if rms > 0 else m
