"""Pins of the oracle's twins against the exact recurrence and closed forms.

The FP64 oracle's two twins serve as arbiters: ``sosfilt_ld`` (x87 long
double) judges FP64 results where FP64 rounding itself exceeds 1e-12, and
``sosfilt_f32arith`` (plain FP32) gives the FP32 floor that the reports and
some tolerances quote.  Agreement with the FP64 oracle cannot show either
property (a long-double twin built in double, or an FP32 twin that
accumulates in double, would agree just as well), so each is pinned here
against something that does not depend on the oracle:

* the exact result of the recurrence in dyadic integer arithmetic
  (``tests/exact_dyadic.py``), and the closed-form impulse response of a
  conjugate pole pair, r^n sin((n+1) theta)/sin(theta) (Section II's
  second-order recurrence), evaluated at 50 digits for the poles of the
  coefficients as rounded to FP64;
* the error of scipy's own single-precision ``sosfilt`` on the same draw.

``sosfilt_batch`` (one host thread per channel) is pinned by closed-form
impulse responses of channels that differ in length and poles, which also
catches channels swapped or cut.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from paper_2607_14054_amd import workloads as W

from exact_dyadic import Exact, exact_cascade


def pole_row(r, theta, b=(1.0, 0.0, 0.0)):
    return [b[0], b[1], b[2], 1.0, -2.0 * r * math.cos(theta), r * r]


def closed_form_impulse(row, n, dps=50):
    """h[k] = rho^k sin((k+1) phi) / sin(phi) for b = (1, 0, 0), with rho and
    phi the pole radius and angle of the row's FP64 coefficients
    (a2 = rho^2, a1 = -2 rho cos(phi)), at dps digits."""
    with mpmath.workdps(dps):
        a1, a2 = mpmath.mpf(row[4]), mpmath.mpf(row[5])
        rho = mpmath.sqrt(a2)
        phi = mpmath.acos(-a1 / (2 * rho))
        s = mpmath.sin(phi)
        return np.array([float(rho ** k * mpmath.sin((k + 1) * phi) / s) for k in range(n)])


# ------------------------------------------------------------ long double

def test_ld_beats_fp64_on_slow_pole_closed_form():
    """r = 0.9995, theta = 0.01 (a nearly double pole at z = 1, where FP64
    direct form loses digits): the FP64 oracle is measurably off the
    closed form and the long-double twin is at least 100x closer."""
    row = pole_row(0.9995, 0.01)
    n = 4000
    x = np.zeros(n)
    x[0] = 1.0
    ref = closed_form_impulse(row, n)
    e64 = oracle.rel_rms(oracle.sosfilt(x, [row]), ref)
    eld = oracle.rel_rms(oracle.sosfilt_ld(x, [row]), ref)
    assert e64 > 2e-14, e64          # the case does exercise FP64 rounding
    assert eld * 100 <= e64, (eld, e64)
    assert eld < 1e-15, eld          # long double rounded to FP64 at the end


def test_ld_beats_fp64_exact_dyadic():
    """The same pole and a three-section cascade of slow poles with random
    input, against the exact recurrence in integer arithmetic."""
    row = pole_row(0.9995, 0.01)
    n = 600
    x = np.zeros(n)
    x[0] = 1.0
    ref = np.array([float(v) for v in exact_cascade(x, [row])])
    e64 = oracle.rel_rms(oracle.sosfilt(x, [row]), ref)
    eld = oracle.rel_rms(oracle.sosfilt_ld(x, [row]), ref)
    assert e64 > 2e-14 and eld * 100 <= e64, (e64, eld)
    # the closed form agrees with the exact recurrence (both pin each other)
    assert oracle.rel_rms(closed_form_impulse(row, n), ref) < 1e-15

    sos = W.make_sos(3, 0.99, 0.9995, 5)
    x = W.make_signal(500, 3, np.float64)
    ref = np.array([float(v) for v in exact_cascade(x, sos)])
    e64 = oracle.rel_rms(oracle.sosfilt(x, sos), ref)
    eld = oracle.rel_rms(oracle.sosfilt_ld(x, sos), ref)
    assert eld * 100 <= e64, (eld, e64)


# ------------------------------------------------------------ FP32 twin

# Sections with short dyadic coefficients (stable: |a2| < 1, |a1| < 1 + a2)
# and small integer inputs: every product and partial sum of the first
# samples has a short mantissa.
DYADIC_SOS = np.array([[1.0, 0.5, 0.25, 1.0, -0.5, 0.25],
                       [0.5, -1.0, 0.5, 1.0, 0.25, 0.125],
                       [2.0, 0.0, -1.0, 1.0, -1.0, 0.5]])


@pytest.mark.parametrize("K", [1, 2, 3])
def test_f32arith_is_exact_where_fp32_is_exact(K):
    """Where every FP32 operation of the recurrence is exact (all
    intermediates of at most 24 significant bits, exponents in range), the
    FP32 twin must equal the exact result and the FP64 oracle bit for bit.
    Pins the twin's recurrence (terms, signs, delays, section order)
    without reference to the oracle."""
    sos = DYADIC_SOS[:K]
    rng = np.random.default_rng(11 + K)
    x_all = rng.integers(-4, 5, size=64).astype(np.float64)
    # the longest prefix on which FP32 arithmetic is exact
    n = 0
    for m in range(1, x_all.size + 1):
        ex = Exact()
        ex.cascade(x_all[:m], sos)
        if ex.max_bits > 24 or ex.min_exp < -126 or ex.max_exp > 127:
            break
        n = m
    assert n >= 6, n   # the case is not vacuous
    x = x_all[:n]
    ref = np.array([float(v) for v in exact_cascade(x, sos)])
    y32 = oracle.sosfilt_f32arith(x.astype(np.float32), sos)
    assert np.array_equal(y32.astype(np.float64), ref)
    assert np.array_equal(oracle.sosfilt(x, sos), ref)


def test_f32arith_error_is_single_precision_error():
    """On draws of the headline cascade shape (K = 8, r in [0.8, 0.98]) the
    FP32 twin's error against the FP64 oracle is that of an independent
    single-precision cascade, scipy.signal.sosfilt on float32 data and
    coefficients (a DF2T evaluation: different rounding, same precision),
    within a factor of 4 either way.  A twin that accumulated in FP64, or
    that filtered with FP64 coefficients and inputs, would be orders of
    magnitude closer and fail; one that rounded to a shorter type would be
    orders of magnitude further."""
    sig = pytest.importorskip("scipy.signal")
    x = W.make_signal(1 << 18, 0, np.float32)
    for seed in range(4):
        sos = W.make_sos(8, 0.8, 0.98, seed)
        ref = oracle.sosfilt(x, sos)
        e_twin = oracle.rel_rms(oracle.sosfilt_f32arith(x, sos), ref)
        ys = sig.sosfilt(sos.astype(np.float32), x)
        assert ys.dtype == np.float32
        e_scipy = oracle.rel_rms(ys, ref)
        assert 0.25 <= e_twin / e_scipy <= 4.0, (seed, e_twin, e_scipy)
        assert e_twin > 1e-7, e_twin   # well above FP64 arithmetic's error


# ------------------------------------------------------------ threaded batch

def test_batch_channels_match_closed_forms():
    """Channels of different lengths, each an impulse through its own pole
    pair: every output matches its own closed form (so no channel is
    swapped, cut or shared between threads), with more channels than
    threads."""
    params = [(0.9, 0.3), (0.5, 2.0), (0.8, 1.0), (0.95, 0.05), (0.7, 2.9), (0.6, 1.5),
              (0.85, 0.7)]
    lengths = [300, 17, 1, 999, 64, 250, 511]
    xs, soss, refs = [], [], []
    for (r, th), n in zip(params, lengths):
        x = np.zeros(n)
        x[0] = 1.0
        xs.append(x)
        soss.append(np.array([pole_row(r, th)]))
        k = np.arange(n)
        refs.append(r ** k * np.sin((k + 1) * th) / math.sin(th))
    ys = oracle.sosfilt_batch(xs, soss, threads=3)
    assert len(ys) == len(xs)
    for y, ref, n in zip(ys, refs, lengths):
        assert y.shape == (n,)
        assert np.max(np.abs(y - ref)) < 1e-13 * max(1.0, float(np.max(np.abs(ref))))
