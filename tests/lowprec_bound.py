"""A-priori error bounds of block filtering with FP16 / BF16 Toeplitz products
(test infrastructure; the numbers come from the error model below and the
FP64 oracle, never from the kernel).

Block filtering (Section IV, eq. block_filtering_equation) forms each block
of 16 outputs of a section as y_n = H v_n + (terms from the previous block),
H the lower-triangular Toeplitz matrix of the section's first 16
impulse-response samples h_0..h_15.  Only the product H v_n is formed in the
product type; the rest is FP64, and the last two rows of every block (the
values carried into the next block) are formed in FP64 too.  So a section's
output is its exact output plus a product error e_k in the other rows, and
that error is an input perturbation of every later section.

Per output sample p of section k (v: the section's input; the block holding
p is within 15 samples of it, whatever the block partition):

* one rounding per operand (slices S = 1): H and v (scaled by a power of
  two) are rounded FP64 -> FP32 -> product type (relative error
  eps = u_pt + u_32 + u_pt u_32, plus half the subnormal spacing in
  absolute terms for FP16), the products are exact in FP32 and the 16-term
  sum is rounded in FP32 (at most 2 gamma_16 of the sum of magnitudes, a
  factor 2 over the round-to-nearest bound):
      |e_k[p]| <= (2 eps + eps^2 + 2 gamma_16 (1 + eps)^2) sum_d |h_d| |v[p-d]|
                  + subnormal terms;
* S >= 2 slices of W bits (W = 10 for FP16, 8 for BF16) after a power-of-two
  scale per block: the sums of slice products are exact in FP32, so the
  error is the slices cut off (at most 2 max|h| 2^(-W S) per entry of H and
  2 vmax 2^(-W S) per value of the block, vmax its largest magnitude) and
  the products of order a + b >= S (at most 4.01 (S - 1) 2^(-W S) max|h|
  vmax per term), with t = 2^(-W S):
      |e_k[p]| <= t (2 max|h| sum_{d<16} |v[p-d]| + 2 vmax(p) sum_d |h_d| (1 + 2t)
                     + 16 * 4.01 (S - 1) max|h| vmax(p))
                  + 2^-48 sum_d |h_d| |v[p-d]|   (the FP64 sums of orders),
  vmax(p) the largest |v| within 15 samples of p.

The bound is carried through the cascade: with B_k the bound on the error of
section k's input (B_1 = 0, v_k the exact input from the oracle), section k
sees inputs of magnitude at most |v_k| + B_k, and
    B_{k+1} = |h_k| * B_k + E_k(|v_k| + B_k),
|h_k| * the convolution with the magnitude of section k's whole impulse
response.  The output bound adds the final rounding to the I/O type and the
FP64 arithmetic of the rest of the method (2^-29 of the plain FP32 cascade's
error, the ratio of the two unit roundoffs, times 64).

The l2 form (a second, coarser check on the whole signal; the elementwise
bound is the tighter of the two): ||e||_2 grows by at most
the peak gain max_w |H_k(e^jw)| through section k (Parseval; the sections
are scaled to unit peak gain), so
    L_{k+1} = peak_k L_k + ||E_k||_2.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.signal as sg

import oracle

U32 = 2.0 ** -24
U_PT = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
SLICE_BITS = {"f16": 10, "bf16": 8}
F16_HALF_SUBNORMAL = 2.0 ** -25
F16_MAX = 65504.0


def _impulse(row, n):
    d = np.zeros(n)
    d[0] = 1.0
    return oracle.sosfilt(d, np.asarray(row, dtype=np.float64).reshape(1, 6))


def _decay_length(row, n_max):
    """Samples after which |impulse response| stays below 1e-18 of its peak."""
    a1, a2 = row[4] / row[3], row[5] / row[3]
    r = math.sqrt(max(abs(a2), 1e-300))
    if r <= 0.0 or r >= 1.0:
        return n_max
    return int(min(n_max, 64 + math.ceil(math.log(1e-18) / math.log(r)) * 2))


def _window_max(a, half):
    """max of a over [p - half, p + half]."""
    from scipy.ndimage import maximum_filter1d
    return maximum_filter1d(a, size=2 * half + 1, mode="constant", cval=0.0)


def _peak_gain(row):
    w = np.linspace(0.0, math.pi, 1 << 15)
    z1 = np.exp(-1j * w)
    b0, b1, b2, a0, a1, a2 = row
    return float(np.max(np.abs((b0 + b1 * z1 + b2 * z1 * z1) / (a0 + a1 * z1 + a2 * z1 * z1))))


def _input_scales(sos, n_imp):
    """The S = 1 input scale of each section: the power of two nearest the
    inverse white-noise RMS gain of the sections before it."""
    scales = []
    d = np.zeros(n_imp)
    d[0] = 1.0
    for k in range(sos.shape[0]):
        g = math.sqrt(float(np.sum(d * d)))
        scales.append(2.0 ** -round(math.log2(g)))
        d = oracle.sosfilt(d, sos[k].reshape(1, 6))
    return scales


def _product_error_bound(v_mag, h16, dtype, S, scale):
    """Bound on |e_k| per sample for a section with first taps h16, input
    magnitudes at most v_mag."""
    conv = sg.fftconvolve(v_mag, np.abs(h16))[:v_mag.shape[0]]   # sum_d |h_d| |v[p-d]|
    hmax = float(np.max(np.abs(h16)))
    if S == 1:
        u = U_PT[dtype]
        eps = u + U32 + u * U32
        g16 = 16 * U32 / (1 - 16 * U32)
        E = (2 * eps + eps * eps + 2 * g16 * (1 + eps) ** 2) * conv
        if dtype == "f16":
            # absolute subnormal rounding of the scaled input and of H
            E += F16_HALF_SUBNORMAL / scale * np.sum(np.abs(h16)) * (1 + eps)
            E += F16_HALF_SUBNORMAL * sg.fftconvolve(v_mag, np.ones(16))[:v_mag.shape[0]] * (1 + eps)
        return E
    W = SLICE_BITS[dtype]
    t = 2.0 ** (-W * S)
    vmax = _window_max(v_mag, 15)
    vsum = sg.fftconvolve(v_mag, np.ones(16))[:v_mag.shape[0]]   # sum of |v| over the 16 samples back
    h1 = float(np.sum(np.abs(h16)))
    return t * (2 * hmax * vsum + 2 * vmax * h1 * (1 + 2 * t) + 16 * 4.01 * (S - 1) * hmax * vmax) \
        + 2.0 ** -48 * conv


def error_bounds(x, sos, dtype, S):
    """(elementwise bound, l2 bound) on |y - y_exact| for block filtering of
    x (its values as given) through sos with `dtype` products and S slices,
    and y_exact = oracle.sosfilt(x, sos).  Output rounding to the I/O type
    and the FP64 allowance are not included (see output_allowance)."""
    sos = np.asarray(sos, dtype=np.float64)
    sos = sos / sos[:, 3:4]
    v = np.asarray(x, dtype=np.float64)
    n = v.shape[0]
    B = np.zeros(n)
    L2 = 0.0
    scales = _input_scales(sos, 1 << 16) if S == 1 else [1.0] * sos.shape[0]
    for k in range(sos.shape[0]):
        row = sos[k]
        h16 = _impulse(row, 16)
        E = _product_error_bound(np.abs(v) + B, h16, dtype, S, scales[k])
        if S == 1 and dtype == "f16" and float(np.max(np.abs(v) + B)) * scales[k] >= F16_MAX:
            E = np.full(n, np.inf)   # the scaled input may leave FP16's range: no bound
        hk = np.abs(_impulse(row, _decay_length(row, n)))
        B = sg.fftconvolve(B, hk)[:n] + E
        L2 = _peak_gain(row) * 1.0001 * L2 + float(np.linalg.norm(E))
        v = oracle.sosfilt(v, row.reshape(1, 6))
    return B, L2


def output_allowance(y_exact, x, sos, io_dtype="f32"):
    """Elementwise allowance for the final rounding to the I/O type and the
    FP64 arithmetic of the rest of the method."""
    floor = oracle.rel_rms(oracle.sosfilt_f32arith(np.asarray(x, dtype=np.float32), sos), y_exact)
    rms = float(np.sqrt(np.mean(np.asarray(y_exact) ** 2)))
    u_io = U32 if io_dtype == "f32" else 2.0 ** -53
    return u_io * np.abs(y_exact) + 64 * 2.0 ** -29 * max(floor, 1e-7) * rms
