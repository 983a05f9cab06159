"""Block filtering with low-precision Toeplitz products (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product.
It shares no code with the HIP path.

What is modelled.  Block filtering (Section IV, eq. block_filtering_equation)
maps each block of L samples of a section's input v to its output by

    y_n = H v_n + (response to the last two inputs and outputs before block n),

H the L x L lower-triangular Toeplitz matrix of the section's first L
impulse-response samples.  The precision study runs only the dense product
H v_n at reduced precision; everything else stays FP64.  The rounding points
modelled here (the precision reading of the block-filtering product):

* every entry of H and of v_n is rounded first to FP32, then to the product
  type (FP16: 11 significand bits, BF16: 8), round to nearest even; H in the
  type's own exponent range, v_n with an unbounded exponent (below);
* the products are exact in FP32, and their sum is rounded once to FP32;
* the last two rows of every block (the values that carry into the next
  block) are taken from the FP64 product, so no rounding enters the
  block-to-block recurrence;
* the terms from the previous block's inputs and outputs are FP64.

So the section output is the FP64 output plus, in rows 0..L-3 of every
block, the rounding error of that row's product; that error is not fed back
into the recurrence, but it is the next section's input.

The inputs v_n are rounded with an unbounded exponent: the product's input
is scaled by a power of two to about unit size for white input, such a
scale does not change a rounding that stays in the normal range, and at
unit size FP16's subnormal range (below 6.1e-5) only holds values whose
rounding error is below 3e-8 in absolute terms.  H is not scaled, so its
entries are rounded in the type's own range.

Parity of this model with the plain definition is pinned in the tests: with
no rounding it reproduces ``oracle.sosfilt``; its rounding agrees with
numpy's float16 and torch's bfloat16 conversions; its products agree with a
dense float32 evaluation of the same block system.
"""
from __future__ import annotations

import numpy as np

from . import sosfilt as _sosfilt

# significand bits (with the implicit one) of the product types
SIGNIFICAND_BITS = {"f16": 11, "bf16": 8}


def round_significand(a, bits: int) -> np.ndarray:
    """Round float64 values to `bits` significand bits, nearest even, with an
    unbounded exponent (zeros, infinities and NaNs pass through)."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                      # a = m * 2^e, 0.5 <= |m| < 1
    scaled = np.ldexp(m, bits)              # |scaled| in [2^(bits-1), 2^bits)
    return np.ldexp(np.rint(scaled), e - bits)   # rint rounds half to even


def to_product_type(a, pt: str, bounded: bool = True) -> np.ndarray:
    """The value a reaches in the product type: FP64 -> FP32 -> pt, nearest
    even.  bounded: with the type's own exponent range (FP16 subnormals
    below 6.1e-5, overflow past 65504; BF16 has FP32's range); otherwise with
    an unbounded exponent."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    if bounded and pt == "f16":
        with np.errstate(over="ignore"):
            return f.astype(np.float16).astype(np.float64)
    return round_significand(f.astype(np.float64), SIGNIFICAND_BITS[pt])


def impulse_response(row, L: int) -> np.ndarray:
    """First L samples of one section's impulse response (Section II's
    recurrence applied to a unit impulse, FP64)."""
    d = np.zeros(L)
    d[0] = 1.0
    return _sosfilt(d, np.asarray(row, dtype=np.float64).reshape(1, 6))


def toeplitz_lower(h: np.ndarray) -> np.ndarray:
    """H[m][c] = h[m - c] for c <= m, else 0 (eq. block_filtering_matrices)."""
    L = h.shape[0]
    m = np.arange(L)[:, None] - np.arange(L)[None, :]
    return np.where(m >= 0, h[np.clip(m, 0, L - 1)], 0.0)


def product_error(v: np.ndarray, h: np.ndarray, pt: str, start: int = 0) -> np.ndarray:
    """Rounding error of the low-precision product H v_n, per output sample.

    v: a section's FP64 input; blocks of L = len(h) samples begin at
    `start` + j L for every integer j, samples outside [0, len(v)) read as
    zero.  Rows L-2 and L-1 of every block carry no error."""
    L = h.shape[0]
    n = v.shape[0]
    pad_front = (-start) % L                         # sample 0's row in its block
    total = pad_front + n
    pad_back = (-total) % L
    vb = np.concatenate([np.zeros(pad_front), np.asarray(v, dtype=np.float64), np.zeros(pad_back)])
    V = vb.reshape(-1, L).T                          # column j = block j
    H = toeplitz_lower(h)
    exact = H @ V
    low = (toeplitz_lower(to_product_type(h, pt)) @ to_product_type(V, pt, bounded=False)).astype(np.float32)
    err = low.astype(np.float64) - exact
    err[L - 2:, :] = 0.0
    return err.T.reshape(-1)[pad_front:pad_front + n]


def block_filter_lowprec(x, sos, pt: str, L: int = 16, start: int = 0) -> np.ndarray:
    """Cascade output (FP64) of block filtering with `pt` products.

    x: input (float32 or float64); sos: [K, 6] rows as for ``oracle.sosfilt``
    (each row is normalised by its a0, b0 kept in H); blocks begin at
    `start` + j L in sample coordinates (any integer; the blocks tile the
    whole line, so `start` matters only modulo L)."""
    sos = np.asarray(sos, dtype=np.float64)
    v = np.asarray(x).astype(np.float64)
    for k in range(sos.shape[0]):
        row = sos[k] / sos[k, 3]
        h = impulse_response(row, L)
        y = _sosfilt(v, row.reshape(1, 6))
        v = y + product_error(v, h, pt, start)
    return v
