"""Pins of the low-precision block-filtering model (oracle/lowprec.py).

The model is checked against things other than itself:
* its rounding against numpy's float16 and torch's bfloat16 conversions, and
  against hand-worked ties;
* on operands that every type represents exactly, against the plain FP64
  cascade (the rounding must then be a no-op);
* on a small case, against a per-sample evaluation of the block system that
  assigns samples to blocks, rounds the product rows in numpy float16 /
  torch bfloat16 and keeps the carried rows in FP64 on its own;
* the size of its error, which must scale with the significand width.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import lowprec as LP
from paper_2607_14054_amd import workloads as W

torch = pytest.importorskip("torch")


def test_round_significand_hand_worked_ties():
    u = 2.0 ** -10                      # FP16 spacing at 1
    got = LP.round_significand(np.array([1 + u / 2, 1 + 3 * u / 2, -(1 + u / 2), 1 + u / 2 + 2 ** -30]), 11)
    assert list(got) == [1.0, 1 + 2 * u, -1.0, 1 + u]
    v = 2.0 ** -7                       # BF16 spacing at 1
    got = LP.round_significand(np.array([1 + v / 2, 1 + 3 * v / 2, 3 * 2.0 ** -140]), 8)
    assert list(got) == [1.0, 1 + 2 * v, 3 * 2.0 ** -140]
    assert LP.round_significand(np.array([0.0]), 11)[0] == 0.0


def test_rounding_matches_numpy_float16_and_torch_bfloat16():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(200000) * np.exp2(rng.uniform(-13, 15, 200000))
    a32 = a.astype(np.float32)
    # FP16, normal range: both the bounded and the unbounded forms
    with np.errstate(over="ignore"):
        ref16 = a32.astype(np.float16).astype(np.float64)
    assert np.isinf(ref16).any() and (np.abs(ref16) < 2.0 ** -14).any()   # both range ends are hit
    normal = (np.abs(ref16) >= 2.0 ** -14) & np.isfinite(ref16)
    assert np.array_equal(LP.to_product_type(a, "f16"), ref16)
    assert np.array_equal(LP.to_product_type(a, "f16", bounded=False)[normal], ref16[normal])
    # BF16 (FP32's exponent range)
    refb = torch.from_numpy(a32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(LP.to_product_type(a, "bf16"), refb)
    assert np.array_equal(LP.to_product_type(a, "bf16", bounded=False), refb)


@pytest.mark.parametrize("pt", ["f16", "bf16"])
def test_exactly_representable_operands_round_to_themselves(pt):
    """h[n] = 2^-n (b = [1, 0, 0], a = [1, -1/2, 0]) and small-integer inputs
    are exact in both types, and every block product is exact in FP32: the
    model must then equal the plain FP64 cascade bit for bit."""
    sos = np.array([[1.0, 0.0, 0.0, 1.0, -0.5, 0.0]] * 2)
    x = np.random.default_rng(1).integers(-8, 9, 1000).astype(np.float64)
    for start in (0, 5, -3):
        got = LP.block_filter_lowprec(x, sos[:1], pt, start=start)
        assert np.array_equal(got, oracle.sosfilt(x, sos[:1]))
    # two sections: the first's output has more bits than the types hold, so
    # the second product does round; only the first section is exact
    got = LP.block_filter_lowprec(x, sos, pt)
    assert not np.array_equal(got, oracle.sosfilt(x, sos))


def _block_system_by_hand(v, row, pt, start, L=16):
    """One section of block filtering, per sample: the carried rows and the
    recurrence in FP64, rows 0..L-3 of each block replaced by the rounded
    product plus the same FP64 boundary response."""
    b0, b1, b2, a0, a1, a2 = row / row[3]
    n = len(v)
    h = np.zeros(L)
    x1 = x2 = y1 = y2 = 0.0
    for i in range(L):                       # impulse response, direct form
        xi = 1.0 if i == 0 else 0.0
        yi = b0 * xi + b1 * x1 + b2 * x2 - a1 * y1 - a2 * y2
        x2, x1, y2, y1 = x1, xi, y1, yi
        h[i] = yi

    def rnd(a):
        a32 = np.asarray(a, dtype=np.float32)
        if pt == "f16":
            return a32.astype(np.float16).astype(np.float32)
        return torch.from_numpy(a32).to(torch.bfloat16).to(torch.float32).numpy()

    y = np.zeros(n)
    x1 = x2 = y1 = y2 = 0.0
    for i in range(n):                       # exact recurrence (FP64)
        y[i] = b0 * v[i] + b1 * x1 + b2 * x2 - a1 * y1 - a2 * y2
        x2, x1, y2, y1 = x1, v[i], y1, y[i]
    out = y.copy()
    b = start % L                            # the first block that holds sample 0
    if b:
        b -= L
    while b < n:
        for m in range(L - 2):
            i = b + m
            if not 0 <= i < n:
                continue
            cols = [c for c in range(m + 1) if 0 <= b + c < n]
            hv = sum(h[m - c] * v[b + c] for c in cols)               # FP64 product
            terms = [np.float32(rnd(h[m - c])) * np.float32(rnd(v[b + c])) for c in cols]
            lo = np.float32(math.fsum(float(t) for t in terms))      # one FP32 rounding
            out[i] = y[i] - hv + float(lo)
        b += L
    return out


@pytest.mark.parametrize("pt", ["f16", "bf16"])
@pytest.mark.parametrize("start", [0, 7, -5])
def test_model_matches_block_system_by_hand(pt, start):
    sos = W.make_sos(1, 0.5, 0.95, 11)
    v = W.make_signal(90, 12, np.float64)
    got = LP.block_filter_lowprec(v, sos, pt, start=start)
    ref = _block_system_by_hand(v, sos[0], pt, start)
    scale = np.sqrt(np.mean(ref ** 2))
    assert np.max(np.abs(got - ref)) < 1e-12 * scale
    # and the rounding did change rows 0..13 (the case is not vacuous)
    assert np.max(np.abs(got - oracle.sosfilt(v, sos))) > 1e-6 * scale


def test_error_scales_with_significand_width():
    """Relative RMS error against the exact cascade: about 2^-p times a
    draw-dependent constant, so BF16 (8 bits) sits 3 bits above FP16 (11)."""
    sos = W.make_sos(4, 0.5, 0.9, 13)
    x = W.make_signal(2 ** 14, 14, np.float32)
    ref = oracle.sosfilt(x, sos)
    e16 = oracle.rel_rms(LP.block_filter_lowprec(x, sos, "f16"), ref)
    e8 = oracle.rel_rms(LP.block_filter_lowprec(x, sos, "bf16"), ref)
    assert 1e-6 < e16 < 1e-2
    assert 4 < e8 / e16 < 16
