"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
impulse responses of a conjugate pole pair, the frequency response at steady
state, the DC gain, linearity and time invariance, a dense solve of the banded
Toeplitz system of Section III, extended precision, and finite differences for
the adjoint.  A plausible slip in the oracle (a dropped term, a sign, an
index, a wrong a0 division, a swapped section order in the adjoint) fails at
least one of them; ``test_pins_catch_planted_mistakes`` plants such slips in a
copy of the oracle's recurrence and checks that the pins notice.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2607_14054_amd import workloads as W


def pole_section(r, theta, b=(1.0, 0.0, 0.0)):
    return np.array([[b[0], b[1], b[2], 1.0, -2.0 * r * math.cos(theta), r * r]])


@pytest.mark.parametrize("r,theta", [(0.9, 0.3), (0.5, 2.0), (0.99, math.pi / 2), (0.7, 1.0)])
def test_impulse_response_closed_form(r, theta):
    # b = [1, 0, 0]: h[n] = r^n sin((n+1) theta) / sin(theta)
    n = 400
    x = np.zeros(n); x[0] = 1.0
    h = oracle.sosfilt(x, pole_section(r, theta))
    k = np.arange(n)
    ref = r ** k * np.sin((k + 1) * theta) / math.sin(theta)
    assert np.max(np.abs(h - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))
    # b = [0, 1, 0]: one-sample delay, h[n] = r^(n-1) sin(n theta) / sin(theta)
    h1 = oracle.sosfilt(x, pole_section(r, theta, (0.0, 1.0, 0.0)))
    ref1 = np.zeros(n)
    ref1[1:] = r ** (k[1:] - 1) * np.sin(k[1:] * theta) / math.sin(theta)
    assert np.max(np.abs(h1 - ref1)) < 1e-13 * max(1.0, np.max(np.abs(ref1)))


def test_cascade_impulse_is_convolution_of_sections():
    n = 300
    s1, s2 = pole_section(0.8, 0.4), pole_section(0.6, 2.5, (0.3, -0.2, 0.5))
    x = np.zeros(n); x[0] = 1.0
    h1 = oracle.sosfilt(x, s1)
    h2 = oracle.sosfilt(x, s2)
    h12 = oracle.sosfilt(x, np.vstack([s1, s2]))
    ref = np.convolve(h1, h2)[:n]
    assert np.max(np.abs(h12 - ref)) < 1e-13


def freq_response(sos, w):
    z1 = np.exp(-1j * w)
    H = 1.0 + 0j
    for b0, b1, b2, a0, a1, a2 in sos:
        H *= (b0 + b1 * z1 + b2 * z1 * z1) / (a0 + a1 * z1 + a2 * z1 * z1)
    return H


@pytest.mark.parametrize("w", [0.1, 0.77, 1.9, 3.0])
def test_steady_state_sinusoid(w):
    sos = W.make_sos(8, 0.5, 0.95, 3)
    n = 4000
    t = np.arange(n)
    y = oracle.sosfilt(np.cos(w * t), sos)
    H = freq_response(sos, w)
    # after the transient (0.95^3000 ~ 2e-67) y = |H| cos(w t + arg H)
    ref = np.abs(H) * np.cos(w * t + np.angle(H))
    tail = slice(3000, n)
    # rounding is relative to the unit-amplitude input, not to |H| (which can
    # be deep in the stop band): allow 1e-15 absolute on top of 1e-10 |H|
    assert np.max(np.abs(y[tail] - ref[tail])) < 1e-10 * np.abs(H) + 1e-15
    assert np.abs(H) > 1e-12


def test_dc_gain():
    sos = W.make_sos(4, 0.5, 0.9, 5)
    y = oracle.sosfilt(np.ones(3000), sos)
    g = np.prod([(b0 + b1 + b2) / (a0 + a1 + a2) for b0, b1, b2, a0, a1, a2 in sos])
    assert abs(y[-1] - g) <= 1e-12 * max(abs(g), 1e-300)


def test_linearity_and_time_invariance():
    sos = W.make_sos(8, 0.5, 0.95, 7)
    rng = np.random.default_rng(11)
    x, z = rng.standard_normal(2000), rng.standard_normal(2000)
    y = oracle.sosfilt(2.5 * x - 0.75 * z, sos)
    ref = 2.5 * oracle.sosfilt(x, sos) - 0.75 * oracle.sosfilt(z, sos)
    # the cascade attenuates strongly (unit peak gain per section), so the
    # output carries rounding of O(1) intermediates: 1e-11 relative
    assert oracle.rel_rms(y, ref) < 1e-11
    d = 37
    xs = np.concatenate([np.zeros(d), x])
    ys = oracle.sosfilt(xs, sos)
    assert np.array_equal(ys[:d], np.zeros(d))
    assert oracle.rel_rms(ys[d:], oracle.sosfilt(x, sos)) < 1e-14


def test_a0_normalisation():
    sos = W.make_sos(3, 0.5, 0.95, 9)
    scaled = sos.copy()
    scaled[1] *= 3.0
    scaled[2] *= -0.25
    x = np.random.default_rng(2).standard_normal(500)
    assert oracle.rel_rms(oracle.sosfilt(x, scaled), oracle.sosfilt(x, sos)) < 1e-14


def dense_solution(x, b, a, xs, ys):
    """Section III: A y = B x + B_- x_-1 - A_- y_-1, solved densely."""
    n = len(x)
    A = np.eye(n) + np.diag(np.full(n - 1, a[1]), -1) + np.diag(np.full(n - 2, a[2]), -2)
    B = b[0] * np.eye(n) + np.diag(np.full(n - 1, b[1]), -1) + np.diag(np.full(n - 2, b[2]), -2)
    Am = np.zeros((n, 2)); Am[0] = [a[2], a[1]]; Am[1, 1] = a[2]
    Bm = np.zeros((n, 2)); Bm[0] = [b[2], b[1]]; Bm[1, 1] = b[2]
    rhs = B @ x + Bm @ np.asarray(xs) - Am @ np.asarray(ys)
    return np.linalg.solve(A, rhs)


def test_dense_banded_toeplitz_solve_with_state():
    rng = np.random.default_rng(4)
    sos = W.make_sos(3, 0.5, 0.95, 13)
    sos[:, 0:3] *= 5.0
    n = 200
    x = rng.standard_normal(n)
    zi = rng.standard_normal((3, 4))
    y, zf = oracle.sosfilt(x, sos, zi=zi, return_zf=True)
    u = x
    for k in range(3):
        b, a = sos[k, 0:3], np.array([1.0, sos[k, 4], sos[k, 5]])
        u = dense_solution(u, b, a, zi[k, 0:2], zi[k, 2:4])
    assert oracle.rel_rms(y, u) < 1e-13
    # final state = the last two inputs and outputs of each section
    assert np.allclose(zf[2, 2:4], y[-2:], rtol=0, atol=1e-14 * np.max(np.abs(y)))


def test_state_continuation():
    """Filtering in two pieces with zf -> zi equals one pass."""
    sos = W.make_sos(8, 0.5, 0.95, 21)
    x = np.random.default_rng(5).standard_normal(3000)
    y = oracle.sosfilt(x, sos)
    y1, zf = oracle.sosfilt(x[:1234], sos, return_zf=True)
    y2 = oracle.sosfilt(x[1234:], sos, zi=zf)
    assert np.array_equal(np.concatenate([y1, y2]), y)


def test_extended_precision_agreement_tiny_config():
    c = W.CONFIGS["tiny"]
    sos = W.make_sos(c.K, c.r_lo, c.r_hi, c.seed)
    x = W.make_signal(c.n, c.seed, np.float64)
    assert oracle.rel_rms(oracle.sosfilt(x, sos), oracle.sosfilt_ld(x, sos)) < 1e-12


def test_f32_input_path_matches_promoted_f64():
    sos = W.make_sos(8, 0.8, 0.98, 0)
    x = W.make_signal(5000, 0, np.float32)
    assert np.array_equal(oracle.sosfilt(x, sos), oracle.sosfilt(x.astype(np.float64), sos))


def test_matches_scipy_sosfilt():
    ss = pytest.importorskip("scipy.signal")
    sos = W.make_sos(8, 0.5, 0.95, 0)
    x = W.make_signal(20000, 0)
    assert oracle.rel_rms(oracle.sosfilt(x, sos), ss.sosfilt(sos, x)) < 1e-11


# ---------------------------------------------------------------- adjoint

def loss(x, sos, g):
    return float(np.dot(oracle.sosfilt(x, sos), g))


def test_backward_input_gradient_dense():
    """dL/dx = H^T g with H the dense impulse-response Toeplitz matrix."""
    sos = W.make_sos(3, 0.5, 0.95, 31)
    rng = np.random.default_rng(8)
    n = 150
    x, g = rng.standard_normal(n), rng.standard_normal(n)
    gx, _ = oracle.sosfilt_backward(x, sos, g)
    e = np.zeros(n); e[0] = 1.0
    h = oracle.sosfilt(e, sos)
    H = np.zeros((n, n))
    for i in range(n):
        H[i, :i + 1] = h[i::-1]
    assert oracle.rel_rms(gx, H.T @ g) < 1e-13


def test_backward_coefficient_gradient_finite_differences():
    sos = W.make_sos(3, 0.5, 0.95, 33)
    sos[1, 3] = 1.7          # exercise the a0 chain rule
    sos[1, [0, 1, 2, 4, 5]] *= 1.7
    rng = np.random.default_rng(9)
    n = 256
    x, g = rng.standard_normal(n), rng.standard_normal(n)
    _, gs = oracle.sosfilt_backward(x, sos, g)
    for k in range(3):
        for j in range(6):
            h = 1e-6 * max(1.0, abs(sos[k, j]))
            sp, sm = sos.copy(), sos.copy()
            sp[k, j] += h
            sm[k, j] -= h
            fd = (loss(x, sp, g) - loss(x, sm, g)) / (2 * h)
            assert abs(gs[k, j] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, j, gs[k, j], fd)


def test_backward_input_gradient_finite_differences():
    sos = W.make_sos(8, 0.5, 0.95, 35)
    rng = np.random.default_rng(10)
    n = 64
    x, g = rng.standard_normal(n), rng.standard_normal(n)
    gx, _ = oracle.sosfilt_backward(x, sos, g)
    for i in (0, 1, 17, 63):
        xp, xm = x.copy(), x.copy()
        xp[i] += 1e-4
        xm[i] -= 1e-4
        fd = (loss(xp, sos, g) - loss(xm, sos, g)) / 2e-4
        assert abs(gx[i] - fd) < 1e-8 * max(1.0, abs(fd))


# ------------------------------------------------- planted-mistake check

def _df1_python(x, sos, slip=None):
    """A copy of the oracle's recurrence in Python, with optional slips."""
    y = np.array(x, dtype=np.float64)
    for k, (b0, b1, b2, a0, a1, a2) in enumerate(sos):
        b0, b1, b2, a1, a2 = b0 / a0, b1 / a0, b2 / a0, a1 / a0, a2 / a0
        if slip == "no_a0":
            b0, b1, b2, a1, a2 = b0 * a0, b1 * a0, b2 * a0, a1 * a0, a2 * a0
        x1 = x2 = y1 = y2 = 0.0
        for i in range(len(y)):
            xi = y[i]
            if slip == "sign_a1":
                acc = b0 * xi + b1 * x1 + b2 * x2 + a1 * y1 - a2 * y2
            elif slip == "drop_b2":
                acc = b0 * xi + b1 * x1 - a1 * y1 - a2 * y2
            elif slip == "index":
                acc = b0 * xi + b1 * x2 + b2 * x1 - a1 * y1 - a2 * y2
            else:
                acc = b0 * xi + b1 * x1 + b2 * x2 - a1 * y1 - a2 * y2
            x2, x1, y2, y1 = x1, xi, y1, acc
            y[i] = acc
    return y


@pytest.mark.parametrize("slip", ["sign_a1", "drop_b2", "index", "no_a0"])
def test_pins_catch_planted_mistakes(slip):
    r, theta = 0.9, 0.3
    n = 120
    x = np.zeros(n); x[0] = 1.0
    sec = pole_section(r, theta, (1.0, 0.4, 0.3))
    sec = sec * 2.0                                       # a0 = 2
    good = _df1_python(x, sec)
    assert oracle.rel_rms(good, oracle.sosfilt(x, sec)) < 1e-14
    bad = _df1_python(x, sec, slip)
    # closed form of this section: (1 + 0.4 z^-1 + 0.3 z^-2) / A(z)
    k = np.arange(n)
    h0 = r ** k * np.sin((k + 1) * theta) / math.sin(theta)
    ref = h0.copy()
    ref[1:] += 0.4 * h0[:-1]
    ref[2:] += 0.3 * h0[:-2]
    assert oracle.rel_rms(good, ref) < 1e-13
    assert oracle.rel_rms(bad, ref) > 1e-3


def test_extended_precision_adjoint_pins():
    """The long-double adjoint (the arbiter of FP64 adjoints): its dL/dx
    equals the extended-precision forward cascade run on the time-reversed
    upstream gradient (H^T = J H J for a Toeplitz H, J the reversal), and its
    dL/dsos agrees with the FP64 adjoint to that adjoint's rounding."""
    sos = W.make_sos(8, 0.5, 0.95, 48)
    x = W.make_signal(3000, 41, np.float64)
    g = W.grad_seed_signal(3000, 41, np.float64)
    lx, ls = oracle.sosfilt_backward_ld(x, sos, g)
    ref = oracle.sosfilt_ld(g[::-1].copy(), sos)[::-1]
    assert oracle.rel_rms(lx, ref) < 1e-15
    ox, os_ = oracle.sosfilt_backward(x, sos, g)
    scale = np.max(np.abs(ls), axis=1, keepdims=True)
    assert np.max(np.abs(os_ - ls) / scale) < 1e-9
    assert oracle.rel_rms(ox, lx) < 1e-11
