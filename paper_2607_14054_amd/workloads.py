"""Seeded synthetic inputs for cascaded-biquad filtering.

This module only draws inputs: signals and second-order-section (SOS)
coefficient arrays.  It holds none of the filtering arithmetic, so the FP64
CPU oracle and the HIP path can both take their inputs from here.

Recipe (the paper measures a 16th-order cascade, K = 8, but states neither
its coefficients nor its input signal; Section VIII):

* signal: ``default_rng(seed).standard_normal(n, dtype)``; N(0, 1).
* coefficients: ``default_rng(seed + 1)``; per section, in this order,
  pole radius r ~ U[r_lo, r_hi], pole angle theta ~ U[0, pi], zero angle
  phi ~ U[0, pi].  Denominator a = [1, -2 r cos(theta), r^2] (a conjugate
  pole pair), numerator b = g [1, -2 cos(phi), 1] (a conjugate zero pair on
  the unit circle), with g chosen so that the section's peak magnitude
  response over a dense grid of 2^14 + 1 frequencies on [0, pi] is 1.
* rows follow the SOS convention of Section II: [b0, b1, b2, a0, a1, a2]
  with a0 = 1 and the denominator entering with a minus sign.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAIN_GRID = 2 ** 14 + 1


def _peak_gain(b: np.ndarray, a: np.ndarray) -> float:
    w = np.linspace(0.0, math.pi, GAIN_GRID)
    z1 = np.exp(-1j * w)
    z2 = z1 * z1
    num = b[0] + b[1] * z1 + b[2] * z2
    den = a[0] + a[1] * z1 + a[2] * z2
    return float(np.max(np.abs(num / den)))


def make_sos(K: int, r_lo: float, r_hi: float, seed: int) -> np.ndarray:
    """K x 6 float64 SOS array drawn by the recipe above."""
    rng = np.random.default_rng(seed + 1)
    sos = np.zeros((K, 6), dtype=np.float64)
    for k in range(K):
        r = rng.uniform(r_lo, r_hi)
        theta = rng.uniform(0.0, math.pi)
        phi = rng.uniform(0.0, math.pi)
        a = np.array([1.0, -2.0 * r * math.cos(theta), r * r])
        b = np.array([1.0, -2.0 * math.cos(phi), 1.0])
        b = b / _peak_gain(b, a)
        sos[k, 0:3] = b
        sos[k, 3:6] = a
    return sos


def make_signal(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """x ~ N(0, 1), n samples, drawn directly in ``dtype``."""
    rng = np.random.default_rng(seed)
    dt = np.dtype(dtype)
    if dt == np.float32:
        return rng.standard_normal(n, dtype=np.float32)
    return rng.standard_normal(n, dtype=np.float64).astype(dt, copy=False)


@dataclass
class Config:
    """One workload: a single channel or a batch of channels."""
    name: str
    n: int | None            # samples per channel (None: per-channel lengths)
    dtype: str               # "f32" | "f64"
    K: int | None            # sections (None: per-channel K)
    r_lo: float
    r_hi: float
    channels: int = 1
    seed: int = 0
    N: int = 0               # 0: let the library choose
    extra: dict = field(default_factory=dict)

    @property
    def np_dtype(self):
        return np.float32 if self.dtype == "f32" else np.float64


# The five workloads of the build; sizes follow the paper's K = 8 headline
# cascade.  "tiny" is small enough for the oracle in well under a second.
CONFIGS = {
    "tiny": Config("plain-tiny", 2 ** 16, "f64", 8, 0.5, 0.95, N=8),
    "scale": Config("plain-2^28-f32", 2 ** 28, "f32", 8, 0.8, 0.98),
    "batch": Config("batched-ragged", None, "f32", None, 0.5, 0.95,
                    channels=4096, extra={"log2_lo": 10, "log2_hi": 22,
                                          "K_lo": 1, "K_hi": 16}),
    "precision": Config("precision", 2 ** 20, "f32", 8, 0.9, 0.999,
                        channels=256),
    "grad": Config("adjoint", 2 ** 18, "f32", 8, 0.5, 0.95, channels=64),
}


def batch_lengths(channels: int, log2_lo: float, log2_hi: float,
                  seed: int) -> np.ndarray:
    """Channel lengths, log-uniform in [2^log2_lo, 2^log2_hi]."""
    rng = np.random.default_rng(seed + 3)
    e = rng.uniform(log2_lo, log2_hi, size=channels)
    return np.floor(2.0 ** e).astype(np.int64)


def batch_sections(channels: int, K_lo: int, K_hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed + 4)
    return rng.integers(K_lo, K_hi + 1, size=channels).astype(np.int64)


def grad_seed_signal(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Upstream gradient g ~ N(0, 1) for the loss sum(y * g), seed + 2."""
    return make_signal(n, seed + 2, dtype)
