"""Exact evaluation of the cascade's recurrence (Section II) for pinning the
oracle's extended- and single-precision twins.

Every FP64 number is a dyadic rational m 2^e, and sums and products of
dyadic rationals are dyadic, so the direct-form recurrence run on pairs
(m, e) of Python integers is exact: no rounding anywhere.  The cost grows
with the mantissas (a few hundred to a few thousand samples in seconds),
which is what the pins need.

``max_bits`` reports the longest odd mantissa any intermediate value took,
products and partial sums included: when it is at most 24 (and the
exponents stay in range), a plain FP32 evaluation performs every operation
exactly.
"""
from __future__ import annotations

import math
from fractions import Fraction


def _dy(v: float):
    if v == 0.0:
        return (0, 0)
    m, e = math.frexp(v)
    return (int(m * (1 << 53)), e - 53)


def _norm(a):
    m, e = a
    if m == 0:
        return (0, 0)
    tz = (m & -m).bit_length() - 1   # trailing zero bits
    return (m >> tz, e + tz)


def _add(a, b):
    (m1, e1), (m2, e2) = a, b
    if e1 > e2:
        return ((m1 << (e1 - e2)) + m2, e2)
    return (m1 + (m2 << (e2 - e1)), e1)


def _mul(a, b):
    return (a[0] * b[0], a[1] + b[1])


def _neg(a):
    return (-a[0], a[1])


class Exact:
    def __init__(self):
        self.max_bits = 0
        self.min_exp = 0
        self.max_exp = 0

    def _track(self, a):
        m, e = _norm(a)
        if m:
            self.max_bits = max(self.max_bits, abs(m).bit_length())
            top = e + abs(m).bit_length()   # value < 2^top
            self.min_exp = min(self.min_exp, e)
            self.max_exp = max(self.max_exp, top)
        return (m, e)

    def cascade(self, x, sos):
        """The cascade of rows (b0, b1, b2, 1, a1, a2) applied to x, zero
        initial state; returns exact Fractions."""
        cur = [_dy(float(v)) for v in x]
        for row in sos:
            if float(row[3]) != 1.0:
                raise ValueError("rows must have a0 = 1")
            b0, b1, b2, a1, a2 = (_dy(float(row[i])) for i in (0, 1, 2, 4, 5))
            z = (0, 0)
            x1 = x2 = y1 = y2 = z
            out = []
            for xi in cur:
                t = self._track(_mul(b0, xi))
                t = self._track(_add(t, self._track(_mul(b1, x1))))
                t = self._track(_add(t, self._track(_mul(b2, x2))))
                t = self._track(_add(t, _neg(self._track(_mul(a1, y1)))))
                t = self._track(_add(t, _neg(self._track(_mul(a2, y2)))))
                x2, x1, y2, y1 = x1, xi, y1, t
                out.append(t)
            cur = out
        return [Fraction(m) * (Fraction(2) ** e) for m, e in cur]


def exact_cascade(x, sos):
    return Exact().cascade(x, sos)
