"""The two Newton recurrences the device code uses in place of a division and
the library cube root (CPU only): 1/d from an estimate by two steps
r <- r + r (1 - d r), and J^(-1/3) from an estimate by two steps
y <- y + y (1 - J y^3) / 3.  Each step here is the device's operation
sequence with every fused multiply-add and product rounded once (exact
rationals, then one rounding), starting from estimates no better than the
hardware's (a relative error of 1e-4 for the reciprocal, 3e-7 for the
single-precision exp2/log2 estimate of the cube root).  The results must
lie within two units in the last place of the exact values.
"""
from fractions import Fraction

import numpy as np

ULP = 2.0 ** -52


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def mul(a, b):
    return float(Fraction(a) * Fraction(b))


def recip(d, r):
    for _ in range(2):
        e = fma(-d, r, 1.0)
        r = fma(r, e, r)
    return r


def inv_cbrt(J, y):
    a = abs(J)
    for _ in range(2):
        e = fma(-a, mul(mul(y, y), y), 1.0)
        y = fma(mul(y, e), 1.0 / 3.0, y)
    return y if J > 0 else -y


def samples(rng):
    return np.concatenate([rng.uniform(0.3, 3.0, 400), 10.0 ** rng.uniform(-12, 6, 200)])


def test_reciprocal_within_two_ulps():
    rng = np.random.default_rng(5)
    for d in samples(rng):
        d = float(d)
        r0 = (1.0 / d) * (1.0 + rng.uniform(-1e-4, 1e-4))
        r = recip(d, r0)
        err = abs((Fraction(r) - 1 / Fraction(d)) * Fraction(d))
        assert err <= 2 * ULP, (d, float(err))


def test_inverse_cube_root_within_two_ulps():
    rng = np.random.default_rng(6)
    for J in samples(rng):
        for s in (1.0, -1.0):
            Jv = s * float(J)
            y0 = float(np.float32(abs(Jv) ** (-1.0 / 3.0) * (1.0 + rng.uniform(-3e-7, 3e-7))))
            y = inv_cbrt(Jv, y0)
            assert np.sign(y) == np.sign(Jv)
            # |y^3 J - 1| / 3 is the relative error of y to first order
            err = abs(Fraction(y) ** 3 * Fraction(Jv) - 1) / 3
            assert err <= 2 * ULP, (Jv, float(err))
