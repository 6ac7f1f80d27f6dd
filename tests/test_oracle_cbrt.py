"""Pins of the oracle's correctly rounded cube root (inverse CDF of Eq. 3)."""
import math
from fractions import Fraction

import numpy as np

from oracle.cbrt import cbrt_rn, icbrt


def test_icbrt_exact():
    for n in [0, 1, 7, 8, 26, 27, 28, 10**30, 10**30 - 1, (2**53 + 1) ** 3, (2**53 + 1) ** 3 - 1]:
        y = icbrt(n)
        assert y ** 3 <= n < (y + 1) ** 3


def test_perfect_cubes_exact():
    for k in [1, 2, 3, 5, 7, 11, 1000, 2**17 - 1]:
        for j in [-30, -7, 0, 5]:
            x = math.ldexp(float(k ** 3), 3 * j)
            assert cbrt_rn(x) == math.ldexp(float(k), j)
    assert cbrt_rn(27.0 / 64.0) == 0.75
    assert cbrt_rn(1.0 / 64.0) == 0.25


def _is_nearest(a, y):
    """a^(1/3) lies strictly between the midpoints of y with its neighbours."""
    lo = (Fraction(y) + Fraction(np.nextafter(y, 0.0))) / 2
    hi = (Fraction(y) + Fraction(np.nextafter(y, np.inf))) / 2
    fa = Fraction(a)
    return lo ** 3 < fa < hi ** 3


def test_nearest_by_rational_arithmetic():
    rng = np.random.default_rng(2)
    xs = np.concatenate([rng.uniform(1.0 / 64.0, 1.0, 3000),
                         10.0 ** rng.uniform(-30, 30, 1000),
                         rng.uniform(0, 1, 500) ** 9])
    for x in xs:
        assert _is_nearest(float(x), cbrt_rn(float(x)))


def test_within_one_ulp_of_libm():
    rng = np.random.default_rng(3)
    xs = rng.uniform(1.0 / 64.0, 1.0, 20000)
    got = np.array([cbrt_rn(v) for v in xs])
    ref = np.cbrt(xs)
    assert np.all(np.abs(got - ref) <= np.spacing(ref))


def test_monotone():
    rng = np.random.default_rng(4)
    xs = np.sort(rng.uniform(0.01, 1.0, 5000))
    ys = [cbrt_rn(v) for v in xs]
    assert all(b >= a for a, b in zip(ys, ys[1:]))
