"""Correctly rounded (round-to-nearest-even) FP64 cube root, oracle side.

The inverse-CDF draw of the quadratic distance-ratio density (Sec. III-B,
Eq. 3) needs a cube root.  For the reflection counts to be reproducible bit for
bit, the cube root must be a function of its argument alone, so the oracle uses
the correctly rounded value: the double nearest to the real cube root.  It is
computed here with exact Python integers (no floating point at all):

1. write the argument as an exact rational n / 2^j;
2. pick the exponent e so that Y = floor(cbrt(a) / 2^e) has 53 bits;
3. Y comes from an exact integer cube root;
4. round up iff a exceeds the cube of the midpoint (Y + 1/2) * 2^e, compared as
   integers (ties cannot occur: the cube of an odd 54-bit integer has more
   than 53 significant bits).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import math


def icbrt(n):
    """floor(cbrt(n)) for a non-negative integer n, exactly."""
    if n < 0:
        raise ValueError("negative")
    if n == 0:
        return 0
    # float start, then exact integer correction
    x = int(round(float(n) ** (1.0 / 3.0))) if n < (1 << 1000) else 1 << (n.bit_length() // 3)
    while x * x * x > n:
        x -= 1
    while (x + 1) * (x + 1) * (x + 1) <= n:
        x += 1
    return x


def cbrt_rn(a):
    """Correctly rounded cube root of a finite double a >= 0."""
    a = float(a)
    if not math.isfinite(a) or a < 0.0:
        raise ValueError("cbrt_rn expects a finite non-negative double")
    if a == 0.0:
        return 0.0
    num, den = a.as_integer_ratio()          # den is a power of two
    j = den.bit_length() - 1                 # a = num * 2^-j
    # cbrt(a) ~ 2^(log2(a)/3); choose e so that Y lands in [2^52, 2^53)
    log2a = num.bit_length() - 1 - j
    e = (log2a // 3) - 52
    while True:
        # Y = floor(cbrt(num * 2^(-j - 3e)))
        s = -j - 3 * e
        # floor(cbrt(q)) = floor(cbrt(floor(q))) for q >= 0, because the
        # break points of floor(cbrt(.)) are integer cubes
        y = icbrt(num << s) if s >= 0 else icbrt(num >> (-s))
        if y >= (1 << 53):
            e += 1
            continue
        if y < (1 << 52):
            e -= 1
            continue
        break
    # midpoint (2y + 1) * 2^(e-1); compare a against its cube exactly:
    # a > ((2y+1) 2^(e-1))^3  <=>  num * 2^(-j) > (2y+1)^3 * 2^(3e-3)
    lhs_exp = -j
    rhs_exp = 3 * e - 3
    lhs = num
    rhs = (2 * y + 1) ** 3
    if lhs_exp >= rhs_exp:
        lhs <<= (lhs_exp - rhs_exp)
    else:
        rhs <<= (rhs_exp - lhs_exp)
    if lhs > rhs:
        y += 1
    return math.ldexp(float(y), e)

