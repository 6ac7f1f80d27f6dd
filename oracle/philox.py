"""Philox-4xW-R counter-based generator, oracle side.

Written from the definition in J. K. Salmon, M. A. Moraes, R. O. Dror and
D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11 (Sec. 4.2,
the Philox S-box and key schedule):

* the state is four W-bit words (x0, x1, x2, x3) and the key two W-bit words
  (k0, k1);
* one round multiplies x0 and x2 by the constants M0 and M1 as a full 2W-bit
  product split into (hi, lo), and outputs
  (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0));
* between rounds the key is bumped by the Weyl increments (W0, W1) modulo 2^W;
* Philox-4xW-10 applies ten rounds, round j using key + j*(W0, W1).

The Weyl increments are the W-bit fixed-point fractions of the golden ratio
(phi - 1) and of sqrt(3) - 1; ``weyl_constant`` recomputes them from that
definition with exact integers.  The multipliers are the published constants.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This module has two implementations:
``philox4_ref``   Python integers, any word width (32 or 64).  At W = 64 it is
                  checked bit for bit against numpy's Philox4x64-10 in the
                  tests, which pins the round structure and key schedule.
``philox4x32``    numpy uint64 vectorised W = 32 version for bulk draws; checked
                  against ``philox4_ref`` at W = 32.
"""
import math

import numpy as np

ROUNDS = 10

# Published round multipliers (SC'11, Table 2 / Sec. 4.2).
MULTIPLIERS = {
    32: (0xD2511F53, 0xCD9E8D57),
    64: (0xD2E7470EE14C6C93, 0xCA5A826395121157),
}


def weyl_constant(kind, width):
    """W-bit fixed-point fraction of (phi - 1) ('golden') or sqrt(3) - 1
    ('sqrt3'), truncated: floor(2^W * value), computed with exact integers."""
    scale = 1 << width
    if kind == "golden":
        # (sqrt(5) - 1) / 2 * 2^W  =  (sqrt(5 * 4^W) - 2^W) / 2
        s = math.isqrt(5 * scale * scale)
        return (s - scale) // 2
    if kind == "sqrt3":
        s = math.isqrt(3 * scale * scale)
        return s - scale
    raise ValueError(kind)


WEYL = {
    32: (0x9E3779B9, 0xBB67AE85),
    64: (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B),
}


def _mulhilo(a, b, width):
    prod = a * b
    return prod >> width, prod & ((1 << width) - 1)


def philox4_ref(ctr, key, width=32, rounds=ROUNDS):
    """Philox-4xW-R on one counter, in Python integers.

    ctr: four words, key: two words, each in [0, 2^W).  Returns four words.
    """
    mask = (1 << width) - 1
    m0, m1 = MULTIPLIERS[width]
    w0, w1 = WEYL[width]
    x0, x1, x2, x3 = (int(v) & mask for v in ctr)
    k0, k1 = (int(v) & mask for v in key)
    for j in range(rounds):
        if j > 0:
            k0 = (k0 + w0) & mask
            k1 = (k1 + w1) & mask
        hi0, lo0 = _mulhilo(m0, x0, width)
        hi1, lo1 = _mulhilo(m1, x2, width)
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Vectorised Philox-4x32-R.  Arguments broadcast; returns four uint64
    arrays holding 32-bit words."""
    mask = np.uint64(0xFFFFFFFF)
    sh = np.uint64(32)
    m0, m1 = (np.uint64(v) for v in MULTIPLIERS[32])
    w0, w1 = (np.uint64(v) for v in WEYL[32])
    x0, x1, x2, x3, key0, key1 = np.broadcast_arrays(
        *(np.asarray(v, dtype=np.uint64) & mask for v in (c0, c1, c2, c3, k0, k1)))
    x0, x1, x2, x3 = (v.copy() for v in (x0, x1, x2, x3))
    key0 = key0.copy()
    key1 = key1.copy()
    for j in range(rounds):
        if j > 0:
            key0 = (key0 + w0) & mask
            key1 = (key1 + w1) & mask
        p0 = m0 * x0          # < 2^64: exact in uint64
        p1 = m1 * x2
        hi0, lo0 = p0 >> sh, p0 & mask
        hi1, lo1 = p1 >> sh, p1 & mask
        x0, x1, x2, x3 = hi1 ^ x1 ^ key0, lo1, hi0 ^ x3 ^ key1, lo0
    return x0, x1, x2, x3
