"""Pins of the oracle's Philox-4xW-10 (SC'11 definition).

* the width-generic Python-integer version at W = 64 reproduces numpy's
  Philox4x64-10 bit for bit, which fixes the round function, the key schedule,
  the output order and the round count;
* the Weyl key increments equal their closed-form definition (fixed-point
  golden ratio and sqrt(3) - 1) at both widths;
* the vectorised W = 32 version equals the generic one at W = 32;
* the W = 32 output is uniform (chi-square) and avalanches;
* both widths reproduce the published known-answer vectors of Philox4x32-10
  and Philox4x64-10 (tests/golden/philox_kat.txt), which fixes the
  multipliers and every other constant to the generator's definition.
"""
import numpy as np
import pytest
from scipy import stats

from oracle.philox import MULTIPLIERS, WEYL, philox4_ref, philox4x32, weyl_constant
from tests.golden import philox_kat


@pytest.mark.parametrize("key", [(0, 0), (1, 2), (0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF)])
def test_generic_w64_matches_numpy_philox(key):
    # numpy increments the 256-bit counter before each block: starting from
    # counter c, block j of output is Philox(c + j + 1).
    start = [5, 0, 7, 1 << 63]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(start, dtype=np.uint64))
    raw = [int(v) for v in bg.random_raw(4 * 6)]
    for j in range(6):
        ctr = list(start)
        ctr[0] += j + 1
        got = philox4_ref(ctr, key, width=64)
        assert list(got) == raw[4 * j:4 * j + 4]


def test_weyl_constants_closed_form():
    for width in (32, 64):
        assert WEYL[width] == (weyl_constant("golden", width), weyl_constant("sqrt3", width))


def test_known_answer_vectors_both_widths():
    rows = philox_kat()
    assert sorted({r[0] for r in rows}) == [32, 64] and len(rows) == 6
    for width, ctr, key, want in rows:
        assert list(philox4_ref(ctr, key, width=width)) == want, (width, ctr)


def test_known_answer_vectors_vectorised_w32():
    for width, ctr, key, want in philox_kat():
        if width == 32:
            got = philox4x32(*[np.array([c], dtype=np.uint64) for c in ctr + key])
            assert [int(w[0]) for w in got] == want


def test_multipliers_are_odd_and_full_width():
    for width in (32, 64):
        for m in MULTIPLIERS[width]:
            assert m % 2 == 1 and m.bit_length() == width


def test_vectorised_w32_equals_generic():
    rng = np.random.default_rng(0)
    for _ in range(200):
        c = [int(v) for v in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        k = [int(v) for v in rng.integers(0, 2**32, 2, dtype=np.uint64)]
        want = philox4_ref(c, k, width=32)
        got = [int(v) for v in philox4x32(*c, *k)]
        assert got == list(want)


def test_w32_uniform_chi_square():
    i = np.arange(1 << 16, dtype=np.uint64)
    words = np.concatenate(philox4x32(i, 3, 0, 0, 12345, 678))
    top = (words >> np.uint64(24)).astype(np.int64)          # top byte
    counts = np.bincount(top, minlength=256)
    _, pval = stats.chisquare(counts)
    assert pval > 1e-4
    # every bit is set half the time
    bits = np.stack([(words >> np.uint64(b)) & np.uint64(1) for b in range(32)]).astype(float)
    assert np.all(np.abs(bits.mean(axis=1) - 0.5) < 0.01)


def test_w32_avalanche():
    rng = np.random.default_rng(1)
    flips = []
    for _ in range(300):
        c = [int(v) for v in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        k = [int(v) for v in rng.integers(0, 2**32, 2, dtype=np.uint64)]
        a = philox4_ref(c, k, width=32)
        word, bit = rng.integers(0, 4), rng.integers(0, 32)
        c2 = list(c)
        c2[word] ^= 1 << int(bit)
        b = philox4_ref(c2, k, width=32)
        flips.append(sum(bin(x ^ y).count("1") for x, y in zip(a, b)))
    assert abs(np.mean(flips) - 64.0) < 2.0
