"""Pins of the oracle's paper-literal multi-rate chain (Sec. II, Sec. III-D,
Eq. 7-8; readings R-24..R-27): the rate factors and lengths, the ceil / clamp
rule of the high-rate index on exactly representable delays, the sparse
resampler against a literal zero-stuff / filter / pick implementation on the
dense high-rate impulse train, the high-pass against scipy's Butterworth design
and its -3 dB point, the decimator against a direct per-sample sum and its pass
band, and the chain end to end on a direct path."""
import math

import numpy as np
import pytest

from oracle import framrir as F
from oracle import multirate as M


@pytest.mark.parametrize("fs, rh, rl", [(16000.0, 62, 7), (48000.0, 20, 4), (8000.0, 125, 11), (44100.0, 22, 4)])
def test_rate_factors(fs, rh, rl):
    assert M.rate_factors(fs) == (rh, rl)


def test_lengths():
    assert M.lengths(0.4, 16000.0) == (396800, 44800, 6400)
    assert M.lengths(1.2, 48000.0) == (1152000, 230400, 57600)


def test_high_rate_index_ceil_and_clamp():
    # c0 = 256 m/s and fs = 16 kHz: r_h fs = 992000, so D = 2 m is exactly 7750
    # high-rate samples; a hair more rounds up; the clamp keeps q <= L - 1
    q = M.high_rate_index(np.array([2.0, 2.0 + 1e-12, 0.5]), 256.0, 16000.0)
    assert list(q) == [7750, 7751, 1938]
    assert list(M.clamp_index(q, 7000)) == [6999, 6999, 1938]


def _literal_resample(q, amp, fs, big_l, t_l):
    # zero-stuff the high-rate train by r_l, low-pass with the output-rate
    # pulse sampled on the up-sampled grid, keep every r_h-th sample
    rh, rl = M.rate_factors(fs)
    x = M.impulse_train(q, amp, big_l)
    up = np.zeros(big_l * rl)
    up[::rl] = x
    half = int(math.ceil(40.5 * rh)) - 1
    v = np.arange(-half, half + 1, dtype=np.float64)
    k = F.pulse(v / rh)
    full = np.convolve(up, k)
    idx = np.arange(t_l) * rh + half
    out = np.zeros(t_l)
    ok = idx < len(full)
    out[ok] = full[idx[ok]]
    return out


def test_sparse_resampler_matches_literal():
    fs = 250000.0                      # r_h = 4, r_l = 2: a small dense train
    big_l, t_l, _ = M.lengths(0.002, fs)
    rng = np.random.default_rng(5)
    q = rng.integers(0, big_l, 60)
    amp = rng.uniform(0.1, 1.0, 60)
    want = _literal_resample(q, amp, fs, big_l, t_l)
    got = M.resample_sparse(q, amp, fs, t_l)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_highpass_is_scipy_butterworth():
    from scipy.signal import butter
    for rate in (112000.0, 192000.0, 44000.0):
        b, a = M.butter_hp2(80.0, rate)
        wb, wa = butter(2, 80.0, btype="highpass", fs=rate)
        np.testing.assert_allclose(b, wb, rtol=1e-12)
        np.testing.assert_allclose(a, wa, rtol=1e-12, atol=1e-15)


def test_highpass_response():
    rate = 112000.0
    b, a = M.butter_hp2(80.0, rate)

    def gain(f):
        z = np.exp(-2j * np.pi * f / rate)
        return abs((b[0] + b[1] * z + b[2] * z * z) / (a[0] + a[1] * z + a[2] * z * z))
    assert gain(0.0) < 1e-12
    assert abs(gain(80.0) - 1 / math.sqrt(2.0)) < 1e-9
    assert abs(gain(8000.0) - 1.0) < 1e-6


def test_decimator_matches_direct_sum():
    fs = 16000.0
    _, rl = M.rate_factors(fs)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(3000)
    t_len = 430
    got = M.decimate(x, fs, t_len)
    want = np.zeros(t_len)
    for n in range(t_len):
        for j in range(len(x)):
            u = n * rl - j
            if abs(u) < 40.5 * rl:
                want[n] += x[j] * F.pulse(u / rl)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_decimator_pass_band():
    # a tone at fs / 8 sampled at r_l fs comes out as the same tone at fs,
    # times r_l (the kernel keeps an impulse's height, so its DC gain is
    # sum_u P(u / r_l) = r_l up to the window)
    fs = 16000.0
    _, rl = M.rate_factors(fs)
    f0 = fs / 8
    j = np.arange(7 * 4000)
    x = np.cos(2 * np.pi * f0 * j / (rl * fs))
    y = M.decimate(x, fs, 4000)
    n = np.arange(4000)
    mid = slice(200, 3800)
    np.testing.assert_allclose(y[mid] / rl, np.cos(2 * np.pi * f0 * n / fs)[mid], atol=2e-4)


def test_down_samplers_keep_impulse_height():
    # an impulse of height 1 at an integer position of every grid comes out of
    # each stage as a pulse of peak 1 at the matching sample
    fs = 16000.0
    rh, rl = M.rate_factors(fs)
    h_l = M.resample_sparse(np.array([rh * 10]), np.array([1.0]), fs, 1000)   # q r_l / r_h = 70
    assert np.argmax(h_l) == 70 and abs(h_l[70] - 1.0) < 1e-15
    x = np.zeros(2000)
    x[7 * 50] = 1.0
    y = M.decimate(x, fs, 200)
    assert np.argmax(y) == 50 and abs(y[50] - 1.0) < 1e-15


def test_chain_direct_path():
    # one image (the direct path): the output peaks at the direct-path delay
    # with height P(frac) / D0 (P(frac) in [0.63, 1] for the fractional part of
    # the delay, less a little high-pass droop), and the high-pass removed the mean
    room = F.Room(size=(6.0, 5.0, 3.0), rt60=0.5, fs=16000.0, c=343.0, seed=0,
                  src=np.array([[1.0, 1.2, 1.3]]), mic=np.array([[3.7, 2.1, 1.9]]))
    plan = F.room_plan(room, F.Params(img_lo=0, img_hi=0))
    out = M.multirate_room(plan, room)[0, 0]
    d0 = float(np.linalg.norm(room.src[0] - room.mic[0]))
    t0 = d0 * room.fs / room.c
    assert abs(int(np.argmax(out)) - t0) <= 1.0
    frac = t0 - round(t0)
    assert abs(out.max() * d0 - F.pulse(np.array([frac]))[0]) < 0.04
    assert abs(out.sum()) < 1e-3 * out.max()
