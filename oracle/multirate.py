"""Paper-literal multi-rate rendering (Sec. II, Sec. III-D, Eq. 7-8), plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed, per (source, microphone) channel, in the paper's order:
  r_h = floor(10^6 / fs),  r_l = floor(sqrt(r_h))                        (Sec. II)
  L   = ceil(T60 r_h fs)   high-rate samples                            (Sec. III-D)
  q_i = min(ceil(D_i / c0 * r_h fs), L - 1),  h[q_i] += r^g_i / D_i      (Eq. 7, 8)
        with D_i the image-to-microphone distance of Eq. 1 (reading R-24)
  down-sample h from r_h fs to r_l fs                                    (Sec. II)
  80 Hz high-pass at r_l fs                                              (Sec. II)
  down-sample to fs                                                      (Sec. II)

The paper names the filters but not their designs.  Readings (R-25..R-27):
  - both down-samplers use the 81-tap Hann-windowed sinc of the fractional-delay
    rendering, P(x) = sinc(x) (1 + cos(2 pi x / 81)) / 2, in units of the lower
    rate and unit-peak, so that each keeps the height of an impulse (an image's
    r^g / D comes out as a band-limited pulse of that height, like the impulses
    of Eq. 1 at fs): resampling by r_l / r_h gives
    h_l[j] = sum_q h[q] P(j - q r_l / r_h), decimating by r_l gives
    y[n] = sum_j x[j] P((n r_l - j) / r_l);
  - the high-pass is the second-order Butterworth, bilinear transform with the
    cut-off prewarped to 80 Hz, applied from rest;
  - lengths: T_l = ceil(T60 r_l fs) intermediate samples, T = ceil(T60 fs) out;
    products are taken as T60 (r_h fs) and T60 (r_l fs), r_h fs being exact.
"""
import math

import numpy as np

from . import framrir as F


def rate_factors(fs):
    """(r_h, r_l) = (floor(10^6 / fs), floor(sqrt(r_h))) (Sec. II)."""
    rh = int(math.floor(1.0e6 / fs))
    return rh, math.isqrt(rh)


def lengths(rt60, fs):
    """(L, T_l, T): high-rate, intermediate and output samples per channel."""
    rh, rl = rate_factors(fs)
    return (int(math.ceil(rt60 * (rh * fs))), int(math.ceil(rt60 * (rl * fs))), F.rir_length(rt60, fs))


def high_rate_index(dist, c, fs):
    """q = min(ceil(D / c0 * r_h fs), L - 1) of Eq. 7, given L via the caller's
    T60 (returned unclamped here; clamp with clamp_index)."""
    rh, _ = rate_factors(fs)
    return np.ceil((np.asarray(dist, dtype=np.float64) / c) * (rh * fs)).astype(np.int64)


def clamp_index(q, big_l):
    return np.minimum(q, big_l - 1)


def impulse_train(q, amp, big_l):
    """The high-rate filter of Eq. 8: h[q_i] += r^g_i / D_i on L zeros."""
    h = np.zeros(big_l)
    np.add.at(h, q, amp)
    return h


def resample_sparse(q, amp, fs, t_l):
    """h_l[j] = sum_i A_i P(j - q_i r_l / r_h), j in [0, T_l): the
    r_h -> r_l down-sampling of the impulse train, summed over its non-zero
    samples only (each image's 81 taps around its fractional position)."""
    rh, rl = rate_factors(fs)
    t = (q.astype(np.float64) * rl) / rh
    n, x = F.footprint(t)
    w = np.asarray(amp, dtype=np.float64)[:, None] * F.pulse(x)
    ok = (n >= 0) & (n < t_l)
    return np.bincount(n[ok].astype(np.int64), weights=w[ok], minlength=t_l)[:t_l]


def butter_hp2(fc, rate):
    """Second-order Butterworth high-pass by the bilinear transform with the
    cut-off prewarped (analog prototype s^2 / (s^2 + sqrt(2) w s + w^2)):
    returns (b, a) with a[0] = 1."""
    k = math.tan(math.pi * fc / rate)
    norm = 1.0 + math.sqrt(2.0) * k + k * k
    b0 = 1.0 / norm
    b = np.array([b0, -2.0 * b0, b0])
    a = np.array([1.0, 2.0 * (k * k - 1.0) / norm, (1.0 - math.sqrt(2.0) * k + k * k) / norm])
    return b, a


def highpass(x, fs):
    """80 Hz high-pass at the intermediate rate r_l fs, from rest:
    y[n] = b0 x[n] + b1 x[n-1] + b2 x[n-2] - a1 y[n-1] - a2 y[n-2]."""
    from scipy.signal import lfilter
    _, rl = rate_factors(fs)
    b, a = butter_hp2(80.0, rl * fs)
    return lfilter(b, a, np.asarray(x, dtype=np.float64))


def decimation_kernel(rl):
    """Taps k[u] = P(u / r_l) for |u| < 40.5 r_l (u in intermediate samples),
    centred: index u + half."""
    half = int(math.ceil(40.5 * rl)) - 1
    u = np.arange(-half, half + 1, dtype=np.float64)
    return F.pulse(u / rl), half


def decimate(x, fs, t_len):
    """y[n] = sum_j x[j] P((n r_l - j) / r_l), n in [0, T)."""
    _, rl = rate_factors(fs)
    k, half = decimation_kernel(rl)
    full = np.convolve(np.asarray(x, dtype=np.float64), k)      # full[i] = sum_j x[j] k[i - j]
    idx = np.arange(t_len) * rl + half                          # i = n r_l + half  <=>  u = n r_l - j
    out = np.zeros(t_len)
    ok = idx < len(full)
    out[ok] = full[idx[ok]]
    return out


def multirate_channel(pos, g, mic, r, rt60, fs, c):
    """One channel through the whole chain: Eq. 7-8 at r_h fs, down-sample,
    high-pass, down-sample."""
    big_l, t_l, t_len = lengths(rt60, fs)
    _, dist, _, amp = F.pair_geometry(pos, g, mic, r, fs, c)
    q = clamp_index(high_rate_index(dist, c, fs), big_l)
    h_l = resample_sparse(q, amp, fs, t_l)
    return decimate(highpass(h_l, fs), fs, t_len)


def multirate_room(plan, room):
    """[S, M, T] paper-literal RIRs of one room (image tables from the same
    draws as the band-limited rendering)."""
    _, _, t_len = lengths(room.rt60, room.fs)
    out = np.zeros((len(plan["sources"]), len(room.mic), t_len))
    for s, so in enumerate(plan["sources"]):
        pos = so["pos"].copy()
        pos[0] = room.src[s]
        for m in range(len(room.mic)):
            out[s, m] = multirate_channel(pos, so["g"], room.mic[m], plan["r"], room.rt60, room.fs, room.c)
    return out


def intermediate_room(plan, room):
    """[S, M, T_l] intermediate-rate signals before the high-pass (stage one)."""
    big_l, t_l, _ = lengths(room.rt60, room.fs)
    out = np.zeros((len(plan["sources"]), len(room.mic), t_l))
    for s, so in enumerate(plan["sources"]):
        pos = so["pos"].copy()
        pos[0] = room.src[s]
        for m in range(len(room.mic)):
            _, dist, _, amp = F.pair_geometry(pos, so["g"], room.mic[m], plan["r"], room.fs, room.c)
            q = clamp_index(high_rate_index(dist, room.c, room.fs), big_l)
            out[s, m] = resample_sparse(q, amp, room.fs, t_l)
    return out
