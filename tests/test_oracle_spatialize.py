"""Pins of the spatialisation oracle (oracle/spatialize.py; Sec. IV-A and
readings R-28..R-31): the convolution against its defining double sum, an
impulse through an RIR, the achieved SIR and SNR measured on the scaled
images, the mixture as the sum of the images, and invariance of the result
to the loudness of the dry signals."""
import numpy as np
import pytest

from oracle import spatialize as SP
from paper_2304_08052_amd import workloads as W


def brute_conv(x, h, n):
    y = np.zeros(n)
    for k in range(n):
        for j in range(len(h)):
            if 0 <= k - j < len(x):
                y[k] += h[j] * x[k - j]
    return y


@pytest.mark.parametrize("nx,nh,n", [(7, 5, 11), (13, 4, 9), (5, 9, 20)])
def test_convolution_is_the_defining_sum(nx, nh, n):
    rng = np.random.default_rng(nx * 100 + nh)
    x, h = rng.standard_normal(nx), rng.standard_normal(nh)
    got = SP.convolve_window(x, h, n)
    want = brute_conv(x, h, n)
    assert len(got) == min(n, nx + nh - 1)
    assert np.allclose(got, want[:len(got)], rtol=0, atol=1e-12)


def test_impulse_reproduces_the_rir():
    rng = np.random.default_rng(3)
    h = rng.standard_normal(40)
    x = np.zeros(100)
    x[17] = 1.0
    y = SP.convolve_window(x, h, 100)
    assert np.array_equal(y[17:57], h) and np.all(y[:17] == 0) and np.all(y[57:] == 0)


def _room(seed=1, n=4000, T=900):
    rng = np.random.default_rng(seed)
    rir = rng.standard_normal((3, 4, T)) * np.exp(-np.arange(T) / 200.0)
    sig = rng.standard_normal((3, n))
    sig[1, : n // 4] = 0.0   # the second speaker starts later
    return rir, sig


@pytest.mark.parametrize("sir,snr", [(-6.0, 10.0), (0.0, 15.0), (5.5, 19.0)])
def test_achieved_sir_and_snr(sir, snr):
    rir, sig = _room()
    images, mix, g = SP.spatialize_room(rir, sig, sir, snr, 4000)
    assert g[0] == 1.0
    e = lambda a: float(np.sum(a * a))
    assert abs(10 * np.log10(e(images[0]) / e(images[1])) - sir) < 1e-9
    assert abs(10 * np.log10(e(images[0] + images[1]) / e(images[2])) - snr) < 1e-9
    assert np.array_equal(mix, images[0] + images[1] + images[2])


def test_scaled_images_do_not_depend_on_dry_loudness():
    rir, sig = _room(seed=2)
    a, ma, _ = SP.spatialize_room(rir, sig, 2.0, 12.0, 4000)
    sig2 = sig * np.array([1.0, 3.0, 0.1])[:, None]
    b, mb, _ = SP.spatialize_room(rir, sig2, 2.0, 12.0, 4000)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12) and np.allclose(ma, mb, rtol=1e-12, atol=1e-12)


def test_workload_recipe():
    batch = W.spatial_batch(4, seed=1)
    assert np.all(batch["n_src"] == 3) and np.all(batch["n_mic"] == 4)
    sig, sir, snr = W.spatial_signals(batch, 16000, seed=1)
    assert sig.shape == (4, 3, 16000) and sig.dtype == np.float32
    assert np.all((sir >= -6) & (sir <= 6)) and np.all((snr >= 10) & (snr <= 20))
    for b in range(4):   # the speakers' active spans overlap by at least half their union
        act = [np.flatnonzero(sig[b, s]) for s in (0, 1)]
        lo = [a.min() for a in act]
        hi = [a.max() + 1 for a in act]
        inter = max(0, min(hi) - max(lo))
        union = max(hi) - min(lo)
        assert inter / union >= 0.5 - 1e-3
