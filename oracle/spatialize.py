"""FP64 oracle of the spatialisation and mixing step of the on-the-fly
training set-up (Sec. IV-A): two speech sources and a point-source noise are
each convolved with their multi-channel RIRs, the second speaker is scaled to
the sampled signal-to-interference ratio and the noise to the sampled
signal-to-noise ratio, and the images are summed into the mixture.

TEST INFRASTRUCTURE ONLY: the library never imports, links or runs this
module; tests/, the smoke check and the benchmark's CPU baseline do.

Readings (where the paper does not fix the details):
  R-28  an image is the full linear convolution y = x * h truncated to the
        utterance window of N samples (the RIR tail past the window is cut);
  R-29  the SIR is 10 log10(E1 / E2) with E_s the energy of source s's scaled
        image summed over all microphones and the N samples; speaker 1 is the
        reference (gain 1) and speaker 2 is scaled;
  R-30  the SNR is 10 log10(E_sp / E_n) with E_sp the energy of the speech
        mixture (speaker 1 plus scaled speaker 2, all microphones) and E_n that
        of the scaled noise image;
  R-31  sources 0 and 1 of a room are the speakers, source 2 the noise; the
        speakers' overlap is fixed by where their dry signals sit in the
        window (an input).
"""
import numpy as np


def convolve_window(x, h, n):
    """R-28: y[k] = sum_j h[j] x[k - j] for k < n (np.convolve is that sum)."""
    return np.convolve(np.asarray(x, dtype=np.float64), np.asarray(h, dtype=np.float64))[:n]


def source_images(rir, sig, n):
    """Images y[s, m, :] of the dry signals sig[s] through rir[s, m] (R-28)."""
    S, M, _ = rir.shape
    y = np.zeros((S, M, n))
    for s in range(S):
        for m in range(M):
            y[s, m] = convolve_window(sig[s], rir[s, m], n)
    return y


def mixing_gains(y, sir_db, snr_db):
    """Gains (1, g2, gn) that give the requested SIR (R-29) and SNR (R-30).
    E_sp = sum (y1 + g2 y2)^2 = E1 + 2 g2 E12 + g2^2 E2 (expanded square)."""
    e1 = np.sum(y[0] * y[0])
    e2 = np.sum(y[1] * y[1])
    e12 = np.sum(y[0] * y[1])
    en = np.sum(y[2] * y[2])
    g2 = np.sqrt(e1 / (e2 * 10.0 ** (sir_db / 10.0)))
    esp = e1 + 2.0 * g2 * e12 + g2 * g2 * e2
    gn = np.sqrt(esp / (en * 10.0 ** (snr_db / 10.0)))
    return np.array([1.0, g2, gn])


def spatialize_room(rir, sig, sir_db, snr_db, n):
    """Scaled images [3, M, n] and the mixture [M, n] of one room."""
    y = source_images(rir, sig, n)
    g = mixing_gains(y, sir_db, snr_db)
    images = y * g[:, None, None]
    return images, images.sum(axis=0), g
