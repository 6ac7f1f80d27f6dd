"""Pins of the oracle's early-reverberation filter (Eq. 9, reading R-23): the
window lengths at 16 and 48 kHz, the ceil rule of the direct-path index on an
exactly representable delay and just past it, full reconstruction of a
direct-path-only RIR (its 81-tap pulse lies inside the window), the mask on a
room with images, and zero padding where the window starts before n = 0."""
import numpy as np

from oracle import framrir as F

NONE = F.Params(img_lo=0, img_hi=0)        # direct path only


def _room(src, mics, fs=16000.0, c=320.0, rt60=0.4, prm=NONE, seed=0):
    room = F.Room(size=(6.0, 5.0, 3.0), rt60=rt60, fs=fs, c=c, seed=seed,
                  src=np.asarray([src], dtype=float), mic=np.asarray(mics, dtype=float))
    plan = F.room_plan(room, prm)
    return room, plan, F.render_room(plan, room)


def test_window_lengths():
    # 6 ms and 50 ms: 96 and 800 samples at 16 kHz, 288 and 2400 at 48 kHz
    assert F.early_window(0.0, 16000.0) == (-96, 800)
    assert F.early_window(0.0, 48000.0) == (-288, 2400)
    room, plan, h = _room((1.0, 1.0, 1.0), [(3.0, 1.0, 1.0)])
    early, start = F.early_room(room, h)
    assert early.shape == (1, 1, 96 + 800 + 1)


def test_direct_index_uses_ceil():
    # fs / c = 50 samples per metre; D0 = 2 m exactly gives t0 = 100, so the
    # window starts at 100 - 96 = 4; a hair more distance moves it to 5
    room, plan, h = _room((1.0, 1.0, 1.0), [(3.0, 1.0, 1.0)])
    _, start = F.early_room(room, h)
    assert start[0, 0] == 4
    room, plan, h = _room((1.0, 1.0, 1.0), [(3.0 + 1e-9, 1.0, 1.0)])
    _, start = F.early_room(room, h)
    assert start[0, 0] == 5


def test_direct_path_only_is_reconstructed():
    # without images the whole RIR is the 81-tap pulse at t0 (+-40 samples),
    # which the [-96, +800] window contains: h_e equals h
    room, plan, h = _room((1.0, 1.2, 1.3), [(3.7, 2.1, 1.9), (3.75, 2.1, 1.9)], c=343.0)
    early, start = F.early_room(room, h)
    for m in range(2):
        full = np.zeros(plan["T"])
        lo = int(start[0, m])
        idx = np.arange(lo, lo + early.shape[2])
        ok = (idx >= 0) & (idx < plan["T"])
        full[idx[ok]] = early[0, m][ok]
        np.testing.assert_array_equal(full, h[0, m])


def test_mask_keeps_window_only():
    # with images: inside the window h_e is h, and the energy outside it is
    # what the filter removes (a late tail exists at T60 = 0.6 s)
    room, plan, h = _room((1.0, 1.2, 1.3), [(3.7, 2.1, 1.9)], c=343.0, rt60=0.6,
                          prm=F.Params(img_lo=600, img_hi=600), seed=5)
    early, start = F.early_room(room, h)
    lo = int(start[0, 0])
    w = early.shape[2]
    np.testing.assert_array_equal(early[0, 0], h[0, 0, lo:lo + w])
    e_in = np.sum(early ** 2)
    e_all = np.sum(h ** 2)
    assert 0 < e_in < e_all
    assert np.sum(h[0, 0, lo + w:] ** 2) > 0


def test_window_before_zero_is_zero_padded():
    # D0 = 0.5 m at 50 samples per metre: t0 = 25, the window starts at -71
    room, plan, h = _room((1.0, 1.0, 1.0), [(1.5, 1.0, 1.0)])
    early, start = F.early_room(room, h)
    assert start[0, 0] == 25 - 96
    assert np.all(early[0, 0, :71] == 0.0)
    np.testing.assert_array_equal(early[0, 0, 71:], h[0, 0, :early.shape[2] - 71])
