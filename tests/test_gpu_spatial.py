"""GPU parity of the spatialisation and mixing step (Sec. IV-A, readings
R-28..R-31) against the FP64 oracle: the rendered RIRs (checked by their own
parity tests) are copied to the host and given to the oracle, so this tests
the convolution (overlap-save with a 32768-point FFT in FP32), the gains and
the mixture.  Images and mixtures within 1e-5 relative L2 per channel, gains
within 1e-5 relative; the mixture equals the sum of the stored images bit for
bit."""
import sys

import numpy as np
import pytest

from oracle import spatialize as SP
from paper_2304_08052_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _run(batch, n, seed=0, launch=None):
    import torch
    from paper_2304_08052_amd import framrir as fr
    plan = fr.Plan(batch, launch=launch)
    out, _ = plan.forward()
    sig, sir, snr = W.spatial_signals(batch, n, seed=seed)
    sig_d = torch.from_numpy(sig.reshape(-1, n)).cuda()
    images, mix, gains = plan.spatialize(out, sig_d, torch.from_numpy(sir).cuda(), torch.from_numpy(snr).cuda())
    torch.cuda.synchronize()
    return plan, out.cpu().numpy(), sig, sir, snr, images.cpu().numpy(), mix.cpu().numpy(), gains.cpu().numpy()


def _check_rooms(plan, out, sig, sir, snr, images, mix, gains, rooms, n):
    mo, so = plan.mic_off, plan.src_off
    for b in rooms:
        M, T = int(plan.n_mic[b]), int(plan.T[b])
        rir = out[plan.out_off[b]:plan.out_off[b + 1]].reshape(3, M, T).astype(np.float64)
        want_img, want_mix, want_g = SP.spatialize_room(rir, sig[b].astype(np.float64), float(sir[b]),
                                                       float(snr[b]), n)
        c0 = 3 * mo[b]   # first channel of the room (3 sources per room)
        got_img = images[c0:c0 + 3 * M].reshape(3, M, n)
        e_img = max(rel(got_img[s, m], want_img[s, m]) for s in range(3) for m in range(M))
        e_mix = max(rel(mix[mo[b] + m], want_mix[m]) for m in range(M))
        e_g = np.max(np.abs(gains[so[b]:so[b] + 3] - want_g) / want_g)
        say(f"room {b}: T {T} images {e_img:.2e} mix {e_mix:.2e} gains {e_g:.2e}")
        assert e_img <= TOL and e_mix <= TOL and e_g <= TOL


@pytest.mark.parametrize("n", [16000, 70000])
def test_spatialize_matches_oracle(n):
    """One overlap-save block (1 s) and three blocks (4.4 s), short RIRs so
    that the oracle's direct convolution stays quick."""
    batch = W.spatial_batch(3, seed=5, rt60_range=(0.1, 0.3))
    say(f"spatialize 3 rooms, n = {n}")
    plan, out, sig, sir, snr, images, mix, gains = _run(batch, n, seed=1)
    _check_rooms(plan, out, sig, sir, snr, images, mix, gains, range(3), n)


def test_spatialize_longest_rir_odd_window():
    """The longest RIR the library takes (T60 1.024 s at 16 kHz: 16,384
    samples, so an overlap-save block advances by 16,385) over an odd window
    of 17,001 samples: two blocks, the second one ragged."""
    batch = W.spatial_batch(1, seed=8, rt60_range=(1.024, 1.024))
    n = 17001
    say(f"spatialize the longest RIR, n = {n}")
    plan, out, sig, sir, snr, images, mix, gains = _run(batch, n, seed=3)
    assert int(plan.T[0]) == 16384
    _check_rooms(plan, out, sig, sir, snr, images, mix, gains, range(1), n)


def test_spatialize_full_workload_sampled():
    """The benchmark's workload (256 rooms, 4 s at 16 kHz, T60 up to 0.7 s):
    sampled rooms against the oracle, every room's identities checked."""
    from paper_2304_08052_amd import autotune
    batch = W.spatial_batch(256, seed=0)
    n = 64000
    say("spatialize 256 rooms, 4 s")
    plan, out, sig, sir, snr, images, mix, gains = _run(batch, n, launch=autotune.launch_for(batch))
    mo = plan.mic_off
    for b in range(256):   # the mixture is the sum of the stored images, bit for bit
        M = int(plan.n_mic[b])
        img = images[3 * mo[b]:3 * mo[b] + 3 * M].reshape(3, M, n)
        assert np.array_equal(mix[mo[b]:mo[b] + M], (img[0] + img[1]) + img[2])
    assert np.all(gains[0::3] == 1.0)
    longest = int(np.argmax(plan.T))
    _check_rooms(plan, out, sig, sir, snr, images, mix, gains, (0, longest), n)


def test_spatialize_reproducible_and_rejects():
    import torch
    from paper_2304_08052_amd import framrir as fr
    batch = W.spatial_batch(4, seed=6, rt60_range=(0.1, 0.3))
    a = _run(batch, 20000, seed=2)
    b = _run(batch, 20000, seed=2)
    for x, y in zip(a[5:], b[5:]):
        assert np.array_equal(x, y)
    plan = fr.Plan(W.config4(2))          # one source per room
    with pytest.raises(fr.FramrirError):
        plan.spatial_workspace_bytes(1000)
    long_batch = W.spatial_batch(1, seed=7, fs=48000.0)
    long_batch["rt60"][:] = 5.6           # 268,800 samples: more than 16 partitions of 16,384
    with pytest.raises(fr.FramrirError):
        fr.Plan(long_batch).spatial_workspace_bytes(1000)
    long_batch["rt60"][:] = 1.2           # 57,600 samples: four partitions, accepted
    assert fr.Plan(long_batch).spatial_workspace_bytes(1000) > 0


def test_spatialize_long_rirs_partitioned(oracle_pool):
    """RIRs longer than one FFT half (48 kHz, T60 0.45-1.2 s: 21,600-57,600
    samples, two to four partitions of 16,384) over a 52,000-sample window,
    so that every partition's delayed block spectra enter the sums: images,
    mixtures and gains of every room against the FP64 oracle (its direct
    convolution runs in the worker pool)."""
    from tests import oracle_pool as P
    batch = W.spatial_batch(6, seed=9, rt60_range=(0.45, 1.2), fs=48000.0, n_mic=2)
    n = 52000
    plan, out, sig, sir, snr, images, mix, gains = _run(batch, n, seed=4)
    parts = [(int(t) + 16383) // 16384 for t in plan.T]
    say(f"long RIRs: T {list(plan.T)} partitions {parts}, n = {n}")
    assert max(parts) == 4 and min(parts) >= 2
    mo, so = plan.mic_off, plan.src_off
    jobs = []
    for b in range(len(plan.T)):
        M, T = int(plan.n_mic[b]), int(plan.T[b])
        c0 = 3 * mo[b]
        jobs.append((out[plan.out_off[b]:plan.out_off[b + 1]].reshape(3, M, T), sig[b], float(sir[b]), float(snr[b]),
                     n, images[c0:c0 + 3 * M].reshape(3, M, n), mix[mo[b]:mo[b] + M], gains[so[b]:so[b] + 3]))
    for b, (e_img, e_mix, e_g) in enumerate(oracle_pool.map(P.spatial_errors, jobs, chunksize=1)):
        say(f"room {b}: T {plan.T[b]} images {e_img:.2e} mix {e_mix:.2e} gains {e_g:.2e}")
        assert e_img <= TOL and e_mix <= TOL and e_g <= TOL
