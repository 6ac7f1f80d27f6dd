"""Seeded synthetic room batches.

This module only places rooms, sources and microphones; it holds none of the
method's arithmetic.  Both the HIP path and the FP64 oracle read the arrays it
returns, so the two sides see identical inputs.

The ranges stand in for the paper's simulation set-up (Sec. IV-A): rooms from
3 x 3 x 2.5 m to 10 x 10 x 4 m, T60 in [0.1, 0.7] s, source-to-array distance
0.3-6 m, static sources.  The paper's speech and noise corpora are not used:
this path produces RIRs only.

A batch is a dict of flat numpy arrays:
  size (B,3) f64, rt60 (B,) f64, fs (B,) f64, c (B,) f64,
  r_override (B,) f64 (NaN = use Eq. 2), seed (B,) u64,
  n_src (B,) i32, n_mic (B,) i32,
  src (sum n_src, 3) f64, mic (sum n_mic, 3) f64
"""
import numpy as np

SOUND_SPEED = 343.0
WALL_MARGIN = 0.5        # sources and array centres keep this far from walls


def _empty():
    return dict(size=[], rt60=[], fs=[], c=[], r_override=[], seed=[],
                n_src=[], n_mic=[], src=[], mic=[])


def _finish(d):
    return dict(size=np.asarray(d["size"], dtype=np.float64).reshape(-1, 3),
                rt60=np.asarray(d["rt60"], dtype=np.float64),
                fs=np.asarray(d["fs"], dtype=np.float64),
                c=np.asarray(d["c"], dtype=np.float64),
                r_override=np.asarray(d["r_override"], dtype=np.float64),
                seed=np.asarray(d["seed"], dtype=np.uint64),
                n_src=np.asarray(d["n_src"], dtype=np.int32),
                n_mic=np.asarray(d["n_mic"], dtype=np.int32),
                src=np.asarray(d["src"], dtype=np.float64).reshape(-1, 3),
                mic=np.asarray(d["mic"], dtype=np.float64).reshape(-1, 3))


def circular_array(centre, n_mic, radius, yaw):
    """Horizontal uniform circular array."""
    ang = yaw + 2.0 * np.pi * np.arange(n_mic) / n_mic
    return np.stack([centre[0] + radius * np.cos(ang),
                     centre[1] + radius * np.sin(ang),
                     np.full(n_mic, centre[2])], axis=1)


def linear_array(centre, n_mic, spacing, yaw):
    """Horizontal uniform linear array centred on ``centre``."""
    off = (np.arange(n_mic) - (n_mic - 1) / 2.0) * spacing
    return np.stack([centre[0] + off * np.cos(yaw),
                     centre[1] + off * np.sin(yaw),
                     np.full(n_mic, centre[2])], axis=1)


def _inside(rng, size, margin):
    return np.array([rng.uniform(margin, size[k] - margin) for k in range(3)])


def _add_room(d, rng, size, rt60, fs, seed, n_src, mics, dist_range=(0.3, 6.0)):
    centre = mics.mean(axis=0)
    srcs = []
    for _ in range(n_src):
        for _attempt in range(10000):
            s = _inside(rng, size, WALL_MARGIN)
            if dist_range[0] <= np.linalg.norm(s - centre) <= dist_range[1]:
                break
        else:
            raise RuntimeError("could not place a source")
        srcs.append(s)
    d["size"].append(size)
    d["rt60"].append(rt60)
    d["fs"].append(fs)
    d["c"].append(SOUND_SPEED)
    d["r_override"].append(np.nan)
    d["seed"].append(seed)
    d["n_src"].append(n_src)
    d["n_mic"].append(len(mics))
    d["src"].extend(srcs)
    d["mic"].extend(list(mics))


def config1():
    """One shoebox room 6 x 5 x 3 m, T60 0.4 s, fs 16 kHz, one source at
    (2, 3, 1.5) m, two microphones 5 cm apart along x centred at
    (4, 2.5, 1.2) m, seed 0."""
    d = _empty()
    d["size"].append([6.0, 5.0, 3.0])
    d["rt60"].append(0.4)
    d["fs"].append(16000.0)
    d["c"].append(SOUND_SPEED)
    d["r_override"].append(np.nan)
    d["seed"].append(0)
    d["n_src"].append(1)
    d["n_mic"].append(2)
    d["src"].append([2.0, 3.0, 1.5])
    d["mic"].extend([[3.975, 2.5, 1.2], [4.025, 2.5, 1.2]])
    return _finish(d)


def _uca_rooms(n_rooms, rng, n_src, n_mic, rt60_range, fs_choices, seed0=0,
               size_lo=(3.0, 3.0, 2.5), size_hi=(10.0, 10.0, 4.0), radius=0.05):
    d = _empty()
    for b in range(n_rooms):
        size = np.array([rng.uniform(size_lo[k], size_hi[k]) for k in range(3)])
        rt60 = rng.uniform(*rt60_range)
        fs = float(fs_choices[rng.integers(len(fs_choices))])
        ns = n_src if np.isscalar(n_src) else int(rng.integers(n_src[0], n_src[1] + 1))
        nm = n_mic if np.isscalar(n_mic) else int(rng.integers(n_mic[0], n_mic[1] + 1))
        centre = _inside(rng, size, WALL_MARGIN)
        mics = circular_array(centre, nm, radius, rng.uniform(0.0, 2.0 * np.pi))
        _add_room(d, rng, size, rt60, fs, seed0 + b, ns, mics)
    return _finish(d)


def config2(n_rooms=256):
    """Batched forward: rooms U(3,10) x U(3,10) x U(2.5,4) m, T60 U(0.1,0.7) s,
    fs 16 kHz, 2 sources, 6-mic circular array of radius 5 cm, seeds 0..B-1."""
    rng = np.random.default_rng(1002)
    return _uca_rooms(n_rooms, rng, 2, 6, (0.1, 0.7), (16000.0,))


def config3(n_rooms=64):
    """Long filters: rooms U(8,20) x U(8,20) x U(3,6) m, T60 U(0.6,1.2) s,
    fs 48 kHz, 1 source, 8-mic linear array with 3 cm spacing."""
    rng = np.random.default_rng(1003)
    d = _empty()
    for b in range(n_rooms):
        size = np.array([rng.uniform(8.0, 20.0), rng.uniform(8.0, 20.0), rng.uniform(3.0, 6.0)])
        rt60 = rng.uniform(0.6, 1.2)
        centre = _inside(rng, size, WALL_MARGIN)
        mics = linear_array(centre, 8, 0.03, rng.uniform(0.0, 2.0 * np.pi))
        _add_room(d, rng, size, rt60, 48000.0, b, 1, mics)
    return _finish(d)


def config4(n_rooms=128):
    """Differentiable form: as config2 but 1 source and a 4-mic circular array."""
    rng = np.random.default_rng(1004)
    return _uca_rooms(n_rooms, rng, 1, 4, (0.1, 0.7), (16000.0,))


def config4_target_perturbation(batch):
    """Perturbations that define the target RIR of the differentiable form:
    microphones moved by N(0, 1 cm) per coordinate, reflection coefficient
    raised by 0.05."""
    rng = np.random.default_rng(2004)
    return dict(mic_delta=rng.normal(0.0, 0.01, size=batch["mic"].shape), r_delta=0.05)


def config5(step=0, n_rooms=1024):
    """Mixed on-the-fly stream: fs from {16, 48} kHz, 2-8 mics (circular,
    radius 5 cm), 1-3 sources, T60 U(0.1, 1.0) s, rooms as config2; the
    per-room seed is step * n_rooms + b."""
    rng = np.random.default_rng([1005, step])
    return _uca_rooms(n_rooms, rng, (1, 3), (2, 8), (0.1, 1.0), (16000.0, 48000.0),
                      seed0=step * n_rooms)


def small_mixed(n_rooms=4, seed=7, fs_choices=(16000.0, 48000.0), rt60_range=(0.1, 0.35)):
    """Small mixed batch for parity tests that the oracle finishes in seconds:
    uneven sizes, T60, fs, source and microphone counts."""
    rng = np.random.default_rng([1100, seed])
    return _uca_rooms(n_rooms, rng, (1, 3), (1, 8), rt60_range, fs_choices, seed0=seed * 1000)


def _explicit_room(d, size, rt60, fs, seed, srcs, mics, r=np.nan):
    d["size"].append(list(size))
    d["rt60"].append(rt60)
    d["fs"].append(fs)
    d["c"].append(SOUND_SPEED)
    d["r_override"].append(r)
    d["seed"].append(seed)
    d["n_src"].append(len(srcs))
    d["n_mic"].append(len(mics))
    d["src"].extend([list(v) for v in srcs])
    d["mic"].extend([list(v) for v in mics])


def edge_cases():
    """Rooms at the edges of the admitted inputs, in one batch:
      0  64 microphones (the largest count), circular array of radius 0.2 m, 2 sources;
      1  a source 1 cm from a microphone (near field, direct-path gain 100);
      2  T60 4 ms at 16 kHz: a 64-sample RIR, shorter than the 81-tap pulse;
      3  48 kHz, 13-microphone linear array (ragged microphone groups), 3 sources;
      4  10 x 10 x 4 m room, T60 0.1 s, source 6 m away (direct path late in the RIR);
      5  reflection coefficient 0.95 (near-rigid walls);
      6  reflection coefficient 0.02 (near-anechoic walls)."""
    d = _empty()
    _explicit_room(d, (7.0, 6.0, 3.0), 0.3, 16000.0, 501,
                   [(1.5, 1.2, 1.4), (5.6, 4.9, 2.1)], circular_array((3.5, 3.0, 1.5), 64, 0.2, 0.1))
    _explicit_room(d, (4.0, 4.0, 3.0), 0.25, 16000.0, 502,
                   [(2.01, 2.0, 1.5)], [(2.0, 2.0, 1.5), (2.05, 2.0, 1.5)])
    _explicit_room(d, (3.0, 3.0, 2.5), 0.004, 16000.0, 503,
                   [(1.3, 1.5, 1.2)], [(1.6, 1.5, 1.2)])
    _explicit_room(d, (6.0, 5.0, 3.2), 0.2, 48000.0, 504,
                   [(1.0, 1.0, 1.6), (4.8, 3.9, 1.1), (3.0, 4.2, 2.5)],
                   linear_array((3.2, 2.1, 1.3), 13, 0.03, 0.7))
    _explicit_room(d, (10.0, 10.0, 4.0), 0.1, 16000.0, 505,
                   [(8.5, 5.0, 2.0)], [(2.5, 5.0, 2.0)])
    _explicit_room(d, (5.0, 4.0, 3.0), 0.5, 16000.0, 506,
                   [(1.0, 1.0, 1.0)], [(3.9, 2.8, 1.7), (3.95, 2.8, 1.7)], r=0.95)
    _explicit_room(d, (5.0, 4.0, 3.0), 0.5, 16000.0, 507,
                   [(1.0, 3.0, 2.0), (4.0, 1.0, 1.0)], [(2.5, 2.0, 1.5)], r=0.02)
    return _finish(d)


def spatial_batch(n_rooms=256, seed=0, rt60_range=(0.1, 0.7), fs=16000.0, n_mic=4):
    """Rooms for the spatialisation workload (Sec. IV-A, the speed set-up of
    Table 2): rooms U(3,10) x U(3,10) x U(2.5,4) m, T60 U(0.1,0.7) s, 16 kHz,
    three sources per room (two speakers and a point-source noise) 0.3-6 m
    from the array centre, the 4-microphone linear array of the evaluation
    set (spacings 4, 8, 4 cm), seeds 10000 + b.  fs and n_mic (2: the array's
    inner pair) give the long-RIR variants."""
    rng = np.random.default_rng([1006, seed])
    d = _empty()
    for b in range(n_rooms):
        size = np.array([rng.uniform(3.0, 10.0), rng.uniform(3.0, 10.0), rng.uniform(2.5, 4.0)])
        rt60 = rng.uniform(*rt60_range)
        centre = _inside(rng, size, WALL_MARGIN)
        yaw = rng.uniform(0.0, 2.0 * np.pi)
        off = np.array([-0.08, -0.04, 0.04, 0.08]) if n_mic == 4 else np.array([-0.04, 0.04])
        mics = np.stack([centre[0] + off * np.cos(yaw), centre[1] + off * np.sin(yaw), np.full(len(off), centre[2])],
                        axis=1)
        _add_room(d, rng, size, rt60, float(fs), 10000 + b, 3, mics)
    return _finish(d)


def spatial_signals(batch, n_samples, seed=0):
    """Seeded stand-ins for the dry signals of Sec. IV-A (the paper's speech and
    noise corpora are not used).  Speakers: Gaussian noise under a random
    syllable-rate envelope (2-6 Hz) with silent gaps, active on spans whose
    overlap is at least half of their union; noise: white Gaussian over the
    whole window.  SIR U(-6, 6) dB, SNR U(10, 20) dB.  Returns sig [B, 3, N]
    (float32), sir_db [B], snr_db [B] (float32)."""
    rng = np.random.default_rng([2006, seed])
    B, N = len(batch["rt60"]), n_samples
    sig = np.zeros((B, 3, N), dtype=np.float32)
    t = np.arange(N) / float(batch["fs"][0])
    for b in range(B):
        l1, l2 = (int(rng.uniform(0.75, 1.0) * N) for _ in range(2))
        spans = [(0, l1), (N - l2, N)]
        if rng.uniform() < 0.5:
            spans.reverse()
        for s, (a, e) in enumerate(spans):
            rate = rng.uniform(2.0, 6.0)
            env = np.clip(np.sin(2.0 * np.pi * rate * t + rng.uniform(0, 2 * np.pi)), 0.0, None) ** 2
            x = rng.standard_normal(N) * env * rng.uniform(0.2, 1.0)
            x[:a] = 0.0
            x[e:] = 0.0
            sig[b, s] = x
        sig[b, 2] = rng.standard_normal(N) * rng.uniform(0.05, 0.5)
    sir = rng.uniform(-6.0, 6.0, B).astype(np.float32)
    snr = rng.uniform(10.0, 20.0, B).astype(np.float32)
    return sig, sir, snr


def t60_curriculum_range(epoch, t60_max):
    """T60 range (seconds) for a training epoch (0-based) under the T60
    curriculum of Sec. V: [0.05, 0.10] s at the first epoch, the upper bound
    raised by 0.05 s per epoch until it reaches t60_max."""
    hi = min(t60_max, 0.10 + 0.05 * epoch)
    return 0.05, max(0.05, hi)


def t60_curriculum_sample(epoch, t60_max, n, seed=0):
    """n T60 values drawn uniformly from the epoch's curriculum range (seeded)."""
    lo, hi = t60_curriculum_range(epoch, t60_max)
    return np.random.default_rng([4000, seed, epoch]).uniform(lo, hi, n)


def upstream_grad(shape_total, seed=0):
    """Seeded N(0, 1) FP32 upstream gradient for backward benchmarks."""
    rng = np.random.default_rng([3000, seed])
    return rng.standard_normal(shape_total).astype(np.float32)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
