"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars: Philox words, image counts, cube roots and every FP64 draw quantity
(theta, phi, xhat, p, DR, D, g) bit for bit; positions to FP64 rounding of the
trigonometric functions; RIRs per channel within 1e-5 relative L2 (FP32
kernels vs FP64 oracle).
"""
import math
import sys

import numpy as np
import pytest

from oracle import framrir as F
from oracle.cbrt import cbrt_rn as oracle_cbrt
from oracle.philox import philox4x32 as oracle_philox
from paper_2304_08052_amd import workloads as W

pytestmark = pytest.mark.gpu

RIR_TOL = 1e-5


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _fr():
    from paper_2304_08052_amd import framrir as fr
    return fr


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(got, want):
    den = np.linalg.norm(want)
    return np.linalg.norm(got - want) / den if den > 0 else np.linalg.norm(got)


def oracle_room(batch, b, prm=F.Params(), mic=None, src=None, r=None):
    room = F.rooms_from_batch(batch)[b]
    plan = F.room_plan(room, prm)
    return room, plan, F.render_room(plan, room, mic=mic, src=src, r=r)


def check_rooms(plan, out, batch, rooms, prm=F.Params(), tol=RIR_TOL):
    out_np = out.cpu().numpy()
    worst = 0.0
    for b in rooms:
        _, _, want = oracle_room(batch, b, prm)
        got = out_np[plan.out_off[b]:plan.out_off[b + 1]].reshape(want.shape)
        for s in range(want.shape[0]):
            for m in range(want.shape[1]):
                e = rel_l2(got[s, m], want[s, m])
                worst = max(worst, e)
                assert e <= tol, f"room {b} src {s} mic {m}: rel L2 {e:.3e}"
    return worst


def test_philox_words_bit_exact():
    torch, fr = _torch(), _fr()
    say("philox 1e6 counters")
    rng = np.random.default_rng(10)
    n = 1 << 20
    ctr = rng.integers(0, 2**32, (n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, (n, 2), dtype=np.uint64).astype(np.uint32)
    out = fr.philox4x32(torch.from_numpy(ctr.view(np.int32)).cuda(), torch.from_numpy(key.view(np.int32)).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32).astype(np.uint64)
    want = np.stack(oracle_philox(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], key[:, 0], key[:, 1]), axis=1)
    assert np.array_equal(got, want)


def test_philox_known_answer_vectors():
    torch, fr = _torch(), _fr()
    from tests.golden import philox_kat
    rows = [r for r in philox_kat() if r[0] == 32]
    ctr = np.array([r[1] for r in rows], dtype=np.uint32)
    key = np.array([r[2] for r in rows], dtype=np.uint32)
    out = fr.philox4x32(torch.from_numpy(ctr.view(np.int32)).cuda(), torch.from_numpy(key.view(np.int32)).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    assert [[int(v) for v in g] for g in got] == [r[3] for r in rows]


def test_cbrt_bit_exact():
    torch, fr = _torch(), _fr()
    say("cbrt 2e5 arguments")
    rng = np.random.default_rng(11)
    u = (rng.integers(0, 2**32, 150000).astype(np.float64) + 0.5) * 2.0**-32
    from tests.test_abi_host import near_midpoint_cubes
    x = np.concatenate([1.0 / 64.0 + u * (63.0 / 64.0), u[:20000], 10.0 ** rng.uniform(-300, 300, 30000),
                        np.array([1.0, 8.0, 27.0, 0.125, 2.0, 3.0]), near_midpoint_cubes(2000, seed=5)])
    y = fr.cbrt_rn(torch.from_numpy(x).cuda()).cpu().numpy()
    want = np.array([oracle_cbrt(float(v)) for v in x])
    assert np.array_equal(y.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("tau", [0.25, 0.5, 1.0])
def test_draws_bit_exact(tau):
    torch, fr = _torch(), _fr()
    say(f"draws config2[:12] tau={tau}")
    batch = W.config2(12)
    prm = F.Params(tau=tau)
    plan = fr.Plan(batch, params=dict(tau=tau))
    table, aux, words = plan.draw(aux=True, words=True)
    torch.cuda.synchronize()
    table, aux = table.cpu().numpy(), aux.cpu().numpy()
    words = words.cpu().numpy().view(np.uint32).astype(np.uint64)
    s_glob = 0
    for b, room in enumerate(F.rooms_from_batch(batch)):
        op = F.room_plan(room, prm)
        for so in op["sources"]:
            lo, hi = plan.img_off[s_glob], plan.img_off[s_glob + 1]
            assert hi - lo == so["I"] + 1
            d = so["draws"]
            assert np.array_equal(words[lo + 1:hi], d["words"])
            for col, key in enumerate(["theta", "phi", "xhat", "p", "dr", "dist", "g"]):
                assert np.array_equal(aux[lo + 1:hi, col].view(np.uint64), d[key].view(np.uint64)), key
            assert np.array_equal(table[lo + 1:hi, 3].view(np.uint64), d["g"].view(np.uint64))
            scale = np.maximum(1.0, d["dist"])[:, None]
            assert np.all(np.abs(table[lo + 1:hi, :3] - d["pos"]) <= 4e-15 * scale + 1e-15)
            s_glob += 1


def test_direct_rows_hold_sources():
    torch, fr = _torch(), _fr()
    say("direct-path rows")
    batch = W.small_mixed(5, seed=2)
    plan = fr.Plan(batch)
    table, _, _ = plan.draw()
    table = table.cpu().numpy()
    for s in range(plan.info.n_src):
        row = table[plan.img_off[s]]
        assert np.array_equal(row[:3], batch["src"][s]) and row[3] == 0.0


def test_render_config1():
    torch, fr = _torch(), _fr()
    say("render config1")
    batch = W.config1()
    out, plan, _ = fr.simulate(batch)
    torch.cuda.synchronize()
    worst = check_rooms(plan, out, batch, [0])
    say(f"config1 worst rel L2 {worst:.3e}")


def test_integer_delay_exact_impulse():
    torch, fr = _torch(), _fr()
    say("integer delay")
    batch = dict(size=np.array([[6.0, 5.0, 3.0]]), rt60=np.array([0.4]), fs=np.array([34300.0]),
                 c=np.array([343.0]), r_override=np.array([np.nan]), seed=np.array([0], dtype=np.uint64),
                 n_src=np.array([1]), n_mic=np.array([1]), src=np.array([[1.0, 1.0, 1.0]]),
                 mic=np.array([[2.5, 1.0, 1.0]]))
    out, plan, _ = fr.simulate(batch, params=dict(img_lo=0, img_hi=0))
    h = out.cpu().numpy()
    want = np.zeros_like(h)
    want[150] = np.float32(1.0) / np.float32(1.5)
    assert np.max(np.abs(h - want)) <= 1e-7


@pytest.mark.parametrize("launch", [None, dict(lds_bytes=32768, wg_threads=1024, max_mic_group=3),
                                    dict(lds_bytes=16384, wg_threads=256, max_mic_group=2),
                                    dict(lds_bytes=65536, wg_threads=512, max_mic_group=8, grid_wgs=7),
                                    # bin moments: time-tiled 256-sample blocks, groups of 1-3 microphones
                                    dict(lds_bytes=65536, wg_threads=512, max_mic_group=1, render_path=1),
                                    dict(lds_bytes=131072, wg_threads=1024, max_mic_group=3, render_path=1),
                                    dict(lds_bytes=24576, wg_threads=256, max_mic_group=2, grid_wgs=5,
                                         render_path=1)])
def test_render_small_mixed_tiles(launch):
    torch, fr = _torch(), _fr()
    say(f"render small_mixed launch={launch}")
    batch = W.small_mixed(6, seed=5)
    out, plan, _ = fr.simulate(batch, launch=launch)
    torch.cuda.synchronize()
    worst = check_rooms(plan, out, batch, range(6))
    say(f"small_mixed worst rel L2 {worst:.3e} items {plan.info.n_items}")


def test_render_config2_full_sampled():
    torch, fr = _torch(), _fr()
    say("render config2 B=256 (sampled rooms vs oracle)")
    batch = W.config2()
    out, plan, _ = fr.simulate(batch)
    torch.cuda.synchronize()
    out_np = out.cpu().numpy()
    assert np.all(np.isfinite(out_np))
    rooms = [0, 1, 37, 128, 200, 255]
    worst = check_rooms(plan, out, batch, rooms)
    say(f"config2 worst rel L2 {worst:.3e}")


def test_render_config3_long_filters_sampled():
    torch, fr = _torch(), _fr()
    say("render config3 B=64 48 kHz (sampled rooms)")
    batch = W.config3()
    out, plan, _ = fr.simulate(batch)
    torch.cuda.synchronize()
    assert plan.info.n_items > 64          # time-tiled
    worst = check_rooms(plan, out, batch, [0, 31, 63])
    say(f"config3 worst rel L2 {worst:.3e}")


def test_render_config5_mixed_full_sampled():
    """The mixed stream at full size (1,024 rooms: 16 and 48 kHz, 2-8
    microphones, 1-3 sources, T60 up to 1 s) in its tuned launch shape;
    sampled rooms against the oracle: the first and last, one with 2
    microphones and 1 source, one with 8 microphones and 3 sources, and the
    one with the most output samples (48 kHz, 3 x 8 channels, T60 0.98 s)."""
    from paper_2304_08052_amd import autotune
    torch, fr = _torch(), _fr()
    batch = W.config5(0)
    launch = autotune.launch_for(batch)
    say(f"render config5 B=1024 mixed (sampled rooms) launch={launch}")
    plan = fr.Plan(batch, launch=launch)
    out, _ = plan.forward()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(out.cpu().numpy()))
    rooms = F.rooms_from_batch(batch)
    heaviest = max(range(len(rooms)), key=lambda b: len(rooms[b].src) * len(rooms[b].mic) *
                   F.rir_length(rooms[b].rt60, rooms[b].fs))
    small = next(b for b, r in enumerate(rooms) if len(r.mic) == 2 and len(r.src) == 1)
    large = next(b for b, r in enumerate(rooms) if len(r.mic) == 8 and len(r.src) == 3)
    worst = check_rooms(plan, out, batch, [0, small, large, heaviest, 511, 1023])
    say(f"config5 worst rel L2 {worst:.3e}")


def test_render_perturbed_inputs_table_fixed():
    torch, fr = _torch(), _fr()
    say("render with perturbed mics and r, table fixed")
    batch = W.config4(3)
    pert = W.config4_target_perturbation(batch)
    plan = fr.Plan(batch)
    table, _, _ = plan.draw()
    mic2 = batch["mic"] + pert["mic_delta"]
    r2 = plan.r + pert["r_delta"]
    out = plan.render(table, mic=torch.from_numpy(mic2).cuda(), r=torch.from_numpy(r2).cuda())
    out_np = out.cpu().numpy()
    for b in range(3):
        mo = plan.mic_off
        _, _, want = oracle_room(batch, b, mic=mic2[mo[b]:mo[b + 1]], r=r2[b])
        got = out_np[plan.out_off[b]:plan.out_off[b + 1]].reshape(want.shape)
        for m in range(want.shape[1]):
            assert rel_l2(got[0, m], want[0, m]) <= RIR_TOL


def test_output_fully_written():
    # every sample is written: results do not depend on the buffer's contents
    torch, fr = _torch(), _fr()
    say("output fully written")
    batch = W.small_mixed(4, seed=9)
    plan = fr.Plan(batch, launch=dict(lds_bytes=32768, wg_threads=1024, max_mic_group=3))
    table, _, _ = plan.draw()
    a = plan.render(table, out=torch.full((plan.info.out_floats,), float("nan"), device="cuda"))
    b = plan.render(table, out=torch.full((plan.info.out_floats,), 7.0, device="cuda"))
    assert torch.isfinite(a).all()
    assert torch.allclose(a, b, rtol=1e-6, atol=1e-9)


def test_forward_bitwise_reproducible():
    # fixed-point accumulation: the result does not depend on the order in
    # which the workgroups' atomics land
    torch, fr = _torch(), _fr()
    say("forward determinism")
    batch = W.config2(32)
    plan = fr.Plan(batch)
    table, _, _ = plan.draw()
    a = plan.render(table).clone()
    b = plan.render(table).clone()
    c = fr.Plan(batch, launch=dict(grid_wgs=13)).render(table)
    assert torch.equal(a, b) and torch.equal(a, c)


@pytest.mark.parametrize("which", ["small_mixed", "config2"])
def test_preparation_deterministic(which):
    """The preparation (scales, bucket offsets, delay-ordered rows) is the same
    bytes on every run, and the same whether it draws the rows itself or reads
    them from a drawn table."""
    import torch
    from paper_2304_08052_amd import framrir as fr
    batch = W.small_mixed(6, seed=21) if which == "small_mixed" else W.config2()
    plan = fr.Plan(batch)
    say(f"preparation determinism {which}")
    table, _, _ = plan.draw()
    runs = [plan.prepare(table, ws=plan.workspace(), draw=False).clone() for _ in range(3)]
    t2 = plan.empty_table()
    runs.append(plan.prepare(t2, ws=plan.workspace(), draw=True).clone())
    torch.cuda.synchronize()
    for k, w in enumerate(runs[1:]):
        assert torch.equal(runs[0], w), f"run {k + 1}"
    assert torch.equal(t2, table)
