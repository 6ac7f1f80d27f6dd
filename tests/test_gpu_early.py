"""GPU parity of the early-reverberation windows (Eq. 9, reading R-23):
window starts bit-exact with the oracle's FP64 decision, window values equal
to the rendered RIR samples bit for bit (zero outside [0, T)), and against the
oracle's early filter of its own RIRs within the RIR tolerance."""
import sys

import numpy as np
import pytest

from oracle import framrir as F
from paper_2304_08052_amd import workloads as W

pytestmark = pytest.mark.gpu

RIR_TOL = 1e-5


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def _oracle_starts(batch):
    starts = []
    for rm in F.rooms_from_batch(batch):
        for s in range(len(rm.src)):
            for m in range(len(rm.mic)):
                _, _, t, _ = F.pair_geometry(rm.src[s][None, :], np.zeros(1), rm.mic[m], 0.5, rm.fs, rm.c)
                starts.append(F.early_window(float(t[0]), rm.fs)[0])
    return np.asarray(starts, dtype=np.int64)


def _run(batch, launch=None):
    import torch
    from paper_2304_08052_amd import framrir as fr
    plan = fr.Plan(batch, launch=launch)
    out, table = plan.forward()
    early, start = plan.early(out)
    torch.cuda.synchronize()
    return plan, out.cpu().numpy(), early.cpu().numpy(), start.cpu().numpy()


def _check_windows_equal_output(plan, out, early, start):
    ch = 0
    for b in range(plan.n_rooms):
        T, w = int(plan.T[b]), int(plan.early_width[b])
        h = out[plan.out_off[b]:plan.out_off[b + 1]].reshape(-1, T)
        e = early[plan.early_off[b]:plan.early_off[b + 1]].reshape(-1, w)
        for k in range(h.shape[0]):
            n = start[ch + k] + np.arange(w)
            ok = (n >= 0) & (n < T)
            want = np.zeros(w, dtype=np.float32)
            want[ok] = h[k, n[ok]]
            assert np.array_equal(e[k], want), f"room {b} channel {k}"
        ch += h.shape[0]


def _edge_batch():
    # one room, T = 800: a mic 0.2 m from the source (window starts before 0)
    # and one ~4.4 m away (window runs past T)
    return dict(size=np.array([[6.0, 5.0, 3.0]]), rt60=np.array([0.05]), fs=np.array([16000.0]),
                c=np.array([343.0]), r_override=np.array([np.nan]), seed=np.array([7], dtype=np.uint64),
                n_src=np.array([1], dtype=np.int32), n_mic=np.array([2], dtype=np.int32),
                src=np.array([[2.0, 2.0, 1.5]]), mic=np.array([[2.2, 2.0, 1.5], [5.5, 4.5, 2.5]]))


@pytest.mark.parametrize("which", ["small_mixed", "edges", "edge_cases"])
def test_early_matches_oracle(which):
    batch = dict(small_mixed=lambda: W.small_mixed(6, seed=31), edges=_edge_batch,
                 edge_cases=W.edge_cases)[which]()
    say(f"early windows {which}")
    plan, out, early, start = _run(batch)
    assert np.array_equal(start.astype(np.int64), _oracle_starts(batch))
    _check_windows_equal_output(plan, out, early, start)
    prm = F.Params()
    for b, rm in enumerate(F.rooms_from_batch(batch)):
        h = F.render_room(F.room_plan(rm, prm), rm)
        want, wstart = F.early_room(rm, h)
        got = early[plan.early_off[b]:plan.early_off[b + 1]].reshape(want.shape)
        errs = [np.linalg.norm(got[s, m] - want[s, m]) / np.linalg.norm(want[s, m])
                for s in range(want.shape[0]) for m in range(want.shape[1])]
        say(f"room {b}: worst channel rel-L2 {max(errs):.2e}")
        assert max(errs) <= RIR_TOL
    if which == "edges":
        assert start[0] < 0 and start[1] + plan.early_width[0] > plan.T[0]


@pytest.mark.parametrize("which", ["config2", "config3"])
def test_early_full_workloads(which):
    from paper_2304_08052_amd import autotune
    batch = W.config2() if which == "config2" else W.config3()
    say(f"early windows {which}")
    plan, out, early, start = _run(batch, launch=autotune.launch_for(batch))
    assert np.array_equal(start.astype(np.int64), _oracle_starts(batch))
    _check_windows_equal_output(plan, out, early, start)


@pytest.mark.parametrize("which,launch", [
    ("edges", None),
    ("edge_cases", None),
    ("small_mixed", dict(lds_bytes=16384, wg_threads=256, max_mic_group=2)),   # many time tiles
    ("small_mixed", dict(lds_bytes=65536, wg_threads=512, max_mic_group=2, render_path=1)),
    ("edge_cases", dict(lds_bytes=65536, wg_threads=512, max_mic_group=1, render_path=1)),
    ("config2", "tuned"),
])
def test_early_fused_in_render(which, launch):
    """framrir_forward_early: the windows come from the render pass itself
    (every output sample stored once more when it lies in its channel's
    window, the edge items writing the zeros and the start indices): the RIRs
    equal framrir_forward's and the windows and starts equal framrir_early's,
    bit for bit, in both render paths and under time tiling."""
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    batch = dict(small_mixed=lambda: W.small_mixed(6, seed=31), edges=_edge_batch, edge_cases=W.edge_cases,
                 config2=W.config2)[which]()
    if launch == "tuned":
        launch = autotune.launch_for(batch)
    say(f"fused early windows {which} launch={launch}")
    plan = fr.Plan(batch, launch=launch)
    early_f = torch.full((plan.info.early_floats,), float("nan"), dtype=torch.float32, device="cuda")
    start_f = torch.full((plan.info.n_chan,), -7, dtype=torch.int32, device="cuda")
    out_f, _, early_f, start_f = plan.forward_early(early=early_f, start=start_f)
    out, _ = plan.forward()
    early, start = plan.early(out)
    torch.cuda.synchronize()
    assert torch.equal(out_f, out)
    assert torch.equal(start_f, start)
    assert torch.equal(early_f, early), "fused windows differ from the separate early kernel"
    assert np.array_equal(start.cpu().numpy().astype(np.int64), _oracle_starts(batch))
