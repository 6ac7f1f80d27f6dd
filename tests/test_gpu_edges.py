"""GPU parity at the edges of the admitted inputs (workloads.edge_cases):
64 microphones, a source 1 cm from a microphone, a 64-sample RIR (shorter
than the 81-tap pulse), ragged microphone groups at 48 kHz, a late direct
path, near-rigid and near-anechoic walls; and the largest image count
(65535 per source).  Draws bit-exact, RIRs within 1e-5 relative L2 per
channel, gradients within 1e-4 relative per tensor, against the FP64 oracle."""
import sys

import numpy as np
import pytest

from oracle import framrir as F
from paper_2304_08052_amd import workloads as W

pytestmark = pytest.mark.gpu

RIR_TOL = 1e-5
GRAD_TOL = 1e-4
MAX_IMG = dict(img_lo=65535, img_hi=65535)


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(got, want):
    den = np.linalg.norm(want)
    return np.linalg.norm(got - want) / den if den > 0 else np.linalg.norm(got)


def _render(batch, launch=None, params=None):
    import torch
    from paper_2304_08052_amd import framrir as fr
    plan = fr.Plan(batch, launch=launch, params=params)
    out, table = plan.forward()
    torch.cuda.synchronize()
    return plan, out.cpu().numpy(), table.cpu().numpy()


def _check_room(plan, out, rm, op, b, mics=None):
    """Channels of room b (all microphones, or the listed ones) against the oracle."""
    mics = np.arange(len(rm.mic)) if mics is None else np.asarray(mics)
    want = F.render_room(op, rm, mic=rm.mic[mics])
    got = out[plan.out_off[b]:plan.out_off[b + 1]].reshape(len(rm.src), len(rm.mic), op["T"])[:, mics]
    worst = 0.0
    for s in range(want.shape[0]):
        for j, m in enumerate(mics):
            e = rel_l2(got[s, j], want[s, j])
            worst = max(worst, e)
            assert e <= RIR_TOL, f"room {b} src {s} mic {m}: rel L2 {e:.3e}"
    return worst


def _check_draws(plan, table, rooms, oplans):
    """Reflection counts bit-exact; each source's direct-path row holds the source."""
    s_glob = 0
    for b, op in enumerate(oplans):
        for s_local, so in enumerate(op["sources"]):
            lo, hi = plan.img_off[s_glob], plan.img_off[s_glob + 1]
            assert hi - lo == so["I"] + 1
            assert np.array_equal(table[lo + 1:hi, 3].view(np.uint64), so["draws"]["g"].view(np.uint64))
            assert np.array_equal(table[lo, :3], rooms[b].src[s_local]) and table[lo, 3] == 0.0
            s_glob += 1


@pytest.mark.parametrize("launch", [None, dict(max_mic_group=16),
                                    dict(lds_bytes=8192, wg_threads=256, max_mic_group=3),
                                    dict(lds_bytes=131072, wg_threads=1024, max_mic_group=2, render_path=1),
                                    dict(lds_bytes=65536, wg_threads=512, max_mic_group=1, render_path=1)])
def test_edge_rooms_forward(launch):
    batch = W.edge_cases()
    say(f"edge rooms forward launch={launch}")
    plan, out, table = _render(batch, launch)
    rooms = F.rooms_from_batch(batch)
    oplans = [F.room_plan(rm, F.Params()) for rm in rooms]
    _check_draws(plan, table, rooms, oplans)
    for b, (rm, op) in enumerate(zip(rooms, oplans)):
        e = _check_room(plan, out, rm, op, b)
        say(f"room {b}: T {op['T']} mics {len(rm.mic)} worst rel L2 {e:.2e}")


def test_edge_rooms_largest_image_count():
    """img_lo = img_hi = 65535: every source carries the largest image count;
    the 64- and 13-microphone rooms are checked on their first and last
    microphones (the oracle's cost), the others on every channel."""
    batch = W.edge_cases()
    say("edge rooms, 65535 images per source")
    plan, out, table = _render(batch, params=MAX_IMG)
    rooms = F.rooms_from_batch(batch)
    prm = F.Params(**MAX_IMG)
    assert np.all(np.diff(plan.img_off) == 65536)
    for b, rm in enumerate(rooms):
        op = F.room_plan(rm, prm)
        mics = [0, len(rm.mic) - 1] if len(rm.mic) > 8 else None
        e = _check_room(plan, out, rm, op, b, mics)
        say(f"room {b}: worst rel L2 {e:.2e}")


def test_edge_rooms_backward():
    """Adjoint on the edge rooms (draws fixed) against the oracle adjoint."""
    import torch
    batch = W.edge_cases()
    say("edge rooms backward")
    from paper_2304_08052_amd import framrir as fr
    plan = fr.Plan(batch)
    ws = plan.workspace(backward=True)
    out, table = plan.forward(ws=ws)
    G = W.upstream_grad(plan.info.out_floats, seed=5)
    gm, gs, gr = plan.backward(table, torch.from_numpy(G).cuda(), ws=ws, prepared=True)
    torch.cuda.synchronize()
    gm, gs, gr = gm.cpu().numpy(), gs.cpu().numpy(), gr.cpu().numpy()
    mo, so = plan.mic_off, plan.src_off
    for b, rm in enumerate(F.rooms_from_batch(batch)):
        op = F.room_plan(rm, F.Params())
        gh = G[plan.out_off[b]:plan.out_off[b + 1]].astype(np.float64).reshape(len(rm.src), len(rm.mic), op["T"])
        wm, ws_, wr = F.adjoint_room(op, rm, gh)
        em = np.linalg.norm(gm[mo[b]:mo[b + 1]] - wm) / np.linalg.norm(wm)
        es = np.linalg.norm(gs[so[b]:so[b + 1]] - ws_) / np.linalg.norm(ws_)
        er = abs(gr[b] - wr) / abs(wr)
        say(f"room {b}: mic {em:.2e} src {es:.2e} r {er:.2e}")
        assert em <= GRAD_TOL and es <= GRAD_TOL and er <= GRAD_TOL
