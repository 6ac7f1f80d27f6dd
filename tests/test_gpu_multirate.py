"""GPU parity of the paper-literal multi-rate rendering (Sec. II, Sec. III-D,
Eq. 7-8; readings R-24..R-27) against the FP64 oracle: the intermediate signal
at r_l fs (impulses on the high-rate grid, down-sampled) and the output at fs
after the 80 Hz high-pass and the decimation; 1e-5 relative L2 per channel,
the RIR tolerance."""
import sys

import numpy as np
import pytest

from oracle import framrir as F
from oracle import multirate as M
from paper_2304_08052_amd import workloads as W

pytestmark = pytest.mark.gpu

RIR_TOL = 1e-5


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def worst_channel(got, want):
    """Largest per-channel relative L2 error over a room's [S, M, T] RIRs."""
    return max(rel(got[s, m], want[s, m]) for s in range(want.shape[0]) for m in range(want.shape[1]))


def _short_batch():
    # 16 and 48 kHz rooms with short T60 so that the oracle stays quick
    return W.small_mixed(4, seed=17, fs_choices=(16000.0, 48000.0), rt60_range=(0.08, 0.2))


def _check_rooms(batch, plan, out, inter, rooms_to_check):
    out = out.cpu().numpy()
    inter = inter.cpu().numpy()
    mr = plan.info.mr_floats
    prm = F.Params()
    rooms = F.rooms_from_batch(batch)
    mr_off = 0
    offs = []
    for rm in rooms:
        _, t_l, _ = M.lengths(rm.rt60, rm.fs)
        offs.append(mr_off)
        mr_off += len(rm.src) * len(rm.mic) * t_l
    assert mr_off == mr
    for b in rooms_to_check:
        rm = rooms[b]
        op = F.room_plan(rm, prm)
        _, t_l, t_len = M.lengths(rm.rt60, rm.fs)
        n = len(rm.src) * len(rm.mic)
        want_l = M.intermediate_room(op, rm)
        got_l = inter[offs[b]:offs[b] + n * t_l].reshape(want_l.shape)
        e1 = worst_channel(got_l, want_l)
        want = M.multirate_room(op, rm)
        got = out[plan.out_off[b]:plan.out_off[b + 1]].reshape(want.shape)
        e3 = worst_channel(got, want)
        say(f"room {b} fs {rm.fs:.0f}: intermediate {e1:.2e} output {e3:.2e}")
        assert e1 <= RIR_TOL and e3 <= RIR_TOL


def test_multirate_stages_match_oracle():
    import torch
    from paper_2304_08052_amd import framrir as fr
    batch = _short_batch()
    plan = fr.Plan(batch, multirate=True)
    say("multi-rate short batch")
    out, table, inter = plan.forward_multirate()
    torch.cuda.synchronize()
    _check_rooms(batch, plan, out, inter, range(len(batch["rt60"])))


def test_multirate_edge_rooms():
    """64 microphones, a near-field source, a 64-sample RIR (448 intermediate
    samples: less than two filter chunks, one partial decimation tile),
    48 kHz with 13 microphones, extreme reflection coefficients."""
    import torch
    from paper_2304_08052_amd import framrir as fr
    batch = W.edge_cases()
    plan = fr.Plan(batch, multirate=True)
    say("multi-rate edge rooms")
    out, table, inter = plan.forward_multirate()
    torch.cuda.synchronize()
    _check_rooms(batch, plan, out, inter, range(len(batch["rt60"])))


def test_multirate_config2_sampled():
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    batch = W.config2()
    plan = fr.Plan(batch, launch=autotune.launch_for(batch), multirate=True)
    say("multi-rate config2")
    out, table, inter = plan.forward_multirate()
    torch.cuda.synchronize()
    _check_rooms(batch, plan, out, inter, (0, 255))


def test_multirate_reproducible_and_single_rate_calls_refused():
    import torch
    from paper_2304_08052_amd import framrir as fr
    batch = _short_batch()
    plan = fr.Plan(batch, multirate=True)
    a = plan.forward_multirate()[0].clone()
    b = plan.forward_multirate()[0].clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(fr.FramrirError):
        plan.forward()
    with pytest.raises(fr.FramrirError):
        plan.backward(plan.empty_table(), torch.zeros(plan.info.out_floats, device="cuda"))


def test_multirate_every_room_of_the_batched_workload(oracle_pool):
    """Every room of the 256-room batch through the multi-rate chain, in the
    tuned launch shape, against the oracle (worker processes forked before
    the GPU was used): both the intermediate signal and the output, worst
    channel of each room at 1e-5."""
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    from tests import oracle_pool as P
    batch = W.config2()
    plan = fr.Plan(batch, launch=autotune.launch_for(batch), multirate=True)
    say("multi-rate, every room of the 256-room batch")
    out, table, inter = plan.forward_multirate()
    torch.cuda.synchronize()
    out, inter = out.cpu().numpy(), inter.cpu().numpy()
    ones = fr.split_rooms(batch)
    jobs, off = [], 0
    for b, rm in enumerate(F.rooms_from_batch(batch)):
        _, t_l, _ = M.lengths(rm.rt60, rm.fs)
        n = len(rm.src) * len(rm.mic) * t_l
        jobs.append((ones[b], inter[off:off + n], out[plan.out_off[b]:plan.out_off[b + 1]]))
        off += n
    assert off == plan.info.mr_floats
    res = oracle_pool.map(P.multirate_errors, jobs, chunksize=1)
    e1 = np.array([r[0] for r in res])
    e3 = np.array([r[1] for r in res])
    say(f"multi-rate every room: intermediate worst {e1.max():.2e} (room {int(e1.argmax())}), "
        f"output worst {e3.max():.2e} (room {int(e3.argmax())}), output median {np.median(e3):.2e}")
    assert e1.max() <= RIR_TOL and e3.max() <= RIR_TOL


def test_multirate_every_decimation_ratio():
    """One room per r_l from 2 to 12 (6 kHz .. 192 kHz): each r_l has its own
    fragment table, filter half-length, window pad and step count in the
    decimation kernel, so every one the plan accepts apart from the 16 and
    48 kHz rooms above (r_l = 7 and 4) is rendered here against the oracle."""
    import torch
    from paper_2304_08052_amd import framrir as fr
    fss = (6000.0, 8000.0, 11025.0, 22050.0, 32000.0, 96000.0, 192000.0)
    batch = W.small_mixed(len(fss), seed=31, fs_choices=(16000.0,), rt60_range=(0.06, 0.15))
    batch["fs"] = np.array(fss)
    assert sorted(M.rate_factors(f)[1] for f in fss) == [2, 3, 5, 6, 9, 11, 12]
    plan = fr.Plan(batch, multirate=True)
    say("multi-rate, r_l = 2 .. 12")
    out, table, inter = plan.forward_multirate()
    torch.cuda.synchronize()
    _check_rooms(batch, plan, out, inter, range(len(fss)))
