"""GPU checks of the batched launch machinery: hipGraph replay of the
forward + backward step equals eager execution on every replay (with eager
work and synchronisations in between); one fixed-capacity graph replays
different batches; the plain per-room launch path gives the same RIRs."""
import sys

import numpy as np
import pytest

from paper_2304_08052_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def test_graph_replay_equals_eager():
    import torch
    from paper_2304_08052_amd import framrir as fr
    say("graph replay of draw + render + backward")
    batch = W.small_mixed(6, seed=21)
    plan = fr.Plan(batch)
    table, out = plan.empty_table(), plan.empty_out()
    ws, ws_b = plan.workspace(), plan.workspace(backward=True)
    grad = torch.from_numpy(W.upstream_grad(plan.info.out_floats, seed=4)).cuda()
    grads = (torch.empty((plan.info.n_mic, 3), device="cuda"), torch.empty((plan.info.n_src, 3), device="cuda"),
             torch.empty(plan.info.n_rooms, device="cuda"))

    def step():
        plan.draw(table)
        plan.render(table, out=out, ws=ws)
        plan.backward(table, grad, ws=ws_b, grads=grads)

    step()
    torch.cuda.synchronize()
    ref = [out.clone(), table.clone()] + [g.clone() for g in grads]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(4):
        out.fill_(-1.0)
        table.zero_()
        for t in grads:
            t.fill_(7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [out, table] + list(grads)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), f"replay {rep}"
        _ = (out * 2).sum().item()        # eager work between replays


def test_capacity_graph_replays_different_batches():
    import torch
    from paper_2304_08052_amd import framrir as fr
    from paper_2304_08052_amd.stream import GraphStream
    say("fixed-capacity graph over different batches")
    gs = GraphStream(n_rooms=8, n_src_max=3, n_mic_max=8, rt60_max=0.35, fs_max=48000.0, backward=True)
    batches = [W.small_mixed(8, seed=s, rt60_range=(0.1, 0.35)) for s in (31, 32, 33)]
    plans = [fr.Plan(b) for b in batches]
    gs.load(plans[0])
    gs.capture()
    for rep, plan in enumerate(plans + plans[:1]):
        gs.load(plan)
        grad = torch.from_numpy(W.upstream_grad(plan.info.out_floats, seed=rep)).cuda()
        gs.grad[:plan.info.out_floats].copy_(grad)
        gs.replay()
        torch.cuda.synchronize()
        out, gm, gsrc, gr = gs.outputs()
        ref_out, ref_table = plan.forward()
        rm, rs, rr = plan.backward(ref_table, grad)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out), f"batch {rep}: RIRs"
        assert torch.equal(gm, rm) and torch.equal(gsrc, rs) and torch.equal(gr, rr), f"batch {rep}: grads"


def test_per_room_path_equals_batched():
    import torch
    from paper_2304_08052_amd import framrir as fr
    say("per-room launch path vs batched persistent path")
    batch = W.config2(16)
    out_b, plan, _ = fr.simulate(batch)
    pr = fr.PerRoom(batch)
    out_r = pr.forward(torch.empty_like(out_b))
    torch.cuda.synchronize()
    assert torch.equal(out_b, out_r)
