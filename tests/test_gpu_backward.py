"""GPU parity of the adjoint (render backward, draws held fixed) against the
FP64 oracle adjoint and FP64 finite differences: 1e-4 relative per tensor."""
import sys

import numpy as np
import pytest

from oracle import framrir as F
from paper_2304_08052_amd import workloads as W

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _setup(n_rooms, launch=None, params=None):
    import torch
    from paper_2304_08052_amd import framrir as fr
    batch = W.config4(n_rooms)
    pert = W.config4_target_perturbation(batch)
    prm = F.Params(**(params or {}))
    plan = fr.Plan(batch, launch=launch, params=params)
    table, _, _ = plan.draw()
    rooms = F.rooms_from_batch(batch)
    oplans = [F.room_plan(rm, prm) for rm in rooms]
    G = np.zeros(plan.info.out_floats, dtype=np.float32)
    targets = []
    for b, (rm, op) in enumerate(zip(rooms, oplans)):
        mo = plan.mic_off
        h = F.render_room(op, rm)
        tgt = F.render_room(op, rm, mic=rm.mic + pert["mic_delta"][mo[b]:mo[b + 1]], r=op["r"] + pert["r_delta"])
        targets.append(tgt)
        G[plan.out_off[b]:plan.out_off[b + 1]] = (2.0 * (h - tgt)).astype(np.float32).ravel()
    return torch, fr, batch, plan, table, rooms, oplans, G, targets


@pytest.mark.parametrize("launch", [None, dict(lds_bytes=32768, wg_threads=1024, max_mic_group=2),
                                    dict(lds_bytes=65536, wg_threads=512, bwd_wg_threads=1024, bwd_grid_wgs=300),
                                    dict(lds_bytes=65536, wg_threads=512, max_mic_group=2, render_path=1)])
def test_backward_matches_oracle_adjoint(launch):
    torch, fr, batch, plan, table, rooms, oplans, G, _ = _setup(4, launch)
    say(f"backward vs oracle adjoint launch={launch}")
    gm, gs, gr = plan.backward(table, torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    gm, gs, gr = gm.cpu().numpy(), gs.cpu().numpy(), gr.cpu().numpy()
    for b, (rm, op) in enumerate(zip(rooms, oplans)):
        gh = G[plan.out_off[b]:plan.out_off[b + 1]].astype(np.float64).reshape(len(rm.src), len(rm.mic), op["T"])
        wm, ws, wr = F.adjoint_room(op, rm, gh)
        mo, so = plan.mic_off, plan.src_off
        em, es, er = rel(gm[mo[b]:mo[b + 1]], wm), rel(gs[so[b]:so[b + 1]], ws), abs(gr[b] - wr) / abs(wr)
        say(f"room {b}: mic {em:.2e} src {es:.2e} r {er:.2e}")
        assert em <= GRAD_TOL and es <= GRAD_TOL and er <= GRAD_TOL


def test_backward_matches_finite_differences():
    torch, fr, batch, plan, table, rooms, oplans, G, targets = _setup(2, params=dict(img_lo=200, img_hi=400))
    say("backward vs FP64 finite differences")
    gm, gs, gr = plan.backward(table, torch.from_numpy(G).cuda())
    gm, gs, gr = gm.cpu().numpy(), gs.cpu().numpy(), gr.cpu().numpy()
    for b, (rm, op) in enumerate(zip(rooms, oplans)):
        fm, fs_, fr_ = F.fd_grads(op, rm, targets[b], step=1e-6)
        mo, so = plan.mic_off, plan.src_off
        assert rel(gm[mo[b]:mo[b + 1]], fm) <= GRAD_TOL
        assert rel(gs[so[b]:so[b + 1]], fs_) <= GRAD_TOL
        assert abs(gr[b] - fr_) / abs(fr_) <= GRAD_TOL


def test_backward_bitwise_reproducible():
    torch, fr, batch, plan, table, rooms, oplans, G, _ = _setup(3)
    say("backward determinism")
    g = torch.from_numpy(G).cuda()
    a = [t.clone() for t in plan.backward(table, g)]
    b = [t.clone() for t in plan.backward(table, g)]
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_autograd_function():
    import torch
    from paper_2304_08052_amd import framrir as fr
    say("autograd RenderFn")
    batch = W.config4(2)
    plan = fr.Plan(batch)
    table, _, _ = plan.draw()
    mic = plan.mic_dev.clone().requires_grad_(True)
    src = plan.src_dev.clone().requires_grad_(True)
    r = torch.from_numpy(plan.r).cuda().requires_grad_(True)
    out = fr.render_differentiable(plan, table, mic, src, r)
    tgt = torch.randn_like(out)
    loss = ((out - tgt) ** 2).sum()
    loss.backward()
    gm, gs, gr = plan.backward(table, (2 * (out - tgt)).detach())
    assert torch.allclose(mic.grad.float(), gm, rtol=1e-6, atol=0)
    assert torch.allclose(src.grad.float(), gs, rtol=1e-6, atol=0)
    assert torch.allclose(r.grad.float(), gr, rtol=1e-6, atol=0)


def test_backward_prepared_reuses_forward_preparation():
    """framrir_render_backward_prepared after a forward on the same workspace
    equals the standalone backward bit for bit, on two calls in a row."""
    torch, fr, batch, plan, table, rooms, oplans, G, _ = _setup(3)
    say("backward_prepared vs standalone backward")
    g = torch.from_numpy(G).cuda()
    want = [t.clone() for t in plan.backward(table, g)]
    ws = plan.workspace(backward=True)
    out, table2 = plan.forward(ws=ws)
    assert torch.equal(table2, table)
    for call in range(2):
        got = plan.backward(table2, g, ws=ws, prepared=True)
        torch.cuda.synchronize()
        for x, y in zip(got, want):
            assert torch.equal(x, y), f"call {call}"


def test_backward_config2_full_sampled():
    """Full batched workload (256 rooms, 6 mics, 16 kHz) in the launch shape the
    benchmark uses, forward + prepared backward; sampled rooms against the
    FP64 oracle adjoint."""
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    batch = W.config2()
    launch = autotune.launch_for(batch)
    say(f"config2 backward launch={launch}")
    plan = fr.Plan(batch, launch=launch)
    ws = plan.workspace(backward=True)
    out, table = plan.forward(ws=ws)
    G = W.upstream_grad(plan.info.out_floats)
    gm, gs, gr = plan.backward(table, torch.from_numpy(G).cuda(), ws=ws, prepared=True)
    torch.cuda.synchronize()
    gm, gs, gr = gm.cpu().numpy(), gs.cpu().numpy(), gr.cpu().numpy()
    prm = F.Params()
    rooms = F.rooms_from_batch(batch)
    for b in (0, 131, 255):
        rm = rooms[b]
        op = F.room_plan(rm, prm)
        gh = G[plan.out_off[b]:plan.out_off[b + 1]].astype(np.float64).reshape(len(rm.src), len(rm.mic), op["T"])
        wm, ws_, wr = F.adjoint_room(op, rm, gh)
        mo, so = plan.mic_off, plan.src_off
        em, es, er = rel(gm[mo[b]:mo[b + 1]], wm), rel(gs[so[b]:so[b + 1]], ws_), abs(gr[b] - wr) / abs(wr)
        say(f"room {b}: mic {em:.2e} src {es:.2e} r {er:.2e}")
        assert em <= GRAD_TOL and es <= GRAD_TOL and er <= GRAD_TOL


def test_backward_config4_full_sampled():
    """Differentiable workload at full size (128 rooms, 4 mics, loss against a
    perturbed target) in the tuned launch shape: sampled rooms against the
    FP64 oracle adjoint."""
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    batch = W.config4()
    pert = W.config4_target_perturbation(batch)
    launch = autotune.launch_for(batch)
    say(f"config4 backward launch={launch}")
    plan = fr.Plan(batch, launch=launch)
    ws = plan.workspace(backward=True)
    out, table = plan.forward(ws=ws)
    prm = F.Params()
    rooms = F.rooms_from_batch(batch)
    sample = (0, 64, 127)
    h = out.cpu().numpy()
    G = np.zeros(plan.info.out_floats, dtype=np.float32)
    oracle = {}
    for b, rm in enumerate(rooms):
        op = F.room_plan(rm, prm) if b in sample else None
        mo = plan.mic_off
        if b in sample:
            tgt = F.render_room(op, rm, mic=rm.mic + pert["mic_delta"][mo[b]:mo[b + 1]], r=op["r"] + pert["r_delta"])
            G[plan.out_off[b]:plan.out_off[b + 1]] = (2.0 * (h[plan.out_off[b]:plan.out_off[b + 1]]
                                                         - tgt.ravel())).astype(np.float32)
            oracle[b] = (rm, op)
    gm, gs, gr = plan.backward(table, torch.from_numpy(G).cuda(), ws=ws, prepared=True)
    torch.cuda.synchronize()
    gm, gs, gr = gm.cpu().numpy(), gs.cpu().numpy(), gr.cpu().numpy()
    for b, (rm, op) in oracle.items():
        gh = G[plan.out_off[b]:plan.out_off[b + 1]].astype(np.float64).reshape(len(rm.src), len(rm.mic), op["T"])
        wm, ws_, wr = F.adjoint_room(op, rm, gh)
        mo, so = plan.mic_off, plan.src_off
        em, es, er = rel(gm[mo[b]:mo[b + 1]], wm), rel(gs[so[b]:so[b + 1]], ws_), abs(gr[b] - wr) / abs(wr)
        say(f"room {b}: mic {em:.2e} src {es:.2e} r {er:.2e}")
        assert em <= GRAD_TOL and es <= GRAD_TOL and er <= GRAD_TOL
