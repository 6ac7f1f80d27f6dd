"""GPU parity over whole workloads, in the launch shapes the benchmark times.

* The batched forward (256 rooms, 16 kHz, 2 sources, 6 mics) and the
  long-filter batch (64 rooms, 48 kHz, 8 mics, time-tiled): every room, the
  forward (draws fused into the preparation, then the render) per channel
  within 1e-5 relative L2, and the adjoint with the draws held fixed, run on
  the forward's preparation, per room within 1e-4 relative for dL/dmic,
  dL/dsrc and dL/dr.
* The mixed on-the-fly stream (1024 rooms per step, 16/48 kHz, 2-8 mics, 1-3
  sources, T60 up to 1 s) through its fixed-capacity hipGraph of forward +
  backward, in the shipped launch shape: two different batches replayed on
  the one captured graph, each checked on a stratified sample of 64 rooms
  (every sample-rate x microphone-count x source-count class present, the
  heaviest 48 kHz room, the rest drawn at random) to the same bars.

The oracle (FP64) runs in the worker pool forked before the GPU is touched
(tests/oracle_pool.py); only the errors come back.
"""
import sys

import numpy as np
import pytest

from paper_2304_08052_amd import workloads as W
from tests import oracle_pool as P

pytestmark = pytest.mark.gpu

RIR_TOL = 1e-5
GRAD_TOL = 1e-4


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def room_work(batch, plan, b):
    """Tap-updates plus output samples of room b (its share of the work)."""
    s0, s1 = int(plan.src_off[b]), int(plan.src_off[b + 1])
    return int(np.sum(plan.n_img[s0:s1])) * int(batch["n_mic"][b]) * 81 + int(plan.out_off[b + 1] - plan.out_off[b])


def jobs_for(batch, plan, rooms, out, G, gm, gs, gr):
    """One room_errors job per room; out and G are device or host tensors /
    arrays in the packed layout, sliced per room before the copy."""
    from paper_2304_08052_amd import framrir as fr
    ones = fr.split_rooms(batch)

    def host(x, a, b):
        x = x[a:b]
        return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)

    jobs = []
    for b in sorted(rooms, key=lambda b: -room_work(batch, plan, b)):   # heaviest first
        o0, o1 = int(plan.out_off[b]), int(plan.out_off[b + 1])
        m0, m1 = int(plan.mic_off[b]), int(plan.mic_off[b + 1])
        s0, s1 = int(plan.src_off[b]), int(plan.src_off[b + 1])
        jobs.append((b, (ones[b], host(out, o0, o1), None if G is None else host(G, o0, o1),
                         host(gm, m0, m1), host(gs, s0, s1), float(host(gr, b, b + 1)[0]))))
    return jobs


def check_jobs(pool, jobs, label):
    res = pool.map(P.room_errors, [j for _, j in jobs], chunksize=1)
    fwd_worst = bwd_worst = (0.0, None)
    chans = []
    for (b, _), (fwd, bwd) in zip(jobs, res):
        chans.append(fwd.ravel())
        e = float(fwd.max())
        if e > fwd_worst[0]:
            fwd_worst = (e, b)
        assert e <= RIR_TOL, f"{label} room {b}: per-channel rel L2 {fwd.ravel()}"
        if bwd is not None:
            em, es, er = bwd
            if max(bwd) > bwd_worst[0]:
                bwd_worst = (max(bwd), b)
            assert em <= GRAD_TOL and es <= GRAD_TOL and er <= GRAD_TOL, \
                f"{label} room {b}: grad_mic {em:.2e} grad_src {es:.2e} grad_r {er:.2e}"
    chans = np.concatenate(chans)
    say(f"{label}: {len(jobs)} rooms, {chans.size} channels, rel L2 max {chans.max():.2e} (room {fwd_worst[1]}) "
        f"median {np.median(chans):.2e}; gradients worst {bwd_worst[0]:.2e} (room {bwd_worst[1]})")


# the bin-moment render (matrix-core filter) on the same workload
MOMENTS = dict(lds_bytes=65536, wg_threads=512, grid_wgs=0, max_mic_group=2, waves_per_simd=4, render_path=1)


def run_batched(batch, seed, launch=None):
    """The benchmark's forward (prepare with the draws, then render) and the
    adjoint on that preparation, in the tuned launch shape (or `launch`)."""
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    plan = fr.Plan(batch, launch=launch or autotune.launch_for(batch))
    table, out, ws = plan.empty_table(), plan.empty_out(), plan.workspace(backward=True)
    plan.prepare(table, ws=ws, draw=True)
    plan.render_prepared(table, out=out, ws=ws)
    G = W.upstream_grad(plan.info.out_floats, seed=seed)
    gm, gs, gr = plan.backward(table, torch.from_numpy(G).cuda(), ws=ws, prepared=True)
    torch.cuda.synchronize()
    return plan, out, G, gm, gs, gr


@pytest.mark.parametrize("which", ["batched256", "long64", "batched256_moments"])
def test_every_room_forward_backward(which, oracle_pool):
    batch = W.config3() if which == "long64" else W.config2()
    launch = MOMENTS if which.endswith("moments") else None
    say(f"{which}: forward + backward of every room, launch {launch or 'tuned'}")
    plan, out, G, gm, gs, gr = run_batched(batch, seed=11, launch=launch)
    rooms = range(plan.n_rooms)
    check_jobs(oracle_pool, jobs_for(batch, plan, rooms, out, G, gm, gs, gr), which)


def stratified_rooms(batch, plan, n, seed):
    """One room of every (fs, mics, sources) class present, the heaviest
    48 kHz room, then random rooms up to n."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(plan.n_rooms)
    picked, seen = [], set()
    for b in order:
        key = (float(batch["fs"][b]), int(batch["n_mic"][b]), int(batch["n_src"][b]))
        if key not in seen:
            seen.add(key)
            picked.append(int(b))
    hi = [b for b in range(plan.n_rooms) if float(batch["fs"][b]) == 48000.0]
    heaviest = max(hi, key=lambda b: room_work(batch, plan, b))
    if heaviest not in picked:
        picked.append(heaviest)
    for b in order:
        if len(picked) >= n:
            break
        if int(b) not in picked:
            picked.append(int(b))
    return picked, heaviest, len(seen)


def test_mixed_stream_graph_replays(oracle_pool):
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    from paper_2304_08052_amd.stream import GraphStream
    launch = autotune.launch_for_stream(1024, 3, 8, 1.0, 48000.0)
    say(f"mixed stream: fixed-capacity graph, launch {launch}")
    gstream = GraphStream(n_rooms=1024, n_src_max=3, n_mic_max=8, rt60_max=1.0, fs_max=48000.0, launch=launch,
                          backward=True)
    batches = [W.config5(0), W.config5(1)]
    plans = [fr.Plan(b, launch=gstream.launch) for b in batches]
    gstream.load(plans[0])
    gstream.capture()
    for k, (batch, plan) in enumerate(zip(batches, plans)):
        n = plan.info.out_floats
        G = W.upstream_grad(n, seed=50 + k)
        gstream.out.fill_(float("nan"))
        gstream.grad[:n].copy_(torch.from_numpy(G))
        gstream.load(plan)
        gstream.replay()
        torch.cuda.synchronize()
        out, gm, gs, gr = gstream.outputs()
        assert not torch.isnan(out).any(), f"batch {k}: output not fully written"
        rooms, heaviest, classes = stratified_rooms(batch, plan, 64, seed=k)
        say(f"batch {k}: {len(rooms)} rooms over {classes} classes, heaviest 48 kHz room {heaviest} "
            f"(T {plan.T[heaviest]}, {batch['n_mic'][heaviest]} mics, {batch['n_src'][heaviest]} sources)")
        check_jobs(oracle_pool, jobs_for(batch, plan, rooms, out, G, gm, gs, gr), f"mixed batch {k}")
