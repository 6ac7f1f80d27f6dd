"""GPU parity on seeded random batches of unusual shapes: sample rates 8 to 48
kHz (the rates the other tests leave out included), 1 to 8 microphones, 1 to 3
sources, T60 from 0.05 s (400 samples at 8 kHz) to 0.9 s, in the tuned launch
shape, in a small-tile shape that time-tiles every room and in the second
render path (bin moments).  Every room's forward per channel within 1e-5
relative L2 and its adjoint (dL/dmic, dL/dsrc, dL/dr, draws held fixed) within
1e-4 of the FP64 oracle (Eq. 1-6); half of the batches also through the
multi-rate chain (Sec. II, Eq. 7-8), the gradient through the draws and the
early-reverberation windows of Eq. 9.  The oracle runs in the worker pool forked
before the GPU is touched."""
import numpy as np
import pytest

from paper_2304_08052_amd import workloads as W
from tests.test_gpu_full import check_jobs, jobs_for, run_batched, say

pytestmark = pytest.mark.gpu

FS = (8000.0, 11025.0, 16000.0, 22050.0, 32000.0, 44100.0, 48000.0)
SMALL_TILES = dict(lds_bytes=16384, wg_threads=256, grid_wgs=0, max_mic_group=2, waves_per_simd=4)
# the second render path (bin moments, matrix-core pulse filter)
MOMENTS = dict(lds_bytes=65536, wg_threads=512, grid_wgs=0, max_mic_group=2, waves_per_simd=4, render_path=1)


def random_batch(seed):
    rng = np.random.default_rng([2300, seed])
    return W._uca_rooms(4, rng, (1, 3), (1, 8), (0.05, 0.9), FS, seed0=100 * seed)


@pytest.mark.parametrize("seed", range(10))
def test_random_shapes_forward_backward(seed, oracle_pool):
    batch = random_batch(seed)
    launch = MOMENTS if seed >= 8 else SMALL_TILES if seed % 2 else None
    shapes = [(int(batch["fs"][b]), int(batch["n_mic"][b]), int(batch["n_src"][b]), round(float(batch["rt60"][b]), 2))
              for b in range(len(batch["rt60"]))]
    say(f"seed {seed}: rooms (fs, mics, sources, T60) {shapes}, launch {launch or 'tuned'}")
    plan, out, G, gm, gs, gr = run_batched(batch, seed=40 + seed, launch=launch)
    if launch is SMALL_TILES:
        assert plan.info.n_items > 2 * plan.n_rooms   # the small tiles split the rooms in time
    check_jobs(oracle_pool, jobs_for(batch, plan, range(plan.n_rooms), out, G, gm, gs, gr), f"random seed {seed}")


@pytest.mark.parametrize("seed", range(4))
def test_random_shapes_multirate(seed, oracle_pool):
    """The same batches through the paper-literal multi-rate chain (Sec. II,
    Eq. 7-8): intermediate signal and output per channel within 1e-5."""
    import torch
    from oracle import framrir as F
    from oracle import multirate as M
    from paper_2304_08052_amd import framrir as fr
    from tests import oracle_pool as P
    batch = random_batch(seed)
    plan = fr.Plan(batch, multirate=True)
    say(f"seed {seed}: multi-rate, rates {[int(f) for f in batch['fs']]}")
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
    say(f"seed {seed}: intermediate worst {e1.max():.2e}, output worst {e3.max():.2e}")
    assert e1.max() <= 1e-5 and e3.max() <= 1e-5


@pytest.mark.parametrize("seed", range(4))
def test_random_shapes_draws_backward(seed):
    """The gradient through the draws (Eq. 4-6 with the Philox variates fixed)
    on the same shapes, 200-400 images per source, against the oracle's
    adjoint_room_draws: dL/dmic and dL/dsrc per room, dL/dr over the batch,
    within 1e-4."""
    from oracle import framrir as F
    from paper_2304_08052_amd import framrir as fr
    from tests.test_gpu_draws_grad import _check, _grads
    params = dict(img_lo=200, img_hi=400)
    batch = random_batch(seed)
    say(f"seed {seed}: backward through the draws")
    plan = fr.Plan(batch, params=params, launch=SMALL_TILES if seed % 2 else None)
    table, _, _ = plan.draw()
    G = W.upstream_grad(plan.info.out_floats, seed=60 + seed)
    _check(plan, batch, F.Params(**params), G, _grads(plan, table, G))


@pytest.mark.parametrize("seed", range(4))
def test_random_shapes_early_windows(seed):
    """The Eq. 9 windows stored by the render pass itself on the same shapes:
    equal bit for bit to the separate early kernel's, each window equal to its
    span of the rendered RIR (zeros outside [0, T)), and the start indices equal
    to the oracle's."""
    import torch
    from paper_2304_08052_amd import framrir as fr
    from tests.test_gpu_early import _check_windows_equal_output, _oracle_starts
    batch = random_batch(seed)
    say(f"seed {seed}: early windows from the render pass")
    plan = fr.Plan(batch, launch=SMALL_TILES if seed % 2 else None)
    out_f, _, early_f, start_f = plan.forward_early()
    out, _ = plan.forward()
    early, start = plan.early(out)
    torch.cuda.synchronize()
    assert torch.equal(out_f, out) and torch.equal(start_f, start) and torch.equal(early_f, early)
    assert np.array_equal(start.cpu().numpy().astype(np.int64), _oracle_starts(batch))
    _check_windows_equal_output(plan, out.cpu().numpy(), early.cpu().numpy(), start.cpu().numpy())
