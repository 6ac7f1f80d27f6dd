"""A pool of worker processes for the FP64 oracle in the GPU parity tests.

The pool is forked once, at the end of collection, before any test touches
the GPU (conftest.py starts it when a selected test asks for the
``oracle_pool`` fixture), so its workers hold no GPU state.  Each worker runs
single-threaded numpy.  The work functions below take one room as a
single-room batch (paper_2304_08052_amd.framrir.split_rooms), compute the
oracle's RIRs or adjoint for it and compare them with the GPU's values sent
along, returning only the errors.
"""
import multiprocessing as mp
import os

import numpy as np

_POOL = None


def workers():
    """Host cores to use: the process's CPU set, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _init_worker():
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:      # pragma: no cover
        pass


def start():
    global _POOL
    if _POOL is None:
        _POOL = mp.get_context("fork").Pool(workers(), initializer=_init_worker)
    return _POOL


def get():
    if _POOL is None:
        raise RuntimeError("the oracle pool is started at collection time, before the GPU is used")
    return _POOL


def stop():
    global _POOL
    if _POOL is not None:
        _POOL.terminate()
        _POOL.join()
        _POOL = None


def rel_l2(got, want):
    den = np.linalg.norm(want)
    return float(np.linalg.norm(got - want) / den) if den > 0 else float(np.linalg.norm(got))


def _room(one):
    from oracle import framrir as F
    rm = F.rooms_from_batch(one)[0]
    return F, rm, F.room_plan(rm, F.Params())


def forward_errors(job):
    """job = (one-room batch, GPU RIRs [S, M, T] FP32): per-channel relative
    L2 errors [S, M] against the oracle's render (Eq. 1, 8)."""
    one, got = job
    F, rm, op = _room(one)
    want = F.render_room(op, rm)
    got = np.asarray(got, dtype=np.float64).reshape(want.shape)
    return np.array([[rel_l2(got[s, m], want[s, m]) for m in range(want.shape[1])]
                     for s in range(want.shape[0])])


def backward_errors(job):
    """job = (one-room batch, dL/dh [S, M, T] FP32, GPU grad_mic [M, 3],
    grad_src [S, 3], grad_r): relative errors of the three gradients against
    the oracle's adjoint with the draws held fixed."""
    one, g, gm, gs, gr = job
    F, rm, op = _room(one)
    wm, ws, wr = F.adjoint_room(op, rm, np.asarray(g, dtype=np.float64).reshape(len(rm.src), len(rm.mic), op["T"]))
    return (rel_l2(np.ravel(gm), np.ravel(wm)), rel_l2(np.ravel(gs), np.ravel(ws)),
            float(abs(gr - wr) / abs(wr)) if wr != 0 else float(abs(gr)))


def room_errors(job):
    """Forward and backward errors of one room: job = (one-room batch, RIRs,
    dL/dh, grad_mic, grad_src, grad_r); the backward part is skipped when
    dL/dh is None."""
    one, got, g, gm, gs, gr = job
    fwd = forward_errors((one, got))
    bwd = backward_errors((one, g, gm, gs, gr)) if g is not None else None
    return fwd, bwd


def spatial_errors(job):
    """job = (RIRs [3, M, T], dry signals [3, n], SIR dB, SNR dB, n, GPU
    images [3, M, n], GPU mixture [M, n], GPU gains [3]): the worst
    per-channel relative L2 errors of the images and the mixture and the
    worst relative gain error against the spatialisation oracle (R-28..R-31)."""
    from oracle import spatialize as SP
    rir, sig, sir, snr, n, img, mix, g = job
    want_img, want_mix, want_g = SP.spatialize_room(np.asarray(rir, dtype=np.float64), np.asarray(sig, dtype=np.float64),
                                                   sir, snr, n)
    S, M = want_img.shape[:2]
    e_img = max(rel_l2(np.asarray(img[s, m], dtype=np.float64), want_img[s, m]) for s in range(S) for m in range(M))
    e_mix = max(rel_l2(np.asarray(mix[m], dtype=np.float64), want_mix[m]) for m in range(M))
    e_g = float(np.max(np.abs(np.asarray(g, dtype=np.float64) - want_g) / want_g))
    return e_img, e_mix, e_g


def multirate_errors(job):
    """job = (one-room batch, GPU intermediate signal [S, M, T_l], GPU output
    [S, M, T]): the worst per-channel relative L2 errors of both against the
    multi-rate oracle (Sec. II, Eq. 7-8), the output taken through the
    oracle's high-pass and decimation of its own intermediate signal."""
    from oracle import multirate as M
    one, got_l, got = job
    F, rm, op = _room(one)
    want_l = M.intermediate_room(op, rm)
    _, _, t_len = M.lengths(rm.rt60, rm.fs)
    got_l = np.asarray(got_l, dtype=np.float64).reshape(want_l.shape)
    got = np.asarray(got, dtype=np.float64).reshape(want_l.shape[0], want_l.shape[1], t_len)
    e1 = e3 = 0.0
    for s in range(want_l.shape[0]):
        for m in range(want_l.shape[1]):
            e1 = max(e1, rel_l2(got_l[s, m], want_l[s, m]))
            want = M.decimate(M.highpass(want_l[s, m], rm.fs), rm.fs, t_len)
            e3 = max(e3, rel_l2(got[s, m], want))
    return e1, e3
