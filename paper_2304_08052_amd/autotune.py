"""Launch-shape autotuner for the render kernel.

A size class is the set of sample rates, the largest microphone count and the
RIR-length range of a batch (those decide how items split into microphone
groups and time tiles).  For a class, tune() times the render of a
representative batch under each candidate launch shape (LDS tile budget,
threads per workgroup, waves per SIMD, microphones per item, workgroups of
the persistent grid) with HIP events
and keeps the fastest.  Results are cached in a JSON file keyed by the GPU
architecture and the size class: $FRAMRIR_TUNE_CACHE, else
~/.cache/framrir/tune.json.  launch_for() also consults tune_cache.json
shipped beside this module (entries measured on MI355X).
"""
import json
import os

import numpy as np

from . import framrir as fr

N_CU = 256            # MI355X compute units
LDS_PER_CU = 163840   # bytes


def static_lds(threads):
    """The render kernel's static LDS for a workgroup size, bounded from above
    (per wave the bank-ordered pool, 128 pairs x 3 words, and 32 counts)."""
    return 512 + (threads // 64) * (3 * 128 + 32) * 4


def _per_cu_max(lds, threads, waves_per_simd):
    """Workgroups of one shape that fit a compute unit at once."""
    return max(1, min(LDS_PER_CU // (lds + static_lds(threads)), waves_per_simd * 4 // (threads // 64)))


# (LDS tile, threads, waves per SIMD) x microphones per item x resident
# workgroups per CU (the persistent grid is that many per CU)
DEFAULT_CANDIDATES = [
    dict(lds_bytes=lds, wg_threads=t, waves_per_simd=w, max_mic_group=g, grid_wgs=N_CU * k)
    for (lds, t, w) in [(131072, 1024, 4), (98304, 1024, 4), (65536, 1024, 8), (49152, 1024, 8),
                        (40960, 1024, 8), (65536, 512, 4), (49152, 512, 8), (40960, 512, 8), (32768, 256, 4)]
    if lds + static_lds(t) <= LDS_PER_CU
    for g in (8, 4)
    for k in range(1, _per_cu_max(lds, t, w) + 1)
]


def cache_path():
    return os.environ.get("FRAMRIR_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "framrir", "tune.json"))


def arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def size_class(batch):
    T = np.ceil(np.asarray(batch["rt60"]) * np.asarray(batch["fs"])).astype(np.int64)
    fs = sorted({int(v) for v in np.asarray(batch["fs"])})
    t_lo, t_hi = (int(2 ** np.floor(np.log2(T.min()))), int(2 ** np.ceil(np.log2(T.max()))))
    return f"fs={'/'.join(map(str, fs))};mics<={int(np.max(batch['n_mic']))};T={t_lo}-{t_hi}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key, value):
    data = _load()
    data[key] = value
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_render(batch, launch, reps=5, warmup=2, params=None):
    """Median render time (ms) of one batch under one launch shape."""
    import torch
    plan = fr.Plan(batch, params=params, launch=launch)
    table, _, _ = plan.draw()
    out, ws = plan.empty_out(), plan.workspace()
    for _ in range(warmup):
        plan.render(table, out=out, ws=ws)
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.render(table, out=out, ws=ws)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def tune(batch, candidates=None, reps=5, params=None, store=True):
    """Times every candidate render shape on this batch; returns (best launch,
    results).  The backward workgroup size (bwd_wg_threads) is not tuned here:
    shipped entries carry it where a different size measured faster."""
    results = []
    for cand in candidates or DEFAULT_CANDIDATES:
        launch = dict(fr.DEFAULT_LAUNCH, **cand)
        try:
            ms = time_render(batch, launch, reps=reps, params=params)
        except fr.FramrirError:      # shape not valid for this batch
            continue
        results.append((ms, launch))
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    if store:
        _store(f"{arch()}|{size_class(batch)}", dict(launch=best, ms=results[0][0]))
    return best, results


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _lookup(key):
    hit = _load().get(key)
    if hit is None:
        try:
            with open(SHIPPED) as f:
                hit = json.load(f).get(key)
        except (OSError, ValueError):
            hit = None
    return hit


def launch_for(batch, tune_if_missing=False, params=None):
    """The cached best launch for this batch's size class (or the default)."""
    hit = _lookup(f"{arch()}|{size_class(batch)}")
    if hit is not None:
        return dict(fr.DEFAULT_LAUNCH, **hit["launch"])
    if tune_if_missing:
        return tune(batch, params=params)[0]
    return dict(fr.DEFAULT_LAUNCH)


def stream_class(n_rooms, n_src_max, n_mic_max, rt60_max, fs_max):
    """Size class of a fixed-capacity graph step (stream.GraphStream): its
    launch shape serves every batch the capacity admits."""
    return f"stream:rooms={n_rooms};src<={n_src_max};mics<={n_mic_max};rt60<={rt60_max:g};fs<={fs_max:g}"


def launch_for_stream(n_rooms, n_src_max, n_mic_max, rt60_max, fs_max):
    """The shipped or cached launch for a graph step of this capacity (or the default)."""
    hit = _lookup(f"{arch()}|{stream_class(n_rooms, n_src_max, n_mic_max, rt60_max, fs_max)}")
    return dict(fr.DEFAULT_LAUNCH, **hit["launch"]) if hit is not None else dict(fr.DEFAULT_LAUNCH)
