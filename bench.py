#!/usr/bin/env python3
"""Benchmark of batched FRAM-RIR synthesis on one MI355X.

A step is one pass of the device hot path over one batch whose inputs (room
descriptors, positions) are already resident in HBM: the draw stage (image
table) and the render (RIRs) -- forward; the backward step adds the adjoint.
The headline workload is the batched forward: 256 rooms, 2 sources each,
6-microphone circular arrays, 16 kHz.

Prints ONE JSON line (rank 0).  Extra fields: forward+backward time (draws
held fixed, and through the draws) and its ratio to the forward, eager vs
hipGraph step times, the host planning time.
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

METRIC = "multi-channel RIRs/sec at batch 256, 16 kHz; fwd+bwd/fwd ratio; VALU/HBM % peak"

# MI355X peaks (published): HBM3E 8 TB/s; FP32 vector 157.3 TFLOP/s (that
# figure counts packed FP32 instructions, which this library never emits: the
# non-packed rate is 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz = 78.64,
# reported beside it); dense fp16 matrix 2.5 PFLOP/s.
HBM_PEAK_GBS = 8000.0
FP32_PUBLISHED_PEAK_TFLOPS = 157.3
FP32_NONPACKED_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12     # 78.64
FP16_MFMA_PEAK_TFLOPS = 2500.0
FLOPS_PER_TAP = 11          # sub, rcp, 2 mul + FMA (window), FMA, mul, add
# bin-moment render: per 256-sample block 31 MFMA 16x16x32 (16,384 flops each)
MOMENT_MFMA_PER_BLOCK = 31
MOMENT_BLOCK = 256


KERNEL_SOURCES = ["kernels.hip", "framrir_internal.h", "tap_poly.h", "plan.cpp", "plan_internal.h"]
PROFILES = {   # committed counter summaries per render path
    0: dict(hbm=os.path.join(HERE, "profiles", "render_kernel_batched256_hbm.md"),
            valu=os.path.join(HERE, "profiles", "render_kernel_batched256_valu.md")),
    1: dict(hbm=os.path.join(HERE, "profiles", "render_moment_kernel_batched256_hbm.md"),
            valu=os.path.join(HERE, "profiles", "render_moment_kernel_batched256_valu.md")),
}
HBM_PROFILE = PROFILES[0]["hbm"]
VALU_PROFILE = PROFILES[0]["valu"]
SPATIAL_SOURCES = ["spatial.hip", "framrir_internal.h", "plan_internal.h"]
SPATIAL_HBM_PROFILE = os.path.join(HERE, "profiles", "spatial_batched256_hbm.md")


def kernel_sources_sha256(files=None):
    import hashlib
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES if files is None else files):
        with open(os.path.join(HERE, "paper_2304_08052_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def copy_probe(mib):
    """One elementwise kernel of known traffic (mib MiB read, mib MiB written)
    for scaling the FETCH_SIZE / WRITE_SIZE counters of the same run."""
    import torch
    a = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.neg(a, out=b)
    torch.cuda.synchronize()


def measured_spatial_traffic():
    """HBM bytes of one framrir_spatialize call on the training-mixture
    workload from the committed counter passes, or None when the
    spatialisation sources differ from the ones the counters were taken on."""
    try:
        with open(SPATIAL_HBM_PROFILE) as f:
            kv = dict(line.split(" = ", 1) for line in f.read().splitlines() if " = " in line)
    except OSError:
        return None
    if kv.get("workload") != "spatial" or kv.get("source_sha256") != kernel_sources_sha256(SPATIAL_SOURCES):
        return None
    return int(kv["traffic_bytes"])


MULTIRATE_PROFILE = os.path.join(HERE, "profiles", "kernels_multirate256_trace.md")


def measured_multirate_traffic():
    """HBM bytes of the multi-rate filter stages on the batched workload from
    the committed counter passes, or None when the kernel sources differ."""
    try:
        with open(MULTIRATE_PROFILE) as f:
            kv = dict(line.split(" = ", 1) for line in f.read().splitlines() if " = " in line)
    except OSError:
        return None
    if kv.get("workload") != "multirate" or kv.get("source_sha256") != kernel_sources_sha256():
        return None
    return int(kv["traffic_bytes"])


def launch_key(launch):
    """The launch shape as the counter summaries record it."""
    keys = ["lds_bytes", "wg_threads", "grid_wgs", "max_mic_group", "waves_per_simd"]
    if launch.get("render_path", 0):
        keys.append("render_path")
    return " ".join(f"{k}={launch[k]}" for k in keys)


def profile_values(path, workload_name, launch):
    """The key = value lines of a committed rocprofv3 counter summary, or None
    when the kernel sources, the workload or the launch shape differ from the
    ones the counters were taken on."""
    try:
        with open(path) as f:
            kv = dict(line.split(" = ", 1) for line in f.read().splitlines() if " = " in line)
    except OSError:
        return None
    if (kv.get("workload") != workload_name or kv.get("launch") != launch_key(launch)
            or kv.get("source_sha256") != kernel_sources_sha256()):
        return None
    return kv


def _profile_path(kind, launch, default):
    path = PROFILES.get(launch.get("render_path", 0), PROFILES[0])[kind]
    return default if launch.get("render_path", 0) == 0 else path


def measured_traffic(workload_name, launch):
    """HBM bytes per render launch and of the whole forward step (preparation
    + render) from the committed FETCH_SIZE and WRITE_SIZE passes (scaled by
    a copy kernel of known size), or None (profile_values)."""
    kv = profile_values(_profile_path("hbm", launch, HBM_PROFILE), workload_name, launch)
    return int(kv["traffic_bytes"]) if kv else None


def measured_step_traffic(workload_name, launch):
    kv = profile_values(_profile_path("hbm", launch, HBM_PROFILE), workload_name, launch)
    return int(kv["step_traffic_bytes"]) if kv and "step_traffic_bytes" in kv else None


def measured_valu_insts(workload_name, launch):
    """VALU and LDS wave instructions per render launch from the committed
    SQ counter pass, or None (profile_values)."""
    kv = profile_values(_profile_path("valu", launch, VALU_PROFILE), workload_name, launch)
    return (int(kv["valu_wave_insts"]), int(kv["lds_wave_insts"])) if kv else None


def parse_args():
    p = argparse.ArgumentParser(description=__doc__)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="batched", choices=["batched", "long", "mixed", "one", "multirate",
                                                              "spatial"])
    p.add_argument("--cpu-rooms", type=int, default=256,
                   help="rooms of the workload timed through the FP64 oracle (one host core, then all host "
                        "cores; 0 = skip)")
    p.add_argument("--no-graph", action="store_true")
    p.add_argument("--no-backward", action="store_true")
    p.add_argument("--lds-bytes", type=int, default=None)
    p.add_argument("--wg-threads", type=int, default=None)
    p.add_argument("--max-mic-group", type=int, default=None)
    p.add_argument("--waves-per-simd", type=int, default=None)
    p.add_argument("--grid-wgs", type=int, default=None, help="workgroups of the persistent grid (0 = as many as fit)")
    p.add_argument("--bwd-wg-threads", type=int, default=None, help="threads per backward workgroup (0 = as the render)")
    p.add_argument("--bwd-grid-wgs", type=int, default=None, help="workgroups of the backward grid (0 = as many as fit)")
    p.add_argument("--render-path", type=int, default=None, choices=[0, 1],
                   help="render path: 0 scatter, 1 bin moments on the matrix cores")
    p.add_argument("--tune", action="store_true", help="pick the launch shape with the autotuner first")
    p.add_argument("--no-per-room", action="store_true",
                   help="skip the plain per-room launch path (the same kernels, one launch set per room)")
    p.add_argument("--early", action="store_true",
                   help="also time the early-reverberation windows (Eq. 9) of the rendered batch")
    p.add_argument("--copy-probe-mb", type=int, default=0,
                   help="run one plain device copy of this many MiB first (reference for HBM counters)")
    return p.parse_args()


def workload(name):
    from paper_2304_08052_amd import workloads as W
    if name == "batched":
        return W.config2(), ("batched forward: 256 rooms U(3,10)xU(3,10)xU(2.5,4) m, T60 U(0.1,0.7) s, "
                             "16 kHz, 2 sources, 6-mic circular array r=5 cm, seeds 0..255")
    if name == "long":
        return W.config3(), ("long filters: 64 rooms U(8,20)xU(8,20)xU(3,6) m, T60 U(0.6,1.2) s, 48 kHz, "
                             "1 source, 8-mic linear array 3 cm")
    if name == "multirate":
        return W.config2(), ("paper-literal multi-rate rendering of the batched workload (256 rooms, 16 kHz, 2 sources, "
                             "6 mics): impulses on the 992 kHz grid, down-sampled to 112 kHz, 80 Hz high-pass, "
                             "decimated to 16 kHz")
    if name == "mixed":
        return W.config5(0), ("mixed stream: 1024 rooms, fs {16,48} kHz, 2-8 mics, 1-3 sources, "
                              "T60 U(0.1,1.0) s")
    return W.config1(), "one room 6x5x3 m, T60 0.4 s, 16 kHz, 1 source, 2 mics"


def room_slice(batch, b0, b1):
    """Rooms b0 .. b1-1 of a batch, with their sources and microphones."""
    import numpy as np
    s0, s1 = (int(np.sum(batch["n_src"][:b])) for b in (b0, b1))
    m0, m1 = (int(np.sum(batch["n_mic"][:b])) for b in (b0, b1))
    sub = dict(batch)
    for k in ("size", "rt60", "fs", "c", "r_override", "seed", "n_src", "n_mic"):
        sub[k] = batch[k][b0:b1]
    sub["src"] = batch["src"][s0:s1]
    sub["mic"] = batch["mic"][m0:m1]
    return sub


def _oracle_rooms(sub):
    """Worker of cpu_baseline_parallel: the oracle on a few rooms, one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import framrir as F
    with threadpool_limits(limits=1):
        F.simulate(sub)
    return 0


def host_cpu_model():
    """The host CPU as /proc/cpuinfo names it (model name, family / model /
    stepping, clock), with the logical CPUs of the machine and of this
    process's CPU set, or None."""
    try:
        with open("/proc/cpuinfo") as f:
            text = f.read()
    except OSError:
        return None
    first = text.split("\n\n", 1)[0]
    kv = {}
    for line in first.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    name = kv.get("model name")
    if name is None:
        return None
    n_cpu = text.count("processor\t:") or text.count("processor :")
    try:
        n_set = len(os.sched_getaffinity(0))
    except OSError:
        n_set = n_cpu
    parts = [name]
    if "cpu family" in kv and "model" in kv:
        parts.append(f"family {kv['cpu family']} model {kv['model']} stepping {kv.get('stepping', '?')}")
    if "cpu MHz" in kv:
        parts.append(f"{float(kv['cpu MHz']):.0f} MHz")
    parts.append(f"{n_cpu} logical CPUs, {n_set} in this process's CPU set")
    return ", ".join(parts)


def cpu_baseline(batch, n_rooms):
    """The FP64 oracle as it stands, on the first n_rooms rooms, one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import framrir as F
    nb = min(n_rooms, len(batch["rt60"]))
    ns = int(np.sum(batch["n_src"][:nb]))
    sub = room_slice(batch, 0, nb)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        F.simulate(sub)
        dt = time.perf_counter() - t0
    return dict(value=ns / dt, unit="RIR/s", cores=1, kind="oracle", cpu_model=host_cpu_model(),
                sample=f"first {nb} rooms ({ns} multi-channel RIRs) of the same workload, "
                       f"FP64 numpy oracle, {dt:.2f} s on 1 thread")


def cpu_baseline_parallel(batch, n_rooms):
    """The same oracle on the same rooms, one room per task over a pool of
    worker processes (one per available host core, at most 16, each single
    threaded).  Forked before the GPU is touched."""
    import multiprocessing as mp
    import numpy as np
    nb = min(n_rooms, len(batch["rt60"]))
    ns = int(np.sum(batch["n_src"][:nb]))
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    subs = [room_slice(batch, b, b + 1) for b in range(nb)]
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_rooms, subs, chunksize=1)
        dt = time.perf_counter() - t0
    return dict(value=ns / dt, unit="RIR/s", cores=workers, kind="oracle", cpu_model=host_cpu_model(),
                sample=f"first {nb} rooms ({ns} multi-channel RIRs) of the same workload, "
                       f"FP64 numpy oracle, {dt:.2f} s on {workers} single-threaded processes")


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the path shards by room with no "
              f"exchange, and no multi-GPU launcher is provided.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2304_08052_amd import framrir as fr
    from paper_2304_08052_amd import workloads as W

    launch = {}
    if args.lds_bytes:
        launch["lds_bytes"] = args.lds_bytes
    if args.wg_threads:
        launch["wg_threads"] = args.wg_threads
    if args.max_mic_group:
        launch["max_mic_group"] = args.max_mic_group
    if args.waves_per_simd:
        launch["waves_per_simd"] = args.waves_per_simd
    if args.grid_wgs is not None:
        launch["grid_wgs"] = args.grid_wgs
    if args.bwd_wg_threads is not None:
        launch["bwd_wg_threads"] = args.bwd_wg_threads
    if args.bwd_grid_wgs is not None:
        launch["bwd_grid_wgs"] = args.bwd_grid_wgs
    if args.render_path is not None:
        launch["render_path"] = args.render_path
    if args.workload == "spatial":
        return run_spatial(args, launch)
    batch, desc = workload(args.workload)
    if args.workload == "mixed":
        return run_mixed(args, batch, desc, launch)
    if args.workload == "multirate":
        return run_multirate(args, batch, desc, launch)
    # the oracle on all host cores first: its worker processes fork before
    # anything here touches the GPU
    cpu_par = cpu_long = None
    if args.cpu_rooms > 0:
        cpu_par = cpu_baseline_parallel(batch, args.cpu_rooms)
        if args.workload == "batched":
            long_batch, _ = workload("long")
            cpu_long = cpu_baseline_parallel(long_batch, len(long_batch["rt60"]))
            cpu_long["workload"] = "long filters: 64 rooms, 48 kHz, 8 mics, T60 0.6-1.2 s"
    tuned = None
    if not args.tune and not launch:
        from paper_2304_08052_amd import autotune
        launch = autotune.launch_for(batch)
    if args.tune:
        from paper_2304_08052_amd import autotune
        best, best_ms = autotune.tune(batch)
        launch = dict(best, **launch)
        tuned = dict(ms=round(best_ms, 4), **best)
    t0 = time.perf_counter()
    plan = fr.Plan(batch, launch=launch)
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info
    n_rirs = int(np.sum(batch["n_src"]))
    m_per_src = np.repeat(batch["n_mic"], batch["n_src"]).astype(np.int64)
    taps = int(np.sum(plan.n_img.astype(np.int64) * m_per_src)) * fr.FRAMRIR_TAPS
    out_bytes = info.out_floats * 4
    path = plan.launch.get("render_path", 0)

    table = plan.empty_table()
    out = plan.empty_out()
    ws = plan.workspace(backward=not args.no_backward)   # the backward reuses the forward's preparation
    grad = torch.from_numpy(W.upstream_grad(info.out_floats)).cuda()
    stream = torch.cuda.current_stream()
    if args.copy_probe_mb > 0:   # known traffic: N MiB read + N MiB written (one elementwise kernel)
        copy_probe(args.copy_probe_mb)

    # forward step = framrir_forward split in its two launches: draws +
    # preparation, then the render kernel (timed on its own for the roofline).
    # The step without the image table (tab=None: the preparation draws each
    # row again instead of reading the table back) is timed beside it.
    def fwd_step(ev=None, tab=table):
        plan.prepare(tab, ws=ws, draw=True)
        if ev is not None:
            ev[0].record(stream)
        plan.render_prepared(tab, out=out, ws=ws)
        if ev is not None:
            ev[1].record(stream)

    def bwd_step():
        fwd_step()
        plan.backward(table, grad, ws=ws, prepared=True)

    def events(n):
        return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]

    def per_step(fn, n, inner=None):
        """n steps of fn, each between its own pair of events on the launch
        stream; returns the per-step times (ms) and the whole span (ms)."""
        evs = events(n)
        torch.cuda.synchronize()
        for k in range(n):
            evs[k][0].record(stream)
            fn() if inner is None else fn(inner[k])
            evs[k][1].record(stream)
        torch.cuda.synchronize()
        return np.array([a.elapsed_time(b) for a, b in evs]), evs[0][0].elapsed_time(evs[-1][1])

    def pct(a):
        return [float(np.percentile(a, q)) for q in (10, 50, 90)]

    for _ in range(args.warmup):
        fwd_step()
    torch.cuda.synchronize()

    # ---- eager forward, with per-launch render events
    revs = events(args.steps)
    eager_each, _ = per_step(fwd_step, args.steps, inner=revs)
    render_each = np.array([a.elapsed_time(b) for a, b in revs])
    render_ms = float(np.median(render_each))

    # ---- hipGraph-captured forward step (draw + render): the headline
    graph_each = graph_notable_each = None
    if not args.no_graph:
        try:
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            with torch.cuda.stream(side):
                fwd_step()
            stream.wait_stream(side)
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                fwd_step()
            for _ in range(args.warmup):
                g.replay()
            torch.cuda.synchronize()
            graph_each, _ = per_step(g.replay, args.steps)
            gt = torch.cuda.CUDAGraph()   # the same step without an image table
            with torch.cuda.graph(gt):
                fwd_step(tab=None)
            for _ in range(args.warmup):
                gt.replay()
            torch.cuda.synchronize()
            graph_notable_each, _ = per_step(gt.replay, args.steps)
        except Exception as exc:      # graph capture unavailable: report eager only
            print(f"[bench] graph capture failed: {exc}", file=sys.stderr)
            graph_each = None

    # ---- forward + backward (draws held fixed), and through the draws
    fb_each = fbd_each = None
    if not args.no_backward:
        for _ in range(max(1, args.warmup // 2)):
            bwd_step()
        fb_each, _ = per_step(bwd_step, args.steps)

        def bwd_draws_step():
            fwd_step()
            plan.backward_draws(table, grad, ws=ws, prepared=True)
        for _ in range(max(1, args.warmup // 2)):
            bwd_draws_step()
        fbd_each, _ = per_step(bwd_draws_step, args.steps)

    early_ms = None
    if args.early:
        early_buf, start_buf = plan.early(out)
        e_each, _ = per_step(lambda: plan.early(out, early=early_buf, start=start_buf), args.steps)
        early_ms = float(np.median(e_each))

    # ---- the plain per-room launch path on the same GPU (comparator)
    per_room_ms = None
    if not args.no_per_room:
        pr = fr.PerRoom(batch, launch=plan.launch)
        pr_out = torch.empty_like(out)
        for _ in range(2):
            pr.forward(pr_out)
        pr_each, _ = per_step(lambda: pr.forward(pr_out), max(2, args.steps // 10))
        per_room_ms = float(np.median(pr_each))
        fwd_step()
        torch.cuda.synchronize()
        if not torch.equal(pr_out, out):
            raise RuntimeError("per-room path disagrees with the batched path")

    eager_ms = float(np.median(eager_each))
    graph_ms = float(np.median(graph_each)) if graph_each is not None else None
    head_each = graph_each if graph_each is not None else eager_each
    step_ms = float(np.median(head_each))
    fb_ms = float(np.median(fb_each)) if fb_each is not None else None
    fbd_ms = float(np.median(fbd_each)) if fbd_each is not None else None
    value = n_rirs / (step_ms * 1e-3)
    achieved = taps * FLOPS_PER_TAP / (render_ms * 1e-3) / 1e12
    cpu = cpu_baseline(batch, args.cpu_rooms) if args.cpu_rooms > 0 else None
    cpu_long_1 = None
    if args.cpu_rooms > 0 and args.workload == "batched":   # the long-filter workload in full, one core
        long_batch, _ = workload("long")
        cpu_long_1 = cpu_baseline(long_batch, len(long_batch["rt60"]))
        cpu_long_1["workload"] = "long filters: 64 rooms, 48 kHz, 8 mics, T60 0.6-1.2 s"
    traffic = measured_traffic(args.workload, plan.launch)
    step_traffic = measured_step_traffic(args.workload, plan.launch)
    insts = measured_valu_insts(args.workload, plan.launch)
    # a wave64 VALU instruction holds a 16-lane SIMD for 4 clocks: 1,024 SIMDs
    # at 2.4 GHz issue at most 614.4 G wave instructions per second
    valu_issue = insts[0] / (render_ms * 1e-3) / (1024 * 2.4e9 / 4) if insts else None
    # secondary byte model: every image row (32 B) read once per microphone
    # group of its source, every output sample (4 B) written once
    groups = np.repeat(-(-batch["n_mic"] // plan.launch["max_mic_group"]), batch["n_src"]).astype(np.int64)
    row_bytes = int(np.sum(plan.n_img.astype(np.int64) * groups)) * 32 + out_bytes
    mfma = None
    if path == 1:
        blocks = int(info.fir_blocks)
        mflops = blocks * MOMENT_MFMA_PER_BLOCK * 16 * 16 * 32 * 2
        mfma = {"flops_per_launch": mflops, "tflops": mflops / (render_ms * 1e-3) / 1e12,
                "peak": FP16_MFMA_PEAK_TFLOPS, "frac": mflops / (render_ms * 1e-3) / 1e12 / FP16_MFMA_PEAK_TFLOPS,
                "blocks_of_256_samples": blocks}
    kernel = "render_moment_kernel" if path == 1 else "render_kernel"
    prof = _profile_path("hbm", plan.launch, HBM_PROFILE)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "RIR/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "ms_per_step_p10_p50_p90": pct(head_each),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "rooms": int(plan.n_rooms),
            "rirs": n_rirs,
            "samples_out": int(info.out_floats),
            "taps_per_pulse": fr.FRAMRIR_TAPS,
            "image_rows": int(info.n_img),
            "draws": "FP64 bit-exact",
            "launch": plan.launch,
            "render_path": "bin moments (matrix-core FIR)" if path == 1 else "scatter",
            "work_items": int(info.n_items),
            "timed_step": "hipGraph replay of draws + preparation + render" if graph_each is not None
            else "eager draws + preparation + render",
        },
        "roofline": {
            "bound": "alu",
            "kernel": kernel,
            "achieved": achieved,
            "peak": FP32_PUBLISHED_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PUBLISHED_PEAK_TFLOPS,
            "peak_nonpacked": FP32_NONPACKED_PEAK_TFLOPS,
            "frac_nonpacked": achieved / FP32_NONPACKED_PEAK_TFLOPS,
            "peak_nonpacked_derivation": "256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, FP32 without packed "
                                         "instructions",
            "traffic": traffic,
            "traffic_source": os.path.relpath(prof, HERE) if traffic else None,
            "algorithmic_bytes": out_bytes,
            "traffic_over_algorithmic": traffic / out_bytes if traffic else None,
            "step_traffic": step_traffic,
            "step_traffic_over_algorithmic": step_traffic / out_bytes if step_traffic else None,
            "algorithmic_bytes_with_rows": row_bytes,
            "tap_updates_per_launch": taps,
            "flops_per_tap": FLOPS_PER_TAP,
            "render_ms": render_ms,
            "render_ms_p10_p50_p90": pct(render_each),
            "valu_issue_frac_counters": valu_issue,
            "valu_lds_wave_insts_counters": list(insts) if insts else None,
            "counters_source": os.path.relpath(_profile_path("valu", plan.launch, VALU_PROFILE), HERE)
            if insts else None,
            "mfma_fp16": mfma,
            "hbm_write_gbs": out_bytes / (render_ms * 1e-3) / 1e9,
            "hbm_frac": out_bytes / (render_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_par,
        "cpu_baseline_long_filters": cpu_long_1,
        "cpu_baseline_long_filters_all_cores": cpu_long,
        "eager_ms_per_step": eager_ms,
        "eager_ms_p10_p50_p90": pct(eager_each),
        "graph_ms_per_step": graph_ms,
        "graph_without_table_ms_p10_p50_p90": pct(graph_notable_each) if graph_notable_each is not None else None,
        "fwd_bwd_ms_per_step": fb_ms,
        "fwd_bwd_ms_p10_p50_p90": pct(fb_each) if fb_each is not None else None,
        "fwd_bwd_over_fwd": (fb_ms / eager_ms) if fb_ms else None,
        "fwd_bwd_draws_ms_per_step": fbd_ms,
        "per_room_ms_per_step": per_room_ms,
        "per_room_over_batched": (per_room_ms / step_ms) if per_room_ms else None,
        "early_ms": early_ms,
        "plan_host_ms": plan_ms,
        "autotune_top": tuned,
    }
    print(json.dumps(line), flush=True)


def spatial_hbm_bytes(plan, n):
    """Algorithmic HBM bytes of one framrir_spatialize call: the RIR spectra
    (written once, read by each of the channel's blocks), the signal-block
    spectra (written once, read by each microphone of the room), the RIRs and
    signals read, the images written, read for the energies, then read and
    written scaled, and the mixtures written."""
    import numpy as np
    bins = 16385 * 8
    tm = int(np.max(plan.T))
    n_blk = -(-n // (32768 - tm + 1))
    n_chan, n_src, n_mic = plan.info.n_chan, plan.info.n_src, plan.info.n_mic
    spectra = n_chan * bins * (1 + n_blk) + n_src * n_blk * bins + n_chan * n_blk * bins
    inputs = 4 * int(plan.info.out_floats) + 4 * n_src * n_blk * 32768
    images = 4 * 4 * n_chan * n
    return spectra + inputs + images + 4 * n_mic * n


def run_spatial(args, launch):
    """On-the-fly generation of training mixtures (Sec. IV-A, the speed
    experiment of Table 2): per step the RIRs of 256 rooms (3 sources, 4-mic
    array) are synthesised, then the two speakers and the noise are convolved
    with them and mixed at the sampled SIR and SNR (4 s windows at 16 kHz)."""
    import numpy as np
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    from paper_2304_08052_amd import workloads as W
    batch = W.spatial_batch(256)
    n = 64000
    if not launch:
        launch = autotune.launch_for(batch)
    plan = fr.Plan(batch, launch=launch)
    sig, sir, snr = W.spatial_signals(batch, n)
    sig_d = torch.from_numpy(sig.reshape(-1, n)).cuda()
    sir_d, snr_d = torch.from_numpy(sir).cuda(), torch.from_numpy(snr).cuda()
    table, out, ws = plan.empty_table(), plan.empty_out(), plan.workspace()
    images = torch.empty((plan.info.n_chan, n), dtype=torch.float32, device="cuda")
    mix = torch.empty((plan.info.n_mic, n), dtype=torch.float32, device="cuda")
    gains = torch.empty(plan.info.n_src, dtype=torch.float32, device="cuda")
    ws_sp = torch.empty(plan.spatial_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    if args.copy_probe_mb > 0:
        copy_probe(args.copy_probe_mb)

    def spatial():
        plan.spatialize(out, sig_d, sir_d, snr_d, images=images, mix=mix, gains=gains, ws=ws_sp)

    def step():
        plan.forward(table=table, out=out, ws=ws)
        spatial()

    def timed(fn, k):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(k):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    eager_ms = timed(step, args.steps)
    graph_ms = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            step()
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        graph_ms = timed(g.replay, args.steps)
    spatial_ms = timed(spatial, args.steps)
    step_ms = min(eager_ms, graph_ms) if graph_ms else eager_ms
    hbm = spatial_hbm_bytes(plan, n)
    achieved = hbm / (spatial_ms * 1e-3) / 1e9
    line = {
        "metric": "training mixtures/sec generated on the fly (RIRs + spatialisation + SIR/SNR mixing), batch 256",
        "value": 256 / (step_ms * 1e-3), "unit": "mixtures/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "256 rooms U(3,10)xU(3,10)xU(2.5,4) m, T60 U(0.1,0.7) s, 16 kHz, 2 speakers + "
                               "1 noise source, 4-mic linear array (4-8-4 cm), 4 s windows, SIR U(-6,6) dB, "
                               "SNR U(10,20) dB",
                   "rooms": 256, "samples": n, "launch": plan.launch},
        "roofline": {"bound": "hbm", "kernel": "framrir_spatialize (spectra, products + inverse FFTs, energies, "
                                              "mixing)", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_spatial_traffic(),
                     "traffic_source": os.path.relpath(SPATIAL_HBM_PROFILE, HERE) if measured_spatial_traffic()
                     else None, "algorithmic_bytes": hbm,
                     "spatial_ms": spatial_ms},
        "eager_ms_per_step": eager_ms, "graph_ms_per_step": graph_ms,
        "cpu_baseline": None,
    }
    if args.cpu_rooms > 0:
        line["cpu_baseline"] = cpu_baseline_spatial(batch, sig, sir, snr, n, min(4, args.cpu_rooms))
    print(json.dumps(line), flush=True)


def cpu_baseline_spatial(batch, sig, sir, snr, n, n_rooms):
    """The FP64 oracles (RIRs, then spatialisation) on the first n_rooms rooms, one thread."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:      # pragma: no cover
        threadpool_limits = None
    from oracle import framrir as F
    from oracle import spatialize as SP
    rooms = F.rooms_from_batch(batch)[:n_rooms]
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    t0 = time.perf_counter()
    for b, rm in enumerate(rooms):
        h = F.render_room(F.room_plan(rm, F.Params()), rm)
        SP.spatialize_room(h, sig[b].astype(float), float(sir[b]), float(snr[b]), n)
    dt = time.perf_counter() - t0
    if ctx is not None:
        ctx.unregister() if hasattr(ctx, "unregister") else None
    return dict(value=n_rooms / dt, unit="mixtures/s", cores=1, kind="oracle",
                sample=f"first {n_rooms} rooms of the same workload (RIRs and spatialisation), FP64 numpy oracle, "
                       f"{dt:.2f} s on 1 thread")


def run_multirate(args, batch, desc, launch):
    """The paper-literal multi-rate chain on the batched workload: draws,
    render at r_l fs on the high-rate grid, high-pass, decimation."""
    import numpy as np
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    if not launch:
        launch = autotune.launch_for(batch)
    plan = fr.Plan(batch, launch=launch, multirate=True)
    info = plan.info
    table, out = plan.empty_table(), plan.empty_out()
    inter = torch.empty(info.mr_floats, dtype=torch.float32, device="cuda")
    ws = torch.zeros(info.ws_mr_bytes, dtype=torch.uint8, device="cuda")
    if args.copy_probe_mb > 0:
        copy_probe(args.copy_probe_mb)
    stream = torch.cuda.current_stream()

    def step():
        plan.forward_multirate(table=table, inter=inter, out=out, ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(args.steps):
        step()
    b.record(stream)
    torch.cuda.synchronize()
    eager_ms = a.elapsed_time(b) / args.steps
    graph_ms = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            step()
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(args.steps):
            g.replay()
        b.record(stream)
        torch.cuda.synchronize()
        graph_ms = a.elapsed_time(b) / args.steps
    # the stages after the render alone
    a.record(stream)
    for _ in range(args.steps):
        plan.multirate_filter(inter, out=out, ws=ws)
    b.record(stream)
    torch.cuda.synchronize()
    filter_ms = a.elapsed_time(b) / args.steps
    step_ms = min(eager_ms, graph_ms) if graph_ms else eager_ms
    n_rirs = int(np.sum(batch["n_src"]))
    # decimation work: every output sample takes 2 ceil(40.5 r_l) - 1 taps (2 flops each)
    rl = np.array([int(np.sqrt(np.floor(1e6 / f))) for f in batch["fs"]])
    taps = 2 * np.ceil(40.5 * rl) - 1
    dec_flops = float(np.sum(batch["n_src"] * batch["n_mic"] * np.ceil(batch["rt60"] * batch["fs"]) * taps * 2))
    # filter stages: the intermediate signal read twice (chunk-end states, then
    # the decimation windows) and the output written once
    filter_bytes = 4.0 * (2 * int(info.mr_floats) + int(info.out_floats))
    # the counter traffic is for the batched workload only
    mr_traffic = measured_multirate_traffic() if int(info.n_rooms) == 256 else None
    achieved = filter_bytes / (filter_ms * 1e-3) / 1e9
    line = {
        "metric": "multi-channel RIRs/sec, paper-literal multi-rate rendering, batch 256, 16 kHz",
        "value": n_rirs / (step_ms * 1e-3), "unit": "RIR/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "rooms": int(plan.n_rooms), "rirs": n_rirs,
                   "intermediate_samples": int(info.mr_floats), "samples_out": int(info.out_floats),
                   "launch": plan.launch},
        "roofline": {"bound": "hbm", "kernel": "hp_chunk_end + hp_carry + decimate_mfma", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": mr_traffic,
                     "traffic_over_algorithmic": mr_traffic / filter_bytes if mr_traffic else None,
                     "traffic_source": os.path.relpath(MULTIRATE_PROFILE, HERE) if mr_traffic else None,
                     "algorithmic_bytes": filter_bytes, "filter_ms": filter_ms,
                     "decimation_flops": dec_flops,
                     "decimation_flops_rate_tflops": dec_flops / (filter_ms * 1e-3) / 1e12},
        "eager_ms_per_step": eager_ms, "graph_ms_per_step": graph_ms,
    }
    print(json.dumps(line), flush=True)


def _event_ms(fn, reps=10, warmup=3):
    """Milliseconds per call of fn (stream-ordered work) by HIP events on the
    current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def mixed_size_classes(launch):
    """The mixed stream by size class: the 16 kHz and the 48 kHz rooms of its
    first batch, each as a batch of its own in the stream's launch shape, timed
    as eager forward and forward + backward calls.  Per class: RIR/s of the
    forward + backward, and the forward's algorithmic fractions of the FP32
    peak (11 flops per tap-update) and of the HBM bandwidth (output written)."""
    import numpy as np
    import torch
    from paper_2304_08052_amd import framrir as fr
    from paper_2304_08052_amd import workloads as W
    rooms = fr.split_rooms(W.config5(0))
    classes = []
    for fs in (16000.0, 48000.0):
        keep = [r for r in rooms if float(r["fs"][0]) == fs]
        sub = {k: np.concatenate([r[k] for r in keep]) for k in keep[0]}
        plan = fr.Plan(sub, launch=launch)
        info = plan.info
        ws = plan.workspace(backward=True)
        table, out = plan.empty_table(), plan.empty_out()
        grad = torch.from_numpy(W.upstream_grad(info.out_floats, seed=7)).cuda()

        def fwd():
            plan.forward(table=table, out=out, ws=ws)

        def fwd_bwd():
            fwd()
            plan.backward(table, grad, ws=ws, prepared=True)

        fwd_ms, fb_ms = _event_ms(fwd), _event_ms(fwd_bwd)
        taps = int(np.sum(plan.n_img.astype(np.int64) * np.repeat(sub["n_mic"], sub["n_src"]))) * fr.FRAMRIR_TAPS
        classes.append({
            "class": f"fs {fs / 1000:g} kHz", "rooms": len(keep), "rirs": int(info.n_src),
            "samples_out": int(info.out_floats), "fwd_ms": fwd_ms, "fwd_bwd_ms": fb_ms,
            "rirs_per_s_fwd_bwd": info.n_src / (fb_ms * 1e-3),
            "fwd_valu_frac_algorithmic": taps * FLOPS_PER_TAP / (fwd_ms * 1e-3) / 1e12 / FP32_NONPACKED_PEAK_TFLOPS,
            "fwd_hbm_write_frac": info.out_floats * 4 / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        })
    return classes


def run_mixed(args, batch0, desc, launch):
    """Mixed on-the-fly stream: every step renders a new batch of 1024 rooms
    (fs 16/48 kHz, 2-8 mics, 1-3 sources, T60 0.1-1.0 s) through one
    fixed-capacity hipGraph holding draw, render and backward.  Host planning
    of the batches happens before the timed region; inside it each step
    copies its descriptor and positions into the graph's buffers and replays."""
    import numpy as np
    import torch
    from paper_2304_08052_amd import framrir as fr
    from paper_2304_08052_amd import workloads as W
    from paper_2304_08052_amd.stream import GraphStream
    n_batches = min(args.steps, 8)
    if not launch:
        from paper_2304_08052_amd import autotune
        launch = autotune.launch_for_stream(1024, 3, 8, 1.0, 48000.0)
    t0 = time.perf_counter()
    plans = [fr.Plan(W.config5(k), launch=launch) for k in range(n_batches)]
    plan_ms = (time.perf_counter() - t0) * 1e3 / n_batches
    gs = GraphStream(n_rooms=1024, n_src_max=3, n_mic_max=8, rt60_max=1.0, fs_max=48000.0, launch=launch,
                     backward=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3000)
    gs.grad.normal_(generator=gen)          # synthetic upstream dL/dh
    gs.load(plans[0])
    gs.capture()
    stream = torch.cuda.current_stream()
    for k in range(args.warmup):
        gs.load(plans[k % n_batches])
        gs.replay()
    torch.cuda.synchronize()
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_rirs = 0
    t_start.record(stream)
    for k in range(args.steps):
        p = plans[k % n_batches]
        gs.load(p)
        gs.replay()
        n_rirs += p.info.n_src
    t_end.record(stream)
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end) / args.steps
    value = n_rirs / (t_start.elapsed_time(t_end) * 1e-3)
    line = {
        "metric": "multi-channel RIRs/sec, mixed on-the-fly stream, forward + backward per hipGraph replay",
        "value": value, "unit": "RIR/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "rooms_per_step": 1024, "distinct_batches": n_batches,
                   "rirs_per_step": n_rirs / args.steps, "launch": gs.launch,
                   "capacity_out_floats": int(gs.cap.info.out_floats)},
        "plan_host_ms_per_batch": plan_ms,
        "size_classes": mixed_size_classes(gs.launch),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
