"""Host-side logic of bench.py (no GPU): the one-GPU refusal, and the rule
that counter-based figures (HBM traffic, VALU instruction counts) are
reported only while the kernel sources, the workload and the launch shape are
the ones the committed rocprofv3 passes were taken on."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, HERE)

import bench  # noqa: E402

HEADLINE = dict(lds_bytes=65536, wg_threads=512, grid_wgs=512, max_mic_group=4, waves_per_simd=8)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(HERE, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_figures_follow_the_sources_and_the_shape():
    traffic = bench.measured_traffic("batched", HEADLINE)
    insts = bench.measured_valu_insts("batched", HEADLINE)
    assert traffic is not None and insts is not None, "committed counter passes do not match the sources"
    assert 1.0 <= traffic / 166842720 <= 1.2          # within reach of the algorithmic bytes
    assert insts[0] > 0 and insts[1] > 0
    other = dict(HEADLINE, lds_bytes=32768)
    assert bench.measured_traffic("batched", other) is None
    assert bench.measured_valu_insts("batched", other) is None
    assert bench.measured_traffic("long", HEADLINE) is None


def test_sources_hash_changes_with_any_byte(tmp_path, monkeypatch):
    h0 = bench.kernel_sources_sha256()
    src = tmp_path / "paper_2304_08052_amd" / "csrc"
    src.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_2304_08052_amd", "csrc", f), "rb") as fh:
            (src / f).write_bytes(fh.read())
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    assert bench.kernel_sources_sha256() == h0
    p = src / bench.KERNEL_SOURCES[0]
    p.write_bytes(p.read_bytes() + b"\n")
    assert bench.kernel_sources_sha256() != h0


def test_spatial_traffic_matches_the_sources():
    t = bench.measured_spatial_traffic()
    assert t is not None, "committed spatialisation counters do not match the sources"


class _Info:
    n_chan, n_src, n_mic = 12, 3, 4
    out_floats = 3 * 4 * 1000


class _Plan:
    info = _Info()

    class T:
        pass


def test_spatial_byte_model():
    """One room, 3 sources, 4 mics, 1,000-sample RIRs, n = 40,000: two blocks
    of 31,769 outputs; every term of the model counted by hand."""
    import numpy as np
    plan = _Plan()
    plan.T = np.array([1000])
    n = 40000
    bins = 16385 * 8
    n_blk = 2
    spectra = 12 * bins * (1 + n_blk) + 3 * n_blk * bins + 12 * n_blk * bins
    inputs = 4 * 12000 + 4 * 3 * n_blk * 32768
    images = 4 * 4 * 12 * n
    assert bench.spatial_hbm_bytes(plan, n) == spectra + inputs + images + 4 * 4 * n


def test_defaults_are_one_gpu_and_no_probe():
    """Defaults: one GPU, no copy-probe kernel in ordinary runs."""
    saved = sys.argv
    try:
        sys.argv = ["bench.py"]
        args = bench.parse_args()
    finally:
        sys.argv = saved
    assert args.gpus == 1 and args.copy_probe_mb == 0 and args.workload == "batched"
