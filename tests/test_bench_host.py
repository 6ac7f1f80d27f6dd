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


def _profile(path, workload, launch, sha, **values):
    shape = " ".join(f"{k}={launch[k]}" for k in ("lds_bytes", "wg_threads", "grid_wgs", "max_mic_group",
                                                  "waves_per_simd"))
    lines = ["# counters", "```", "kernel = render_kernel", f"workload = {workload}", f"launch = {shape}",
             f"source_sha256 = {sha}"] + [f"{k} = {v}" for k, v in values.items()] + ["```"]
    path.write_text("\n".join(lines) + "\n")


def test_counter_figures_follow_the_sources_and_the_shape(tmp_path, monkeypatch):
    sha = bench.kernel_sources_sha256()
    hbm, valu = tmp_path / "hbm.md", tmp_path / "valu.md"
    _profile(hbm, "batched", HEADLINE, sha, traffic_bytes=168662465)
    _profile(valu, "batched", HEADLINE, sha, valu_wave_insts=63500000, lds_wave_insts=12700000)
    monkeypatch.setattr(bench, "HBM_PROFILE", str(hbm))
    monkeypatch.setattr(bench, "VALU_PROFILE", str(valu))
    assert bench.measured_traffic("batched", HEADLINE) == 168662465
    assert bench.measured_valu_insts("batched", HEADLINE) == (63500000, 12700000)
    other = dict(HEADLINE, lds_bytes=32768)
    assert bench.measured_traffic("batched", other) is None
    assert bench.measured_valu_insts("batched", other) is None
    assert bench.measured_traffic("long", HEADLINE) is None
    _profile(hbm, "batched", HEADLINE, "0" * 64, traffic_bytes=168662465)     # taken on other sources
    assert bench.measured_traffic("batched", HEADLINE) is None


def test_committed_counter_summaries_parse():
    """The committed summaries carry the key = value block bench.py reads
    (whether they still match the sources is decided at run time)."""
    for path, keys in ((bench.HBM_PROFILE, ("traffic_bytes",)),
                       (bench.VALU_PROFILE, ("valu_wave_insts", "lds_wave_insts"))):
        with open(path) as f:
            kv = dict(line.split(" = ", 1) for line in f.read().splitlines() if " = " in line)
        for k in ("kernel", "workload", "launch", "source_sha256") + keys:
            assert k in kv, f"{path}: {k} missing"


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


def test_spatial_traffic_follows_the_sources(tmp_path, monkeypatch):
    prof = tmp_path / "spatial.md"
    sha = bench.kernel_sources_sha256(bench.SPATIAL_SOURCES)
    prof.write_text(f"workload = spatial\nsource_sha256 = {sha}\ntraffic_bytes = 6960000000\n")
    monkeypatch.setattr(bench, "SPATIAL_HBM_PROFILE", str(prof))
    assert bench.measured_spatial_traffic() == 6960000000
    prof.write_text("workload = spatial\nsource_sha256 = 0\ntraffic_bytes = 6960000000\n")
    assert bench.measured_spatial_traffic() is None


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
