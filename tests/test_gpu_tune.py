"""The handle and the tuner through the C ABI: create (gfx950 check, caches)
-> lookup of the shipped entries -> tune over a few candidates on a small
batch (the winner stored under "arch|class" in a temporary cache and read
back by a new handle) -> forward in the tuned shape, bit for bit equal to the
default shape's forward (scatter shapes accumulate the same fixed-point
integers), and a bin-moment candidate within the RIR tolerance."""
import json
import sys

import numpy as np
import pytest

from paper_2304_08052_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def test_create_tune_lookup_forward(tmp_path):
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    cache = tmp_path / "tune.json"
    h = fr.Handle(0, (str(cache), autotune.SHIPPED))
    shipped, found = h.lookup(fr.size_class(W.config2()))
    assert found
    with open(autotune.SHIPPED) as f:
        want = json.load(f)["gfx950|" + fr.size_class(W.config2())]["launch"]
    assert all(shipped[k] == v for k, v in want.items())
    batch = W.small_mixed(6, seed=5)
    cands = [dict(lds_bytes=32768, wg_threads=256, max_mic_group=4, waves_per_simd=4, grid_wgs=512),
             dict(lds_bytes=65536, wg_threads=512, max_mic_group=8, waves_per_simd=8, grid_wgs=512)]
    say(f"tune class {fr.size_class(batch)} over {len(cands)} candidates")
    best, ms = h.tune(batch, candidates=cands, reps=3)
    say(f"best {best} {ms:.4f} ms")
    assert ms > 0.0
    assert any(all(best[k] == c[k] for k in c) for c in cands)
    stored = json.loads(cache.read_text())
    key = "gfx950|" + fr.size_class(batch)
    assert key in stored and stored[key]["launch"]["lds_bytes"] == best["lds_bytes"]
    again, found = fr.Handle(0, (str(cache),)).lookup(fr.size_class(batch))
    assert found and again == best
    out_best, _ = fr.Plan(batch, launch=best).forward()
    out_def, _ = fr.Plan(batch).forward()
    torch.cuda.synchronize()
    assert torch.equal(out_best, out_def)
    # a bin-moment candidate: same RIRs within the tolerance
    mom = dict(lds_bytes=65536, wg_threads=512, max_mic_group=2, waves_per_simd=4, render_path=1)
    best_m, ms_m = h.tune(batch, candidates=[mom], reps=3, size_class="test:moments")
    assert best_m["render_path"] == 1 and ms_m > 0.0
    out_m, _ = fr.Plan(batch, launch=best_m).forward()
    a, b = out_m.cpu().numpy().astype(np.float64), out_def.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)


def test_library_search_on_the_headline_class(tmp_path):
    """The library's own search (scatter and bin-moment shapes) on the
    headline batch returns a valid shape and stores it."""
    from paper_2304_08052_amd import framrir as fr
    cache = tmp_path / "tune.json"
    h = fr.Handle(0, (str(cache),))
    best, ms = h.tune(W.config2(), reps=3)
    say(f"headline search: best {best} {ms:.4f} ms")
    assert ms > 0.0 and best["render_path"] in (0, 1)
    assert "gfx950|" + fr.size_class(W.config2()) in json.loads(cache.read_text())
