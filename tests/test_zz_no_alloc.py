"""The allocation-free forward (framrir_forward_noalloc: the workspace in the
library's static device scratch) against framrir_forward with a caller
workspace, through the C ABI: two calls in a row, the headline batch (256
rooms, 16 kHz, 2 sources, 6 mics; 45 MB of workspace) and then a smaller
mixed batch, each bit for bit (the forward is bitwise reproducible); a plan
whose workspace exceeds the scratch is refused before anything runs."""
import sys

import numpy as np
import pytest

from paper_2304_08052_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def test_forward_noalloc_matches_forward():
    import torch
    from paper_2304_08052_amd import autotune
    from paper_2304_08052_amd import framrir as fr
    for name, batch in (("batched256", W.config2()), ("small_mixed", W.small_mixed(5, seed=23))):
        plan = fr.Plan(batch, launch=autotune.launch_for(batch))
        assert plan.info.ws_bytes <= fr.NOALLOC_SCRATCH_BYTES
        say(f"{name}: {plan.n_rooms} rooms, workspace {plan.info.ws_bytes} bytes")
        want, want_table = plan.forward()
        out = torch.full_like(want, float("nan"))
        table = torch.full_like(want_table, float("nan"))
        plan.forward_noalloc(table, out)
        torch.cuda.synchronize()
        assert torch.equal(table, want_table), f"{name}: image table differs"
        assert torch.equal(out, want), f"{name}: RIRs differ (max abs {float((out - want).abs().max()):.3e})"


def test_forward_noalloc_refuses_large_plans():
    import torch
    from paper_2304_08052_amd import framrir as fr
    batch = W.config5(0)
    plan = fr.Plan(batch)
    assert plan.info.ws_bytes > fr.NOALLOC_SCRATCH_BYTES
    out = torch.empty(8, dtype=torch.float32, device="cuda")
    table = torch.empty((8, 4), dtype=torch.float64, device="cuda")
    # straight through the C ABI (the binding would refuse the small buffers
    # first): the size check comes before anything touches them
    with pytest.raises(fr.FramrirError) as e:
        fr._check(fr.lib().framrir_forward_noalloc(plan._h, fr._ptr(plan.desc), fr._ptr(table), fr._ptr(plan.mic_dev),
                                                   fr._ptr(plan.src_dev), None, fr._ptr(out), fr._stream(None)))
    assert e.value.code == -4 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
