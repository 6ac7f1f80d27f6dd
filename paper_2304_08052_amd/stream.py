"""Fixed-capacity hipGraph step for on-the-fly batches of uneven rooms.

The kernels read every per-batch size (rooms, sources, image rows, work
items, offsets) from the device descriptor, and their grids depend only on
capacities.  So one hipGraph captured with a worst-case capacity plan replays
the draw -> render (-> backward) step for any batch that fits: before each
replay the batch's descriptor and positions are copied into the fixed device
buffers the graph points at.  Argument marshalling only; all work runs in the
library's kernels.
"""
import numpy as np

from . import framrir as fr


def _capacity_batch(n_rooms, n_src, n_mic, rt60, fs, c=343.0):
    """A valid batch with every capacity at its maximum (only its launch
    shapes and sizes are used; its geometry never renders)."""
    size = np.tile([[10.0, 10.0, 4.0]], (n_rooms, 1))
    ang = 2.0 * np.pi * np.arange(n_mic) / n_mic
    mics = np.stack([5.0 + 0.05 * np.cos(ang), 5.0 + 0.05 * np.sin(ang), np.full(n_mic, 1.5)], axis=1)
    srcs = np.stack([np.full(n_src, 3.0), 2.0 + 0.5 * np.arange(n_src), np.full(n_src, 1.5)], axis=1)
    return dict(size=size, rt60=np.full(n_rooms, float(rt60)), fs=np.full(n_rooms, float(fs)),
                c=np.full(n_rooms, float(c)), r_override=np.full(n_rooms, np.nan),
                seed=np.arange(n_rooms, dtype=np.uint64), n_src=np.full(n_rooms, n_src, dtype=np.int32),
                n_mic=np.full(n_rooms, n_mic, dtype=np.int32), src=np.tile(srcs, (n_rooms, 1)),
                mic=np.tile(mics, (n_rooms, 1)))


class GraphStream:
    """Capacity buffers plus one captured step.

    n_rooms, n_src_max, n_mic_max, rt60_max, fs_max bound every batch that
    load() accepts; launch defaults to the tuned shape of that capacity.  backward=True adds the adjoint of an L(h) whose dL/dh is
    the `grad` buffer (filled by the caller)."""

    def __init__(self, n_rooms, n_src_max, n_mic_max, rt60_max, fs_max, params=None, launch=None,
                 backward=True):
        import torch
        self.params = dict(fr.DEFAULT_PARAMS, **(params or {}))
        if launch is None:   # the tuned shape of this capacity class, if one is known
            from .autotune import launch_for_stream
            launch = launch_for_stream(n_rooms, n_src_max, n_mic_max, rt60_max, fs_max)
        self.launch = dict(fr.DEFAULT_LAUNCH, **launch)
        cap_params = dict(self.params, img_lo=self.params["img_hi"])
        self.cap = fr.Plan(_capacity_batch(n_rooms, n_src_max, n_mic_max, rt60_max, fs_max),
                           params=cap_params, launch=self.launch)
        info = self.cap.info
        dev = self.cap.device
        self.backward = backward
        self.desc = torch.zeros(info.desc_bytes, dtype=torch.uint8, device=dev)
        self.table = torch.zeros((info.n_img, 4), dtype=torch.float64, device=dev)
        self.mic = torch.zeros((info.n_mic, 3), dtype=torch.float64, device=dev)
        self.src = torch.zeros((info.n_src, 3), dtype=torch.float64, device=dev)
        self.out = torch.zeros(info.out_floats, dtype=torch.float32, device=dev)
        self.ws = self.cap.workspace(backward=backward)   # the backward reuses the forward's preparation
        self.grad = torch.zeros(info.out_floats, dtype=torch.float32, device=dev)
        self.grads = (torch.zeros((info.n_mic, 3), dtype=torch.float32, device=dev),
                      torch.zeros((info.n_src, 3), dtype=torch.float32, device=dev),
                      torch.zeros(info.n_rooms, dtype=torch.float32, device=dev))
        self.graph = None
        self.plan = None

    def fits(self, plan):
        a, c = plan.info, self.cap.info
        return (plan.params == self.params and plan.launch == self.launch and a.n_rooms <= c.n_rooms
                and a.n_src <= c.n_src and a.n_mic <= c.n_mic and a.n_img <= c.n_img and a.n_items <= c.n_items
                and a.out_floats <= c.out_floats and a.desc_bytes <= c.desc_bytes and a.max_img <= c.max_img)

    def load(self, plan):
        """Copies a batch plan into the capacity buffers (stream-ordered)."""
        if not self.fits(plan):
            raise ValueError("batch exceeds the capacity of this GraphStream")
        self.desc[:plan.info.desc_bytes].copy_(plan.desc, non_blocking=True)
        self.mic[:plan.info.n_mic].copy_(plan.mic_dev, non_blocking=True)
        self.src[:plan.info.n_src].copy_(plan.src_dev, non_blocking=True)
        self.plan = plan

    def step(self):
        """One eager step: draw, render (and backward) of the loaded batch."""
        cap = self.cap
        cap.forward(self.table, mic=self.mic, src=self.src, out=self.out, ws=self.ws, desc=self.desc)
        if self.backward:
            cap.backward(self.table, self.grad, mic=self.mic, src=self.src, ws=self.ws, grads=self.grads,
                         desc=self.desc, prepared=True)

    def capture(self):
        """Captures step() into a hipGraph (after one eager warm-up)."""
        import torch
        if self.plan is None:
            raise RuntimeError("load() a batch before capture()")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.step()
        return self.graph

    def replay(self):
        self.graph.replay()

    def outputs(self):
        """(packed RIRs, grad_mic, grad_src, grad_r) views of the loaded batch."""
        a = self.plan.info
        gm, gs, gr = self.grads
        return self.out[:a.out_floats], gm[:a.n_mic], gs[:a.n_src], gr[:a.n_rooms]
