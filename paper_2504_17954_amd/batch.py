"""Batched training step over many (model, view) jobs, optionally captured as
a HIP graph.

All jobs of a step go through one launch per kernel: projection over every
(job, Gaussian), one binning/sort over every (job, tile), and persistent
render kernels that take (job, tile) items longest-list-first from a device
queue.  The step computes the L1 image gradient elementwise in one launch
(sign(rgba - target) / numel, no reduction kernel), so it can be captured
as a graph and replayed; gradients accumulate over jobs that share
Gaussians (several views of one model).
"""
from __future__ import annotations

import torch

from . import native as N
from . import raster as R


class BatchStep:
    """planes: dict of [d, n] device planes (the concatenated models);
    jobs: raster.Jobs; cams_t: camera table; targets: [n_jobs, 4, H, W]."""

    def __init__(self, planes: dict, cams_t, jobs: R.Jobs, targets: torch.Tensor,
                 settings: R.Settings, model_id=None, edits_t=None, capacity: int | None = None):
        self.planes = planes
        self.cams_t = cams_t
        self.jobs = jobs
        self.targets = targets
        self.model_id = model_id
        self.edits_t = edits_t if edits_t is not None else R.default_edits(cams_t.device)
        self.settings = settings
        dev = cams_t.device
        s = settings
        self.rgba = torch.empty((jobs.n_jobs, 4, s.height, s.width), dtype=torch.float32, device=dev)
        self.dl = torch.empty_like(self.rgba)
        n = planes["mean"].shape[1]
        self.grads = {k: torch.empty((d, n), dtype=torch.float32, device=dev) for k, d in R.PLANE_DIMS.items()}
        self.renderer = R.Renderer(settings, capacity=capacity or (1 << 24), check="sync")
        if tuple(targets.shape) != tuple(self.rgba.shape) or targets.dtype != torch.float32 \
                or not targets.is_contiguous():
            raise ValueError("targets: expected a contiguous float32 [n_jobs, 4, H, W] tensor")
        self.one = torch.ones((), dtype=torch.float32, device=dev)  # dL/d(mean)
        self.graph = None
        # size every buffer (and the pair capacity) with one synchronising pass
        self.renderer.forward(self.planes, self.cams_t, self.jobs, self.model_id, self.edits_t, out=self.rgba)
        self.renderer.grow(int(self.renderer.pairs() * 1.15) + 4096)
        self.renderer.check = "defer"

    def step(self):
        """Forward, L1 image gradient, backward; returns the gradient dict."""
        r = self.renderer
        r.forward(self.planes, self.cams_t, self.jobs, self.model_id, self.edits_t, out=self.rgba)
        N.ivrgs_l1_bwd(self.rgba.data_ptr(), self.targets.data_ptr(), self.rgba.numel(), self.one.data_ptr(),
                       self.dl.data_ptr(), R._stream())
        r.backward(self.planes, self.cams_t, self.jobs, self.rgba, self.dl, self.model_id, self.edits_t,
                   grads=self.grads)
        return self.grads

    def capture(self, warmup: int = 2):
        """Capture step() as a graph (after warm-up on a side stream)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self.step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
        return self.grads

    def verify(self):
        return self.renderer.verify()


def batch_settings(width, height, **kw) -> R.Settings:
    """Settings for batched steps: persistent render kernels on."""
    flags = kw.pop("flags", 0) | N.FLAG_PERSISTENT
    return R.Settings(width, height, flags=flags, **kw)
