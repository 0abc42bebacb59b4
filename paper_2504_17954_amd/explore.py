"""Inverse volume exploration (Sec. 4.6) on the GPU.

The Gaussians of every basic model stay frozen.  The composed model is fitted
to one reference image and its camera by learning a few transformation
parameters:
- per basic model, the palette colour c_p and an opacity scale s_o;
- for the whole composed model, one light-magnitude transform
  lambda * (k_a, k_d, k_s, beta) + b (lambda, b in R^4);
- one orbital light direction from its polar and azimuthal angles.

The paper uses L1 + SSIM.  This loop uses the L1 term (mean |RGBA - target|)
and Adam.

The whole iteration stays on the device, with no host round trip:

    compose_dev -> project -> bin_sort -> render_fwd -> L1 gradient
      -> render_bwd -> compose_bwd, light_bwd -> explore_step

- ivrgs_compose_dev composes the scene under the current edit table.
- ivrgs_explore_step takes the Adam step and rewrites that table for the
  next iteration.
- The optimiser state (parameters, Adam moments, step count) lives in one
  device array.

Parameter vector layout (K models, n = 4K + 10):

    [palette K*3 | s_o K | lambda 4 | b 4 | polar | azimuth]
"""
from __future__ import annotations

import numpy as np
import torch

from . import native as N
from . import raster as R

LEARN_PALETTE, LEARN_OPACITY, LEARN_MAGNITUDE, LEARN_LIGHT = 1, 2, 4, 8
LEARN_ALL = 15


def n_params(K: int) -> int:
    return 4 * K + 10


def initial_theta(palettes, opacity_scales=None, lam=(1, 1, 1, 1), bias=(0, 0, 0, 0), polar=0.0, azimuth=0.0):
    """Parameter vector from its parts (float64, host)."""
    palettes = np.asarray(palettes, np.float64).reshape(-1, 3)
    K = palettes.shape[0]
    s_o = np.ones(K) if opacity_scales is None else np.asarray(opacity_scales, np.float64)
    return np.concatenate([palettes.reshape(-1), s_o, np.asarray(lam, np.float64),
                           np.asarray(bias, np.float64), [polar, azimuth]])


class Explorer:
    """Fits the exploration parameters to `target` ([4, H, W] or [1, 4, H, W]
    device float32) seen from `camera`.

    - models: list of device plane dicts, one per basic model, whose colour
      plane holds the offsets delta-c.
    - base_rows: one edit row per model.  Only the headlight word is used, and
      the light direction of headlight models.
    - theta0: the starting parameter vector.
    """

    def __init__(self, models, base_rows, theta0, camera, target, settings: R.Settings, lr=0.01,
                 beta1=0.9, beta2=0.999, eps=1e-8, learn=LEARN_ALL, capacity=1 << 24, device="cuda"):
        self.device = torch.device(device)
        self.models = list(models)
        self.K = K = len(self.models)
        self.structs = [R.gaussians_struct(m) for m in self.models]
        self.total = sum(s.n for s in self.structs)
        self.edits = R.edit_table(base_rows, self.device)
        if self.edits.shape[0] != K:
            raise ValueError("one base row per model")
        heads = self.edits[:, 15].cpu().numpy().view(np.int32)
        self.orbital = bool((heads == 0).any())
        theta0 = np.asarray(theta0, np.float64)
        if theta0.shape != (n_params(K),):
            raise ValueError(f"theta0: expected {n_params(K)} values")
        self.state = torch.zeros(N.ivrgs_explore_state_words(K), dtype=torch.float32, device=self.device)
        self.state[:n_params(K)] = torch.from_numpy(theta0.astype(np.float32)).to(self.device)
        self.opts = N.ivrgs_explore_opts(lr, beta1, beta2, eps, int(learn))
        # the table from the starting parameters (learn = 0 only rewrites it)
        N.ivrgs_explore_step(None, None, K, N.ivrgs_explore_opts(lr, beta1, beta2, eps, 0),
                             self.state.data_ptr(), self.edits.data_ptr(), R._stream())

        self.settings = settings
        self.cams = R.camera_table([camera], self.device)
        self.jobs = R.Jobs.single(self.total)
        t = target.reshape(1, 4, settings.height, settings.width)
        if t.dtype != torch.float32 or not t.is_cuda:
            raise ValueError("target: expected a float32 device tensor")
        self.target = t.contiguous()
        self.rnd = R.Renderer(settings, capacity=capacity, check="sync", device=self.device)
        self.comp = {k: torch.empty((d, self.total), dtype=torch.float32, device=self.device)
                     for k, d in R.PLANE_DIMS.items()}
        self.mid = torch.empty(self.total, dtype=torch.int32, device=self.device)
        self.comp_struct = N.ivrgs_gaussians(self.total, *[self.comp[k].data_ptr() for k in R.PLANES],
                                             self.mid.data_ptr())
        self.grads = {k: torch.empty((d, self.total), dtype=torch.float32, device=self.device)
                      for k, d in R.PLANE_DIMS.items()}
        self.rgba = torch.empty_like(self.target)
        self.dl = torch.empty_like(self.target)
        self.edit_grad = torch.empty((K, 12), dtype=torch.float32, device=self.device)
        self.light_grad = torch.empty((K, 3), dtype=torch.float32, device=self.device)
        self.iterations = 0

    def step(self):
        """One iteration: render under the current table, L1 gradient,
        backward, edit and light gradients, Adam step (rewrites the table)."""
        s = R._stream()
        N.ivrgs_compose_dev(self.structs, self.K, self.edits.data_ptr(), self.comp_struct, s)
        self.rnd.forward(self.comp, self.cams, self.jobs, model_id=self.mid, edits_t=self.edits, out=self.rgba)
        # dL/dRGBA of mean |RGBA - target|
        torch.sub(self.rgba, self.target, out=self.dl)
        self.dl.sign_().mul_(1.0 / self.dl.numel())
        self.rnd.backward(self.comp, self.cams, self.jobs, self.rgba, self.dl, model_id=self.mid,
                          edits_t=self.edits, grads=self.grads)
        R.compose_bwd(self.models, self.grads, out=self.edit_grad)
        lg = None
        if self.orbital:
            self.rnd.light_grad(self.comp, self.cams, self.jobs, model_id=self.mid, edits_t=self.edits,
                                out=self.light_grad)
            lg = self.light_grad.data_ptr()
        N.ivrgs_explore_step(self.edit_grad.data_ptr(), lg, self.K, self.opts, self.state.data_ptr(),
                             self.edits.data_ptr(), s)
        self.iterations += 1

    def run(self, iters: int):
        for _ in range(iters):
            self.step()

    def loss(self) -> float:
        """L1 loss of the last rendered image (before the last step; syncs)."""
        return float((self.rgba - self.target).abs().mean())

    def theta(self) -> np.ndarray:
        return self.state[:n_params(self.K)].double().cpu().numpy()
