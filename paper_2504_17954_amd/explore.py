"""Inverse volume exploration (Sec. 4.6) on the GPU.

The Gaussians of every basic model stay frozen.  The composed model is fitted
to one reference image and its camera by learning a few transformation
parameters:
- per basic model, the palette colour c_p and an opacity scale s_o;
- for the whole composed model, one light-magnitude transform
  lambda * (k_a, k_d, k_s, beta) + b (lambda, b in R^4);
- one orbital light direction from its polar and azimuthal angles.

The objective is the paper's combination of L1 and SSIM, weighted as the
appendix weights the photometric loss: (1 - lam) mean |RGBA - target| +
lam (1 - SSIM), lam = 0.2, over colour and alpha.  The optimiser is Adam.

The whole iteration stays on the device, with no host round trip:

    compose_dev -> project -> bin_sort -> render_fwd -> ssim_fwd
      -> photometric_grad -> render_bwd -> compose_bwd, light_bwd
      -> explore_step

- ivrgs_compose_dev composes the scene under the current edit table.
- ivrgs_photometric_grad writes dL/dRGBA of both terms in one launch.
- ivrgs_explore_step takes the Adam step and rewrites that table for the
  next iteration.
- The optimiser state (parameters, Adam moments, step count) lives in one
  device array.
- The pair capacity is sized once, from a binning of the starting
  parameters with headroom; iterations never read the pair count back, and
  `run` checks once at its end that no binning overflowed (`verify`).

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
SSIM_WEIGHT = 0.2


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
                 beta1=0.9, beta2=0.999, eps=1e-8, learn=LEARN_ALL, capacity=1 << 22, lam=SSIM_WEIGHT,
                 headroom=2.0, device="cuda"):
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
        if not 0.0 <= lam <= 1.0:
            raise ValueError("lam must lie in [0, 1]")
        self.lam = float(lam)
        self.comp = {k: torch.empty((d, self.total), dtype=torch.float32, device=self.device)
                     for k, d in R.PLANE_DIMS.items()}
        self.mid = torch.empty(self.total, dtype=torch.int32, device=self.device)
        self.comp_struct = N.ivrgs_gaussians(self.total, *[self.comp[k].data_ptr() for k in R.PLANES],
                                             self.mid.data_ptr())
        # size the pair capacity once: bin the starting scene with the
        # host check (it regrows on overflow), then leave headroom for the
        # opacity and light edits and stop reading the count back
        self.rnd = R.Renderer(settings, capacity=capacity, check="sync", device=self.device)
        N.ivrgs_compose_dev(self.structs, K, self.edits.data_ptr(), self.comp_struct, R._stream())
        self.rnd.project_and_bin(self.rnd.make_batch(self.comp, self.mid, self.edits, self.cams, self.jobs))
        need = self.rnd.pairs()
        if int(need * headroom) + 1024 > self.rnd.capacity:
            self.rnd.grow(int(need * headroom) + 1024)
        self.rnd.check = "defer"
        self.ssim_ws = torch.empty(N.ivrgs_ssim_workspace_size(4, settings.height, settings.width),
                                   dtype=torch.uint8, device=self.device)
        self.ssim_val = torch.zeros((), dtype=torch.float32, device=self.device)
        self.grads = {k: torch.empty((d, self.total), dtype=torch.float32, device=self.device)
                      for k, d in R.PLANE_DIMS.items()}
        self.rgba = torch.empty_like(self.target)
        self.dl = torch.empty_like(self.target)
        self.edit_grad = torch.empty((K, 12), dtype=torch.float32, device=self.device)
        self.light_grad = torch.empty((K, 3), dtype=torch.float32, device=self.device)
        self.iterations = 0

    def step(self):
        """One iteration: render under the current table, SSIM and the
        photometric gradient, backward, edit and light gradients, Adam step
        (rewrites the table)."""
        s = R._stream()
        N.ivrgs_compose_dev(self.structs, self.K, self.edits.data_ptr(), self.comp_struct, s)
        self.rnd.forward(self.comp, self.cams, self.jobs, model_id=self.mid, edits_t=self.edits, out=self.rgba)
        H, W = self.settings.height, self.settings.width
        N.ivrgs_ssim_fwd(self.rgba.data_ptr(), self.target.data_ptr(), 4, H, W, self.ssim_val.data_ptr(),
                         self.ssim_ws.data_ptr(), self.ssim_ws.numel(), s)
        N.ivrgs_photometric_grad(self.rgba.data_ptr(), self.target.data_ptr(), 4, H, W, self.lam,
                                 self.dl.data_ptr(), self.ssim_ws.data_ptr(), self.ssim_ws.numel(), s)
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

    def run(self, iters: int, verify: bool = True):
        """`iters` iterations, then (verify=True) one check that no binning
        overflowed the pair capacity (waits for the stream)."""
        for _ in range(iters):
            self.step()
        if verify:
            self.verify()

    def verify(self) -> int:
        """Raise if a binning since the last check overflowed the pair
        capacity (an overflowing view renders nothing, so its iterations are
        void); else return the pairs of the last binning.  Waits."""
        return self.rnd.verify()

    def loss(self) -> float:
        """Photometric loss of the last rendered image (before the last
        step): (1 - lam) mean |RGBA - target| + lam (1 - SSIM).  Waits."""
        l1 = float((self.rgba - self.target).abs().mean())
        return (1.0 - self.lam) * l1 + self.lam * (1.0 - float(self.ssim_val))

    def theta(self) -> np.ndarray:
        return self.state[:n_params(self.K)].double().cpu().numpy()
