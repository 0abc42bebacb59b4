"""Learned culling of Gaussians per view.

Labels come from the rasterizer itself: a Gaussian is "visible" in a view if
its largest compositing weight T*alpha over the view's pixels reaches 1/255
(`ivrgs_render_fwd` with a maxw output).  Removing a Gaussian whose weight
stays below w changes any pixel by at most 2 w per unit colour, so the label
bounds each culled Gaussian's own error; the PSNR of culled against plain
renders measures what the misses add up to.

An MLP 10 -> 64 -> 64 -> 1 (ReLU) on (mean, log-scale, opacity, unit
direction to the camera) is trained in FP32 with torch; inference runs in the
`ivrgs_cull` kernel on BF16 matrix cores, followed by an ordered compaction
whose survivor count goes straight into the device job table.  Full
rasterisation (threshold -inf) is the fallback and the reference.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import native as N
from . import raster as R

N_FEAT = 10
HIDDEN = 64
VISIBLE = 1.0 / 255.0


def static_features(planes: dict) -> torch.Tensor:
    """[n, 7]: mean, log-scale, opacity."""
    return torch.cat([planes["mean"].T, planes["log_scale"].T, planes["opacity"].T], 1)


def view_dirs(planes: dict, cam_row: torch.Tensor) -> torch.Tensor:
    """[n, 3] unit direction from each Gaussian to the camera centre."""
    Rm = cam_row[:9].reshape(3, 3)
    c = -(Rm.T @ cam_row[9:12])
    d = c[None, :] - planes["mean"].T
    return d / d.norm(dim=1, keepdim=True)


def collect_labels(planes: dict, cams_t: torch.Tensor, width: int, height: int,
                   renderer: R.Renderer | None = None) -> torch.Tensor:
    """[views, n] uint8 labels: max T*alpha of each Gaussian >= 1/255."""
    n = planes["mean"].shape[1]
    rnd = renderer or R.Renderer(R.Settings(width, height))
    out = torch.empty((cams_t.shape[0], n), dtype=torch.uint8, device=cams_t.device)
    with torch.no_grad():
        for v in range(cams_t.shape[0]):
            _, maxw = rnd.forward(planes, cams_t, R.Jobs.single(n, camera=v), edits_t=R.default_edits(cams_t.device),
                                  want_maxw=True, fwd_only=True)
            out[v] = (maxw[:n] >= VISIBLE).to(torch.uint8)
    return out


class MLP(torch.nn.Module):
    def __init__(self):
        super().__init__()
        self.l1 = torch.nn.Linear(N_FEAT, HIDDEN)
        self.l2 = torch.nn.Linear(HIDDEN, HIDDEN)
        self.l3 = torch.nn.Linear(HIDDEN, 1)

    def forward(self, x):
        return self.l3(torch.relu(self.l2(torch.relu(self.l1(x))))).squeeze(-1)


def train(planes: dict, cams_t: torch.Tensor, labels: torch.Tensor, steps: int = 3000, batch: int = 65536,
          lr: float = 2e-3, seed: int = 0):
    """Fit the MLP on random (view, Gaussian) pairs.  Returns (model, mean,
    std) with the input normalisation statistics."""
    g = torch.Generator(device=cams_t.device)
    g.manual_seed(seed)
    torch.manual_seed(seed)
    dev = cams_t.device
    stat = static_features(planes)
    n, V = stat.shape[0], cams_t.shape[0]
    # normalisation statistics from a sample
    vs = torch.randint(0, V, (min(V, 16),), generator=g, device=dev)
    sample = torch.cat([torch.cat([stat, view_dirs(planes, cams_t[v])], 1) for v in vs.tolist()])
    mean, std = sample.mean(0), sample.std(0).clamp_min(1e-6)
    model = MLP().to(dev)
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)
    pos = labels.float().mean().clamp(1e-3, 1 - 1e-3)
    for _ in range(steps):
        v = torch.randint(0, V, (batch,), generator=g, device=dev)
        i = torch.randint(0, n, (batch,), generator=g, device=dev)
        cr = cams_t[v]
        Rm = cr[:, :9].reshape(-1, 3, 3)
        c = -(Rm.transpose(1, 2) @ cr[:, 9:12, None])[:, :, 0]
        d = c - planes["mean"].T[i]
        d = d / d.norm(dim=1, keepdim=True)
        x = (torch.cat([stat[i], d], 1) - mean) / std
        y = labels[v, i].float()
        loss = torch.nn.functional.binary_cross_entropy_with_logits(
            model(x), y, pos_weight=((1 - pos) / pos).sqrt())
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        sched.step()
    return model, mean, std


def to_bf16_bits(x: torch.Tensor) -> torch.Tensor:
    """float32 -> bf16 bit patterns (round to nearest even) as int16."""
    u = x.float().contiguous().view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r & 0xFFFF).to(torch.int32).to(torch.int16)


@dataclass
class CullWeights:
    w1: torch.Tensor   # [64, 16] int16 bf16 bits
    b1: torch.Tensor   # [64] float32
    w2: torch.Tensor   # [64, 64] int16
    b2: torch.Tensor
    w3: torch.Tensor
    b3: float
    threshold: float = 0.0

    def struct(self) -> N.ivrgs_culler:
        return N.ivrgs_culler(self.w1.data_ptr(), self.b1.data_ptr(), self.w2.data_ptr(), self.b2.data_ptr(),
                              self.w3.data_ptr(), float(self.b3), float(self.threshold))


def pack(model: MLP, mean: torch.Tensor, std: torch.Tensor, threshold: float = 0.0) -> CullWeights:
    """Fold the input normalisation into the first layer and pack BF16."""
    with torch.no_grad():
        W1 = model.l1.weight / std[None, :]
        b1 = model.l1.bias - (model.l1.weight * (mean / std)[None, :]).sum(1)
        w1 = torch.zeros((HIDDEN, 16), dtype=torch.float32, device=W1.device)
        w1[:, :N_FEAT] = W1
        # detached copies: the packed weights must not alias the parameters
        return CullWeights(to_bf16_bits(w1).contiguous(), b1.detach().float().clone(),
                           to_bf16_bits(model.l2.weight.detach()).contiguous(),
                           model.l2.bias.detach().float().clone(),
                           model.l3.weight[0].detach().float().clone(), float(model.l3.bias[0]), threshold)


class Culler:
    """Runs `ivrgs_cull` and renders the survivors."""

    def __init__(self, weights: CullWeights, n: int, device="cuda"):
        self.w = weights
        self.n = n
        self.index = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        self.logits = torch.empty(max(n, 1), dtype=torch.float32, device=device)
        self.ws = torch.empty(N.ivrgs_cull_workspace_size(n), dtype=torch.uint8, device=device)

    def run(self, planes: dict, cams_t: torch.Tensor, jobs: R.Jobs, camera: int, job: int = 0,
            want_logits: bool = False):
        g = R.gaussians_struct(planes)
        N.ivrgs_cull(g, cams_t.data_ptr(), camera, self.w.struct(), self.index.data_ptr(), jobs.device.data_ptr(),
                     job, self.logits.data_ptr() if want_logits else None, self.ws.data_ptr(), self.ws.numel(),
                     R._stream())
        return self.index

    def render(self, renderer: R.Renderer, planes: dict, cams_t: torch.Tensor, jobs: R.Jobs, camera: int,
               out=None):
        """Cull then forward-render one view; jobs must be a one-job table whose
        host count is n (an upper bound) and whose device count the cull writes."""
        self.run(planes, cams_t, jobs, camera)
        return renderer.forward(planes, cams_t, jobs, edits_t=R.default_edits(cams_t.device),
                                gauss_index=self.index, out=out, fwd_only=True)


def calibrate_threshold(culler: Culler, planes: dict, cams_t: torch.Tensor, labels: torch.Tensor,
                        recall: float = 0.999, views=None) -> float:
    """Largest threshold whose recall of visible Gaussians on the given views
    (using the kernel's own BF16 logits) is at least `recall`."""
    n = planes["mean"].shape[1]
    vals = []
    jobs = R.Jobs.single(n)
    for v in (views if views is not None else range(cams_t.shape[0])):
        jobs.device[0, 0] = v
        culler.run(planes, cams_t, jobs, v, want_logits=True)
        vals.append(culler.logits[:n][labels[v].bool()].clone())
    pos = torch.cat(vals)
    if pos.numel() == 0:
        return -math.inf
    return float(torch.quantile(pos.float()[torch.randperm(pos.numel(), device=pos.device)[:1 << 24]],
                                1.0 - recall))


def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    """PSNR of RGB clamped to [0, 1], peak 1."""
    d = (a[:3].clamp(0, 1) - b[:3].clamp(0, 1)).float()
    mse = float((d * d).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def loss_from_psnr(q_db: float, model_psnr_db: float = 36.44) -> float:
    """PSNR loss (dB) against ground truth when a culling error of PSNR q is
    added to a model error of PSNR p: 10 log10(1 + 10^((p - q)/10))."""
    if math.isinf(q_db):
        return 0.0
    return 10.0 * math.log10(1.0 + 10.0 ** ((model_psnr_db - q_db) / 10.0))
