"""Training losses of the basic models, in torch on the maps the kernels
render (the image, and the auxiliary maps of `aux.render_aux`):

  - photometric: (1 - lam) L1 + lam (1 - SSIM) on the colour and alpha
    channels (Sec. 4.2), lam = 0.2;
  - normal consistency ||N - N~|| between the rendered normal map and the
    pseudo-normal of the rendered depth under local planarity (Eq. 5, Eq. 6);
  - sparsity: L1 of the rendered offset-colour map (Sec. 4.3);
  - bilateral smoothness |grad K| exp(-|grad c_gt|) of the shading-term maps
    (Eq. 7);
  - opacity L1 over the Gaussians (Sec. 4.3).

Weights (appendix): L1 and SSIM combine as 0.8 and 0.2, the opacity L1 is
scaled by 0.1, and the normal consistency and the other regularisers by
0.01.  The editable stage adds its regularisers to the base stage's loss.

Readings where the paper is silent: SSIM after Wang et al. (2004), an 11x11
Gaussian window of sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, averaged over the
windows that lie inside the image (the HIP kernels behind ivrgs_ssim_fwd /
ivrgs_ssim_bwd / ivrgs_photometric_grad, the target taken as a constant);
depth and normal maps are divided by the
alpha map before use (pixels with alpha <= 0.5 are left out); the
pseudo-normal is the cross product of the central differences of the
back-projected points, turned to face the camera and taken to world space;
image gradients are forward differences, |grad c_gt| the mean over colour
channels of their absolute values.
"""
from __future__ import annotations

import torch

from . import native as N
from .raster import _stream


class _SsimFn(torch.autograd.Function):
    """Mean SSIM of a device image against a constant target: argument
    marshalling around the HIP kernels (the forward keeps per-window partial
    derivatives in its workspace for the backward)."""

    @staticmethod
    def forward(ctx, x, y):
        c, h, w = (int(v) for v in x.shape)
        nbytes = N.ivrgs_ssim_workspace_size(c, h, w)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        out = torch.empty((), dtype=torch.float32, device=x.device)
        N.ivrgs_ssim_fwd(x.data_ptr(), y.data_ptr(), c, h, w, out.data_ptr(), ws.data_ptr(), nbytes, _stream())
        ctx.save_for_backward(x, y, ws)
        return out

    @staticmethod
    def backward(ctx, g):
        x, y, ws = ctx.saved_tensors
        c, h, w = (int(v) for v in x.shape)
        gx = torch.empty_like(x)
        g = g.to(torch.float32).contiguous()
        N.ivrgs_ssim_bwd(x.data_ptr(), y.data_ptr(), c, h, w, g.data_ptr(), gx.data_ptr(), ws.data_ptr(),
                         ws.numel(), _stream())
        return gx, None


def _check_pair(x, y):
    if not (x.is_cuda and y.is_cuda):
        raise ValueError("expected device tensors (the kernels run on the GPU; the CPU reference is "
                         "the oracle's, not part of this package)")
    if x.dim() != 3 or y.shape != x.shape or x.dtype != torch.float32 or y.dtype != torch.float32 \
            or y.device != x.device:
        raise ValueError("expected float32 [C, H, W] image and target of one shape and device")
    if x.shape[1] < 11 or x.shape[2] < 11:
        raise ValueError("height and width must be at least 11")


def ssim(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Mean SSIM of two device images [C, H, W] with values in [0, 1],
    through the HIP kernels (float32, 11x11 window of sigma 1.5; no gradient
    to the target)."""
    _check_pair(x, y)
    return _SsimFn.apply(x.contiguous(), y.detach().contiguous())


class _PhotometricFn(torch.autograd.Function):
    """(1 - lam) mean |x - y| + lam (1 - SSIM(x, y)); the backward is one
    launch of ivrgs_photometric_grad over the SSIM forward's workspace."""

    @staticmethod
    def forward(ctx, x, y, lam):
        c, h, w = (int(v) for v in x.shape)
        nbytes = N.ivrgs_ssim_workspace_size(c, h, w)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        s = torch.empty((), dtype=torch.float32, device=x.device)
        N.ivrgs_ssim_fwd(x.data_ptr(), y.data_ptr(), c, h, w, s.data_ptr(), ws.data_ptr(), nbytes, _stream())
        ctx.save_for_backward(x, y, ws)
        ctx.lam = lam
        return (1 - lam) * (x - y).abs().mean() + lam * (1 - s)

    @staticmethod
    def backward(ctx, g):
        x, y, ws = ctx.saved_tensors
        c, h, w = (int(v) for v in x.shape)
        gx = torch.empty_like(x)
        N.ivrgs_photometric_grad(x.data_ptr(), y.data_ptr(), c, h, w, ctx.lam, gx.data_ptr(), ws.data_ptr(),
                                 ws.numel(), _stream())
        return gx * g, None, None


def photometric(rgba: torch.Tensor, target: torch.Tensor, lam: float = 0.2) -> torch.Tensor:
    """(1 - lam) mean |rgba - target| + lam (1 - SSIM), colour and alpha
    (device tensors; no gradient to the target)."""
    _check_pair(rgba, target)
    return _PhotometricFn.apply(rgba.contiguous(), target.detach().contiguous(), float(lam))


def pseudo_normal(depth: torch.Tensor, alpha: torch.Tensor, cam) -> tuple[torch.Tensor, torch.Tensor]:
    """World-space unit normals [3, H, W] of the alpha-normalised depth map
    under local planarity, and the mask of pixels where they are defined."""
    H, W = depth.shape
    dev, dt = depth.device, depth.dtype
    ok = alpha > 0.5
    d = torch.where(ok, depth / alpha.clamp_min(1e-6), torch.zeros_like(depth))
    ys, xs = torch.meshgrid(torch.arange(H, dtype=dt, device=dev) + 0.5,
                            torch.arange(W, dtype=dt, device=dev) + 0.5, indexing="ij")
    P = torch.stack([(xs - cam.cx) / cam.fx * d, (ys - cam.cy) / cam.fy * d, d])  # camera space
    dx = torch.zeros_like(P)
    dy = torch.zeros_like(P)
    dx[:, :, 1:-1] = (P[:, :, 2:] - P[:, :, :-2]) / 2
    dy[:, 1:-1, :] = (P[:, 2:, :] - P[:, :-2, :]) / 2
    n = torch.cross(dx, dy, dim=0)
    n = n / n.norm(dim=0, keepdim=True).clamp_min(1e-12)
    n = torch.where((n * P).sum(0, keepdim=True) > 0, -n, n)  # face the camera
    valid = ok.clone()
    valid[:, [0, -1]] = False
    valid[[0, -1], :] = False
    valid &= ok.roll(1, 0) & ok.roll(-1, 0) & ok.roll(1, 1) & ok.roll(-1, 1)
    R = torch.as_tensor(cam.R, dtype=dt, device=dev)
    return torch.einsum("ji,jhw->ihw", R, n), valid  # R^T n: camera to world


def normal_consistency(normal_map: torch.Tensor, depth: torch.Tensor, alpha: torch.Tensor, cam) -> torch.Tensor:
    """Mean over valid pixels of || N / |N| - N~ ||_2 (Eq. 6)."""
    pn, valid = pseudo_normal(depth.detach(), alpha.detach(), cam)
    nn_ = normal_map / normal_map.norm(dim=0, keepdim=True).clamp_min(1e-12)
    diff = (nn_ - pn).norm(dim=0)
    return diff[valid].mean() if valid.any() else normal_map.sum() * 0


def sparsity(delta_c_map: torch.Tensor) -> torch.Tensor:
    """L1 of the rendered offset-colour map."""
    return delta_c_map.abs().mean()


def bilateral_smoothness(k_maps: torch.Tensor, gt_rgb: torch.Tensor) -> torch.Tensor:
    """Mean over maps and pixels of |grad K| exp(-|grad c_gt|) (Eq. 7),
    forward differences in x and y."""
    gx = (k_maps[:, :, 1:] - k_maps[:, :, :-1]).abs()
    gy = (k_maps[:, 1:, :] - k_maps[:, :-1, :]).abs()
    wx = torch.exp(-(gt_rgb[:, :, 1:] - gt_rgb[:, :, :-1]).abs().mean(0))
    wy = torch.exp(-(gt_rgb[:, 1:, :] - gt_rgb[:, :-1, :]).abs().mean(0))
    return (gx * wx).mean() + (gy * wy).mean()


def opacity_l1(opacity: torch.Tensor) -> torch.Tensor:
    return opacity.abs().mean()


W_OPACITY = 0.1  # the L1 regulariser of the editable stage
W_REG = 0.01     # normal consistency and the other regularisers


def base_loss(rgba, target, depth, normal_map, cam) -> torch.Tensor:
    """Base-3DGS stage: photometric + 0.01 normal consistency (maps of one
    view: rgba [4, H, W], depth [H, W], normal_map [3, H, W])."""
    return photometric(rgba, target) + W_REG * normal_consistency(normal_map, depth, rgba[3], cam)


def editable_loss(rgba, target, maps, opacity, cam) -> torch.Tensor:
    """Editable stage: the base loss plus 0.1 opacity L1 and 0.01 (offset-
    colour sparsity + bilateral smoothness of the four shading maps).  maps
    [11, H, W] from aux.render_aux with aux.editable_attributes: depth, unit
    normal (3), delta-c (3), k_a, k_d, k_s, beta."""
    return (base_loss(rgba, target, maps[0], maps[1:4], cam) + W_OPACITY * opacity_l1(opacity)
            + W_REG * (sparsity(maps[4:7]) + bilateral_smoothness(maps[7:11], target[:3])))
