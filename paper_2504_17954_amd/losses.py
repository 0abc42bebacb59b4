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
windows that lie inside the image (on the device: the HIP kernels behind
ivrgs_ssim_fwd / ivrgs_ssim_bwd, the target taken as a constant; the torch
form below serves CPU tensors); depth and normal maps are divided by the
alpha map before use (pixels with alpha <= 0.5 are left out); the
pseudo-normal is the cross product of the central differences of the
back-projected points, turned to face the camera and taken to world space;
image gradients are forward differences, |grad c_gt| the mean over colour
channels of their absolute values.
"""
from __future__ import annotations

import torch
import torch.nn.functional as F

from . import native as N
from .raster import _stream


def _gauss_window(size: int, sigma: float, dtype, device):
    x = torch.arange(size, dtype=dtype, device=device) - (size - 1) / 2
    g = torch.exp(-(x * x) / (2 * sigma * sigma))
    return g / g.sum()


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


def ssim(x: torch.Tensor, y: torch.Tensor, window: int = 11, sigma: float = 1.5) -> torch.Tensor:
    """Mean SSIM of two images [C, H, W] with values in [0, 1].  Device
    tensors go through the HIP kernels (float32, 11x11 window of sigma 1.5;
    no gradient to the target)."""
    if x.is_cuda:
        if window != 11 or sigma != 1.5:
            raise ValueError("the device SSIM takes the 11x11 window of sigma 1.5")
        if x.dim() != 3 or y.shape != x.shape or x.dtype != torch.float32 or y.dtype != torch.float32 \
                or y.device != x.device:
            raise ValueError("ssim: expected float32 [C, H, W] image and target of one shape and device")
        if x.shape[1] < 11 or x.shape[2] < 11:
            raise ValueError("ssim: height and width must be at least 11")
        return _SsimFn.apply(x.contiguous(), y.detach().contiguous())
    c = x.shape[0]
    g = _gauss_window(window, sigma, x.dtype, x.device)
    wx = g.view(1, 1, 1, window).expand(c, 1, 1, window)
    wy = g.view(1, 1, window, 1).expand(c, 1, window, 1)

    def blur(t):
        return F.conv2d(F.conv2d(t[None], wx, groups=c), wy, groups=c)[0]  # 'valid' windows only

    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return s.mean()


def photometric(rgba: torch.Tensor, target: torch.Tensor, lam: float = 0.2) -> torch.Tensor:
    """(1 - lam) mean |rgba - target| + lam (1 - SSIM), colour and alpha."""
    return (1 - lam) * (rgba - target).abs().mean() + lam * (1 - ssim(rgba, target))


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
