"""Training regularisers of the editable Gaussians on the rendered maps of one
view, plain FP64 torch on the CPU, gradients by autograd.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the product
path; it shares no code with the HIP library.

Terms (the appendix weights them 0.01 each, the opacity L1 0.1):
  - normal consistency (Eq. 6): the mean over valid pixels of
    || N / |N| - N~ ||_2, N the composited normal map (Eq. 5), N~ the
    pseudo-normal of the rendered depth under local planarity, held fixed;
  - sparsity of the offset colour (Sec. 4.3): mean |delta-c map|;
  - bilateral smoothness of the shading-term maps (Eq. 7): the mean of
    |grad K| exp(-|grad c_gt|) over the four maps and the pixels, x and y
    forward differences each averaged over their own entries and summed;
  - opacity L1 (Sec. 4.3): mean |o| over the Gaussians.

Readings where the paper is silent (the same on the GPU side):
  - depth and the pseudo-normal: the depth map is alpha-weighted, so the
    depth is depth / alpha at pixels with alpha > 0.5; each pixel centre
    (x + 1/2, y + 1/2) back-projects to P = d ((x + 1/2 - cx) / fx,
    (y + 1/2 - cy) / fy, 1) in camera space; N~ is the normalised cross
    product of the central differences (P[x+1] - P[x-1]) / 2 and
    (P[y+1] - P[y-1]) / 2, negated when it points away from the camera
    (N~ . P > 0), and taken to world space with R^T;
  - a pixel is valid when it and its four neighbours have alpha > 0.5 and
    it is not on the image border; invalid pixels carry no term and N~ = 0
    there; with no valid pixel the term is 0;
  - |N| is clamped below at 1e-12 before the division;
  - |grad c_gt| is the mean over the three colour channels of the absolute
    forward difference of the target;
  - |x| has the derivative sign(x), 0 at 0; ||v||_2 has the gradient 0 at 0.
"""
from __future__ import annotations

import numpy as np
import torch

ALPHA_VALID = 0.5
NORM_FLOOR = 1e-12


def _t(a):
    return torch.as_tensor(np.asarray(a, np.float64))


def valid_mask(alpha: torch.Tensor) -> torch.Tensor:
    """Pixels with a pseudo-normal: alpha > 0.5 there and at the four
    neighbours, not on the border."""
    ok = alpha > ALPHA_VALID
    v = torch.zeros_like(ok)
    v[1:-1, 1:-1] = ok[1:-1, 1:-1] & ok[:-2, 1:-1] & ok[2:, 1:-1] & ok[1:-1, :-2] & ok[1:-1, 2:]
    return v


def pseudo_normal(depth, alpha, cam) -> tuple[torch.Tensor, torch.Tensor]:
    """(N~ [3, H, W] in world space, zero where invalid; valid mask [H, W])."""
    depth, alpha = _t(depth), _t(alpha)
    H, W = depth.shape
    ok = alpha > ALPHA_VALID
    d = torch.where(ok, depth / torch.where(ok, alpha, torch.ones_like(alpha)), torch.zeros_like(depth))
    ys = torch.arange(H, dtype=torch.float64)[:, None] + 0.5
    xs = torch.arange(W, dtype=torch.float64)[None, :] + 0.5
    P = torch.stack([(xs - float(cam.cx)) / float(cam.fx) * d, (ys - float(cam.cy)) / float(cam.fy) * d, d])
    tx = torch.zeros_like(P)
    ty = torch.zeros_like(P)
    tx[:, :, 1:-1] = (P[:, :, 2:] - P[:, :, :-2]) / 2
    ty[:, 1:-1, :] = (P[:, 2:, :] - P[:, :-2, :]) / 2
    n = torch.linalg.cross(tx, ty, dim=0)
    nn = torch.linalg.vector_norm(n, dim=0)
    valid = valid_mask(alpha)
    n = torch.where(valid[None], n / torch.where(nn > 0, nn, torch.ones_like(nn))[None], torch.zeros_like(n))
    n = torch.where((n * P).sum(0, keepdim=True) > 0, -n, n)
    R = _t(np.asarray(cam.R, np.float64))
    return torch.einsum("ji,jhw->ihw", R, n), valid


def normal_consistency(normal_map: torch.Tensor, pn: torch.Tensor, valid: torch.Tensor) -> torch.Tensor:
    """Mean over valid pixels of || N / max(|N|, 1e-12) - N~ ||_2."""
    if not bool(valid.any()):
        return normal_map.sum() * 0.0
    nrm = torch.linalg.vector_norm(normal_map, dim=0, keepdim=True).clamp_min(NORM_FLOOR)
    diff = torch.linalg.vector_norm(normal_map / nrm - pn, dim=0)
    return diff[valid].mean()


def sparsity(delta_c: torch.Tensor) -> torch.Tensor:
    return delta_c.abs().mean()


def bilateral_smoothness(k_maps: torch.Tensor, target_rgb: torch.Tensor) -> torch.Tensor:
    gx = (k_maps[:, :, 1:] - k_maps[:, :, :-1]).abs()
    gy = (k_maps[:, 1:, :] - k_maps[:, :-1, :]).abs()
    wx = torch.exp(-(target_rgb[:, :, 1:] - target_rgb[:, :, :-1]).abs().mean(0))
    wy = torch.exp(-(target_rgb[:, 1:, :] - target_rgb[:, :-1, :]).abs().mean(0))
    return (gx * wx).mean() + (gy * wy).mean()


def opacity_l1(opacity: torch.Tensor) -> torch.Tensor:
    return opacity.abs().mean()


def terms(depth, alpha, normal_map, delta_c, shade_maps, target_rgb, opacity, cam, grad_terms=None):
    """The four terms [normal consistency, sparsity, smoothness, opacity L1],
    the valid pixel count, N~, and (grad_terms given: upstream gradients of
    the four terms) the gradients with respect to the normal map, the
    offset-colour map, the shading maps and the opacities (autograd; the
    depth and alpha maps and the target get none)."""
    pn, valid = pseudo_normal(depth, alpha, cam)
    nm = _t(normal_map).requires_grad_(True)
    dc = _t(delta_c).requires_grad_(True)
    km = _t(shade_maps).requires_grad_(True)
    op = _t(opacity).requires_grad_(True)
    vals = torch.stack([normal_consistency(nm, pn, valid), sparsity(dc),
                        bilateral_smoothness(km, _t(target_rgb)), opacity_l1(op)])
    out = {"terms": vals.detach().numpy(), "count": int(valid.sum()), "pseudo_normal": pn.numpy(),
           "valid": valid.numpy()}
    if grad_terms is not None:
        (vals * _t(grad_terms)).sum().backward()
        out.update(grad_normal=nm.grad.numpy(), grad_delta_c=dc.grad.numpy(), grad_shade=km.grad.numpy(),
                   grad_opacity=op.grad.numpy())
    return out
