"""Training losses of the basic models on the maps the kernels render (the
image, and the auxiliary maps of `aux.render_aux`), as autograd Functions
around the HIP kernels (argument marshalling only):

  - photometric: (1 - lam) L1 + lam (1 - SSIM) on the colour and alpha
    channels (Sec. 4.2), lam = 0.2 (ivrgs_ssim_fwd, ivrgs_photometric_grad);
  - the regularisers of one view in one pass (ivrgs_reg_fwd / ivrgs_reg_bwd):
    normal consistency ||N - N~|| between the rendered normal map and the
    pseudo-normal of the rendered depth under local planarity (Eq. 5, Eq. 6),
    sparsity of the offset-colour map (Sec. 4.3), bilateral smoothness
    |grad K| exp(-|grad c_gt|) of the shading-term maps (Eq. 7), opacity L1
    over the Gaussians (Sec. 4.3).

Weights (appendix): L1 and SSIM combine as 0.8 and 0.2, the opacity L1 is
scaled by 0.1, and the normal consistency and the other regularisers by
0.01.  The editable stage adds its regularisers to the base stage's loss.

Readings where the paper is silent: SSIM after Wang et al. (2004), an 11x11
Gaussian window of sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, averaged over the
windows that lie inside the image, the target taken as a constant; depth
maps are divided by the alpha map before use (pixels with alpha <= 0.5 and
their neighbours are left out); the pseudo-normal is the cross product of
the central differences of the back-projected points, turned to face the
camera and taken to world space; image gradients are forward differences,
|grad c_gt| the mean over colour channels of their absolute values.
"""
from __future__ import annotations

import numpy as np
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


class _L1Fn(torch.autograd.Function):
    """mean |x - y| through ivrgs_l1_fwd / ivrgs_l1_bwd (no gradient to y)."""

    @staticmethod
    def forward(ctx, x, y):
        n = x.numel()
        ws = torch.empty(N.ivrgs_l1_workspace_size(n), dtype=torch.uint8, device=x.device)
        out = torch.empty((), dtype=torch.float32, device=x.device)
        N.ivrgs_l1_fwd(x.data_ptr(), y.data_ptr(), n, out.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
        ctx.save_for_backward(x, y)
        return out

    @staticmethod
    def backward(ctx, g):
        x, y = ctx.saved_tensors
        gx = torch.empty_like(x)
        g = g.to(torch.float32).contiguous()
        N.ivrgs_l1_bwd(x.data_ptr(), y.data_ptr(), x.numel(), g.data_ptr(), gx.data_ptr(), _stream())
        return gx, None


def l1(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """mean |x - y| of two float32 device tensors of one shape (the L1 term
    of the photometric loss; no gradient to y), through the HIP kernels."""
    if not (x.is_cuda and y.is_cuda):
        raise ValueError("expected device tensors (the kernels run on the GPU; the CPU reference is "
                         "the oracle's, not part of this package)")
    if y.shape != x.shape or x.dtype != torch.float32 or y.dtype != torch.float32 or y.device != x.device:
        raise ValueError("expected float32 tensors of one shape and device")
    if x.numel() == 0:
        raise ValueError("mean of an empty tensor")
    return _L1Fn.apply(x.contiguous(), y.detach().contiguous())


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
        l1w = torch.empty(N.ivrgs_l1_workspace_size(x.numel()), dtype=torch.uint8, device=x.device)
        m = torch.empty((), dtype=torch.float32, device=x.device)
        N.ivrgs_l1_fwd(x.data_ptr(), y.data_ptr(), x.numel(), m.data_ptr(), l1w.data_ptr(), l1w.numel(), _stream())
        return (1 - lam) * m + lam * (1 - s)

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


def camera_struct(cam) -> N.ivrgs_camera:
    """The ABI camera of an object with .row() (16 float32 words) or a row."""
    row = cam.row() if hasattr(cam, "row") else np.asarray(cam, np.float32)
    return N.ivrgs_camera.from_buffer_copy(np.ascontiguousarray(row, np.float32).tobytes())


def _reg_maps(depth, alpha, normal, delta_c, shade, target, opacity) -> N.ivrgs_reg_maps:
    H, W = (int(v) for v in alpha.shape)
    m = N.ivrgs_reg_maps()
    for name, t, shape in (("depth", depth, (H, W)), ("alpha", alpha, (H, W)), ("normal", normal, (3, H, W)),
                           ("delta_c", delta_c, (3, H, W)), ("shade", shade, (4, H, W)),
                           ("target", target, (3, H, W))):
        if t is None:
            continue
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == shape
                and t.device == alpha.device):
            raise ValueError(f"{name}: expected a contiguous float32 device tensor of shape {shape}")
        setattr(m, name, t.data_ptr())
    if opacity is not None:
        if not (opacity.is_cuda and opacity.dtype == torch.float32 and opacity.is_contiguous()):
            raise ValueError("opacity: expected a contiguous float32 device tensor")
        m.opacity, m.n_gauss = opacity.data_ptr(), opacity.numel()
    m.height, m.width = H, W
    return m


class _RegFn(torch.autograd.Function):
    """The four regulariser terms of one view through ivrgs_reg_fwd /
    ivrgs_reg_bwd (argument marshalling only); no gradient to the depth,
    the alpha map or the target."""

    @staticmethod
    def forward(ctx, cam, depth, alpha, normal, delta_c, shade, target, opacity):
        m = _reg_maps(depth, alpha, normal, delta_c, shade, target, opacity)
        c = camera_struct(cam)
        ws = torch.empty(max(N.ivrgs_reg_workspace_size(m), 1), dtype=torch.uint8, device=alpha.device)
        terms = torch.empty(5, dtype=torch.float32, device=alpha.device)
        N.ivrgs_reg_fwd(m, c, terms.data_ptr(), None, ws.data_ptr(), ws.numel(), _stream())
        ctx.cam = cam
        ctx.save_for_backward(depth, alpha, normal, delta_c, shade, target, opacity, terms)
        return terms[:4]

    @staticmethod
    def backward(ctx, g):
        depth, alpha, normal, delta_c, shade, target, opacity, terms = ctx.saved_tensors
        m = _reg_maps(depth, alpha, normal, delta_c, shade, target, opacity)
        g = g.to(torch.float32).contiguous()
        outs = [None if t is None or not need else torch.empty_like(t)
                for t, need in zip((normal, delta_c, shade, opacity), ctx.needs_input_grad[3:5] +
                                   ctx.needs_input_grad[5:6] + ctx.needs_input_grad[7:8])]
        N.ivrgs_reg_bwd(m, camera_struct(ctx.cam), terms.data_ptr(), g.data_ptr(),
                        *[None if o is None else o.data_ptr() for o in outs], _stream())
        gn, gd, gs, go = outs
        return None, None, None, gn, gd, gs, None, go


def regularisers(depth, alpha, cam, normal=None, delta_c=None, shade=None, target=None,
                 opacity=None) -> torch.Tensor:
    """[normal consistency (Eq. 6), offset-colour sparsity, bilateral
    smoothness (Eq. 7), opacity L1] of one view's maps (device float32:
    depth, alpha [H, W]; normal [3, H, W]; delta_c [3, H, W]; shade
    [4, H, W] with the target colour [3, H, W]; opacity [n]); a term whose
    input is None is 0.  Differentiable in the normal, offset-colour and
    shading maps and the opacities."""
    if opacity is not None:
        opacity = opacity.reshape(-1)
    return _RegFn.apply(cam, depth.contiguous(), alpha.contiguous(), normal, delta_c, shade,
                        None if target is None else target.detach().contiguous(), opacity)


def pseudo_normal(depth: torch.Tensor, alpha: torch.Tensor, cam) -> tuple[torch.Tensor, int]:
    """World-space pseudo-normal map N~ [3, H, W] of the alpha-normalised
    depth (0 where undefined) and the number of pixels where it is defined,
    from the kernel of ivrgs_reg_fwd (waits for the count)."""
    m = _reg_maps(depth.contiguous(), alpha.contiguous(), None, None, None, None, None)
    ws = torch.empty(max(N.ivrgs_reg_workspace_size(m), 1), dtype=torch.uint8, device=alpha.device)
    terms = torch.empty(5, dtype=torch.float32, device=alpha.device)
    pn = torch.empty((3,) + tuple(alpha.shape), dtype=torch.float32, device=alpha.device)
    N.ivrgs_reg_fwd(m, camera_struct(cam), terms.data_ptr(), pn.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    return pn, int(terms[4].item())


W_OPACITY = 0.1  # the L1 regulariser of the editable stage
W_REG = 0.01     # normal consistency and the other regularisers


def base_loss(rgba, target, depth, normal_map, cam) -> torch.Tensor:
    """Base-3DGS stage: photometric + 0.01 normal consistency (maps of one
    view: rgba [4, H, W], depth [H, W], normal_map [3, H, W])."""
    t = regularisers(depth, rgba[3], cam, normal=normal_map)
    return photometric(rgba, target) + W_REG * t[0]


_WEIGHTS = {}


def _editable_weights(device, lam: float) -> torch.Tensor:
    """Device weights of [SSIM, L1, normal consistency, sparsity,
    smoothness, opacity L1] in the editable-stage loss (its constant lam
    added separately)."""
    key = (str(device), float(lam))
    if key not in _WEIGHTS:
        _WEIGHTS[key] = torch.tensor([-lam, 1.0 - lam, W_REG, W_REG, W_REG, W_OPACITY], dtype=torch.float32,
                                     device=device)
    return _WEIGHTS[key]


class _EditableLossFn(torch.autograd.Function):
    """The editable-stage loss of one view: one kernel pass gives the SSIM
    and L1 means (ivrgs_photometric_fwd), the regulariser kernels add their
    four terms into the same device vector, and one dot product with the
    weights combines them.  Backward: the upstream gradient times the
    weights (one device vector), the photometric gradient of the image with
    those weights (ivrgs_photometric_grad_dev) and the regularisers'
    gradients of the maps (written into one buffer, zeros for the depth
    channel) and the opacities."""

    @staticmethod
    def forward(ctx, rgba, target, maps, opacity, cam, lam):
        c, h, w = (int(v) for v in rgba.shape)
        dev = rgba.device
        nbytes = N.ivrgs_photometric_workspace_size(c, h, w)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        # [SSIM, L1, the four regulariser terms, valid-pixel count, unused]
        terms = torch.empty(8, dtype=torch.float32, device=dev)
        base = terms.data_ptr()
        N.ivrgs_photometric_fwd(rgba.data_ptr(), target.data_ptr(), c, h, w, base, ws.data_ptr(), nbytes,
                                _stream())
        m = _reg_maps(maps[0], rgba[3], maps[1:4], maps[4:7], maps[7:11], target[:3], opacity)
        rws = torch.empty(max(N.ivrgs_reg_workspace_size(m), 1), dtype=torch.uint8, device=dev)
        N.ivrgs_reg_fwd(m, camera_struct(cam), base + 8, None, rws.data_ptr(), rws.numel(), _stream())
        wv = _editable_weights(dev, lam)
        ctx.cam = cam
        ctx.save_for_backward(rgba, target, maps, opacity, ws, terms, wv)
        return torch.dot(terms[:6], wv) + lam

    @staticmethod
    def backward(ctx, g):
        rgba, target, maps, opacity, ws, terms, wv = ctx.saved_tensors
        c, h, w = (int(v) for v in rgba.shape)
        gw = wv * g  # dL/d(each term)
        gx = torch.empty_like(rgba)
        N.ivrgs_photometric_grad_dev(rgba.data_ptr(), target.data_ptr(), c, h, w, gw.data_ptr(), gx.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _stream())
        gmaps = torch.empty_like(maps)
        gop = torch.empty_like(opacity)
        m = _reg_maps(maps[0], rgba[3], maps[1:4], maps[4:7], maps[7:11], target[:3], opacity)
        N.ivrgs_reg_bwd(m, camera_struct(ctx.cam), terms.data_ptr() + 8, gw.data_ptr() + 8,
                        gmaps[1].data_ptr(), gmaps[4].data_ptr(), gmaps[7].data_ptr(), gop.data_ptr(), _stream(),
                        gmaps[0].data_ptr())
        return gx, None, gmaps, gop, None, None


def editable_loss(rgba, target, maps, opacity, cam, lam: float = 0.2) -> torch.Tensor:
    """Editable stage: the base loss plus 0.1 opacity L1 and 0.01 (offset-
    colour sparsity + bilateral smoothness of the four shading maps).  rgba
    [4, H, W] and target [4, H, W]; maps [11, H, W] from aux.render_editable
    (or aux.render_aux with aux.editable_attributes): depth, unit normal (3),
    delta-c (3), k_a, k_d, k_s, beta; opacity the Gaussians' opacities."""
    _check_pair(rgba, target)
    if maps.dim() != 3 or maps.shape[0] != 11 or tuple(maps.shape[1:]) != tuple(rgba.shape[1:]):
        raise ValueError("maps: expected [11, H, W] of the image's size")
    return _EditableLossFn.apply(rgba.contiguous(), target.detach().contiguous(), maps.contiguous(),
                                 opacity.reshape(-1).contiguous(), cam, float(lam))
