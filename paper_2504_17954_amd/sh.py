"""SH colour of base 3DGS (Sec. 3, Sec. 4.2): argument marshalling around
ivrgs_sh_color / ivrgs_sh_color_bwd, and an autograd Function so the colour
plane can feed `raster.rasterize` in a base-model training step.  With the
shading terms (k_a, k_d, k_s) = (1, 0, 0) the projection passes the colour
through unchanged (`base_shade`)."""
from __future__ import annotations

import numpy as np
import torch

from . import native as N
from .raster import _stream


def n_coeffs(degree: int) -> int:
    if not 0 <= degree <= 3:
        raise ValueError("SH degree must be 0..3")
    return (degree + 1) ** 2


def camera_struct(cam) -> N.ivrgs_camera:
    row = cam.row() if hasattr(cam, "row") else np.asarray(cam, np.float32)
    return N.ivrgs_camera.from_buffer_copy(np.ascontiguousarray(row, np.float32)[:16].tobytes())


def _check(sh, mean, degree):
    K = n_coeffs(degree)
    n = int(mean.shape[1])
    for name, t, rows in (("sh", sh, 3 * K), ("mean", mean, 3)):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != (rows, n):
            raise ValueError(f"{name}: expected contiguous float32 [{rows}, n] on the device")
    return n


def color(sh: torch.Tensor, mean: torch.Tensor, cam, degree: int = 3) -> torch.Tensor:
    """[3, n] colour from coefficients sh [3K, n] (row 3k + c: coefficient
    k of channel c) seen from `cam`."""
    n = _check(sh, mean, degree)
    out = torch.empty((3, n), dtype=torch.float32, device=mean.device)
    N.ivrgs_sh_color(sh.data_ptr(), degree, mean.data_ptr(), n, camera_struct(cam), out.data_ptr(), _stream())
    return out


def color_bwd(sh, mean, cam, degree, grad_color, grad_mean=None):
    """dL/dsh [3K, n]; the mean's gradient is added into grad_mean if given."""
    n = _check(sh, mean, degree)
    grad_color = grad_color.contiguous()
    gs = torch.empty_like(sh)
    N.ivrgs_sh_color_bwd(sh.data_ptr(), degree, mean.data_ptr(), n, camera_struct(cam), grad_color.data_ptr(),
                         gs.data_ptr(), None if grad_mean is None else grad_mean.data_ptr(), _stream())
    return gs


class SHColor(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sh, mean, cam, degree):
        ctx.save_for_backward(sh, mean)
        ctx.cam, ctx.degree = cam, degree
        return color(sh, mean, cam, degree)

    @staticmethod
    def backward(ctx, grad_color):
        sh, mean = ctx.saved_tensors
        gm = torch.zeros_like(mean) if ctx.needs_input_grad[1] else None
        gs = color_bwd(sh, mean, ctx.cam, ctx.degree, grad_color, gm)
        return gs, gm, None, None


def base_shade(n: int, device) -> torch.Tensor:
    """Shading planes (k_a, k_d, k_s, beta) = (1, 0, 0, 1): the projection's
    Blinn-Phong step then returns the colour plane as it is."""
    s = torch.zeros((4, n), dtype=torch.float32, device=device)
    s[0] = 1.0
    s[3] = 1.0
    return s
