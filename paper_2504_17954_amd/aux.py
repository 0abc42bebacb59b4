"""Auxiliary maps for the training losses (Eq. 5 depth and normal maps; the
offset-colour and shading-term maps of Sec. 4.3): argument marshalling
around ivrgs_render_aux_fwd / ivrgs_render_aux_bwd and an autograd Function.
The compositing and its backward run in the HIP kernels."""
from __future__ import annotations

import torch

from . import native as N
from .raster import PLANES, PLANE_DIMS, Jobs, Renderer, _stream, default_edits


class _AuxFn(torch.autograd.Function):
    """Forward: project, bin and composite the maps.  Backward: attribute
    gradients and geometry gradients (through alpha and the depth)."""

    @staticmethod
    def forward(ctx, renderer, cams_t, jobs, model_id, edits_t, gauss_index, n_attr, attr, *planes):
        pl = dict(zip(PLANES, planes))
        batch = renderer.make_batch(pl, model_id, edits_t, cams_t, jobs, gauss_index)
        proj, bins = renderer.bins_for(batch)  # the image's bins when it was rendered from the same inputs
        s = renderer.settings
        A = ctx.n_attr = int(n_attr)
        aux = torch.empty((jobs.n_jobs, 1 + A, s.height, s.width), dtype=torch.float32, device=renderer.device)
        N.ivrgs_render_aux_fwd(batch, s.params(), proj, bins, attr.data_ptr() if A else None, A, aux.data_ptr(),
                               _stream())
        ctx.renderer, ctx.jobs, ctx.generation = renderer, jobs, renderer.generation
        ctx.has_mid, ctx.has_idx = model_id is not None, gauss_index is not None
        ctx.save_for_backward(cams_t, model_id if model_id is not None else torch.empty(0), edits_t,
                              gauss_index if gauss_index is not None else torch.empty(0), attr, aux, *planes)
        return aux

    @staticmethod
    def backward(ctx, grad_aux):
        saved = ctx.saved_tensors
        cams_t, mid, edits_t, idx, attr, aux = saved[:6]
        planes = dict(zip(PLANES, saved[6:]))
        r = ctx.renderer
        batch = r.make_batch(planes, mid if ctx.has_mid else None, edits_t, cams_t, ctx.jobs,
                             idx if ctx.has_idx else None)
        if r.generation != ctx.generation:  # the renderer's buffers were reused: bin again
            proj, bins = r.project_and_bin(batch)
        else:
            proj, bins = r._structs(batch)
        n = int(planes["mean"].shape[1])
        grads = {k: torch.zeros((d, n), dtype=torch.float32, device=r.device) for k, d in PLANE_DIMS.items()}
        gattr = torch.zeros_like(attr)
        A = ctx.n_attr
        g = N.ivrgs_gaussians(n, *[grads[k].data_ptr() for k in PLANES], None)
        N.ivrgs_render_aux_bwd(batch, r.settings.params(), proj, bins, attr.data_ptr() if A else None, A,
                               aux.data_ptr(), grad_aux.contiguous().data_ptr(), gattr.data_ptr() if A else None, g,
                               r.ws.data_ptr(), r.ws.numel(), _stream())
        return (None, None, None, None, None, None, None, gattr, *[grads[k] for k in PLANES])


def render_aux(planes: dict, attr: torch.Tensor, cams_t, jobs: Jobs, renderer: Renderer, model_id=None,
               edits_t=None, gauss_index=None, n_attr: int | None = None) -> torch.Tensor:
    """Differentiable maps [n_jobs, 1 + n_attr, H, W]: channel 0 the
    camera-space depth, then the first n_attr columns of the attribute rows
    attr [n, S] (float32, contiguous, S a multiple of 4, 16-byte aligned;
    n_attr defaults to S), each composited with the image's weights
    T_i alpha_i."""
    if attr.dtype != torch.float32 or attr.dim() != 2 or not attr.is_contiguous() or not attr.is_cuda:
        raise ValueError("attr: expected contiguous float32 rows [n, S] on the device")
    S = int(attr.shape[1])
    A = S if n_attr is None else int(n_attr)
    if S % 4 or not 0 <= A <= 15 or S != (A + 3) // 4 * 4 or attr.data_ptr() % 16:
        raise ValueError("attr: rows of n_attr <= 15 values padded to a multiple of 4, 16-byte aligned")
    if edits_t is None:
        edits_t = default_edits(renderer.device)
    return _AuxFn.apply(renderer, cams_t, jobs, model_id, edits_t, gauss_index, A, attr,
                        *[planes[k] for k in PLANES])


EDITABLE_ATTRS = 10  # unit normal 3, delta-c 3, k_a, k_d, k_s, beta
EDITABLE_STRIDE = 12  # row stride of the editable attribute rows


def _check_editable_planes(normal, color, shade):
    n = int(normal.shape[1]) if normal.dim() == 2 else -1
    for name, t, d in (("normal", normal, 3), ("color", color, 3), ("shade", shade, 4)):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == (d, n)):
            raise ValueError(f"{name}: expected a contiguous float32 device tensor [{d}, n]")
    return n


class _EditAttrFn(torch.autograd.Function):
    """Attribute rows [n, 12] from the normal, colour and shade planes
    (ivrgs_editable_attr_fwd) and their backward (ivrgs_editable_attr_bwd)."""

    @staticmethod
    def forward(ctx, normal, color, shade):
        n = _check_editable_planes(normal, color, shade)
        attr = torch.empty((n, EDITABLE_STRIDE), dtype=torch.float32, device=normal.device)
        N.ivrgs_editable_attr_fwd(normal.data_ptr(), color.data_ptr(), shade.data_ptr(), n, attr.data_ptr(),
                                  _stream())
        ctx.save_for_backward(normal)
        return attr

    @staticmethod
    def backward(ctx, g):
        (normal,) = ctx.saved_tensors
        n = int(normal.shape[1])
        g = g.contiguous()
        gn = torch.zeros_like(normal)
        gc = torch.zeros((3, n), dtype=torch.float32, device=normal.device)
        gs = torch.zeros((4, n), dtype=torch.float32, device=normal.device)
        N.ivrgs_editable_attr_bwd(normal.data_ptr(), n, g.data_ptr(), gn.data_ptr(), gc.data_ptr(), gs.data_ptr(),
                                  _stream())
        return gn, gc, gs


def editable_attributes(planes: dict) -> torch.Tensor:
    """The attribute rows of the editable-Gaussian training losses, [n, 12]
    (EDITABLE_ATTRS values and two pad columns): the unit normal (3),
    delta-c (3, the colour plane of a basic model), k_a, k_d, k_s, beta —
    made by the HIP kernel, differentiable in the planes."""
    return _EditAttrFn.apply(planes["normal"], planes["color"], planes["shade"])


class _EditableFn(torch.autograd.Function):
    """The image and the eleven maps of the editable stage from one
    projection and binning, in one walk (ivrgs_render_fwd_aux).  Backward: one call takes the image's and the
    maps' gradients to the planes and the attribute rows
    (ivrgs_render_bwd_aux); the rows' gradient then goes back to the normal,
    colour and shade planes (ivrgs_editable_attr_bwd), so the planes get one
    gradient each."""

    @staticmethod
    def forward(ctx, renderer, cams_t, jobs, edits_t, *planes):
        pl = dict(zip(PLANES, planes))
        n = int(pl["mean"].shape[1])
        attr = torch.empty((n, EDITABLE_STRIDE), dtype=torch.float32, device=renderer.device)
        N.ivrgs_editable_attr_fwd(pl["normal"].data_ptr(), pl["color"].data_ptr(), pl["shade"].data_ptr(), n,
                                  attr.data_ptr(), _stream())
        rgba, maps = renderer.forward_maps(pl, cams_t, jobs, attr, EDITABLE_ATTRS, edits_t)
        ctx.renderer, ctx.jobs, ctx.generation = renderer, jobs, renderer.generation
        ctx.save_for_backward(cams_t, edits_t, rgba, attr, maps, *planes)
        return rgba, maps

    @staticmethod
    def backward(ctx, g_rgba, g_maps):
        saved = ctx.saved_tensors
        cams_t, edits_t, rgba, attr, maps = saved[:5]
        planes = dict(zip(PLANES, saved[5:]))
        r = ctx.renderer
        n = int(planes["mean"].shape[1])
        batch = r.make_batch(planes, None, edits_t, cams_t, ctx.jobs)
        proj, bins = r.prepare_backward(batch, rebin=r.generation != ctx.generation)
        grads = {k: torch.empty((d, n), dtype=torch.float32, device=r.device) for k, d in PLANE_DIMS.items()}
        gattr = torch.empty_like(attr)
        g = N.ivrgs_gaussians(n, *[grads[k].data_ptr() for k in PLANES], None)
        N.ivrgs_render_bwd_aux(batch, r.settings.params(), proj, bins, rgba.data_ptr(),
                               g_rgba.contiguous().data_ptr(), attr.data_ptr(), EDITABLE_ATTRS, maps.data_ptr(),
                               g_maps.contiguous().data_ptr(), gattr.data_ptr(), g, r.ws.data_ptr(), r.ws.numel(),
                               _stream())
        N.ivrgs_editable_attr_bwd(planes["normal"].data_ptr(), n, gattr.data_ptr(), grads["normal"].data_ptr(),
                                  grads["color"].data_ptr(), grads["shade"].data_ptr(), _stream())
        return (None, None, None, None, *[grads[k] for k in PLANES])


def render_editable(planes: dict, cams_t, jobs: Jobs, renderer: Renderer, edits_t=None):
    """Differentiable image [n_jobs, 4, H, W] and editable-stage maps
    [n_jobs, 11, H, W] (depth, unit normal, delta-c, k_a, k_d, k_s, beta) of
    the job batch, from one binning; the same values as rasterize followed
    by render_aux over editable_attributes."""
    if edits_t is None:
        edits_t = default_edits(renderer.device)
    return _EditableFn.apply(renderer, cams_t, jobs, edits_t, *[planes[k] for k in PLANES])
