"""Vector-quantised editable Gaussians (Sec. 4.4) and their composition
(Sec. 4.5): argument marshalling around ivrgs_vq_fit, ivrgs_vq_assign and
ivrgs_vq_compose; the k-means and the decode run in the HIP kernels.

A quantised basic model keeps mean and normal exact and stores one byte per
component of every other attribute, an index into that attribute's scalar
codebook (eight codebooks: log_scale, quat, opacity, delta-c, k_a, k_d, k_s,
beta)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import native as N
from .raster import PLANES, PLANE_DIMS, _stream

# index planes [15, n]: the rows of these float planes, in this order
INDEX_PLANES = (("log_scale", 3), ("quat", 4), ("opacity", 1), ("color", 3), ("shade", 4))
# codebook read by each index plane
PLANE_BOOK = (0, 0, 0, 1, 1, 1, 1, 2, 3, 3, 3, 4, 5, 6, 7)
N_BOOKS = 8


def _dev_f32(name, t):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous float32 device tensor")


def fit(values: torch.Tensor, k: int = 256, iters: int = 10, workspace: torch.Tensor | None = None):
    """k-means codebook (ascending, [k] float32) of the values (any shape,
    all components of one attribute) and the uint8 index of every value."""
    _dev_f32("values", values)
    n = values.numel()
    cb = torch.empty(k, dtype=torch.float32, device=values.device)
    idx = torch.empty(n, dtype=torch.uint8, device=values.device)
    need = N.ivrgs_vq_workspace_size(n, k)
    if need == 0:
        raise ValueError(f"codebook size {k} outside 1..256")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=values.device)
    N.ivrgs_vq_fit(values.data_ptr() if n else None, n, k, iters, cb.data_ptr(),
                   idx.data_ptr() if n else None, workspace.data_ptr(), workspace.numel(), _stream())
    return cb, idx.view(values.shape)


def fit_batch(values: list, k: int = 256, iters: int = 10):
    """`fit` of several attributes at once (one launch per step for up to
    eight of them); each result equals `fit` of that attribute alone."""
    for t in values:
        _dev_f32("values", t)
    if not values:
        return []
    dev = values[0].device
    if any(t.device != dev for t in values):
        raise ValueError("fit_batch: all values on one device")
    out = [(torch.empty(k, dtype=torch.float32, device=dev), torch.empty(t.numel(), dtype=torch.uint8, device=dev))
           for t in values]
    books = [N.ivrgs_vq_book(t.data_ptr() if t.numel() else None, t.numel(), cb.data_ptr(),
                             idx.data_ptr() if t.numel() else None) for t, (cb, idx) in zip(values, out)]
    need = N.ivrgs_vq_fit_batch_workspace_size(books, k)
    if need == 0:
        raise ValueError(f"codebook size {k} outside 1..256")
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    N.ivrgs_vq_fit_batch(books, k, iters, ws.data_ptr(), ws.numel(), _stream())
    return [(cb, idx.view(t.shape)) for t, (cb, idx) in zip(values, out)]


def assign(values: torch.Tensor, codebook: torch.Tensor) -> torch.Tensor:
    """uint8 index of the nearest codebook entry of every value."""
    _dev_f32("values", values)
    _dev_f32("codebook", codebook)
    idx = torch.empty(values.shape, dtype=torch.uint8, device=values.device)
    n = values.numel()
    N.ivrgs_vq_assign(values.data_ptr() if n else None, n, codebook.data_ptr(), codebook.numel(),
                      idx.data_ptr() if n else None, _stream())
    return idx


@dataclass
class QuantizedModel:
    mean: torch.Tensor      # [3, n] float32
    normal: torch.Tensor    # [3, n] float32
    index: torch.Tensor     # [15, n] uint8
    codebook: torch.Tensor  # [8, k] float32

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in (self.mean, self.normal, self.index, self.codebook))

    def struct(self) -> N.ivrgs_vq_model:
        n = self.n
        for name, t, shape, dt in (("mean", self.mean, (3, n), torch.float32),
                                   ("normal", self.normal, (3, n), torch.float32),
                                   ("index", self.index, (15, n), torch.uint8),
                                   ("codebook", self.codebook, (N_BOOKS, self.codebook.shape[-1]), torch.float32)):
            if not t.is_cuda or t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name}: expected contiguous {dt} {shape} on the device")
        return N.ivrgs_vq_model(n, self.mean.data_ptr(), self.normal.data_ptr(), self.index.data_ptr(),
                                self.codebook.data_ptr(), int(self.codebook.shape[1]))


def quantize(planes: dict, k: int = 256, iters: int = 10) -> QuantizedModel:
    """Quantise one basic model: one k-means fit per codebook over all the
    components that share it, the eight fits side by side."""
    n = int(planes["mean"].shape[1])
    dev = planes["mean"].device
    rows = torch.cat([planes[name].reshape(d, n) for name, d in INDEX_PLANES]).contiguous()
    books = torch.empty((N_BOOKS, k), dtype=torch.float32, device=dev)
    index = torch.empty((15, n), dtype=torch.uint8, device=dev)
    spans, p = [], 0
    for b in range(N_BOOKS):
        cnt = PLANE_BOOK.count(b)  # the planes of one book are adjacent
        spans.append((p, cnt))
        p += cnt
    fits = fit_batch([rows[p:p + cnt] for p, cnt in spans], k, iters)
    for b, ((p, cnt), (cb, idx)) in enumerate(zip(spans, fits)):
        books[b] = cb
        index[p:p + cnt] = idx
    return QuantizedModel(planes["mean"].contiguous(), planes["normal"].contiguous(), index, books)


def compose(models: list, edits, device="cuda"):
    """Composition and editing of quantised basic models (Sec. 4.5), each
    decoded inside the compose kernel.  Returns (planes, model_id) like
    raster.compose."""
    structs = [m.struct() for m in models]
    rows = [r.row() if hasattr(r, "row") else np.asarray(r, np.float32) for r in edits]
    if len(rows) != len(structs):
        raise ValueError("one edit row per model")
    es = [N.ivrgs_model_edit.from_buffer_copy(np.ascontiguousarray(r, np.float32).tobytes()) for r in rows]
    total = sum(s.n for s in structs)
    out = {k: torch.empty((d, total), dtype=torch.float32, device=device) for k, d in PLANE_DIMS.items()}
    mid = torch.empty(total, dtype=torch.int32, device=device)
    o = N.ivrgs_gaussians(total, *[out[k].data_ptr() for k in PLANES], mid.data_ptr())
    N.ivrgs_vq_compose(structs, len(structs), es, o, _stream())
    return out, mid
