"""Torch-facing API of the HIP rasterizer.

PyTorch provides device memory and streams; every step of the pipeline runs
in libivrgs.so (see include/ivrgs.h):

    compose(models, edits)            -> composed planes + model ids (Sec. 4.5)
    Renderer.forward(...)             project -> bin_sort -> render_fwd
    Renderer.backward(...)            render_bwd (recompute, nothing stored per pixel)
    rasterize(...)                    torch.autograd.Function around the two

Planes are float32 CUDA (HIP) tensors of shape [k, n] (component-major).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import native as N

PLANES = N.PLANES
PLANE_DIMS = dict(zip(N.PLANES, N.PLANE_DIMS))


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check_plane(name, t, n=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: expected a device tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous float32")
    d = PLANE_DIMS[name]
    if t.dim() != 2 or t.shape[0] != d or (n is not None and t.shape[1] != n):
        raise ValueError(f"{name}: expected shape [{d}, n], got {tuple(t.shape)}")


def gaussians_struct(planes: dict, model_id=None) -> N.ivrgs_gaussians:
    n = int(planes["mean"].shape[1])
    for k in PLANES:
        _check_plane(k, planes[k], n)
    if model_id is not None and (model_id.dtype != torch.int32 or model_id.numel() != n
                                 or not model_id.is_contiguous()):
        raise ValueError("model_id: expected contiguous int32 of length n")
    return N.ivrgs_gaussians(n, *[planes[k].data_ptr() for k in PLANES], _ptr(model_id))


@dataclass
class Settings:
    """Compositing constants and launch shape (see ivrgs_params)."""
    width: int
    height: int
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    lowpass: float = 0.3
    z_near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)
    fwd_px: int = 0
    bwd_px: int = 0
    sort_chunk: int = 0
    flags: int = 0
    persist_per_cu: int = 0

    def params(self) -> N.ivrgs_params:
        p = N.ivrgs_params()
        p.alpha_min, p.alpha_max, p.T_min = self.alpha_min, self.alpha_max, self.T_min
        p.lowpass, p.z_near = self.lowpass, self.z_near
        p.bg = (N.C.c_float * 3)(*self.bg)
        p.width, p.height, p.tile = self.width, self.height, 16
        p.flags, p.fwd_px, p.bwd_px, p.sort_chunk = self.flags, self.fwd_px, self.bwd_px, self.sort_chunk
        p.persist_per_cu = self.persist_per_cu
        return p


def edit_table(rows, device="cuda") -> torch.Tensor:
    """[K, 16] float32 device table of edit rows (palette 3, opacity scale,
    shade scale 4, shade bias 4, light dir 3, headlight as int32 bits)."""
    arr = np.stack([r.row() if hasattr(r, "row") else np.asarray(r, np.float32) for r in rows])
    return torch.from_numpy(np.ascontiguousarray(arr, np.float32)).to(device)


def camera_table(cams, device="cuda") -> torch.Tensor:
    arr = np.stack([c.row() if hasattr(c, "row") else np.asarray(c, np.float32) for c in cams])
    return torch.from_numpy(np.ascontiguousarray(arr, np.float32)).to(device)


@dataclass
class Jobs:
    """Job table: (camera, gauss_begin, gauss_count, rec_begin) per job."""
    host: np.ndarray
    device: torch.Tensor = field(default=None)

    def __post_init__(self):
        self.host = np.ascontiguousarray(self.host, np.int32).reshape(-1, 4)
        if self.device is None:
            self.device = torch.from_numpy(self.host.copy()).to("cuda")

    @property
    def n_jobs(self) -> int:
        return int(self.host.shape[0])

    @property
    def n_records(self) -> int:
        return int(self.host[:, 2].sum())

    @property
    def max_count(self) -> int:
        return int(self.host[:, 2].max()) if self.n_jobs else 0

    @staticmethod
    def ranges(cameras, begins, counts) -> "Jobs":
        cameras, begins, counts = (np.asarray(v, np.int64) for v in (cameras, begins, counts))
        rec = np.concatenate([[0], np.cumsum(counts)[:-1]])
        return Jobs(np.stack([cameras, begins, counts, rec], 1))

    @staticmethod
    def single(n: int, camera: int = 0) -> "Jobs":
        return Jobs.ranges([camera], [0], [n])

    @staticmethod
    def views(n: int, cameras) -> "Jobs":
        cameras = list(cameras)
        return Jobs.ranges(cameras, [0] * len(cameras), [n] * len(cameras))

    @staticmethod
    def models_by_views(model_sizes, n_views: int) -> "Jobs":
        """Job (m, v): model m's Gaussians (concatenated in model order) seen
        by camera v; jobs ordered model-major."""
        starts = np.concatenate([[0], np.cumsum(model_sizes)[:-1]])
        cams, begins, counts = [], [], []
        for m, (s, c) in enumerate(zip(starts, model_sizes)):
            for v in range(n_views):
                cams.append(v)
                begins.append(s)
                counts.append(c)
        return Jobs.ranges(cams, begins, counts)


class Renderer:
    """Owns the device buffers of one pipeline instance (records, bins,
    workspace).  Buffers grow on demand and are reused across calls.

    check: "sync" reads the device pair count after binning and re-bins with a
    larger capacity if it overflowed (one host sync per call); "defer" never
    syncs, and `verify()` reports an overflow afterwards."""

    def __init__(self, settings: Settings, capacity: int = 1 << 22, check: str = "sync",
                 device="cuda"):
        self.settings = settings
        self.device = torch.device(device)
        self.capacity = int(capacity)
        self.check = check
        self.n_records = -1
        self.n_jobs = -1
        self.rec = self.rect = self.depth = self.tile_start = self.sorted = self.status = self.ws = None
        self.nonfinite = None
        self.generation = 0
        self._key = None
        self._bin_fp = None  # inputs of the binning the buffers hold
        self._ckpt_generation = None  # binning whose list checkpoints the workspace holds

    # -- buffers ----------------------------------------------------------
    def _ensure(self, batch: N.ivrgs_batch):
        p = self.settings.params()
        tiles = N.ivrgs_tiles_per_job(p)
        if tiles <= 0:
            raise ValueError("invalid settings")
        dev = self.device
        R, J = int(batch.n_records), int(batch.n_jobs)
        if self.rec is None or self.rec.shape[0] < max(R, 1):
            self._bin_fp = None
            self.rec = torch.empty((max(R, 1), 16), dtype=torch.float32, device=dev)
            self.rect = torch.empty((max(R, 1), 2), dtype=torch.int32, device=dev)
            self.depth = torch.empty(max(R, 1), dtype=torch.int32, device=dev)
        n_tiles = J * tiles
        if self.tile_start is None or self.tile_start.numel() < n_tiles + 1:
            self._bin_fp = None
            self.tile_start = torch.empty(n_tiles + 1, dtype=torch.int32, device=dev)
        if self.sorted is None or self.sorted.numel() < max(self.capacity, 1):
            self._bin_fp = None
            self.sorted = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        if self.status is None:
            self.status = torch.zeros(8, dtype=torch.int64, device=dev)
            self.nonfinite = torch.zeros(1, dtype=torch.int64, device=dev)
        need = N.ivrgs_workspace_size(batch, p, self.capacity)
        if need == 0:
            raise ValueError("ivrgs_workspace_size rejected the batch")
        if self.ws is None or self.ws.numel() < need:
            self._bin_fp = None
            self._ckpt_generation = None
            self.ws = torch.empty(need, dtype=torch.uint8, device=dev)

    def grow(self, capacity: int):
        self.capacity = int(capacity)
        self.sorted = None
        self.ws = None
        self._bin_fp = None

    @staticmethod
    def _fingerprint(batch):
        """Identity of a batch's inputs: storage, in-place version, shape and
        type of every tensor it points into, and the job counts.  None for
        index-gathered jobs: the culler rewrites their index and job counts
        on the device, which no version records."""
        planes, model_id, edits_t, cams_t, jobs_dev, gauss_index = batch._keep
        if gauss_index is not None:
            return None
        ts = [planes[k] for k in PLANES] + [model_id, edits_t, cams_t, jobs_dev]
        return tuple(None if t is None else (t.data_ptr(), t._version, tuple(t.shape), t.dtype) for t in ts) + \
            (int(batch.n_jobs), int(batch.max_job_count), int(batch.n_records))

    def bins_for(self, batch):
        """The projection and bins of `batch`: those the buffers hold when the
        last binning had the same inputs, unchanged since (a render of other
        per-Gaussian outputs over the image's lists), else a new binning."""
        fp = self._fingerprint(batch)
        if fp is not None and fp == self._bin_fp:
            return self._structs(batch)
        return self.project_and_bin(batch)

    def _structs(self, batch):
        proj = N.ivrgs_projected(self.rec.data_ptr(), self.rect.data_ptr(), self.depth.data_ptr(),
                                 self.nonfinite.data_ptr())
        bins = N.ivrgs_bins(self.tile_start.data_ptr(), self.sorted.data_ptr(), self.capacity,
                            self.status.data_ptr())
        return proj, bins

    @staticmethod
    def make_batch(planes, model_id, edits_t, cams_t, jobs: Jobs, gauss_index=None):
        """Marshal the tensors into an ivrgs_batch.  The struct holds raw
        device pointers and a reference to every tensor they point into, so
        the tensors live as long as the struct."""
        g = gaussians_struct(planes, model_id)
        if edits_t is None:
            raise ValueError("an edit table (at least one row) is required")
        if edits_t.dtype != torch.float32 or edits_t.dim() != 2 or edits_t.shape[1] != 16:
            raise ValueError("edits: expected float32 [K, 16]")
        if cams_t.dtype != torch.float32 or cams_t.dim() != 2 or cams_t.shape[1] != 16:
            raise ValueError("cameras: expected float32 [V, 16]")
        if gauss_index is not None and gauss_index.dtype != torch.int32:
            raise ValueError("gauss_index: expected int32")
        if jobs.n_jobs and (jobs.host[:, 0].max() >= cams_t.shape[0] or jobs.host[:, 0].min() < 0):
            raise ValueError("job camera index out of range")
        if gauss_index is None and jobs.n_jobs and \
                (jobs.host[:, 1] + jobs.host[:, 2]).max() > g.n:
            raise ValueError("job Gaussian range out of bounds")
        if gauss_index is not None and jobs.n_jobs and \
                (jobs.host[:, 1] + jobs.host[:, 2]).max() > gauss_index.numel():
            raise ValueError("job index range out of bounds")
        b = N.ivrgs_batch()
        b.g = g
        b.gauss_index = _ptr(gauss_index)
        b.edits = edits_t.data_ptr()
        b.n_models = int(edits_t.shape[0])
        b.cameras = cams_t.data_ptr()
        b.jobs = jobs.device.data_ptr()
        b.n_jobs = jobs.n_jobs
        b.max_job_count = jobs.max_count
        b.n_records = jobs.n_records
        b._keep = (planes, model_id, edits_t, cams_t, jobs.device, gauss_index)
        return b

    # -- pipeline ---------------------------------------------------------
    def project_and_bin(self, batch):
        self._ensure(batch)
        p = self.settings.params()
        s = _stream()
        proj, bins = self._structs(batch)
        N.ivrgs_project(batch, p, proj, s)
        N.ivrgs_bin_sort(batch, p, proj, bins, self.ws.data_ptr(), self.ws.numel(), s)
        if self.check == "sync":
            # an overflow reports the capacity it needed; growing to it can
            # reveal the next requirement (pairs once the binning's block
            # entries fit), so a few rounds may be needed
            for _ in range(4):
                st = self.status[:2].cpu()
                if not int(st[1]) & N.DEV_E_CAPACITY:
                    break
                self.grow(int(int(st[0]) * 1.25) + 1024)
                self._ensure(batch)
                proj, bins = self._structs(batch)
                # the overflow is handled: drop it from the sticky words
                self.status[4:6].zero_()
                N.ivrgs_bin_sort(batch, p, proj, bins, self.ws.data_ptr(), self.ws.numel(), s)
        self.generation += 1
        self._bin_fp = self._fingerprint(batch)
        return proj, bins

    def forward(self, planes, cams_t, jobs: Jobs, model_id=None, edits_t=None, gauss_index=None,
                want_maxw: bool = False, out=None, fwd_only: bool = False):
        """Render the batch.  fwd_only=True (a render nothing will
        differentiate) stores no list checkpoints for the backward; a later
        backward() of such a render recomputes them."""
        batch = self.make_batch(planes, model_id, edits_t, cams_t, jobs, gauss_index)
        proj, bins = self.project_and_bin(batch)
        s = self.settings
        rgba = out if out is not None else torch.empty(
            (jobs.n_jobs, 4, s.height, s.width), dtype=torch.float32, device=self.device)
        maxw = torch.zeros(max(jobs.n_records, 1), dtype=torch.float32, device=self.device) \
            if want_maxw else None
        p = s.params()
        if fwd_only:
            p.flags |= N.FLAG_FWD_ONLY
        N.ivrgs_render_fwd(batch, p, proj, bins, rgba.data_ptr(), _ptr(maxw),
                           self.ws.data_ptr(), self.ws.numel(), _stream())
        self._ckpt_generation = None if fwd_only else self.generation
        self._key = (id(batch), self.generation)
        return (rgba, maxw) if want_maxw else rgba

    def forward_maps(self, planes, cams_t, jobs: Jobs, attr, n_attr: int, edits_t=None):
        """Project, bin, then the image and the auxiliary maps (depth and the
        first n_attr columns of the attribute rows attr [n, S]) in one walk
        (ivrgs_render_fwd_aux); the image is the one forward() gives, and the
        workspace holds its list checkpoints for the backward.  Returns
        (rgba [n_jobs, 4, H, W], maps [n_jobs, 1 + n_attr, H, W])."""
        batch = self.make_batch(planes, None, edits_t, cams_t, jobs)
        proj, bins = self.project_and_bin(batch)
        s = self.settings
        rgba = torch.empty((jobs.n_jobs, 4, s.height, s.width), dtype=torch.float32, device=self.device)
        maps = torch.empty((jobs.n_jobs, 1 + n_attr, s.height, s.width), dtype=torch.float32, device=self.device)
        N.ivrgs_render_fwd_aux(batch, s.params(), proj, bins, attr.data_ptr() if n_attr else None, n_attr,
                               rgba.data_ptr(), maps.data_ptr(), self.ws.data_ptr(), self.ws.numel(), _stream())
        self._ckpt_generation = self.generation
        self._key = (id(batch), self.generation)
        return rgba, maps

    def prepare_backward(self, batch, rebin: bool = False):
        """The projection and bins a backward of `batch` reads, with the
        forward's list checkpoints in the workspace: with rebin (the buffers
        were reused since the forward) the records and bins are recomputed,
        and the checkpoints are when they are not those of this binning (the
        recomputed image comes out bit-identical and is discarded)."""
        if rebin:
            proj, bins = self.project_and_bin(batch)
        else:
            self._ensure(batch)
            proj, bins = self._structs(batch)
        if rebin or self._ckpt_generation != self.generation:
            s = self.settings
            scratch = torch.empty((int(batch.n_jobs), 4, s.height, s.width), dtype=torch.float32,
                                  device=self.device)
            N.ivrgs_render_fwd(batch, s.params(), proj, bins, scratch.data_ptr(), None,
                               self.ws.data_ptr(), self.ws.numel(), _stream())
            self._ckpt_generation = self.generation
        return proj, bins

    def backward(self, planes, cams_t, jobs: Jobs, rgba, dl, model_id=None, edits_t=None,
                 gauss_index=None, rebin: bool = False, grads=None):
        batch = self.make_batch(planes, model_id, edits_t, cams_t, jobs, gauss_index)
        proj, bins = self.prepare_backward(batch, rebin)
        n = batch.g.n
        if grads is None:
            grads = {k: torch.empty((d, n), dtype=torch.float32, device=self.device)
                     for k, d in PLANE_DIMS.items()}
        gs = N.ivrgs_gaussians(n, *[grads[k].data_ptr() for k in PLANES], None)
        if not (rgba.is_contiguous() and dl.is_contiguous()):
            raise ValueError("rgba and dl must be contiguous")
        N.ivrgs_render_bwd(batch, self.settings.params(), proj, bins, rgba.data_ptr(), dl.data_ptr(),
                           gs, self.ws.data_ptr(), self.ws.numel(), _stream())
        return grads

    def light_grad(self, planes, cams_t, jobs: Jobs, model_id=None, edits_t=None, gauss_index=None, out=None):
        """dL/d(orbital light direction) per model [n_models, 3] for the
        gradient of the last backward() on the same inputs (reads the record
        gradients it left in the workspace)."""
        batch = self.make_batch(planes, model_id, edits_t, cams_t, jobs, gauss_index)
        self._ensure(batch)
        proj, _ = self._structs(batch)
        if out is None:
            out = torch.empty((batch.n_models, 3), dtype=torch.float32, device=self.device)
        N.ivrgs_light_bwd(batch, self.settings.params(), proj, out.data_ptr(), self.ws.data_ptr(),
                          self.ws.numel(), _stream())
        return out

    def verify(self):
        """Raise if a binning since the last check overflowed the pair
        capacity (waits for the stream); else return the largest pair count
        they required."""
        bins = N.ivrgs_bins(self.tile_start.data_ptr(), _ptr(self.sorted), self.capacity, self.status.data_ptr())
        err, need = N.ivrgs_get_error(bins, _stream())
        if err & N.DEV_E_CAPACITY:
            raise N.IvrgsError(f"pair capacity {self.capacity} exceeded: {need} pairs needed")
        if err:
            raise N.IvrgsError(f"device error bits {err:#x}")
        return need

    def pairs(self) -> int:
        return int(self.status[0].item())

    def nonfinite_count(self) -> int:
        """Gaussian-views culled for a NaN or infinite value since the
        renderer was created (or since `clear_nonfinite`).  Waits."""
        return 0 if self.nonfinite is None else int(self.nonfinite.item())

    def clear_nonfinite(self):
        if self.nonfinite is not None:
            self.nonfinite.zero_()


class _RasterFn(torch.autograd.Function):
    """Forward: project, bin, composite.  Backward: recompute the per-pixel
    compositing from the saved output image (no per-pixel state is saved);
    if the renderer's buffers were reused meanwhile, the projection and the
    bins are recomputed too."""

    @staticmethod
    def forward(ctx, renderer, cams_t, jobs, model_id, edits_t, gauss_index, *planes):
        pl = dict(zip(PLANES, planes))
        rgba = renderer.forward(pl, cams_t, jobs, model_id, edits_t, gauss_index)
        ctx.renderer, ctx.jobs = renderer, jobs
        ctx.generation = renderer.generation
        ctx.save_for_backward(cams_t, model_id if model_id is not None else torch.empty(0),
                              edits_t, gauss_index if gauss_index is not None else torch.empty(0),
                              rgba, *planes)
        ctx.has_mid = model_id is not None
        ctx.has_idx = gauss_index is not None
        return rgba

    @staticmethod
    def backward(ctx, grad_rgba):
        saved = ctx.saved_tensors
        cams_t, mid, edits_t, idx, rgba = saved[:5]
        planes = dict(zip(PLANES, saved[5:]))
        r = ctx.renderer
        rebin = r.generation != ctx.generation
        grads = r.backward(planes, cams_t, ctx.jobs, rgba, grad_rgba.contiguous(),
                           mid if ctx.has_mid else None, edits_t, idx if ctx.has_idx else None,
                           rebin=rebin)
        return (None, None, None, None, None, None, *[grads[k] for k in PLANES])


def rasterize(planes: dict, cams_t, jobs: Jobs, renderer: Renderer, model_id=None,
              edits_t=None, gauss_index=None) -> torch.Tensor:
    """Differentiable render of the job batch -> RGBA [n_jobs, 4, H, W]."""
    if edits_t is None:
        edits_t = default_edits(renderer.device)
    return _RasterFn.apply(renderer, cams_t, jobs, model_id, edits_t, gauss_index,
                           *[planes[k] for k in PLANES])


_DEFAULT_EDITS = {}


def default_edits(device) -> torch.Tensor:
    """One identity row with the headlight on."""
    key = str(device)
    if key not in _DEFAULT_EDITS:
        r = np.zeros(16, np.float32)
        r[3] = 1.0
        r[4:8] = 1.0
        r.view(np.int32)[15] = 1
        _DEFAULT_EDITS[key] = torch.from_numpy(r[None].copy()).to(device)
    return _DEFAULT_EDITS[key]


def compose(models: list, edits, device="cuda"):
    """Composition and editing of basic models (Sec. 4.5) on the device.
    models: list of plane dicts (color plane = delta-c); edits: list of edit
    rows (objects with .row() or 16-float arrays).  Returns (planes, model_id)."""
    ns = [int(m["mean"].shape[1]) for m in models]
    total = sum(ns)
    out = {k: torch.empty((d, total), dtype=torch.float32, device=device) for k, d in PLANE_DIMS.items()}
    mid = torch.empty(total, dtype=torch.int32, device=device)
    compose_into(models, edits, out, mid)
    return out, mid


def compose_bwd(models: list, grads: dict, out=None):
    """Gradients of each model's edit parameters [n_models, 12] (palette 3,
    opacity scale, shade scale 4, shade bias 4; Sec. 4.6) from the gradients
    of the composed set (composition order)."""
    structs = [gaussians_struct(m) for m in models]
    total = sum(s.n for s in structs)
    for k in PLANES:
        _check_plane(k, grads[k], total)
    g = N.ivrgs_gaussians(total, *[grads[k].data_ptr() for k in PLANES], None)
    if out is None:
        out = torch.empty((len(models), 12), dtype=torch.float32, device=grads["color"].device)
    N.ivrgs_compose_bwd(structs, len(structs), g, out.data_ptr(), _stream())
    return out


def compose_into(models: list, edits, out: dict, mid: torch.Tensor):
    structs = [gaussians_struct(m) for m in models]
    rows = [r.row() if hasattr(r, "row") else np.asarray(r, np.float32) for r in edits]
    es = [N.ivrgs_model_edit.from_buffer_copy(np.ascontiguousarray(r, np.float32).tobytes())
          for r in rows]
    total = sum(s.n for s in structs)
    o = N.ivrgs_gaussians(total, *[out[k].data_ptr() for k in PLANES], mid.data_ptr())
    N.ivrgs_compose(structs, len(structs), es, o, _stream())
