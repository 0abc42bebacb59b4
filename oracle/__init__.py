"""CPU FP64 oracle of the editable-Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library; the two only consume the same seeded inputs.

`ivrgs_oracle.c` holds the definition (projection Sec. 3 / Eq. 1, Blinn-Phong
Eq. 3, compositing Eq. 2, composition and edits Sec. 4.5); this module loads
it with ctypes and adds the composition step (Sec. 4.5) and the gradients of
the edit parameters that inverse volume exploration learns (Sec. 4.6) in
numpy FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ivrgs_oracle.c")
_LIB = os.path.join(_HERE, "libivrgs_oracle.so")

PLANES = ("mean", "log_scale", "quat", "opacity", "normal", "color", "shade")
DIMS = (3, 3, 4, 1, 3, 3, 4)
P_FIELDS = ("valid", "z32", "mx", "my", "cov00", "cov01", "cov11", "q00", "q01", "q11",
            "o", "r", "g", "b", "extx", "exty", "tx", "ty", "tz", "nl", "nh", "dm", "kappa", "ergb")
P_WIDTH = len(P_FIELDS)
REC_FIELDS = ("mx", "my", "q00", "q01", "q11", "o", "r", "g", "b")
AMB_ALPHA_MIN, AMB_T_MIN, AMB_ALPHA_MAX, AMB_SHADE, AMB_MANY = 1, 2, 4, 8, 16


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Gauss(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_void_p) for k in PLANES] + [("model_id", C.c_void_p)]


class _Cam(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float)]


class _Params(C.Structure):
    _fields_ = [("alpha_min", C.c_double), ("alpha_max", C.c_double), ("T_min", C.c_double),
                ("lowpass", C.c_double), ("z_near", C.c_double), ("bg", C.c_double * 3),
                ("width", C.c_int32), ("height", C.c_int32)]


@dataclass
class Params:
    """Compositing constants (readings of the paper, which is silent on
    them): alpha cap 0.99, skip below 1/255, stop before T < 1e-4, EWA
    low-pass 0.3 px^2 on the diagonal, near plane 0.2, black background."""
    width: int
    height: int
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    lowpass: float = 0.3
    z_near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def c(self) -> _Params:
        p = _Params()
        p.alpha_min, p.alpha_max, p.T_min = self.alpha_min, self.alpha_max, self.T_min
        p.lowpass, p.z_near = self.lowpass, self.z_near
        p.bg = (C.c_double * 3)(*self.bg)
        p.width, p.height = self.width, self.height
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        for name in ("og_project", "og_jacobian", "og_render", "og_backward", "og_light_grad"):
            getattr(_lib, name).restype = C.c_int
        _lib.og_num_threads.restype = C.c_int
    return _lib


def num_threads() -> int:
    return int(lib().og_num_threads())


class _Inputs:
    """Keeps contiguous float32 copies alive for the duration of a call."""

    def __init__(self, planes: dict, model_id, edits, cam):
        self.planes = {k: np.ascontiguousarray(planes[k], np.float32) for k in PLANES}
        n = self.planes["mean"].shape[1]
        for k, d in zip(PLANES, DIMS):
            if self.planes[k].shape != (d, n):
                raise ValueError(f"plane {k} has shape {self.planes[k].shape}, want {(d, n)}")
        self.mid = None if model_id is None else np.ascontiguousarray(model_id, np.int32)
        self.g = _Gauss(n, *[self.planes[k].ctypes.data for k in PLANES],
                        None if self.mid is None else self.mid.ctypes.data)
        if edits is None:
            e = np.zeros((1, 16), np.float32)
            e[0].view(np.int32)[15] = 1
            edits = e
        self.edits = np.ascontiguousarray(np.atleast_2d(edits), np.float32)
        row = cam.row() if hasattr(cam, "row") else np.asarray(cam, np.float32)
        self.cam = _Cam.from_buffer_copy(np.ascontiguousarray(row, np.float32).tobytes())
        self.n = n

    def args(self):
        return (C.byref(self.g), self.edits.ctypes.data_as(C.c_void_p),
                C.c_int(self.edits.shape[0]), C.byref(self.cam))


def project(planes, cam, params: Params, model_id=None, edits=None) -> np.ndarray:
    """Per-Gaussian projection diagnostics [n, P_WIDTH] (fields P_FIELDS)."""
    inp = _Inputs(planes, model_id, edits, cam)
    out = np.zeros((inp.n, P_WIDTH), np.float64)
    prm = params.c()
    lib().og_project(*inp.args(), C.byref(prm), out.ctypes.data_as(C.c_void_p))
    return out


def jacobian(planes, cam, params: Params, i: int, model_id=None, edits=None):
    """9x21 Jacobian of (mx, my, q00, q01, q11, o, r, g, b) w.r.t. the 21
    parameters of Gaussian i (complex step)."""
    inp = _Inputs(planes, model_id, edits, cam)
    jac = np.zeros((9, 21), np.float64)
    prm = params.c()
    valid = lib().og_jacobian(*inp.args(), C.byref(prm), C.c_int64(i),
                              jac.ctypes.data_as(C.c_void_p))
    return jac, bool(valid)


def _pix(pix):
    if pix is None:
        return None
    return np.ascontiguousarray(np.asarray(pix, np.int32).reshape(-1, 2))


def render(planes, cam, params: Params, model_id=None, edits=None, pix=None,
           use_box: bool = True, want_maxw: bool = False, want_proj: bool = False):
    """Render the whole image (pix None -> rgba [4, H, W]) or the listed
    pixels (pix [m, 2] of (x, y) -> rgba [m, 4]).  Returns a dict with
    rgba, flags (ambiguity bits per pixel), alt / n_alt (the images of the
    other branches of up to two ambiguous decisions per pixel, [.., 3, 4]),
    maxw (per Gaussian, optional), stats (composited pairs, kept Gaussians,
    evaluated pairs)."""
    inp = _Inputs(planes, model_id, edits, cam)
    p = _pix(pix)
    npix = params.width * params.height if p is None else p.shape[0]
    rgba = np.zeros((npix, 4), np.float64)
    flags = np.zeros(npix, np.int32)
    alt = np.zeros((npix, 3, 4), np.float64)
    n_alt = np.zeros(npix, np.int32)
    maxw = np.zeros(inp.n, np.float64) if want_maxw else None
    stats = np.zeros(3, np.int64)
    proj = np.zeros((inp.n, P_WIDTH), np.float64) if want_proj else None
    prm = params.c()
    vp = C.c_void_p
    lib().og_render(*inp.args(), C.byref(prm), C.c_int64(npix),
                    None if p is None else p.ctypes.data_as(vp), C.c_int(int(use_box)),
                    rgba.ctypes.data_as(vp), flags.ctypes.data_as(vp), alt.ctypes.data_as(vp),
                    n_alt.ctypes.data_as(vp), None if maxw is None else maxw.ctypes.data_as(vp),
                    stats.ctypes.data_as(vp), None if proj is None else proj.ctypes.data_as(vp))
    if p is None:
        H, W = params.height, params.width
        rgba = rgba.reshape(H, W, 4).transpose(2, 0, 1).copy()
        flags = flags.reshape(H, W)
        alt = alt.reshape(H, W, 3, 4)
        n_alt = n_alt.reshape(H, W)
    return {"rgba": rgba, "flags": flags, "alt": alt, "n_alt": n_alt, "maxw": maxw,
            "stats": stats, "proj": proj}


def image_error(gpu, ref):
    """Max-abs error of a GPU image against the oracle, accepting for each
    pixel the primary result or any of its ambiguous-branch alternatives.
    Pixels the oracle cannot resolve (more than two ambiguous decisions, or
    ill-conditioned shading) are excluded.  gpu: [4, H, W] or [m, 4] like
    ref["rgba"].  Returns (max error, excluded pixel count, pixels that
    matched an alternative)."""
    g = np.asarray(gpu, np.float64)
    r = ref["rgba"]
    if r.ndim == 3:
        g = g.transpose(1, 2, 0).reshape(-1, 4)
        r = r.transpose(1, 2, 0).reshape(-1, 4)
    flags = ref["flags"].reshape(-1)
    alt = ref["alt"].reshape(-1, 3, 4)
    n_alt = ref["n_alt"].reshape(-1)
    excl = (flags & (AMB_MANY | AMB_SHADE)) != 0
    err = np.abs(g - r).max(1)
    used = 0
    for k in range(3):
        has = n_alt > k
        e = np.abs(g - alt[:, k]).max(1)
        better = has & (e < err)
        used += int(better.sum())
        err = np.where(better, e, err)
    keep = ~excl
    return (float(err[keep].max()) if keep.any() else 0.0), int(excl.sum()), used


def grad_mask(ref):
    """Pixels whose upstream gradient may be used for a gradient comparison:
    no ambiguous decision, no active-cap ambiguity, no ill-conditioned shading."""
    return ref["flags"] == 0


def backward(planes, cam, params: Params, dl, model_id=None, edits=None, pix=None):
    """Gradient of L = sum(dl * RGBA).  dl: [4, H, W] for the whole image or
    [m, 4] matching pix.  Returns (grads: dict plane -> [d, n] float64,
    grad_rec: [n, 9] w.r.t. REC_FIELDS)."""
    inp = _Inputs(planes, model_id, edits, cam)
    p = _pix(pix)
    if p is None:
        d = np.ascontiguousarray(np.asarray(dl, np.float64).transpose(1, 2, 0).reshape(-1, 4))
    else:
        d = np.ascontiguousarray(np.asarray(dl, np.float64).reshape(-1, 4))
    npix = d.shape[0]
    grad = np.zeros((21, inp.n), np.float64)
    grad_rec = np.zeros((inp.n, 9), np.float64)
    prm = params.c()
    lib().og_backward(*inp.args(), C.byref(prm), C.c_int64(npix),
                      None if p is None else p.ctypes.data_as(C.c_void_p),
                      d.ctypes.data_as(C.c_void_p), grad_rec.ctypes.data_as(C.c_void_p),
                      grad.ctypes.data_as(C.c_void_p))
    out, k = {}, 0
    for name, dim in zip(PLANES, DIMS):
        out[name] = grad[k:k + dim]
        k += dim
    return out, grad_rec


def compose(models_planes, edit_rows):
    """Composition and editing (Sec. 4.5), FP64 then rounded to FP32:
    concatenate the basic models in order; per model m,
      c_v = c_p[m] + delta-c,  o' = s_o[m] * o,
      (k_a, k_d, k_s, beta)' = lambda[m] * (k_a, k_d, k_s, beta) + b[m]
    (the inverse-exploration form of the light-magnitude edit, Sec. 4.6).
    Returns (planes float32, model_id int32)."""
    edit_rows = np.asarray(edit_rows, np.float32).reshape(-1, 16)
    out = {k: [] for k in PLANES}
    mids = []
    for m, pl in enumerate(models_planes):
        e = edit_rows[m].astype(np.float64)
        n = pl["mean"].shape[1]
        for k in ("mean", "log_scale", "quat", "normal"):
            out[k].append(np.asarray(pl[k], np.float32))
        out["color"].append((e[0:3, None] + pl["color"].astype(np.float64)).astype(np.float32))
        out["opacity"].append((e[3] * pl["opacity"].astype(np.float64)).astype(np.float32))
        out["shade"].append((e[4:8, None] * pl["shade"].astype(np.float64)
                             + e[8:12, None]).astype(np.float32))
        mids.append(np.full(n, m, np.int32))
    planes = {k: np.ascontiguousarray(np.concatenate(v, axis=1)) for k, v in out.items()}
    return planes, np.concatenate(mids)


def light_grad(planes, cam, params: Params, grad_rec, model_id=None, edits=None):
    """dL/d(orbital light direction) of each model, [n_models, 3] FP64, with
    respect to the unnormalised direction stored in the edit row (Sec. 4.6
    learns the light direction), from the record gradients of backward()."""
    inp = _Inputs(planes, model_id, edits, cam)
    gr = np.ascontiguousarray(grad_rec, np.float64).reshape(inp.n, 9)
    out = np.zeros((inp.edits.shape[0], 3), np.float64)
    prm = params.c()
    lib().og_light_grad(*inp.args(), C.byref(prm), gr.ctypes.data_as(C.c_void_p),
                        out.ctypes.data_as(C.c_void_p))
    return out


def compose_bwd(models_planes, edit_rows, grads):
    """Gradients of the edit parameters of each model (Sec. 4.5 edits, learned
    by inverse exploration, Sec. 4.6) from the gradients of the composed set
    (grads: dict plane -> [d, N] in composition order), FP64:
      dL/dc_p[m]     = sum_{i in m} dL/dc_v[i]
      dL/ds_o[m]     = sum_{i in m} dL/do'[i] * o[i]
      dL/dlambda[m]  = sum_{i in m} dL/dk'[i] * k[i]   (per component)
      dL/db[m]       = sum_{i in m} dL/dk'[i]
    Returns [n_models, 12]: palette (3), opacity scale, shade scale (4),
    shade bias (4), the order of the edit row."""
    out = np.zeros((len(models_planes), 12), np.float64)
    off = 0
    for m, pl in enumerate(models_planes):
        n = pl["mean"].shape[1]
        sl = slice(off, off + n)
        gc = np.asarray(grads["color"], np.float64)[:, sl]
        go = np.asarray(grads["opacity"], np.float64)[:, sl]
        gk = np.asarray(grads["shade"], np.float64)[:, sl]
        out[m, 0:3] = gc.sum(1)
        out[m, 3] = (go[0] * np.asarray(pl["opacity"], np.float64)[0]).sum()
        out[m, 4:8] = (gk * np.asarray(pl["shade"], np.float64)).sum(1)
        out[m, 8:12] = gk.sum(1)
        off += n
    return out


def l1_loss(x, y):
    """The L1 term of the photometric loss (Sec. 4.2): mean |x - y| over all
    entries, in FP64."""
    d = np.asarray(x, np.float64) - np.asarray(y, np.float64)
    return float(np.abs(d).sum() / d.size)


def l1_loss_grad(rgba, target):
    """Gradient of mean |RGBA - target| over 4HW entries (sign(0) = 0)."""
    return np.sign(rgba - target) / rgba.size
