"""Dense FP64 second opinion of the rasterizer, in plain PyTorch CPU ops.

TEST INFRASTRUCTURE ONLY.  Written separately from `ivrgs_oracle.c`, with
different formulations where the definition allows:
  - rotation from the Hamilton product q e_j q^* applied to the basis vectors
    (not the closed-form matrix);
  - the 2x2 conic by torch.linalg.inv;
  - compositing with the Gaussian loop outside and all pixels updated at once
    (Eq. 2), no pixel box: every kept Gaussian is evaluated at every pixel;
  - gradients by torch autograd instead of the hand-derived backward.
Only for tiny scenes (N <= a few hundred, images <= 64x64).
"""
from __future__ import annotations

import numpy as np
import torch

from . import PLANES, Params


def _qmul(a, b):
    aw, av = a[..., :1], a[..., 1:]
    bw, bv = b[..., :1], b[..., 1:]
    w = aw * bw - (av * bv).sum(-1, keepdim=True)
    v = aw * bv + bw * av + torch.cross(av, bv, dim=-1)
    return torch.cat([w, v], -1)


def rotation(q):
    """[n,4] (w,x,y,z) -> [n,3,3], column j = q e_j q^* for the unit q."""
    q = q / q.norm(dim=-1, keepdim=True)
    conj = q * torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=q.dtype)
    cols = []
    for j in range(3):
        e = torch.zeros_like(q)
        e[:, 1 + j] = 1.0
        cols.append(_qmul(_qmul(q, e), conj)[:, 1:])
    return torch.stack(cols, dim=-1)


def depth_keys(mean32: np.ndarray, cam_row: np.ndarray) -> np.ndarray:
    """FP32 depth key ((R20 x + R21 y) + R22 z) + t2, rounded per operation."""
    R = cam_row[:9].astype(np.float32).reshape(3, 3)
    t2 = np.float32(cam_row[11])
    x, y, z = (mean32[i].astype(np.float32) for i in range(3))
    return ((R[2, 0] * x + R[2, 1] * y) + R[2, 2] * z) + t2


def render(planes_t: dict, cam_row, params: Params, model_id=None, edit_rows=None,
           planes_np: dict | None = None, attr_t=None):
    """planes_t: dict of float64 tensors [d, n] (may require grad).
    Returns rgba [4, H, W] (float64 tensor), the kept-Gaussian order and a
    decision signature (changes iff the set of composited pairs changes).
    With attr_t (float64 [A, n]): also the auxiliary maps [1 + A, H, W]
    composited with the same weights T_i alpha_i (Eq. 5 for depth and normal,
    and the offset-colour and shading maps of Sec. 4.3): channel 0 the
    camera-space depth of each Gaussian, then the A attributes; no
    background term."""
    cam_row = np.asarray(cam_row, np.float32)
    n = planes_t["mean"].shape[1]
    mean = planes_t["mean"].T
    s = torch.exp(planes_t["log_scale"].T)
    Rq = rotation(planes_t["quat"].T)
    Sig = Rq @ torch.diag_embed(s * s) @ Rq.transpose(1, 2)
    W = torch.tensor(cam_row[:9].reshape(3, 3), dtype=torch.float64)
    tw = torch.tensor(cam_row[9:12], dtype=torch.float64)
    fx, fy, cx, cy = (float(v) for v in cam_row[12:16])
    t = mean @ W.T + tw
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * tx / tz ** 2], -1),
                     torch.stack([zero, fy / tz, -fy * ty / tz ** 2], -1)], 1)
    M = J @ W
    S2 = M @ Sig @ M.transpose(1, 2) + params.lowpass * torch.eye(2, dtype=torch.float64)
    Q = torch.linalg.inv(S2)
    mx = fx * tx / tz + cx
    my = fy * ty / tz + cy

    # Blinn-Phong (Eq. 3) per Gaussian
    cam_c = -(W.T @ tw)
    v = cam_c[None, :] - mean
    v = v / v.norm(dim=-1, keepdim=True)
    if edit_rows is None:
        edit_rows = np.zeros((1, 16), np.float32)
        edit_rows[0].view(np.int32)[15] = 1
    edit_rows = np.asarray(edit_rows, np.float32).reshape(-1, 16)
    mid = np.zeros(n, np.int64) if model_id is None else np.asarray(model_id, np.int64)
    head = edit_rows[:, 15].view(np.int32)[mid] != 0
    ld = edit_rows[mid, 12:15].astype(np.float64)
    lnorm = np.linalg.norm(ld, axis=1, keepdims=True)
    ld = ld / np.where(lnorm > 0, lnorm, 1.0)
    l = torch.where(torch.tensor(head)[:, None], v, torch.tensor(ld))
    nrm = planes_t["normal"].T
    nrm = nrm / nrm.norm(dim=-1, keepdim=True)
    nl = (nrm * l).sum(-1)
    hsum = v + l
    hlen = hsum.norm(dim=-1, keepdim=True)
    hdir = hsum / torch.where(hlen > 0, hlen, torch.ones_like(hlen))
    nh = (nrm * hdir).sum(-1).abs()
    ka, kd, ks, beta = planes_t["shade"]
    gate = (nl.abs() > 0) & (hlen[:, 0] > 0) & (nh > 0)
    spec = torch.where(gate, ks * torch.where(gate, nh, torch.ones_like(nh)) ** beta,
                       torch.zeros_like(nh))
    cv = planes_t["color"]
    rgb = ka[None] * cv + kd[None] * cv * nl.abs()[None] + spec[None]
    o = planes_t["opacity"][0]

    src = planes_np if planes_np is not None else {k: planes_t[k].detach().numpy().astype(np.float32)
                                                  for k in PLANES}
    z32 = depth_keys(src["mean"], cam_row)
    det = (S2[:, 0, 0] * S2[:, 1, 1] - S2[:, 0, 1] * S2[:, 1, 0]).detach().numpy()
    keep = (z32.astype(np.float64) > params.z_near) & (det > 0)
    idx = np.arange(n)[keep]
    order = idx[np.lexsort((idx, z32[keep]))]

    H, Wd = params.height, params.width
    ys, xs = np.meshgrid(np.arange(H) + 0.5, np.arange(Wd) + 0.5, indexing="ij")
    px = torch.tensor(xs.reshape(-1))
    py = torch.tensor(ys.reshape(-1))
    P = px.shape[0]
    T = torch.ones(P, dtype=torch.float64)
    Cc = torch.zeros(3, P, dtype=torch.float64)
    A = torch.zeros(P, dtype=torch.float64)
    aux = None if attr_t is None else torch.zeros(1 + attr_t.shape[0], P, dtype=torch.float64)
    alive = torch.ones(P, dtype=torch.bool)
    sig = 0
    pix_id = torch.arange(1, P + 1, dtype=torch.int64)
    for i in order.tolist():
        dx = px - mx[i]
        dy = py - my[i]
        power = -0.5 * (Q[i, 0, 0] * dx * dx + (Q[i, 0, 1] + Q[i, 1, 0]) * dx * dy
                        + Q[i, 1, 1] * dy * dy)
        raw = o[i] * torch.exp(power)
        alpha = torch.minimum(raw, torch.full_like(raw, params.alpha_max))
        use = alive & (alpha >= params.alpha_min)
        Tn = T * (1.0 - alpha)
        stop = use & (Tn < params.T_min)
        alive = alive & ~stop
        comp = use & ~stop
        sig += int(((i + 1) * 1000003 + pix_id)[comp].sum()) + 7 * int(comp.sum())
        w = torch.where(comp, T * alpha, torch.zeros_like(T))
        Cc = Cc + w[None] * rgb[:, i:i + 1]
        A = A + w
        if aux is not None:
            vals = torch.cat([tz[i:i + 1], attr_t[:, i]])
            aux = aux + w[None] * vals[:, None]
        T = torch.where(comp, Tn, T)
    bg = torch.tensor(params.bg, dtype=torch.float64)[:, None]
    out = torch.cat([Cc + T[None] * bg, A[None]], 0).reshape(4, H, Wd)
    if aux is not None:
        return out, order, sig, aux.reshape(-1, H, Wd)
    return out, order, sig


NORMAL_FLOOR = 1e-12  # lower clamp of a normal's length before it is divided out


def editable_attributes(normal, color, shade):
    """Attribute planes [10, n] that the editable-stage maps composite
    (Sec. 4.3; the normal map of Eq. 5): the unit normal (the normal plane
    over its Euclidean length, clamped below at NORMAL_FLOOR), delta-c (the
    colour plane of a basic model) and k_a, k_d, k_s, beta (the shade
    plane).  float64 tensors [k, n]; differentiable by autograd."""
    length = normal.norm(dim=0, keepdim=True).clamp_min(NORMAL_FLOOR)
    return torch.cat([normal / length, color, shade])


def to_tensors(planes: dict, requires_grad: bool = False) -> dict:
    return {k: torch.tensor(np.asarray(planes[k], np.float64), requires_grad=requires_grad)
            for k in PLANES}
