"""Inverse volume exploration (Sec. 4.6) in FP64, for the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With every Gaussian attribute frozen, the composed model is fitted to one
reference image by learning a small set of transformation parameters:
  - per basic model m: the palette colour c_p[m] (3) and an opacity scale
    s_o[m] (colour and opacity edits of Sec. 4.5);
  - for the whole composed model: one light-magnitude transform
    lambda (4), b (4) applied as lambda * (k_a, k_d, k_s, beta) + b to every
    model, and one orbital light direction given by a polar angle t and an
    azimuth p, d = (sin t cos p, sin t sin p, cos t) in world space.
The optimiser is Adam (Kingma and Ba, 2015, Algorithm 1).  The objective is
the paper's combination of L1 and SSIM (Sec. 4.6), with the weights the
appendix gives the photometric loss: (1 - lam) mean |RGBA - target| +
lam (1 - SSIM(RGBA, target)), lam = 0.2, over the colour and alpha channels
(SSIM from `oracle.ssim`, the target held fixed).

Parameter vector layout (K models, n = 4K + 10):
  [palette K*3 | s_o K | lambda 4 | b 4 | t | p]
"""
from __future__ import annotations

import numpy as np

from . import backward, compose, compose_bwd, light_grad, render
from . import ssim as S

SSIM_WEIGHT = 0.2  # lam: the appendix weights L1 and SSIM 0.8 and 0.2
LEARN_PALETTE, LEARN_OPACITY, LEARN_MAGNITUDE, LEARN_LIGHT = 1, 2, 4, 8
LEARN_ALL = 15


def n_params(K: int) -> int:
    return 4 * K + 10


def light_direction(t: float, p: float) -> np.ndarray:
    """Unit vector of polar angle t (from +z) and azimuth p (from +x toward +y)."""
    return np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])


def rows_from_params(theta, base_rows):
    """Edit rows (float32 [K, 16]) for parameter vector theta.  base_rows
    supplies each model's headlight word and, for headlight models, the light
    direction it keeps; orbital models take d(t, p)."""
    base = np.asarray(base_rows, np.float32).reshape(-1, 16)
    K = base.shape[0]
    th = np.asarray(theta, np.float64)
    rows = base.copy()
    rows[:, 0:3] = th[0:3 * K].reshape(K, 3)
    rows[:, 3] = th[3 * K:4 * K]
    rows[:, 4:8] = th[4 * K:4 * K + 4]
    rows[:, 8:12] = th[4 * K + 4:4 * K + 8]
    orbital = base[:, 15].view(np.int32) == 0
    rows[orbital, 12:15] = light_direction(th[4 * K + 8], th[4 * K + 9])
    return rows


def render_params(models_planes, base_rows, theta, cam, prm):
    """Render of the composed model under parameters theta (oracle dict)."""
    rows = rows_from_params(theta, base_rows)
    comp, mid = compose(models_planes, rows)
    return render(comp, cam, prm, model_id=mid, edits=rows)


def param_grad(models_planes, base_rows, theta, cam, prm, dl):
    """Gradient of L = sum(dl * RGBA) with respect to theta (FP64 [4K + 10]):
    the per-model sums of the composed set's gradients, summed again over the
    models for the shared lambda, b and light, then chained through d(t, p)."""
    K = len(models_planes)
    th = np.asarray(theta, np.float64)
    rows = rows_from_params(th, base_rows)
    comp, mid = compose(models_planes, rows)
    grads, grad_rec = backward(comp, cam, prm, dl, model_id=mid, edits=rows)
    eg = compose_bwd(models_planes, rows, grads)  # [K, 12]
    lg = light_grad(comp, cam, prm, grad_rec, model_id=mid, edits=rows)  # [K, 3]
    return assemble(eg, lg, th)


def assemble(eg, lg, theta):
    """Parameter-vector gradient from the per-model edit-row gradients eg
    [K, 12] (palette 3, opacity scale, shade scale 4, shade bias 4) and the
    per-model light-direction gradients lg [K, 3]."""
    eg = np.asarray(eg, np.float64)
    lg = np.asarray(lg, np.float64)
    th = np.asarray(theta, np.float64)
    K = eg.shape[0]
    g = np.zeros(n_params(K))
    g[0:3 * K] = eg[:, 0:3].reshape(-1)
    g[3 * K:4 * K] = eg[:, 3]
    g[4 * K:4 * K + 4] = eg[:, 4:8].sum(0)
    g[4 * K + 4:4 * K + 8] = eg[:, 8:12].sum(0)
    gd = lg.sum(0)
    t, p = th[4 * K + 8], th[4 * K + 9]
    g[4 * K + 8] = gd @ np.array([np.cos(t) * np.cos(p), np.cos(t) * np.sin(p), -np.sin(t)])
    g[4 * K + 9] = gd @ np.array([-np.sin(t) * np.sin(p), np.sin(t) * np.cos(p), 0.0])
    return g


def photometric(rgba, target, lam=SSIM_WEIGHT):
    """(1 - lam) mean |rgba - target| + lam (1 - SSIM(rgba, target)) and its
    gradient with respect to rgba (sign(0) = 0; the target gets none)."""
    rgba = np.asarray(rgba, np.float64)
    target = np.asarray(target, np.float64)
    l1 = float(np.abs(rgba - target).mean())
    dl = (1.0 - lam) * np.sign(rgba - target) / rgba.size
    loss = (1.0 - lam) * l1
    if lam != 0.0:
        s, ds = S.ssim_and_grad(rgba, target)
        loss += lam * (1.0 - s)
        dl = dl - lam * ds
    return loss, dl


def loss_and_grad(models_planes, base_rows, theta, cam, prm, target, lam=SSIM_WEIGHT):
    """Photometric loss (L1 + SSIM, `photometric`) under theta, its gradient
    with respect to theta, and the render."""
    out = render_params(models_planes, base_rows, theta, cam, prm)
    loss, dl = photometric(out["rgba"], target, lam)
    return loss, param_grad(models_planes, base_rows, theta, cam, prm, dl), out


def learn_mask(K: int, learn: int) -> np.ndarray:
    mask = np.zeros(n_params(K), bool)
    if learn & LEARN_PALETTE:
        mask[0:3 * K] = True
    if learn & LEARN_OPACITY:
        mask[3 * K:4 * K] = True
    if learn & LEARN_MAGNITUDE:
        mask[4 * K:4 * K + 8] = True
    if learn & LEARN_LIGHT:
        mask[4 * K + 8:] = True
    return mask


def adam_update(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, mask=None):
    """Adam step number t (1-based): biased moment estimates, their bias
    corrections, then theta - lr * m_hat / (sqrt(v_hat) + eps).  Entries with
    mask False are left untouched (moments included).  Returns new copies."""
    theta, m, v = (np.array(a, np.float64) for a in (theta, m, v))
    g = np.asarray(g, np.float64)
    sel = np.ones(theta.shape, bool) if mask is None else np.asarray(mask, bool)
    m[sel] = beta1 * m[sel] + (1.0 - beta1) * g[sel]
    v[sel] = beta2 * v[sel] + (1.0 - beta2) * g[sel] ** 2
    m_hat = m[sel] / (1.0 - beta1 ** t)
    v_hat = v[sel] / (1.0 - beta2 ** t)
    theta[sel] = theta[sel] - lr * m_hat / (np.sqrt(v_hat) + eps)
    return theta, m, v


def explore(models_planes, base_rows, theta0, cam, prm, target, iters, lr=0.01, beta1=0.9,
            beta2=0.999, eps=1e-8, learn=LEARN_ALL, lam=SSIM_WEIGHT):
    """Run `iters` Adam steps from theta0.  Returns (thetas [iters + 1, n],
    losses [iters]) where losses[i] is the loss at thetas[i]."""
    K = len(models_planes)
    mask = learn_mask(K, learn)
    theta = np.asarray(theta0, np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    thetas, losses = [theta.copy()], []
    for it in range(1, iters + 1):
        loss, g, _ = loss_and_grad(models_planes, base_rows, theta, cam, prm, target, lam)
        losses.append(loss)
        theta, m, v = adam_update(theta, g, m, v, it, lr, beta1, beta2, eps, mask)
        thetas.append(theta.copy())
    return np.stack(thetas), np.array(losses)
