"""View-dependent colour from spherical-harmonic (SH) coefficients: the colour
model of base 3DGS (Sec. 3; Sec. 4.2 keeps it for the base model), plain FP64
torch on the CPU, gradients by autograd.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the product
path; it shares no code with the HIP library.

The paper says only that the view-dependent colour is parameterised by SH
coefficients as in the original 3DGS.  Readings (the same on the GPU side):
  - degree L in 0..3, K = (L + 1)^2 coefficients per colour channel, stored
    as planes [K][3][n] (coefficient, channel, Gaussian);
  - the real basis built from the complex harmonics with the Condon-Shortley
    phase: Y_l^0; sqrt(2) Re Y_l^m for m > 0; sqrt(2) Im Y_l^|m| for m < 0;
    ordered by l, then m = -l .. l;
  - the direction d = (mean - C) / |mean - C| from the camera centre C,
    held in FP32 like the camera row (d = 0 when the mean sits on it);
  - colour_c = max(sum_k Y_k(d) f_kc + 1/2, 0).
Below, each basis function is written out as a polynomial in (x, y, z) = d,
with its normalisation from the square roots; the tests pin them to SciPy's
complex harmonics.
"""
from __future__ import annotations

import math

import numpy as np
import torch

_S = math.sqrt
_PI = math.pi
# normalisations of the real basis, band by band
N0 = 1.0 / (2.0 * _S(_PI))
N1 = _S(3.0 / (4.0 * _PI))
N2 = (0.5 * _S(15.0 / _PI), 0.25 * _S(5.0 / _PI), 0.25 * _S(15.0 / _PI))
N3 = (0.25 * _S(35.0 / (2.0 * _PI)), 0.5 * _S(105.0 / _PI), 0.25 * _S(21.0 / (2.0 * _PI)),
      0.25 * _S(7.0 / _PI), 0.25 * _S(105.0 / _PI))


def n_coeffs(degree: int) -> int:
    if not 0 <= degree <= 3:
        raise ValueError("SH degree must be 0..3")
    return (degree + 1) ** 2


def basis(d, degree: int):
    """[K, n] real SH basis at the unit directions d [3, n] (torch or numpy)."""
    t = torch.as_tensor(d, dtype=torch.float64)
    x, y, z = t[0], t[1], t[2]
    one = torch.ones_like(x)
    ys = [N0 * one]
    if degree >= 1:
        ys += [-N1 * y, N1 * z, -N1 * x]
    if degree >= 2:
        a, b, c = N2
        ys += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, c * (x * x - y * y)]
    if degree >= 3:
        e, f, g, h, j = N3
        ys += [-e * y * (3 * x * x - y * y), f * x * y * z, -g * y * (4 * z * z - x * x - y * y),
               h * z * (2 * z * z - 3 * x * x - 3 * y * y), -g * x * (4 * z * z - x * x - y * y),
               j * z * (x * x - y * y), -e * x * (x * x - 3 * y * y)]
    return torch.stack(ys)


def camera_centre(cam) -> np.ndarray:
    """C = -R^T t for x_cam = R x_world + t, evaluated in FP64 from the FP32
    camera row and held in FP32 (returned as float64), like the camera row
    itself: a mean stored at the centre then has d = 0 on both sides."""
    row = cam.row() if hasattr(cam, "row") else np.asarray(cam, np.float32)
    R = np.asarray(row[:9], np.float64).reshape(3, 3)
    t = np.asarray(row[9:12], np.float64)
    return (-R.T @ t).astype(np.float32).astype(np.float64)


def _colour(sh, mean, centre, degree):
    v = mean - centre[:, None]
    r2 = (v * v).sum(0)
    on = r2 > 0  # masked before the square root, so no gradient flows through sqrt(0)
    r = torch.sqrt(torch.where(on, r2, torch.ones_like(r2)))
    d = torch.where(on, v / r, torch.zeros_like(v))
    Y = basis(d, degree)                             # [K, n]
    K = Y.shape[0]
    f = sh.reshape(K, 3, -1)                         # [K, 3, n]
    raw = (Y[:, None, :] * f).sum(0) + 0.5           # [3, n]
    return torch.clamp(raw, min=0.0), raw


def color(sh, mean, cam, degree: int) -> np.ndarray:
    """[3, n] colour of every Gaussian seen from the camera, FP64."""
    K = n_coeffs(degree)
    shp = torch.as_tensor(np.asarray(sh, np.float64).reshape(K * 3, -1))
    mp = torch.as_tensor(np.asarray(mean, np.float64))
    c, _ = _colour(shp, mp, torch.as_tensor(camera_centre(cam)), degree)
    return c.numpy()


def color_bwd(sh, mean, cam, degree: int, grad_color):
    """(dL/dsh [K*3, n], dL/dmean [3, n]) from dL/dcolour [3, n], by autograd
    through the clamp (derivative 0 where the clamp is active, including
    raw == 0)."""
    K = n_coeffs(degree)
    shp = torch.tensor(np.asarray(sh, np.float64).reshape(K * 3, -1), requires_grad=True)
    mp = torch.tensor(np.asarray(mean, np.float64), requires_grad=True)
    _, raw = _colour(shp, mp, torch.as_tensor(camera_centre(cam)), degree)
    g = torch.as_tensor(np.asarray(grad_color, np.float64)) * (raw > 0)
    raw.backward(g)
    gm = mp.grad.numpy() if mp.grad is not None else np.zeros(mp.shape)  # degree 0: no direction dependence
    return shp.grad.numpy(), gm
