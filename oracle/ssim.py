"""SSIM term of the photometric loss (Sec. 4.2; in the appendix it enters
with weight 0.2 beside 0.8 L1), plain FP64 torch on the CPU, the gradient by
autograd.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the product
path; it shares no code with the HIP library.

The paper names the D-SSIM term without restating the index.  Reading (the
same on the GPU side): the structural-similarity index of Wang et al. (2004)
as 3DGS training uses it:
  - per channel, every valid 11x11 window (no padding), Gaussian weights
    w[i, j] = g[i] g[j], g[k] proportional to exp(-(k - 5)^2 / (2 * 1.5^2)),
    summing to 1;
  - window moments mx = sum w x, Exx = sum w x^2, Exy = sum w x y (and the
    same for y); sxx = Exx - mx^2, sxy = Exy - mx my;
  - S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)),
    C1 = 0.01^2, C2 = 0.03^2 (unit dynamic range);
  - the index is the mean of S over windows and channels.
The window sums are one 2-D cross-correlation (torch conv2d, FP64) with the
full 11x11 window; the tests pin it to explicit window loops.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window() -> torch.Tensor:
    """The 11x11 weights w[i, j] = g[i] g[j] (FP64, sum 1)."""
    d = torch.arange(WINDOW, dtype=torch.float64) - (WINDOW - 1) / 2
    g = torch.exp(-d * d / (2 * SIGMA * SIGMA))
    g = g / g.sum()
    return torch.outer(g, g)


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """S per channel and window, [C, H - 10, W - 10], for x, y [C, H, W]."""
    c = x.shape[0]
    w = window().to(x.dtype).expand(c, 1, WINDOW, WINDOW)

    def wsum(t):
        return F.conv2d(t[None], w, groups=c)[0]

    mx, my = wsum(x), wsum(y)
    sxx = wsum(x * x) - mx * mx
    syy = wsum(y * y) - my * my
    sxy = wsum(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim(x: np.ndarray, y: np.ndarray) -> float:
    """Mean SSIM of two images [C, H, W] (FP64)."""
    return float(ssim_map(torch.as_tensor(np.asarray(x, np.float64)),
                          torch.as_tensor(np.asarray(y, np.float64))).mean())


def ssim_and_grad(x: np.ndarray, y: np.ndarray) -> tuple[float, np.ndarray]:
    """Mean SSIM and its gradient with respect to x (the target y fixed)."""
    xt = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
    s = ssim_map(xt, torch.as_tensor(np.asarray(y, np.float64))).mean()
    s.backward()
    return float(s.detach()), xt.grad.numpy()
