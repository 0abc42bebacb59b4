"""GPU parity of the L1 term of the photometric loss (Sec. 4.2) through
ivrgs_l1_fwd / ivrgs_l1_bwd against the FP64 oracle: the mean within 1e-6
relative (FP32 differences summed in FP64, one FP32 rounding at the end),
the gradient sign(x - y) g / n within one FP32 rounding of the oracle's
value; lengths around the workgroup slice and vector width, a misaligned
start, exact ties, and the 4 x 800 x 800 RGBA of the training step; the
mean is the same bit for bit on repeated calls."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_17954_amd import losses as L
from paper_2504_17954_amd import native as N

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    N.load()
    return torch.device("cuda:0")


def check(x, y, dev, g=1.0):
    xd = torch.from_numpy(x).to(dev).requires_grad_(True)
    yd = torch.from_numpy(y).to(dev)
    m = L.l1(xd, yd)
    (m * g).backward()
    got, ref = float(m.item()), O.l1_loss(x, y)
    assert abs(got - ref) <= 1e-6 * abs(ref) + 1e-30, (got, ref)
    gref = O.l1_loss_grad(x.astype(np.float64), y.astype(np.float64)) * g
    gx = xd.grad.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gx - gref) <= 2 ** -23 * np.abs(gref)), np.abs(gx - gref).max()
    return got


@pytest.mark.parametrize("n", [1, 3, 4, 1023, 1024, 4095, 4097, 12289, 5 * 4096 * 1024 + 7])
def test_l1_matches_oracle(dev, n):
    say(f"l1 n={n}")
    rng = np.random.default_rng(n % 1000)
    x = rng.uniform(0, 1, n).astype(np.float32)
    y = rng.uniform(0, 1, n).astype(np.float32)
    y[::7] = x[::7]  # exact ties: zero gradient
    check(x, y, dev, g=0.75)


def test_l1_misaligned_start(dev):
    """Views that start one float into an allocation take the scalar path."""
    rng = np.random.default_rng(1)
    n = 50_001
    xa = torch.from_numpy(rng.uniform(0, 1, n + 1).astype(np.float32)).to(dev)
    ya = torch.from_numpy(rng.uniform(0, 1, n + 1).astype(np.float32)).to(dev)
    x, y = xa[1:], ya[1:]
    assert x.data_ptr() % 16 != 0
    ws = torch.empty(N.ivrgs_l1_workspace_size(n), dtype=torch.uint8, device=dev)
    out = torch.empty((), dtype=torch.float32, device=dev)
    N.ivrgs_l1_fwd(x.data_ptr(), y.data_ptr(), n, out.data_ptr(), ws.data_ptr(), ws.numel(), 0)
    ref = O.l1_loss(x.cpu().numpy(), y.cpu().numpy())
    assert abs(float(out.item()) - ref) <= 1e-6 * ref


def test_l1_full_rgba_repeatable(dev):
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 1, (4, 800, 800)).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1).astype(np.float32)
    a = check(x, y, dev)
    xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    b = [float(L.l1(xd, yd).item()) for _ in range(3)]
    assert all(np.float32(v).view(np.uint32) == np.float32(a).view(np.uint32) for v in b)


def test_l1_nan_difference_gives_nan_gradient(dev):
    x = torch.tensor([0.5, float("nan"), 0.25], device=dev, requires_grad=True)
    y = torch.tensor([0.25, 0.0, 0.25], device=dev)
    L.l1(x, y).backward()
    g = x.grad.cpu().numpy()
    assert g[0] == np.float32(1 / 3) and np.isnan(g[1]) and g[2] == 0.0
