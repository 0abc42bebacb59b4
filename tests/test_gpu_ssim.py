"""GPU parity of the SSIM term of the photometric loss (Sec. 4.2) through
ivrgs_ssim_fwd / ivrgs_ssim_bwd against the FP64 oracle: the mean within
1e-5, the gradient within 1e-3 relative plus 1e-5 of its largest magnitude;
several 16x16 tiles with ragged edges, the single-window image, and the full
800x800 RGBA of the training step."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle import explore as OX
from oracle import ssim as OS
from paper_2504_17954_amd import losses as L
from paper_2504_17954_amd import native as N

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def pair(shape, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, shape)
    y = np.clip(0.7 * x + 0.3 * rng.uniform(0, 1, shape) + rng.normal(0, 0.05, shape), 0, 1)
    return x.astype(np.float32), y.astype(np.float32)


def run(x, y, dev):
    xd = torch.from_numpy(x).to(dev).requires_grad_(True)
    yd = torch.from_numpy(y).to(dev)
    v = L.ssim(xd, yd)
    v.backward()
    return float(v.detach()), xd.grad.cpu().numpy()


@pytest.mark.parametrize("shape,seed", [((3, 11, 11), 1), ((4, 40, 52), 2), ((1, 27, 100), 3), ((4, 100, 130), 4)])
def test_ssim_matches_oracle(dev, shape, seed):
    x, y = pair(shape, seed)
    say(f"ssim {shape}")
    want, gwant = OS.ssim_and_grad(x.astype(np.float64), y.astype(np.float64))
    got, g = run(x, y, dev)
    assert abs(got - want) <= 1e-5, (got, want)
    tol = 1e-3 * np.abs(gwant) + 1e-5 * np.abs(gwant).max()
    bad = np.abs(g - gwant) > tol
    say(f"  mean {got:.7f} vs {want:.7f}; gradient outside {bad.sum()} / {g.size}, "
        f"worst {(np.abs(g - gwant) / tol).max():.3f}")
    assert not bad.any()


def test_ssim_full_size_rgba(dev):
    """The 800x800 RGBA of a training view: mean and gradient at every pixel."""
    x, y = pair((4, 800, 800), 5)
    say("ssim 4x800x800")
    want, gwant = OS.ssim_and_grad(x.astype(np.float64), y.astype(np.float64))
    got, g = run(x, y, dev)
    assert abs(got - want) <= 1e-5, (got, want)
    tol = 1e-3 * np.abs(gwant) + 1e-5 * np.abs(gwant).max()
    bad = np.abs(g - gwant) > tol
    say(f"  mean {got:.7f} vs {want:.7f}; gradient outside {bad.sum()} / {g.size}")
    assert not bad.any()


def test_ssim_identity_is_exactly_one(dev):
    x, _ = pair((4, 64, 80), 6)
    xd = torch.from_numpy(x).to(dev)
    assert float(L.ssim(xd, xd.clone())) == 1.0


def test_ssim_twice_on_one_workspace_is_deterministic(dev):
    x, y = pair((4, 90, 70), 7)
    a, ga = run(x, y, dev)
    b, gb = run(x, y, dev)
    assert a == b and np.array_equal(ga, gb)


def test_ssim_shape_errors(dev):
    x = torch.zeros((2, 10, 40), device=dev)
    with pytest.raises(ValueError):
        L.ssim(x, x)
    # the C ABI itself: too small an image, too small a workspace, null pointers
    assert N.ivrgs_ssim_workspace_size(2, 10, 40) == 0
    ws = torch.empty(16, dtype=torch.uint8, device=dev)
    out = torch.empty((), device=dev)
    with pytest.raises(N.IvrgsError):
        N.ivrgs_ssim_fwd(x.data_ptr(), x.data_ptr(), 2, 10, 40, out.data_ptr(), ws.data_ptr(), 16, None)
    y = torch.zeros((2, 20, 40), device=dev)
    with pytest.raises(N.IvrgsError):
        N.ivrgs_ssim_fwd(y.data_ptr(), y.data_ptr(), 2, 20, 40, out.data_ptr(), ws.data_ptr(), 16, None)
    with pytest.raises(N.IvrgsError):
        N.ivrgs_ssim_fwd(None, y.data_ptr(), 2, 20, 40, out.data_ptr(), ws.data_ptr(), 16, None)
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape,seed,lam", [((3, 11, 11), 11, 0.2), ((4, 40, 52), 12, 0.2),
                                            ((4, 100, 130), 13, 0.0), ((2, 27, 100), 14, 1.0),
                                            ((4, 800, 800), 15, 0.2)])
def test_photometric_grad_matches_oracle(dev, shape, seed, lam):
    """ivrgs_photometric_grad: the gradient of (1 - lam) mean|x - y| +
    lam (1 - SSIM) against the oracle's (the exploration objective, and the
    photometric term of training), through the C ABI; the autograd Function
    of the losses gives the same gradient and the loss value."""
    x, y = pair(shape, seed)
    y[:, :3, :5] = x[:, :3, :5]  # exact ties: sign(0) = 0 on both sides
    say(f"photometric grad {shape} lam={lam}")
    want, gwant = OX.photometric(x.astype(np.float64), y.astype(np.float64), lam)
    c, h, w = shape
    xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    nbytes = N.ivrgs_ssim_workspace_size(c, h, w)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    s = torch.empty((), device=dev)
    g = torch.full_like(xd, float("nan"))
    N.ivrgs_ssim_fwd(xd.data_ptr(), yd.data_ptr(), c, h, w, s.data_ptr(), ws.data_ptr(), nbytes, None)
    N.ivrgs_photometric_grad(xd.data_ptr(), yd.data_ptr(), c, h, w, lam, g.data_ptr(), ws.data_ptr(), nbytes,
                             None)
    g = g.cpu().numpy()
    tol = 1e-3 * np.abs(gwant) + 1e-5 * np.abs(gwant).max()
    bad = np.abs(g - gwant) > tol
    say(f"  gradient outside {bad.sum()} / {g.size}, worst {(np.abs(g - gwant) / tol).max():.3f}")
    assert not bad.any()
    xr = xd.clone().requires_grad_(True)
    loss = L.photometric(xr, yd, lam)
    loss.backward()
    assert abs(float(loss.detach()) - want) <= 1e-5 * max(1.0, abs(want))
    assert torch.equal(xr.grad.cpu(), torch.from_numpy(g))


def test_photometric_grad_argument_errors(dev):
    x = torch.zeros((4, 20, 20), device=dev)
    nbytes = N.ivrgs_ssim_workspace_size(4, 20, 20)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    for lam in (-0.1, 1.5, float("nan")):
        with pytest.raises(N.IvrgsError):
            N.ivrgs_photometric_grad(x.data_ptr(), x.data_ptr(), 4, 20, 20, lam, x.data_ptr(), ws.data_ptr(),
                                     nbytes, None)
    with pytest.raises(N.IvrgsError):
        N.ivrgs_photometric_grad(x.data_ptr(), x.data_ptr(), 4, 20, 20, 0.2, x.data_ptr(), ws.data_ptr(), 16,
                                 None)
    with pytest.raises(N.IvrgsError):
        N.ivrgs_photometric_grad(x.data_ptr(), x.data_ptr(), 4, 20, 9, 0.2, x.data_ptr(), ws.data_ptr(),
                                 nbytes, None)
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape,seed", [((3, 11, 11), 21), ((4, 40, 52), 22), ((2, 27, 100), 23),
                                        ((4, 171, 202), 24)])
def test_photometric_fwd_and_device_weights_match_oracle(dev, shape, seed):
    """ivrgs_photometric_fwd: the SSIM mean and the L1 mean from one pass
    (the L1 over every pixel, the rows and columns past the last tile of
    windows included) against the oracles; ivrgs_photometric_grad_dev: the
    gradient of w0 SSIM + w1 L1 with the weights read on the device."""
    x, y = pair(shape, seed)
    y[:, :2, :3] = x[:, :2, :3]  # exact ties: sign(0) = 0 on both sides
    c, h, w = shape
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    s_want, ds = OS.ssim_and_grad(x64, y64)
    l1_want = O.l1_loss(x64, y64)
    _, dl1 = OX.photometric(x64, y64, 0.0)  # gradient of the L1 mean
    xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    nbytes = N.ivrgs_photometric_workspace_size(c, h, w)
    assert nbytes >= N.ivrgs_ssim_workspace_size(c, h, w)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = torch.full((2,), float("nan"), device=dev)
    N.ivrgs_photometric_fwd(xd.data_ptr(), yd.data_ptr(), c, h, w, out.data_ptr(), ws.data_ptr(), nbytes, None)
    wts = (-0.37, 1.9)
    wd = torch.tensor(wts, dtype=torch.float32, device=dev)
    g = torch.full_like(xd, float("nan"))
    N.ivrgs_photometric_grad_dev(xd.data_ptr(), yd.data_ptr(), c, h, w, wd.data_ptr(), g.data_ptr(),
                                 ws.data_ptr(), nbytes, None)
    s_got, l1_got = (float(v) for v in out.cpu())
    say(f"photometric {shape}: SSIM {s_got:.7f} vs {s_want:.7f}, L1 {l1_got:.7f} vs {l1_want:.7f}")
    assert abs(s_got - s_want) <= 1e-5
    assert abs(l1_got - l1_want) <= 1e-5 * l1_want
    gwant = wts[0] * ds + wts[1] * dl1
    g = g.cpu().numpy()
    tol = 1e-3 * np.abs(gwant) + 1e-5 * np.abs(gwant).max()
    bad = np.abs(g - gwant) > tol
    say(f"  gradient outside {bad.sum()} / {g.size}, worst {(np.abs(g - gwant) / tol).max():.3f}")
    assert not bad.any()
