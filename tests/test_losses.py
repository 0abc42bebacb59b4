"""The training losses (Sec. 4.2, 4.3; Eq. 6, 7) against brute force and
closed forms, on the CPU."""
import numpy as np
import pytest
import torch

from paper_2504_17954_amd import inputs as I
from paper_2504_17954_amd import losses as L


def test_ssim_refuses_host_tensors():
    """The package has no CPU SSIM: the CPU reference is the oracle's
    (oracle/ssim.py, pinned in test_oracle_ssim.py)."""
    x = torch.rand((4, 20, 24))
    with pytest.raises(ValueError):
        L.ssim(x, x)
    with pytest.raises(ValueError):
        L.photometric(x, x)


def test_pseudo_normal_of_a_plane_is_its_normal():
    cam = I.look_at((0.4, -3.0, 1.0), width=48, height=40)
    n_c = np.array([0.2, -0.3, -1.0])
    n_c /= np.linalg.norm(n_c)  # facing the camera (negative z in camera space)
    c = -2.5  # plane n . P = c in camera space
    ys, xs = np.meshgrid(np.arange(40) + 0.5, np.arange(48) + 0.5, indexing="ij")
    rays = np.stack([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy, np.ones_like(xs)])
    depth = c / np.einsum("i,ihw->hw", n_c, rays)
    alpha = np.full_like(depth, 0.9)
    pn, valid = L.pseudo_normal(torch.from_numpy(depth * alpha), torch.from_numpy(alpha), cam)
    want = np.asarray(cam.R, np.float64).T @ n_c  # world space
    got = pn.numpy()[:, valid.numpy()]
    assert valid.sum() == 38 * 46
    np.testing.assert_allclose(got, np.repeat(want[:, None], got.shape[1], 1), atol=1e-9)


def test_normal_consistency_is_zero_on_agreeing_maps():
    cam = I.look_at((0.0, -3.0, 0.0), width=24, height=24)
    depth = torch.full((24, 24), 2.0, dtype=torch.float64)
    alpha = torch.ones((24, 24), dtype=torch.float64)
    pn, _ = L.pseudo_normal(depth, alpha, cam)
    assert L.normal_consistency(pn * 0.7, depth, alpha, cam).item() < 1e-12


def test_bilateral_smoothness_and_sparsity_closed_forms():
    k = torch.zeros((4, 10, 12), dtype=torch.float64)
    gt = torch.rand((3, 10, 12), dtype=torch.float64, generator=torch.Generator().manual_seed(3))
    assert L.bilateral_smoothness(k, gt).item() == 0.0
    k[0] = torch.arange(12, dtype=torch.float64)[None, :] * 0.5  # slope 0.5 along x
    flat = torch.zeros_like(gt)
    # only the x differences of one map of four: mean 0.5 over a quarter of the entries
    assert abs(L.bilateral_smoothness(k, flat).item() - 0.5 / 4) < 1e-12
    edge = flat.clone()
    edge[:, :, 6:] = 1.0  # a unit step in every channel between columns 5 and 6
    want = 0.5 * (10 * 10 + 10 * np.exp(-1.0)) / (4 * 10 * 11)
    assert abs(L.bilateral_smoothness(k, edge).item() - want) < 1e-12
    assert abs(L.sparsity(torch.tensor([[-1.0, 2.0], [0.5, -0.5]])).item() - 1.0) < 1e-12
