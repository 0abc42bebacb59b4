"""Pins of the regulariser oracle (oracle/regularisers.py: Eq. 5-7, Sec.
4.3) against closed forms, exact geometry and finite differences, on the
CPU."""
import numpy as np
import pytest
import torch

from oracle import regularisers as G
from paper_2504_17954_amd import inputs as I


def plane_depth(cam, n_c, c, H, W):
    """Depth map of the camera-space plane n_c . P = c (exact, FP64)."""
    ys, xs = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    rays = np.stack([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy, np.ones_like(xs)])
    return c / np.einsum("i,ihw->hw", n_c, rays)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_pseudo_normal_of_a_plane_is_its_normal(sign):
    """Differences of points of a plane lie in the plane, so the cross
    product of the central differences is parallel to its normal whatever
    the perspective: N~ = R^T n (facing the camera) at every valid pixel,
    for either orientation of n."""
    H, W = 40, 48
    cam = I.look_at((0.4, -3.0, 1.0), width=W, height=H)
    n_c = np.array([0.2, -0.3, -1.0])
    n_c /= np.linalg.norm(n_c)  # facing the camera: negative z in camera space
    depth = plane_depth(cam, n_c, -2.5, H, W)
    alpha = np.full((H, W), 0.9)
    pn, valid = G.pseudo_normal(depth * alpha, alpha, cam)
    # the same plane written with the opposite normal gives the same N~
    pn2, _ = G.pseudo_normal(plane_depth(cam, sign * -n_c, sign * 2.5, H, W) * alpha, alpha, cam)
    want = np.asarray(cam.R, np.float64).T @ n_c
    assert int(valid.sum()) == (H - 2) * (W - 2)
    got = pn.numpy()[:, valid.numpy()]
    np.testing.assert_allclose(got, np.repeat(want[:, None], got.shape[1], 1), atol=1e-9)
    np.testing.assert_allclose(pn2.numpy(), pn.numpy(), atol=1e-9)
    assert np.all(pn.numpy()[:, ~valid.numpy()] == 0.0)


def test_valid_mask_by_hand():
    """alpha <= 0.5 at one pixel removes it and its four neighbours; the
    border is never valid; alpha exactly 0.5 is not enough."""
    a = np.full((7, 9), 0.8)
    a[3, 4] = 0.2
    a[5, 7] = 0.5
    v = G.valid_mask(torch.as_tensor(a)).numpy()
    want = np.zeros((7, 9), bool)
    want[1:-1, 1:-1] = True
    for (y, x) in [(3, 4), (2, 4), (4, 4), (3, 3), (3, 5), (5, 7), (4, 7), (5, 6)]:
        want[y, x] = False
    assert np.array_equal(v, want)


def test_normal_consistency_closed_forms():
    H, W = 24, 20
    cam = I.look_at((0.0, -3.0, 0.0), width=W, height=H)
    depth = np.full((H, W), 2.0)
    alpha = np.ones((H, W))
    pn, valid = G.pseudo_normal(depth, alpha, cam)
    # a fronto-parallel plane: N~ = -z of the camera in world space
    want = -np.asarray(cam.R, np.float64)[2]
    np.testing.assert_allclose(pn.numpy()[:, valid.numpy()], np.repeat(want[:, None], int(valid.sum()), 1),
                               atol=1e-12)
    assert float(G.normal_consistency(pn * 0.7, pn, valid)) < 1e-12
    # a constant normal map at angle theta from N~: 2 sin(theta / 2), any length
    th = 0.7
    axis = np.cross(want, [0.0, 0.0, 1.0])
    axis /= np.linalg.norm(axis)
    n1 = want * np.cos(th) + np.cross(axis, want) * np.sin(th)
    nm = torch.as_tensor(np.repeat(3.0 * n1[:, None, None], H, 1).repeat(W, 2))
    assert abs(float(G.normal_consistency(nm, pn, valid)) - 2 * np.sin(th / 2)) < 1e-12
    # no valid pixel: 0
    none = torch.zeros((H, W), dtype=torch.bool)
    assert float(G.normal_consistency(nm, pn, none)) == 0.0


def test_sparsity_smoothness_opacity_closed_forms():
    k = torch.zeros((4, 10, 12), dtype=torch.float64)
    gt = torch.rand((3, 10, 12), dtype=torch.float64, generator=torch.Generator().manual_seed(3))
    assert float(G.bilateral_smoothness(k, gt)) == 0.0
    k[0] = torch.arange(12, dtype=torch.float64)[None, :] * 0.5  # slope 0.5 along x in one map of four
    flat = torch.zeros_like(gt)
    assert abs(float(G.bilateral_smoothness(k, flat)) - 0.5 / 4) < 1e-12
    edge = flat.clone()
    edge[:, :, 6:] = 1.0  # a unit step in every colour channel between columns 5 and 6
    want = 0.5 * (10 * 10 + 10 * np.exp(-1.0)) / (4 * 10 * 11)
    assert abs(float(G.bilateral_smoothness(k, edge)) - want) < 1e-12
    # the y differences count over their own entries: slope 0.25 along y in one map
    ky = torch.zeros_like(k)
    ky[2] = torch.arange(10, dtype=torch.float64)[:, None] * 0.25
    assert abs(float(G.bilateral_smoothness(ky, flat)) - 0.25 / 4) < 1e-12
    assert abs(float(G.sparsity(torch.tensor([[-1.0, 2.0], [0.5, -0.5]]))) - 1.0) < 1e-12
    assert abs(float(G.opacity_l1(torch.tensor([0.25, -0.75, 2.0, 0.0]))) - 0.75) < 1e-12


def test_gradients_against_finite_differences():
    H, W = 14, 17
    cam = I.look_at((0.3, -3.5, 0.6), width=W, height=H)
    m = {k: v.astype(np.float64) for k, v in I.view_maps(H, W, 5).items()}
    gt = np.array([0.7, 1.3, -0.4, 2.0])
    out = G.terms(m["depth"], m["alpha"], m["normal"], m["delta_c"], m["shade"], m["target"], m["opacity"], cam,
                  grad_terms=gt)
    assert out["count"] > 50

    def total(key, arr):
        mm = dict(m)
        mm[key] = arr
        o = G.terms(mm["depth"], mm["alpha"], mm["normal"], mm["delta_c"], mm["shade"], mm["target"],
                    mm["opacity"], cam)
        return float(o["terms"] @ gt)

    rng = np.random.default_rng(0)
    for key, gk in [("normal", "grad_normal"), ("delta_c", "grad_delta_c"), ("shade", "grad_shade"),
                    ("opacity", "grad_opacity")]:
        arr = m[key]
        for flat in rng.choice(arr.size, 12, replace=False):
            idx = np.unravel_index(flat, arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            a, b = arr.copy(), arr.copy()
            a[idx] += h
            b[idx] -= h
            fd = (total(key, a) - total(key, b)) / (2 * h)
            assert abs(fd - out[gk][idx]) <= 1e-6 * max(1.0, abs(fd)), (key, idx, fd, out[gk][idx])
    # the normal gradient at a valid pixel written out: (n (n . N~) - N~) / (L |N|) / count
    y, x = np.argwhere(out["valid"])[7]
    N = m["normal"][:, y, x]
    nh = N / np.linalg.norm(N)
    pn = out["pseudo_normal"][:, y, x]
    L = np.linalg.norm(nh - pn)
    want = gt[0] * (nh * (nh @ pn) - pn) / (L * np.linalg.norm(N)) / out["count"]
    np.testing.assert_allclose(out["grad_normal"][:, y, x], want, rtol=1e-10, atol=1e-14)
    # the depth, alpha and target get no gradient and invalid pixels no normal gradient
    assert np.all(out["grad_normal"][:, ~out["valid"]] == 0.0)
