"""Pins of the auxiliary-map oracle (Eq. 5 depth and normal maps, the
offset-colour and shading maps of Sec. 4.3): the dense FP64 formulation
against the C oracle's image and closed forms."""
import numpy as np
import torch

import oracle as O
from oracle import dense as D
from paper_2504_17954_amd import inputs as I


def scene(n, seed, width=40, height=32):
    m = I.small_scene(n, seed, log_scale_mu=-2.6)
    planes = I.plain_planes(m)
    cam = I.look_at((0.3, -3.6, 0.9), width=width, height=height)
    return planes, cam, O.Params(width, height)


def test_colour_as_attribute_reproduces_the_rgb_image():
    planes, cam, prm = scene(150, 31)
    n = planes["mean"].shape[1]
    planes["shade"] = np.tile(np.array([[1.0], [0.0], [0.0], [1.0]], np.float32), (1, n))  # colour passes through
    ref = O.render(planes, cam, prm)
    pt = D.to_tensors(planes)
    _, _, _, aux = D.render(pt, cam.row(), prm, attr_t=pt["color"])
    ok = ref["flags"] == 0
    np.testing.assert_allclose(aux[1:4].numpy()[:, ok], ref["rgba"][:3][:, ok], atol=1e-9)


def test_constant_attribute_is_the_alpha_map():
    planes, cam, prm = scene(120, 32)
    pt = D.to_tensors(planes)
    rgba, _, _, aux = D.render(pt, cam.row(), prm, attr_t=torch.ones((2, 120), dtype=torch.float64))
    np.testing.assert_allclose(aux[1].numpy(), rgba[3].numpy(), atol=1e-12)
    np.testing.assert_allclose(aux[2].numpy(), rgba[3].numpy(), atol=1e-12)


def test_depth_of_one_gaussian_over_alpha_is_its_depth():
    planes, cam, prm = scene(1, 33)
    planes["mean"][:, 0] = (0.1, 0.2, -0.1)
    planes["opacity"][:] = 0.8
    planes["log_scale"][:] = -1.5
    pt = D.to_tensors(planes)
    rgba, _, _, aux = D.render(pt, cam.row(), prm, attr_t=torch.zeros((0, 1), dtype=torch.float64))
    a = rgba[3].numpy()
    z = (np.asarray(cam.R, np.float64) @ planes["mean"][:, 0].astype(np.float64) + cam.t)[2]
    hit = a > 0
    assert hit.sum() > 20
    np.testing.assert_allclose(aux[0].numpy()[hit] / a[hit], z, rtol=1e-12)


def test_attribute_gradient_is_the_compositing_weight():
    planes, cam, prm = scene(60, 34)
    pt = D.to_tensors(planes)
    attr = torch.zeros((1, 60), dtype=torch.float64, requires_grad=True)
    rgba, _, _, aux = D.render(pt, cam.row(), prm, attr_t=attr)
    aux[1].sum().backward()
    # d(sum over pixels of sum_i w_i a_i)/da_i = sum over pixels of w_i; their
    # total is the summed alpha map
    np.testing.assert_allclose(attr.grad.sum().item(), rgba[3].sum().item(), rtol=1e-12)


def test_editable_attributes_closed_forms():
    """The attribute rows of the editable stage: unit normals along the
    normal plane, unchanged by a positive scale, colour and shade passed
    through, the floor at a zero normal; the derivative of the normalisation
    (I - u u^T) / |n|: zero along u, 1 / |n| across it, identity for the
    colour and shade rows."""
    rng = np.random.default_rng(71)
    n = 50
    nrm = torch.tensor(rng.normal(size=(3, n)))
    col = torch.tensor(rng.uniform(-1, 1, size=(3, n)))
    sh = torch.tensor(rng.uniform(0, 1, size=(4, n)))
    a = D.editable_attributes(nrm, col, sh)
    assert a.shape == (10, n)
    u = a[:3]
    np.testing.assert_allclose(u.norm(dim=0).numpy(), 1.0, atol=1e-14)
    np.testing.assert_allclose(torch.linalg.cross(u, nrm, dim=0).numpy(), 0.0, atol=1e-13)
    assert bool(((u * nrm).sum(0) > 0).all())
    np.testing.assert_allclose(D.editable_attributes(3.5 * nrm, col, sh).numpy(), a.numpy(), atol=1e-14)
    np.testing.assert_array_equal(a[3:6].numpy(), col.numpy())
    np.testing.assert_array_equal(a[6:].numpy(), sh.numpy())
    z = D.editable_attributes(torch.zeros((3, 2), dtype=torch.float64), col[:, :2], sh[:, :2])
    np.testing.assert_array_equal(z[:3].numpy(), 0.0)
    # derivative of the rows through autograd against the closed form
    nr = nrm.clone().requires_grad_(True)
    cr = col.clone().requires_grad_(True)
    sr = sh.clone().requires_grad_(True)
    u0 = (nrm / nrm.norm(dim=0, keepdim=True)).numpy()
    g_perp = np.cross(u0.T, rng.normal(size=(n, 3))).T  # across u
    for g_u, expect in ((u0 * 2.0, np.zeros((3, n))), (g_perp, g_perp / np.linalg.norm(nrm.numpy(), axis=0))):
        g = torch.zeros((10, n), dtype=torch.float64)
        g[:3] = torch.tensor(g_u)
        g[3:] = torch.tensor(rng.normal(size=(7, n)))
        nr.grad = cr.grad = sr.grad = None
        D.editable_attributes(nr, cr, sr).backward(g)
        np.testing.assert_allclose(nr.grad.numpy(), expect, atol=1e-12)
        np.testing.assert_array_equal(cr.grad.numpy(), g[3:6].numpy())
        np.testing.assert_array_equal(sr.grad.numpy(), g[6:].numpy())
