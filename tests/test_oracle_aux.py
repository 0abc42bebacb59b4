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
