"""Pins of the SH colour oracle (base 3DGS colour model, Sec. 3 / Sec. 4.2):
the basis against SciPy's complex harmonics and against the properties of
the real orthonormal basis; colour special cases; gradients against finite
differences."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import sh as S
from paper_2504_17954_amd import inputs as I


def unit_dirs(n, seed):
    v = np.random.default_rng(seed).normal(size=(3, n))
    return v / np.linalg.norm(v, axis=0)


def test_basis_matches_scipy_complex_harmonics():
    d = unit_dirs(500, 1)
    theta = np.arccos(np.clip(d[2], -1, 1))  # polar
    phi = np.arctan2(d[1], d[0])             # azimuth
    ref = []
    for l in range(4):
        for m in range(-l, l + 1):
            y = sp.sph_harm_y(l, abs(m), theta, phi)
            ref.append(y.real if m == 0 else math.sqrt(2) * (y.real if m > 0 else y.imag))
    np.testing.assert_allclose(S.basis(d, 3).numpy(), np.array(ref), atol=1e-12)


def test_basis_is_orthonormal_on_the_sphere():
    # Gauss-Legendre in cos(theta) x uniform azimuth: exact for these degrees
    u, w = np.polynomial.legendre.leggauss(16)
    phi = np.arange(32) * 2 * np.pi / 32
    U, P = np.meshgrid(u, phi, indexing="ij")
    s = np.sqrt(1 - U ** 2)
    d = np.stack([s * np.cos(P), s * np.sin(P), U]).reshape(3, -1)
    wt = (w[:, None] * np.full(32, 2 * np.pi / 32)[None, :]).ravel()
    Y = S.basis(d, 3).numpy()
    np.testing.assert_allclose((Y * wt) @ Y.T, np.eye(16), atol=1e-12)


def test_addition_theorem_per_band():
    Y = S.basis(unit_dirs(200, 2), 3).numpy()
    for l in range(4):
        band = Y[l * l:(l + 1) * (l + 1)]
        np.testing.assert_allclose((band ** 2).sum(0), (2 * l + 1) / (4 * np.pi), rtol=1e-12)


def test_condon_shortley_signs_of_band_one():
    k = math.sqrt(3 / (4 * math.pi))
    Y = S.basis(np.eye(3), 1).numpy()  # columns: +x, +y, +z
    np.testing.assert_allclose(Y[1], [0, -k, 0], atol=1e-15)  # m = -1 ~ -y
    np.testing.assert_allclose(Y[2], [0, 0, k], atol=1e-15)   # m = 0 ~ z
    np.testing.assert_allclose(Y[3], [-k, 0, 0], atol=1e-15)  # m = 1 ~ -x


def test_camera_centre_and_constant_colour():
    cam = I.look_at((0.0, -3.0, 0.5), width=32, height=32)
    C = S.camera_centre(cam)
    np.testing.assert_allclose(C, [0.0, -3.0, 0.5], atol=1e-5)
    rng = np.random.default_rng(3)
    n = 50
    mean = rng.normal(size=(3, n)).astype(np.float32)
    sh = np.zeros((16 * 3, n), np.float32)
    want = rng.uniform(0, 1, (3, n))
    sh[0:3] = (want - 0.5) / S.N0  # the constant band alone
    np.testing.assert_allclose(S.color(sh, mean, cam, 3), want, atol=1e-6)
    sh[0:3] = -2.0 / S.N0  # raw colour -1.5: clamped at zero
    np.testing.assert_array_equal(S.color(sh, mean, cam, 3), 0.0)


def test_mean_on_the_camera_centre_uses_the_constant_band():
    cam = I.look_at((1.0, 2.0, 3.0), width=32, height=32)
    C = S.camera_centre(cam)
    mean = np.array(C, np.float64).reshape(3, 1)
    sh = np.random.default_rng(4).normal(size=(48, 1))
    got = S.color(sh, mean, cam, 3)
    np.testing.assert_allclose(got[:, 0], np.maximum(sh[0:3, 0] * S.N0 + 0.5, 0), atol=1e-12)
    gs, gm = S.color_bwd(sh, mean, cam, 3, np.ones((3, 1)))
    assert np.all(np.isfinite(gs)) and np.all(gm == 0)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_gradients_match_finite_differences(degree):
    rng = np.random.default_rng(10 + degree)
    K, n = S.n_coeffs(degree), 40
    cam = I.look_at((0.3, -3.5, 1.2), width=32, height=32)
    mean = rng.normal(scale=0.6, size=(3, n))
    sh = rng.normal(scale=0.3, size=(K * 3, n))
    g = rng.normal(size=(3, n))
    raw = S.color(sh, mean, cam, degree)
    keep = np.all(raw > 1e-3, axis=0) | np.all(raw == 0, axis=0)
    gs, gm = S.color_bwd(sh, mean, cam, degree, g)
    h = 1e-6
    loss = lambda s, m: float((S.color(s, m, cam, degree) * g).sum())
    for i in np.flatnonzero(keep)[:6]:
        for a in range(3):
            mp, mm = mean.copy(), mean.copy()
            mp[a, i] += h
            mm[a, i] -= h
            assert abs((loss(sh, mp) - loss(sh, mm)) / (2 * h) - gm[a, i]) < 1e-6
        for kc in range(0, K * 3, max(1, K * 3 // 5)):
            sp_, sm = sh.copy(), sh.copy()
            sp_[kc, i] += h
            sm[kc, i] -= h
            assert abs((loss(sp_, mean) - loss(sm, mean)) / (2 * h) - gs[kc, i]) < 1e-6
    # colour depends only on the direction: the mean gradient is tangent
    v = mean - S.camera_centre(cam)[:, None]
    np.testing.assert_allclose((gm * v).sum(0), 0.0, atol=1e-10)
