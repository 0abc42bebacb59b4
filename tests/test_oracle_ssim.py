"""Pins of the SSIM oracle (the D-SSIM term of Sec. 4.2) to what the index's
definition fixes: identity, closed forms for constant images, explicit
window loops, finite differences of the gradient."""
import numpy as np

from oracle import ssim as S


def test_window_is_normalised_symmetric_gaussian():
    w = S.window().numpy()
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(w, w.T, rtol=0, atol=0)
    np.testing.assert_allclose(w, w[::-1, ::-1], rtol=0, atol=0)
    # ratio of neighbouring weights along a row: exp(-((k+1-5)^2 - (k-5)^2) / 4.5)
    r = w[5, 6] / w[5, 5]
    assert abs(r - np.exp(-1 / 4.5)) < 1e-14


def test_identity_is_one_with_zero_gradient():
    x = np.random.default_rng(1).uniform(0, 1, (3, 17, 20))
    v, g = S.ssim_and_grad(x, x)
    assert abs(v - 1.0) < 1e-12
    assert np.abs(g).max() < 1e-10  # a maximum of the index


def test_constant_images_closed_form():
    a, b = 0.3, 0.7
    x = np.full((2, 13, 15), a)
    y = np.full((2, 13, 15), b)
    want = (2 * a * b + S.C1) / (a * a + b * b + S.C1)  # variances vanish: the C2 factor is C2 / C2
    assert abs(S.ssim(x, y) - want) < 1e-11  # FP64 rounding of the window sums, over C2


def test_matches_explicit_window_loops():
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (2, 12, 14))
    y = np.clip(x + rng.normal(0, 0.2, x.shape), 0, 1)
    g = np.array([np.exp(-((k - 5) ** 2) / 4.5) for k in range(11)])
    g /= g.sum()
    vals = []
    for c in range(2):
        for i in range(12 - 10):
            for j in range(14 - 10):
                mx = my = exx = eyy = exy = 0.0
                for u in range(11):
                    for v in range(11):
                        wt = g[u] * g[v]
                        a, b = x[c, i + u, j + v], y[c, i + u, j + v]
                        mx += wt * a
                        my += wt * b
                        exx += wt * a * a
                        eyy += wt * b * b
                        exy += wt * a * b
                sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
                vals.append((2 * mx * my + 1e-4) * (2 * sxy + 9e-4) / ((mx * mx + my * my + 1e-4) * (sxx + syy + 9e-4)))
    assert len(vals) == 2 * 2 * 4
    assert abs(S.ssim(x, y) - np.mean(vals)) < 1e-13


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (2, 14, 16))
    y = rng.uniform(0, 1, (2, 14, 16))
    _, g = S.ssim_and_grad(x, y)
    h = 1e-6
    for c, i, j in [(0, 0, 0), (1, 7, 8), (0, 13, 15), (1, 3, 12), (0, 10, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += h
        xm[c, i, j] -= h
        fd = (S.ssim(xp, y) - S.ssim(xm, y)) / (2 * h)
        assert abs(fd - g[c, i, j]) < 1e-8 + 1e-6 * abs(fd), (c, i, j, fd, g[c, i, j])
