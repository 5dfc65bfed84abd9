"""Pins of the oracle's D-SSIM (the object scene's loss, L1 + 0.2 D-SSIM): the window, the
constants C1 and C2, the zero padding and the per-pixel statistics, each against a value the
definition of SSIM fixes on its own (closed forms for constant and checkerboard images, a corner
pixel under zero padding, and a direct double loop over the window at sampled pixels), plus
central finite differences of the loss gradient. The paper only names an RGB difference as the
loss; the form pinned here is the 3D Gaussian Splatting one the workload uses."""
import math

import numpy as np
import pytest
import torch

import oracle

C1, C2 = 0.01 ** 2, 0.03 ** 2
SIGMA = 1.5


def _w1():
    w = oracle.gaussian_window().numpy()
    return w.sum(1)          # the 1-D factor (rows of a separable window sum to it)


def test_window_is_a_normalised_separable_gaussian_of_sigma_1_5():
    w = oracle.gaussian_window().numpy()
    assert w.shape == (11, 11)
    assert abs(w.sum() - 1.0) < 1e-15
    w1 = _w1()
    assert np.allclose(w, np.outer(w1, w1), rtol=0, atol=1e-17)
    assert np.allclose(w1, w1[::-1], rtol=0, atol=1e-18)
    # A Gaussian's neighbouring samples at x and x + 1 have the ratio exp(-(2x + 1) / (2 sigma^2)).
    x = np.arange(-5, 5)
    assert np.allclose(np.log(w1[1:] / w1[:-1]), -(2 * x + 1) / (2 * SIGMA ** 2), rtol=0, atol=1e-13)
    # Second moment: sigma^2 = 2.25 less the truncated tails beyond |x| = 5 (about 0.01 here).
    m2 = float((w1 * np.arange(-5, 6) ** 2).sum())
    assert 2.25 - 0.02 < m2 < 2.25


def test_constant_images_interior_closed_form():
    # Away from the border every window statistic of a constant image is exact: mu = the value,
    # sigma = 0, so SSIM = (2ab + C1) / (a^2 + b^2 + C1).
    a = np.array([0.2, 0.5, 0.9])
    b = np.array([0.3, 0.05, 0.9])
    x = torch.tensor(np.broadcast_to(a[:, None, None], (3, 24, 30)).copy())
    y = torch.tensor(np.broadcast_to(b[:, None, None], (3, 24, 30)).copy())
    s = oracle.ssim_map(x, y).numpy()
    want = (2 * a * b + C1) / (a * a + b * b + C1)
    interior = s[:, 5:-5, 5:-5]
    assert np.allclose(interior, want[:, None, None], rtol=1e-12, atol=0)


def test_checkerboard_against_constant_closed_form():
    # x = a everywhere, y = a + d z with z = (-1)^(i+j). At an interior pixel the window mean of
    # z is (-1)^(i+j) s with s = (sum_u w1(u) (-1)^u)^2 and z^2 = 1, so
    #   mu_y = a + d z s, sigma_y^2 = d^2 (1 - s^2), sigma_x = sigma_xy = 0,
    #   SSIM = (2 a mu_y + C1) C2 / ((a^2 + mu_y^2 + C1)(d^2 (1 - s^2) + C2)).
    a, d = 0.4, 0.03
    H, W = 22, 26
    z = (-1.0) ** (np.arange(H)[:, None] + np.arange(W)[None, :])
    x = torch.tensor(np.full((3, H, W), a))
    y = torch.tensor(np.broadcast_to(a + d * z, (3, H, W)).copy())
    w1 = _w1()
    s = float((w1 * (-1.0) ** np.arange(-5, 6)).sum()) ** 2
    mu_y = a + d * z * s
    want = (2 * a * mu_y + C1) * C2 / ((a * a + mu_y * mu_y + C1) * (d * d * (1 - s * s) + C2))
    got = oracle.ssim_map(x, y).numpy()
    assert np.allclose(got[:, 5:-5, 5:-5], want[None, 5:-5, 5:-5], rtol=1e-10, atol=0)


def test_zero_padding_at_the_corner():
    # Zero padding: at pixel (0, 0) only the quarter u, v >= 0 of the window sees the image, with
    # weight S = (sum_{u>=0} w1(u))^2. For constant images a, b:
    #   mu = a S, sigma_x^2 = a^2 S (1 - S), sigma_xy = a b S (1 - S).
    a, b = 0.7, 0.3
    x = torch.tensor(np.full((3, 16, 16), a))
    y = torch.tensor(np.full((3, 16, 16), b))
    w1 = _w1()
    S = float(w1[5:].sum()) ** 2
    mx, my = a * S, b * S
    vx, vy, cxy = a * a * S * (1 - S), b * b * S * (1 - S), a * b * S * (1 - S)
    want = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
    got = oracle.ssim_map(x, y).numpy()
    assert np.allclose(got[:, 0, 0], want, rtol=1e-12, atol=0)
    # an edge pixel (row 0, interior column): S = sum_{u>=0} w1(u)
    S = float(w1[5:].sum())
    mx, my = a * S, b * S
    vx, vy, cxy = a * a * S * (1 - S), b * b * S * (1 - S), a * b * S * (1 - S)
    want = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
    assert np.allclose(got[:, 0, 8], want, rtol=1e-12, atol=0)


def _ssim_at(x, y, c, i, j):
    """SSIM at one pixel from the definition: window-weighted means, variances and covariance of
    the two images over the 11x11 neighbourhood, pixels outside the image counting as zero."""
    H, W = x.shape[1:]
    mx = my = exx = eyy = exy = 0.0
    for u in range(-5, 6):
        for v in range(-5, 6):
            wt = math.exp(-(u * u + v * v) / (2 * SIGMA ** 2))
            p, q = i + u, j + v
            xv = x[c, p, q] if 0 <= p < H and 0 <= q < W else 0.0
            yv = y[c, p, q] if 0 <= p < H and 0 <= q < W else 0.0
            mx += wt * xv
            my += wt * yv
            exx += wt * xv * xv
            eyy += wt * yv * yv
            exy += wt * xv * yv
    norm = sum(math.exp(-(u * u) / (2 * SIGMA ** 2)) for u in range(-5, 6)) ** 2
    mx, my, exx, eyy, exy = (t / norm for t in (mx, my, exx, eyy, exy))
    vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
    return (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))


def test_direct_loop_at_sampled_pixels():
    rng = np.random.default_rng(11)
    x = rng.uniform(size=(3, 17, 19))
    y = np.clip(x + 0.1 * rng.standard_normal(x.shape), 0, 1)
    got = oracle.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    pix = [(0, 0, 0), (1, 16, 18), (2, 8, 9), (0, 3, 17), (1, 12, 2), (2, 5, 5)] + \
        [(int(rng.integers(3)), int(rng.integers(17)), int(rng.integers(19))) for _ in range(10)]
    for c, i, j in pix:
        assert abs(got[c, i, j] - _ssim_at(x, y, c, i, j)) < 1e-12, (c, i, j)
    # the loss uses the mean over all 3HW values
    assert abs(float(oracle.ssim(torch.tensor(x), torch.tensor(y))) - got.mean()) < 1e-15


@pytest.mark.parametrize("kind", ["l1", "l1_dssim"])
def test_loss_gradient_central_differences(kind):
    rng = np.random.default_rng(12)
    img = rng.uniform(0.2, 0.8, size=(3, 14, 15))
    tgt = img + rng.choice([-1.0, 1.0], size=img.shape) * rng.uniform(0.05, 0.2, size=img.shape)
    _, g = oracle.loss_and_grad(img, tgt, kind)
    h = 1e-5
    for c, i, j in [(0, 0, 0), (1, 7, 7), (2, 13, 14), (0, 4, 11), (1, 10, 1)]:
        xp, xm = img.copy(), img.copy()
        xp[c, i, j] += h
        xm[c, i, j] -= h
        fd = (oracle.loss_and_grad(xp, tgt, kind)[0] - oracle.loss_and_grad(xm, tgt, kind)[0]) / (2 * h)
        assert abs(fd - g[c, i, j]) <= 1e-7 * abs(g[c, i, j]) + 1e-12, (c, i, j, fd, g[c, i, j])
