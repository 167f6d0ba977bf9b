"""Pins of the training-loss oracle (oracle/loss.py) to facts outside it:
finite differences of its own value, the identity SSIM(x, x) = 1, the
closed form for constant images, and a brute-force SSIM written from the
centred definition with explicit loops.  CPU only."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import loss


def test_window_is_a_normalised_gaussian():
    w = loss.window()
    assert w.shape == (11, 11)
    assert abs(w.sum() - 1.0) < 1e-15
    # separable, symmetric, ratio of neighbours exp(-(2r+1)/(2 sigma^2))
    g = w[5] / w[5].sum()
    for r in range(5):
        assert abs(g[5 + r + 1] / g[5 + r] - math.exp(-(2 * r + 1) / (2 * 1.5 ** 2))) < 1e-14
    np.testing.assert_allclose(w, np.outer(w.sum(axis=1), w.sum(axis=0)), atol=1e-16)


def test_identical_images():
    x = np.random.default_rng(1).uniform(0, 1, (3, 20, 17))
    L, g, parts = loss.loss_one(x, x)
    assert L == 0.0 and parts["ssim"] == pytest.approx(1.0, abs=1e-14)
    assert np.abs(g).max() < 1e-15


def test_constant_images_closed_form():
    """Away from the border, two constant images a, b give
    SSIM = (2ab + C1) / (a^2 + b^2 + C1) (no variance, no covariance)."""
    a, b = 0.7, 0.2
    x = np.full((40, 40), a)
    y = np.full((40, 40), b)
    S = loss.ssim_terms(x, y)[0]
    expect = (2 * a * b + loss.C1) / (a * a + b * b + loss.C1)
    np.testing.assert_allclose(S[5:-5, 5:-5], expect, rtol=1e-12)
    L, _, parts = loss.loss_one(np.stack([x] * 3), np.stack([y] * 3))
    assert parts["l1"] == pytest.approx(0.5, abs=1e-15)
    assert parts["l2"] == pytest.approx(0.25, abs=1e-15)


def test_ssim_against_centred_bruteforce():
    """SSIM map from explicit loops over each pixel's zero-padded window with
    the centred variance and covariance, against the moment form."""
    rng = np.random.default_rng(2)
    H, W = 9, 14
    x, y = rng.uniform(0, 1, (H, W)), rng.uniform(0, 1, (H, W))
    w = loss.window()
    xp, yp = np.pad(x, 5), np.pad(y, 5)
    S = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            wx, wy = xp[i:i + 11, j:j + 11], yp[i:i + 11, j:j + 11]
            mx, my = (w * wx).sum(), (w * wy).sum()
            vx, vy = (w * (wx - mx) ** 2).sum(), (w * (wy - my) ** 2).sum()
            cxy = (w * (wx - mx) * (wy - my)).sum()
            S[i, j] = ((2 * mx * my + loss.C1) * (2 * cxy + loss.C2) /
                       ((mx * mx + my * my + loss.C1) * (vx + vy + loss.C2)))
    np.testing.assert_allclose(loss.ssim_terms(x, y)[0], S, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("seed", [0, 3])
def test_gradient_against_finite_differences(seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (3, 8, 12))
    y = rng.uniform(0, 1, (3, 8, 12))
    _, g, _ = loss.loss_one(x, y)
    h = 1e-6
    fd = np.zeros_like(x)
    for idx in np.ndindex(x.shape):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd[idx] = (loss.loss_one(xp, y)[0] - loss.loss_one(xm, y)[0]) / (2 * h)
    assert np.abs(fd - g).max() < 1e-8 * max(1.0, np.abs(g).max()) + 1e-9


def test_crop_gradient_is_exact():
    """The full-size GPU test samples the oracle's gradient through crops
    reaching two window radii around a pixel; on a small image that agrees
    with the whole-image gradient, at the border as well as inside."""
    from tests.test_gpu_loss import _crop_grad
    rng = np.random.default_rng(4)
    x, y = rng.uniform(0, 1, (3, 40, 57)), rng.uniform(0, 1, (3, 40, 57))
    _, g, _ = loss.loss_one(x, y)
    for py, px in [(0, 0), (39, 56), (20, 30), (3, 50), (12, 11)]:
        np.testing.assert_allclose(_crop_grad(x, y, py, px, x.size), g[:, py, px],
                                   rtol=1e-12, atol=1e-18)
