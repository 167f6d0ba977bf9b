"""Pins of the training-step oracles (oracle/adam.py, oracle/densify.py) to
facts outside them: Adam's closed forms and torch.optim.Adam in FP64 on the
CPU; the support radius of known covariances; the NDC scaling of the
gradient norm; a table of hand-decided densification cases.  CPU only."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import adam, densify


def test_adam_first_step_is_signed_lr():
    """With zero moments the first bias-corrected step is lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = adam.step(np.ones(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(th, 1.0 - 0.01 * g / (np.abs(g) + adam.EPS), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient_moves_lr_per_step():
    """Under a constant gradient both bias-corrected moments are exact, so
    every step moves lr * sign(g) (up to eps)."""
    g = np.array([2.0, -7.0])
    th, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, 30):
        th, m, v = adam.step(th, g, m, v, t, lr=0.5)
    np.testing.assert_allclose(th, -0.5 * 29 * np.sign(g), rtol=1e-12)


def test_adam_matches_torch_optim():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    th0 = rng.normal(size=50)
    p = torch.nn.Parameter(torch.tensor(th0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=0.003, betas=(0.9, 0.999), eps=1e-15)
    th, m, v = th0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        g = rng.normal(size=50) * (t % 3 + 0.1)
        p.grad = torch.tensor(g)
        opt.step()
        th, m, v = adam.step(th, g, m, v, t, lr=0.003)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def _one_pair_acc(g, cov, W, H, ext, visible=True):
    acc = densify.new_acc(1)
    return densify.accumulate(acc, [0], [0], [visible], np.array([g]), np.array([cov]), [W],
                              [H], ext)


def test_stats_ndc_gradient_norm():
    """A gradient of (1, 0) per pixel on a 200-wide image is 100 per NDC unit;
    (0, 1) on a 50-high one is 25."""
    acc = _one_pair_acc((1.0, 0.0), (1.0, 0.0, 1.0), 200, 50, 2.5)
    assert acc["grad"][0] == pytest.approx(100.0, rel=1e-15)
    acc = _one_pair_acc((0.0, 1.0), (1.0, 0.0, 1.0), 200, 50, 2.5)
    assert acc["grad"][0] == pytest.approx(25.0, rel=1e-15)
    acc = _one_pair_acc((3.0, 4.0), (1.0, 0.0, 1.0), 2, 2, 2.5)
    assert acc["grad"][0] == pytest.approx(5.0, rel=1e-15)


def test_stats_support_radius():
    """Diagonal covariance: r = ext * sqrt(max(a, c)); a covariance built as
    R diag(l1, l2) R^T: r = ext * sqrt(max(l1, l2)); over the larger image side."""
    acc = _one_pair_acc((0.0, 0.0), (4.0, 0.0, 9.0), 300, 100, 2.5)
    assert acc["max_extent"][0] == pytest.approx(2.5 * 3.0 / 300, rel=1e-14)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    S = R @ np.diag([16.0, 0.25]) @ R.T
    acc = _one_pair_acc((0.0, 0.0), (S[0, 0], S[0, 1], S[1, 1]), 64, 128, 1.5)
    assert acc["max_extent"][0] == pytest.approx(1.5 * 4.0 / 128, rel=1e-13)


def test_stats_visibility_and_max():
    """Three views, visible in two: count 2, gradient sums, extent the max."""
    acc = densify.new_acc(2)
    densify.accumulate(acc, [0, 0, 0, 1], [0, 1, 2, 2], [True, False, True, False],
                       np.array([[1.0, 0.0], [9.0, 9.0], [0.0, 2.0], [5.0, 5.0]]),
                       np.array([[1.0, 0.0, 1.0], [100.0, 0.0, 1.0], [4.0, 0.0, 1.0],
                                 [1.0, 0.0, 1.0]]),
                       [10, 20, 10], [10, 20, 10], 1.0)
    assert acc["count"].tolist() == [2, 0]
    assert acc["grad"][0] == pytest.approx(5.0 + 10.0)
    assert acc["max_extent"][0] == pytest.approx(2.0 / 10)
    assert acc["grad"][1] == 0 and acc["max_extent"][1] == 0


def test_select_table():
    """Each rule in isolation, with scene scale 2 and the 3DLS thresholds:
    tau_grad 2e-4, small means s <= 0.012, big means s > 0.8."""
    D, S, P = densify.DUPLICATE, densify.SPLIT, densify.PRUNE
    cases = [
        # grad sum, count, max extent, max scale, opacity, grow2d, prune_big -> action
        (3e-4, 1, 0.0, 0.01, 0.5, False, False, D),        # high, small
        (3e-4, 1, 0.0, 0.02, 0.5, False, False, S),        # high, not small
        (3e-4, 2, 0.0, 0.01, 0.5, False, False, 0),        # average 1.5e-4: low
        (2e-4, 1, 0.0, 0.01, 0.5, False, False, 0),        # not strictly above
        (0.0, 0, 0.0, 0.01, 0.5, False, False, 0),         # never visible
        (3e-4, 1, 0.06, 0.01, 0.5, True, False, S),        # big on screen: split, not duplicate
        (0.0, 1, 0.06, 0.01, 0.5, True, False, S),         # screen rule needs no gradient
        (0.0, 1, 0.06, 0.01, 0.5, False, False, 0),        # screen rule off
        (0.0, 1, 0.0, 0.01, 0.02, False, False, P),        # transparent
        (0.0, 1, 0.0, 0.01, 0.025, False, False, 0),       # at tau_op: kept
        (0.0, 1, 0.0, 0.9, 0.5, False, True, P),           # big in 3D
        (0.0, 1, 0.2, 0.01, 0.5, False, True, P),          # big on screen
        (0.0, 1, 0.2, 0.9, 0.5, False, False, 0),          # prune_big off
        (3e-4, 1, 0.0, 0.9, 0.01, False, True, S | P),     # split and pruned
    ]
    n = len(cases)
    acc = densify.new_acc(n)
    scales = np.zeros((n, 3))
    opac = np.zeros(n)
    for i, (gs, cnt, ext, s, o, *_r) in enumerate(cases):
        acc["grad"][i], acc["count"][i], acc["max_extent"][i] = gs, cnt, ext
        scales[i] = [s * 0.5, s, s * 0.25]
        opac[i] = o
    for i, (*_a, g2, pb, want) in enumerate(cases):
        got = densify.select({k: v[i:i + 1] for k, v in acc.items()}, scales[i:i + 1],
                             opac[i:i + 1], 2.0, grow2d=g2, prune_big=pb)
        assert int(got[0]) == want, (i, cases[i], int(got[0]))


def test_thresholds_match_the_table():
    assert densify.THRESH_3DLS == dict(grad=0.0002, s2g=0.05, s3g=0.006, s2p=0.15, s3p=0.4,
                                       op=0.025)
    assert densify.THRESH_3DGS["s3g"] == 0.01 and densify.THRESH_3DGS["op"] == 0.005
