"""The training loss of the paper's implementation section and its gradient
with respect to the rendered image (FP64; test infrastructure like the rest
of this package).

Per camera, over its 3 x H x W rendered image x and target y (N = 3 H W):
  L = 0.6 L1 + 0.2 L2 + 0.2 (1 - SSIM)
  L1 = mean |x - y|,  L2 = mean (x - y)^2,
  SSIM = mean over channels and pixels of the SSIM map of Wang et al. (2004).
The paper gives the weights (6:2:2) and the three terms but not the SSIM
window; this takes the usual one of the 3DGS lineage: an 11 x 11 Gaussian
window of sigma 1.5 normalised to sum 1, zero padding at the border (the
window sum is not renormalised there), C1 = 0.01^2 and C2 = 0.03^2 for a
data range of 1.  A batch of cameras adds its per-camera losses.  The L1
term's derivative at x = y is taken as 0.

SSIM map, with local moments over the window w:
  mx = w * x, my = w * y, sxx = w * x^2, syy = w * y^2, sxy = w * xy,
  S = (2 mx my + C1)(2 (sxy - mx my) + C2)
      / ((mx^2 + my^2 + C1)(sxx - mx^2 + syy - my^2 + C2)).
Its derivative with respect to pixel p of x collects, over the pixels q whose
window covers p, w(p - q) (dS_q/dmx + 2 x_p dS_q/dsxx + y_p dS_q/dsxy).
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

W_L1, W_L2, W_SSIM = 0.6, 0.2, 0.2
C1, C2 = 0.01 ** 2, 0.03 ** 2
WIN, SIGMA = 11, 1.5


def window() -> np.ndarray:
    """The 11 x 11 Gaussian window (outer product of the normalised 1D one)."""
    r = np.arange(WIN) - WIN // 2
    g = np.exp(-(r * r) / (2.0 * SIGMA * SIGMA))
    g = g / g.sum()
    return np.outer(g, g)


def _filt(img, w):
    return ndimage.correlate(img, w, mode="constant", cval=0.0)


def ssim_terms(x, y):
    """SSIM map and its partial derivatives dS/dmx, dS/dsxx, dS/dsxy for one
    H x W channel."""
    w = window()
    mx, my = _filt(x, w), _filt(y, w)
    sxx, syy, sxy = _filt(x * x, w), _filt(y * y, w), _filt(x * y, w)
    a1 = 2.0 * mx * my + C1
    a2 = 2.0 * (sxy - mx * my) + C2
    b1 = mx * mx + my * my + C1
    b2 = (sxx - mx * mx) + (syy - my * my) + C2
    d = b1 * b2
    S = a1 * a2 / d
    dmx = (2.0 * my * (a2 - a1) - 2.0 * mx * S * (b2 - b1)) / d
    dsxx = -S / b2
    dsxy = 2.0 * a1 / d
    return S, dmx, dsxx, dsxy


def loss_one(x, y):
    """Loss and dL/dx of one camera; x, y are [3, H, W]."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = x.size
    diff = x - y
    l1 = np.abs(diff).mean()
    l2 = (diff * diff).mean()
    w = window()
    s_sum = 0.0
    g = W_L1 * np.sign(diff) / n + W_L2 * 2.0 * diff / n
    for ch in range(x.shape[0]):
        S, dmx, dsxx, dsxy = ssim_terms(x[ch], y[ch])
        s_sum += S.sum()
        dS = _filt(dmx, w) + 2.0 * x[ch] * _filt(dsxx, w) + y[ch] * _filt(dsxy, w)
        g[ch] -= W_SSIM * dS / n
    ssim = s_sum / n
    return W_L1 * l1 + W_L2 * l2 + W_SSIM * (1.0 - ssim), g, dict(l1=l1, l2=l2, ssim=ssim)


def loss_cameras(images, targets):
    """Sum of the per-camera losses and the per-camera gradients; images and
    targets are lists of [3, H, W] arrays."""
    total = 0.0
    grads = []
    for x, y in zip(images, targets):
        l, g, _ = loss_one(x, y)
        total += l
        grads.append(g)
    return total, grads
