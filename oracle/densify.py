"""Densification statistics and the grow / prune decision with the paper's
3DLS thresholds (implementation section, densification-threshold table), in
FP64.  Test infrastructure like the rest of this package.

The paper changes only the thresholds of the 3DGS procedure (Kerbl et al.
2023, adaptive density control) and names six of them: the gradient
threshold, 2D and 3D grow thresholds, 2D and 3D prune thresholds and the
opacity prune threshold.  This follows the usual reading of those names:

Statistics, per splat i, accumulated over every (camera, splat) pair in
which the splat is visible (its support touches at least one tile):
  grad[i]        += |(dL/dx * W/2, dL/dy * H/2)|, the norm of the gradient of
                    the projected centre in normalised device coordinates
                    (x spans W pixels over 2 NDC units),
  count[i]       += 1,
  max_extent[i]   = max(max_extent[i], r / max(W, H)), r the semi-major axis
                    of the support ellipse in pixels: extent * sqrt(lambda_max)
                    of the (dilated) 2D covariance, extent the kernel's
                    support radius in D' units (lambda for the linear kernel).

Decision, per splat, with s = max of its three scales and S the scene scale:
  high      = grad / count > tau_grad (false when count = 0)
  small     = s <= tau_s3g * S
  split     = (high and not small) or (grow2d and max_extent > tau_s2g)
  duplicate = high and small and not split
  prune     = opacity < tau_op, or (prune_big and (s > tau_s3p * S or
              max_extent > tau_s2p))
grow2d and prune_big switch the screen-size rules on (the training schedule
decides when).  Applying the decision (drawing children, compacting) belongs
to the training loop.
"""
from __future__ import annotations

import numpy as np

THRESH_3DLS = dict(grad=0.0002, s2g=0.05, s3g=0.006, s2p=0.15, s3p=0.4, op=0.025)
THRESH_3DGS = dict(grad=0.0002, s2g=0.05, s3g=0.01, s2p=0.15, s3p=0.1, op=0.005)

DUPLICATE, SPLIT, PRUNE = 1, 2, 4


def new_acc(n):
    return dict(grad=np.zeros(n), count=np.zeros(n, np.int64), max_extent=np.zeros(n))


def accumulate(acc, splat_of_pair, cam_of_pair, visible, g_mean2d, cov2d, widths, heights,
               ext):
    """Add one backward pass's statistics.  Per pair m: its splat and camera,
    visibility, dL/d(projected centre) [M, 2] in pixels and the dilated 2D
    covariance [M, 3] as (a, b, c) of [[a, b], [b, c]]; ext is the kernel's
    support radius in D' units."""
    for m in range(len(splat_of_pair)):
        if not visible[m]:
            continue
        i, c = int(splat_of_pair[m]), int(cam_of_pair[m])
        W, H = float(widths[c]), float(heights[c])
        gx, gy = float(g_mean2d[m][0]), float(g_mean2d[m][1])
        acc["grad"][i] += np.hypot(gx * W / 2.0, gy * H / 2.0)
        acc["count"][i] += 1
        a, b, cc = (float(v) for v in cov2d[m])
        lam = np.linalg.eigvalsh(np.array([[a, b], [b, cc]]))[-1]
        r = ext * np.sqrt(lam)
        acc["max_extent"][i] = max(acc["max_extent"][i], r / max(W, H))
    return acc


def select(acc, scales, opacity, scene_scale, th=THRESH_3DLS, grow2d=False, prune_big=False):
    """Action bits per splat: DUPLICATE, SPLIT, PRUNE.  scales [N, 3],
    opacity [N] (activated)."""
    n = len(opacity)
    out = np.zeros(n, np.uint8)
    for i in range(n):
        cnt = int(acc["count"][i])
        high = cnt > 0 and acc["grad"][i] / cnt > th["grad"]
        s = float(np.max(scales[i]))
        small = s <= th["s3g"] * scene_scale
        ext = float(acc["max_extent"][i])
        split = (high and not small) or (grow2d and ext > th["s2g"])
        if split:
            out[i] |= SPLIT
        elif high and small:
            out[i] |= DUPLICATE
        if opacity[i] < th["op"] or (prune_big and (s > th["s3p"] * scene_scale or ext > th["s2p"])):
            out[i] |= PRUNE
    return out
