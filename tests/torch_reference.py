"""A second, differentiable transcription of the forward pass in PyTorch FP64,
used only to pin the oracle's hand-derived reverse pass against autograd.

Untiled and unsorted-by-tile: every visible splat is evaluated at every pixel
in depth order.  Strict blending only (no alpha floor, no early stop), so the
composite is a smooth function of the parameters away from kinks.
"""
from __future__ import annotations

import math

import torch

SQ = math.sqrt
PI = math.pi


def sh_basis(d, degree):
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    c0 = 1.0 / (2.0 * SQ(PI))
    out = [torch.full_like(x, c0)]
    if degree >= 1:
        c1 = SQ(3.0 / (4.0 * PI))
        out += [-c1 * y, c1 * z, -c1 * x]
    if degree >= 2:
        a, b, c = SQ(15.0 / PI) / 2, SQ(5.0 / PI) / 4, SQ(15.0 / PI) / 4
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, c * (x * x - y * y)]
    if degree >= 3:
        a, b, c = SQ(35.0 / (2 * PI)) / 4, SQ(105.0 / PI) / 2, SQ(21.0 / (2 * PI)) / 4
        d3, e = SQ(7.0 / PI) / 4, SQ(105.0 / PI) / 4
        out += [-a * y * (3 * x * x - y * y), b * x * y * z, -c * y * (4 * z * z - x * x - y * y),
                d3 * z * (2 * z * z - 3 * x * x - 3 * y * y), -c * x * (4 * z * z - x * x - y * y),
                e * z * (x * x - y * y), -a * x * (x * x - 3 * y * y)]
    return torch.stack(out, dim=1)


def render(means, scales, quats, opac, sh, degree, viewmat, intrin, W, H, order,
           lam=2.5, eps=0.3, clip=1.3, alpha_max=0.99, ags=False, ags_arg=0, ags_scope=0):
    """Image [3, H, W] for one camera.  ``order`` lists the visible splats in
    depth order.

    Adaptive gradient scaling (ags) leaves the value unchanged and multiplies
    gradients by omega per (pixel, splat) pair, written as
    v.detach() + omega (v - v.detach()): with ags_scope 0 on the kernel value
    L' (the geometric path only), with ags_scope 1 on alpha and on the pair's
    colour weight (every gradient of the pair)."""
    q = quats / quats.norm(dim=1, keepdim=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)
    Mm = R * scales[:, None, :]
    Sig = Mm @ Mm.transpose(1, 2)
    Wr, tv = viewmat[:, :3], viewmat[:, 3]
    t = means @ Wr.T + tv
    fx, fy, cx, cy = intrin
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    mx = fx * tx / tz + cx
    my = fy * ty / tz + cy
    limx = clip * 0.5 * W / fx
    limy = clip * 0.5 * H / fy
    uc = torch.clamp(tx / tz, -limx, limx)
    vc = torch.clamp(ty / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * uc / tz], 1),
                     torch.stack([zero, fy / tz, -fy * vc / tz], 1)], 1)
    T = J @ Wr
    cov = T @ Sig @ T.transpose(1, 2)
    a = cov[:, 0, 0] + eps
    b = cov[:, 0, 1]
    c = cov[:, 1, 1] + eps
    det = a * c - b * b
    A, B, Cc = c / det, -b / det, a / det
    campos = -Wr.T @ tv
    v = means - campos
    d = v / v.norm(dim=1, keepdim=True)
    Y = sh_basis(d, degree)
    rgb = torch.clamp((Y[:, :, None] * sh[:, : Y.shape[1], :]).sum(1) + 0.5, min=0.0)

    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64), torch.arange(W, dtype=torch.float64),
                            indexing="ij")
    px = xs.reshape(-1) + 0.5
    py = ys.reshape(-1) + 0.5
    o = order
    dx = px[:, None] - mx[o][None, :]
    dy = py[:, None] - my[o][None, :]
    qf = A[o] * dx * dx + 2 * B[o] * dx * dy + Cc[o] * dy * dy
    D = torch.sqrt(torch.clamp(qf, min=1e-300))
    L = torch.clamp(1 - D / lam, min=0.0)
    om = None
    if ags:
        arg = D if ags_arg == 0 else D / lam
        om = torch.exp(-arg * arg).detach()
        if ags_scope == 0:
            L = L.detach() + om * (L - L.detach())
    alpha = torch.clamp(opac[o][None, :] * L, max=alpha_max)
    if ags and ags_scope == 1:
        alpha = alpha.detach() + om * (alpha - alpha.detach())
    one = 1 - alpha
    Tb = torch.cat([torch.ones_like(one[:, :1]), torch.cumprod(one, dim=1)[:, :-1]], dim=1)
    wgt = alpha * Tb
    col = rgb[o]
    if ags and ags_scope == 1:
        img = wgt @ col.detach() + (wgt.detach() * om) @ (col - col.detach())
    else:
        img = wgt @ col
    return img.T.reshape(3, H, W)
