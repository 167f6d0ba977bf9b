"""FP64 projection of splats into one camera, and its reverse pass.

Forward (Sec. 3.1):
  Eq. 2   Sigma = R S S^T R^T, R from the normalised quaternion, S = diag(scale)
  Eq. 3   Sigma' = J W Sigma W^T J^T with W the world-to-camera rotation and J
          the local affine Jacobian of the pinhole map at the splat centre
  Eq. 4   Sigma_2D = top-left 2x2 block of Sigma'
  Eq. 5/11 use Sigma_2D^-1 (the "conic") in the 2D Mahalanobis distance.
Not in the paper (3DGS framework it keeps): Sigma_2D is dilated by eps2d on its
diagonal, the tangent used in J is clamped to clip x the half field of view,
and the colour is the degree <= 3 SH expansion + 0.5, clamped at 0.

All inputs are the FP32 arrays, upcast to FP64; every step below runs in FP64.
"""
from __future__ import annotations

import numpy as np

from . import sh as shmod


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrix [..., 3, 3] of unit quaternions q = (w, x, y, z)."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1 - 2 * (y * y + z * z)
    r[..., 0, 1] = 2 * (x * y - w * z)
    r[..., 0, 2] = 2 * (x * z + w * y)
    r[..., 1, 0] = 2 * (x * y + w * z)
    r[..., 1, 1] = 1 - 2 * (x * x + z * z)
    r[..., 1, 2] = 2 * (y * z - w * x)
    r[..., 2, 0] = 2 * (x * z - w * y)
    r[..., 2, 1] = 2 * (y * z + w * x)
    r[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def _camera(viewmat, intrin):
    vm = np.asarray(viewmat, np.float64)
    fx, fy, cx, cy = (float(v) for v in np.asarray(intrin, np.float64))
    return vm[:, :3], vm[:, 3], fx, fy, cx, cy


def project(means, scales, quats, sh, sh_degree, viewmat, intrin, width, height, cfg):
    """Project splats into one camera.  Returns a dict of FP64 arrays:

    t [N,3] camera-space centre; mean2d [N,2]; cov2d [N,3] (a, b, c) of the
    dilated Sigma_2D = [[a, b], [b, c]]; conic [N,3] (A, B, C) of its inverse so
    that D'^2 = A dx^2 + 2 B dx dy + C dy^2; rgb [N,3]; plus intermediates
    (R, Sigma, T, unclipped masks, SH direction) used by the reverse pass.
    Culling is not decided here (the FP32 binning sequence decides it).
    """
    mu = np.asarray(means, np.float64)
    s = np.asarray(scales, np.float64)
    q = np.asarray(quats, np.float64)
    qn = np.linalg.norm(q, axis=-1, keepdims=True)
    qh = q / qn
    R = quat_to_rot(qh)
    M = R * s[:, None, :]                    # M = R diag(s)
    Sigma = M @ np.swapaxes(M, 1, 2)          # Eq. 2

    Wr, tv, fx, fy, cx, cy = _camera(viewmat, intrin)
    t = mu @ Wr.T + tv
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    mean2d = np.stack([fx * tx / tz + cx, fy * ty / tz + cy], axis=-1)

    clip = float(cfg.clip)
    limx = clip * 0.5 * float(width) / fx
    limy = clip * 0.5 * float(height) / fy
    u, v = tx / tz, ty / tz
    uc, vc = np.clip(u, -limx, limx), np.clip(v, -limy, limy)
    J = np.zeros((len(mu), 2, 3))
    J[:, 0, 0] = fx / tz
    J[:, 0, 2] = -fx * uc / tz
    J[:, 1, 1] = fy / tz
    J[:, 1, 2] = -fy * vc / tz
    T = J @ Wr                                 # J W  (Eq. 3)
    cov = T @ Sigma @ np.swapaxes(T, 1, 2)     # top-left 2x2 block (Eq. 4)
    eps = float(cfg.eps2d)
    a = cov[:, 0, 0] + eps
    b = 0.5 * (cov[:, 0, 1] + cov[:, 1, 0])
    c = cov[:, 1, 1] + eps
    det = a * c - b * b
    conic = np.stack([c / det, -b / det, a / det], axis=-1)

    campos = -Wr.T @ tv
    vdir = mu - campos
    dist = np.linalg.norm(vdir, axis=-1, keepdims=True)
    d = vdir / dist
    Y = shmod.basis(d, sh_degree)              # [N, K]
    shc = np.asarray(sh, np.float64)[:, : Y.shape[1], :]
    raw = np.einsum("nk,nkc->nc", Y, shc) + 0.5
    rgb = np.maximum(raw, 0.0)
    return dict(t=t, mean2d=mean2d, cov2d=np.stack([a, b, c], -1), conic=conic,
                rgb=rgb, rgb_raw=raw, R=R, M=M, Sigma=Sigma, T=T, J=J,
                u_free=np.abs(u) < limx, v_free=np.abs(v) < limy, uc=uc, vc=vc,
                qh=qh, qn=qn[:, 0], d=d, dist=dist[:, 0], Y=Y, Wr=Wr,
                fx=fx, fy=fy, scales=s)


def cov2d_grad(conic, g_conic):
    """Gradient w.r.t. the 2D covariance (a, b, c of [[a, b], [b, c]], b one
    parameter) from the gradient w.r.t. the conic (A, B, C) = its inverse:
    for a symmetric matrix and its inverse, dL/dcov = -conic (dL/dconic) conic,
    with the off-diagonal gradient split over both slots."""
    n = len(conic)
    A, B, C = conic[:, 0], conic[:, 1], conic[:, 2]
    conm = np.empty((n, 2, 2))
    conm[:, 0, 0], conm[:, 0, 1], conm[:, 1, 0], conm[:, 1, 1] = A, B, B, C
    gcm = np.empty((n, 2, 2))
    gcm[:, 0, 0] = g_conic[:, 0]
    gcm[:, 0, 1] = gcm[:, 1, 0] = 0.5 * g_conic[:, 1]
    gcm[:, 1, 1] = g_conic[:, 2]
    gcov = -conm @ gcm @ conm
    return np.stack([gcov[:, 0, 0], 2.0 * gcov[:, 0, 1], gcov[:, 1, 1]], axis=1)


def project_backward(p, sh, sh_degree, g_mean2d, g_conic, g_rgb):
    """Chain rule from per-pair 2D gradients to splat parameters.

    g_mean2d [N,2]; g_conic [N,3] w.r.t. (A, B, C) with D'^2 = A dx^2 +
    2 B dx dy + C dy^2; g_rgb [N,3].  Returns (g_means [N,3], g_scales [N,3],
    g_quats [N,4], g_sh [N,K,3]).  Opacity passes straight through.
    """
    return project_backward_cov(p, sh, sh_degree, g_mean2d, cov2d_grad(p["conic"], g_conic),
                                g_rgb)


def project_backward_cov(p, sh, sh_degree, g_mean2d, gc, g_rgb):
    """project_backward with the 2D shape gradient given w.r.t. the dilated
    covariance (a, b, c of [[a, b], [b, c]], b one parameter)."""
    n = len(p["t"])
    gcov = np.empty((n, 2, 2))
    gcov[:, 0, 0] = gc[:, 0]
    gcov[:, 0, 1] = gcov[:, 1, 0] = 0.5 * gc[:, 1]
    gcov[:, 1, 1] = gc[:, 2]
    T, Sigma, Wr = p["T"], p["Sigma"], p["Wr"]
    g_T = 2.0 * gcov @ T @ Sigma
    g_Sigma = np.swapaxes(T, 1, 2) @ gcov @ T
    g_J = g_T @ Wr.T                           # T = J W
    tx, ty, tz = p["t"][:, 0], p["t"][:, 1], p["t"][:, 2]
    fx, fy = p["fx"], p["fy"]
    g_t = np.zeros((n, 3))
    # J00 = fx/tz, J11 = fy/tz
    g_t[:, 2] += g_J[:, 0, 0] * (-fx / tz**2) + g_J[:, 1, 1] * (-fy / tz**2)
    # J02 = -fx u'/tz with u' = tx/tz when unclipped, else constant
    uf, vf = p["u_free"], p["v_free"]
    g_t[:, 0] += np.where(uf, g_J[:, 0, 2] * (-fx / tz**2), 0.0)
    g_t[:, 2] += np.where(uf, g_J[:, 0, 2] * (2 * fx * tx / tz**3),
                          g_J[:, 0, 2] * (fx * p["uc"] / tz**2))
    g_t[:, 1] += np.where(vf, g_J[:, 1, 2] * (-fy / tz**2), 0.0)
    g_t[:, 2] += np.where(vf, g_J[:, 1, 2] * (2 * fy * ty / tz**3),
                          g_J[:, 1, 2] * (fy * p["vc"] / tz**2))
    # mean2d = (fx tx/tz + cx, fy ty/tz + cy)
    g_t[:, 0] += g_mean2d[:, 0] * fx / tz
    g_t[:, 1] += g_mean2d[:, 1] * fy / tz
    g_t[:, 2] += -g_mean2d[:, 0] * fx * tx / tz**2 - g_mean2d[:, 1] * fy * ty / tz**2
    g_means = g_t @ Wr                          # t = W mu + t_w

    # Sigma = M M^T, M = R diag(s)
    M, R, s = p["M"], p["R"], p["scales"]
    g_M = 2.0 * g_Sigma @ M
    g_scales = np.einsum("nrc,nrc->nc", g_M, R)
    g_R = g_M * s[:, None, :]
    w, x, y, z = (p["qh"][:, i] for i in range(4))
    G = g_R
    g_qh = np.stack([
        2 * (-z * G[:, 0, 1] + y * G[:, 0, 2] + z * G[:, 1, 0] - x * G[:, 1, 2]
             - y * G[:, 2, 0] + x * G[:, 2, 1]),
        2 * (y * G[:, 0, 1] + z * G[:, 0, 2] + y * G[:, 1, 0] - 2 * x * G[:, 1, 1]
             - w * G[:, 1, 2] + z * G[:, 2, 0] + w * G[:, 2, 1] - 2 * x * G[:, 2, 2]),
        2 * (-2 * y * G[:, 0, 0] + x * G[:, 0, 1] + w * G[:, 0, 2] + x * G[:, 1, 0]
             + z * G[:, 1, 2] - w * G[:, 2, 0] + z * G[:, 2, 1] - 2 * y * G[:, 2, 2]),
        2 * (-2 * z * G[:, 0, 0] - w * G[:, 0, 1] + x * G[:, 0, 2] + w * G[:, 1, 0]
             - 2 * z * G[:, 1, 1] + y * G[:, 1, 2] + x * G[:, 2, 0] + y * G[:, 2, 1]),
    ], axis=-1)
    qh = p["qh"]
    g_quats = (g_qh - qh * np.sum(qh * g_qh, -1, keepdims=True)) / p["qn"][:, None]

    # colour: rgb = max(0, sum_k Y_k(d) sh_k + 0.5), d = (mu - campos)/|mu - campos|
    live = p["rgb_raw"] > 0.0
    g_raw = np.where(live, g_rgb, 0.0)
    Y = p["Y"]
    g_sh = Y[:, :, None] * g_raw[:, None, :]
    dY = shmod.basis_grad(p["d"], sh_degree)    # [N, K, 3]
    shc = np.asarray(sh, np.float64)[:, : Y.shape[1], :]
    g_d = np.einsum("nc,nkc,nkj->nj", g_raw, shc, dY)
    d = p["d"]
    g_v = (g_d - d * np.sum(d * g_d, -1, keepdims=True)) / p["dist"][:, None]
    g_means = g_means + g_v
    return g_means, g_scales, g_quats, g_sh
