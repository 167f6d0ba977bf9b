"""Front-to-back compositing with the linear kernel (or another kernel of the
family in the appendix), and its reverse pass.

For a pixel centre x and a splat with projected centre mu', inverse 2D
covariance ("conic") and opacity o:
  D'  = sqrt((x - mu')^T Sigma_2D^-1 (x - mu'))            Eq. 11
  L'  = max(0, 1 - D'/lambda)                               Eq. 10 with DA, Eq. 12
        (another kernel: f(D'/lambda), cut at D' = extent, config.py)
  alpha = min(alpha_max, o * L')                            Eq. 6 (alpha = o * kernel)
  C(x) = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j)         Eq. 6
The splats are taken in the order of the pixel's tile list (binning.py).
Blending rules the paper keeps from 3DGS without printing them (Sec. 3.2):
a splat with alpha <= 0 or alpha < alpha_min is skipped; a splat that would
take the transmittance T below t_min stops the pixel and is not added.  The
output is C + T_final * bg.

The reverse pass differentiates that composite (Sec. 4.1 names a hand-written
backward kernel; Sec. 3.3.2, Eq. 13-14, adds the adaptive gradient scaling
omega(D') = exp(-D'^2) applied to the gradient through L').
"""
from __future__ import annotations

import numpy as np

from .config import extent

CHUNK = 512
FLAG_REL = 1e-4


def _tile_pixels(tx, ty, width, height, cfg):
    x0, y0 = tx * cfg.tile_w, ty * cfg.tile_h
    xs = np.arange(x0, min(x0 + cfg.tile_w, width))
    ys = np.arange(y0, min(y0 + cfg.tile_h, height))
    py, px = np.meshgrid(ys, xs, indexing="ij")
    return px.ravel(), py.ravel()


def kernel_value(q, cfg):
    """f(D'/lambda) of the configured kernel at q = D'^2 (a negative q, from
    rounding at a splat's centre, counts as 0), zero from the support cut
    q >= extent^2 on.  Returns (D', f)."""
    q = np.maximum(np.asarray(q, np.float64), 0.0)
    D = np.sqrt(q)
    lam = cfg.lambda_
    x = D / lam
    k = cfg.kernel
    if k == "linear":
        f = 1.0 - x
    elif k == "gaussian":
        f = np.exp(-q / (2.0 * lam * lam))
    elif k == "laplacian":
        f = np.exp(-x)
    elif k == "cosine":
        f = 0.5 * (1.0 + np.cos(np.pi * np.minimum(x, 1.0)))
    else:   # quadratic
        f = 1.0 - q / (lam * lam)
    e = extent(cfg)
    f = np.where(q < e * e, np.maximum(f, 0.0), 0.0)
    return D, f


def kernel_slope(D, f, cfg):
    """df/dq inside the support (q = D'^2), from D' and f.  Where f is not
    differentiable in q (the centre of the kernels with a cusp or a sqrt, and
    every point outside the support) the slope is 0."""
    D = np.asarray(D, np.float64)
    lam = cfg.lambda_
    k = cfg.kernel
    inside = f > 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        if k == "linear":
            g = np.where(D > 0.0, -1.0 / (2.0 * lam * D), 0.0)
        elif k == "gaussian":
            g = -f / (2.0 * lam * lam)
        elif k == "laplacian":
            g = np.where(D > 0.0, -f / (2.0 * lam * D), 0.0)
        elif k == "cosine":
            g = np.where(D > 0.0, -np.pi * np.sin(np.pi * D / lam) / (4.0 * lam * D), 0.0)
        else:   # quadratic
            g = np.full(D.shape, -1.0 / (lam * lam))
    return np.where(inside, g, 0.0)


def _pair_terms(px, py, mean2d, conic, opac, cfg):
    """Per (pixel, splat) quantities, all FP64: dx, dy, D, L' (the kernel value
    f), o*L', alpha."""
    dx = (px[:, None] + 0.5) - mean2d[None, :, 0]
    dy = (py[:, None] + 0.5) - mean2d[None, :, 1]
    A, B, C = conic[None, :, 0], conic[None, :, 1], conic[None, :, 2]
    q = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy
    D, L = kernel_value(q, cfg)
    raw = opac[None, :] * L
    alpha = np.minimum(cfg.alpha_max, raw)
    return dx, dy, D, L, raw, alpha


def composite_tile(ids, px, py, mean2d, conic, opac, rgb, cfg, want_pairs=False):
    """Composite the pixels (px, py) of one tile over its sorted splat list
    ``ids`` (indices into the per-camera arrays).

    Returns dict with C [P,3], T [P], last [P] (1 + position in ``ids`` of the
    last contributing splat, 0 if none), flag [P] (some skip/stop decision of
    that pixel lies within a relative margin FLAG_REL of its threshold),
    jump [P] (a bound on how far the pixel's colour can move if those
    decisions went the other way, in units of max|colour - background|: the
    transmittance-weighted alpha alpha T of every splat whose skip or stop
    decision is flagged, plus t_min for a flagged stop, after which the rest
    of the list adds less than t_min; the alpha clamp is continuous and adds
    nothing) and, if ``want_pairs``, the per-pair arrays of contributing pairs
    for the reverse pass.
    """
    P = len(px)
    C = np.zeros((P, 3))
    T = np.ones(P)
    last = np.zeros(P, np.int64)
    flag = np.zeros(P, bool)
    jump = np.zeros(P)
    done = np.zeros(P, bool)
    amin, amax, tmin = cfg.alpha_min, cfg.alpha_max, cfg.t_min
    pairs = []
    for k0 in range(0, len(ids), CHUNK):
        if done.all():
            break
        sl = ids[k0:k0 + CHUNK]
        dx, dy, D, L, raw, alpha = _pair_terms(px, py, mean2d[sl], conic[sl], opac[sl], cfg)
        valid = (alpha > 0.0) & (alpha >= amin) & ~done[:, None]
        a_eff = np.where(valid, alpha, 0.0)
        Tincl = T[:, None] * np.cumprod(1.0 - a_eff, axis=1)      # T after each pair
        stop = valid & (Tincl < tmin)
        has_stop = stop.any(axis=1)
        s_idx = np.where(has_stop, np.argmax(stop, axis=1), len(sl))
        kk = np.arange(len(sl))[None, :]
        contrib = valid & (kk < s_idx[:, None])
        Texcl = np.concatenate([T[:, None], Tincl[:, :-1]], axis=1)  # T before each pair
        w = np.where(contrib, a_eff * Texcl, 0.0)
        C += w @ rgb[sl]
        # decision margins, up to and including the stopping pair
        upto = (kk <= s_idx[:, None]) & ~done[:, None]
        m = upto & (raw > 0.0)
        if amin > 0:
            fa = m & (np.abs(alpha - amin) < FLAG_REL * amin)
            flag |= fa.any(axis=1)
            jump += np.sum(np.where(fa, alpha * Texcl, 0.0), axis=1)
        flag |= (m & (np.abs(raw - amax) < FLAG_REL * amax)).any(axis=1)
        if tmin > 0:
            ft = upto & valid & (np.abs(Tincl - tmin) < FLAG_REL * tmin)
            flag |= ft.any(axis=1)
            jump += np.sum(np.where(ft, alpha * Texcl + tmin, 0.0), axis=1)
        if cfg.kernel == "gaussian":
            # the 3-sigma cut is a jump of alpha (o * e^-4.5)
            e2 = extent(cfg) ** 2
            fg = upto & (np.abs(D * D - e2) < FLAG_REL * e2)
            flag |= fg.any(axis=1)
            a_cut = opac[sl][None, :] * kernel_value(e2 * (1.0 - FLAG_REL), cfg)[1]
            jump += np.sum(np.where(fg, np.minimum(amax, a_cut) * Texcl, 0.0), axis=1)
        any_c = contrib.any(axis=1)
        last_local = np.where(any_c, len(sl) - np.argmax(contrib[:, ::-1], axis=1), 0)
        last = np.where(any_c, k0 + last_local, last)
        # transmittance after the last contributing pair of this chunk
        idx_last = np.where(any_c, last_local - 1, 0)
        T = np.where(any_c, Tincl[np.arange(P), idx_last], T)
        if want_pairs:
            pp, kk2 = np.nonzero(contrib)
            pairs.append(dict(p=pp, k=kk2 + k0, id=sl[kk2], dx=dx[pp, kk2], dy=dy[pp, kk2],
                              D=D[pp, kk2], L=L[pp, kk2], raw=raw[pp, kk2],
                              alpha=alpha[pp, kk2], Tb=Texcl[pp, kk2]))
        done |= has_stop
    out = dict(C=C, T=T, last=last, flag=flag, jump=jump)
    if want_pairs:
        if pairs:
            out["pairs"] = {k: np.concatenate([d[k] for d in pairs]) for k in pairs[0]}
        else:
            out["pairs"] = None
    return out


def reverse_tile(res, G, mean2d, conic, opac, rgb, cfg, n_splats, GA=None):
    """Reverse pass over one tile's contributing pairs.

    G [P,3] = dL/d(image) at the tile's pixels; GA [P] (optional) = dL/dA for
    the accumulated opacity A = 1 - T_final = 1 - prod_i (1 - alpha_i), whose
    derivative w.r.t. alpha_i is T_final / (1 - alpha_i).  Returns per-splat arrays
    (length n_splats) g_rgb [.,3], g_opac [.], g_conic [.,3] (w.r.t. A, B, C),
    g_mean2d [.,2]."""
    g_rgb = np.zeros((n_splats, 3))
    g_o = np.zeros(n_splats)
    g_con = np.zeros((n_splats, 3))
    g_mu = np.zeros((n_splats, 2))
    pr = res["pairs"]
    if pr is None:
        return g_rgb, g_o, g_con, g_mu
    bg = np.asarray(cfg.bg, np.float64)
    # order pairs by (pixel, list position) to form the suffix sums per pixel
    order = np.lexsort((pr["k"], pr["p"]))
    p, ids = pr["p"][order], pr["id"][order]
    alpha, Tb = pr["alpha"][order], pr["Tb"][order]
    c_i = rgb[ids]
    contrib = c_i * (alpha * Tb)[:, None]
    # suffix within each pixel: S_i = sum_{j > i, same pixel} contrib_j + T_final bg
    csum = np.cumsum(contrib[::-1], axis=0)[::-1]
    # subtract each pixel's tail beyond its own block
    starts = np.r_[0, np.nonzero(np.diff(p))[0] + 1]
    ends = np.r_[starts[1:], len(p)]
    blk_end = np.repeat(ends, ends - starts)
    tail = np.vstack([csum, np.zeros((1, 3))])[blk_end]
    S = csum - contrib - tail + res["T"][p][:, None] * bg[None, :]
    Gp = G[p]
    dL_drgb = Gp * (alpha * Tb)[:, None]
    dL_dalpha = Tb * np.sum(Gp * c_i, axis=1) - np.sum(Gp * S, axis=1) / (1.0 - alpha)
    if GA is not None:
        dL_dalpha = dL_dalpha + np.asarray(GA, np.float64)[p] * res["T"][p] / (1.0 - alpha)
    raw, L, D = pr["raw"][order], pr["L"][order], pr["D"][order]
    unclamped = raw < cfg.alpha_max
    dL_do = np.where(unclamped, L * dL_dalpha, 0.0)
    dL_dL = np.where(unclamped, opac[ids] * dL_dalpha, 0.0)
    dL_dq = dL_dL * kernel_slope(D, L, cfg)
    if cfg.ags:
        arg = D if cfg.ags_arg == 0 else D / cfg.lambda_
        omega = np.exp(-arg * arg)
        dL_dq = dL_dq * omega
        if cfg.ags_scope == 1:
            dL_drgb = dL_drgb * omega[:, None]
            dL_do = dL_do * omega
    dx, dy = pr["dx"][order], pr["dy"][order]
    A, B, C = conic[ids, 0], conic[ids, 1], conic[ids, 2]
    gc = np.stack([dL_dq * dx * dx, dL_dq * 2.0 * dx * dy, dL_dq * dy * dy], axis=1)
    gm = np.stack([-2.0 * dL_dq * (A * dx + B * dy), -2.0 * dL_dq * (B * dx + C * dy)], axis=1)
    np.add.at(g_rgb, ids, dL_drgb)
    np.add.at(g_o, ids, dL_do)
    np.add.at(g_con, ids, gc)
    np.add.at(g_mu, ids, gm)
    return g_rgb, g_o, g_con, g_mu


def composite_bruteforce(width, height, order, mean2d, conic, opac, rgb, cfg):
    """Untiled composite by plain per-pixel loops over ``order`` (all visible
    splats of the camera in depth order).  For small cases only."""
    C = np.zeros((height, width, 3))
    Tout = np.ones((height, width))
    for py in range(height):
        for px in range(width):
            T = 1.0
            acc = np.zeros(3)
            for i in order:
                dx = px + 0.5 - mean2d[i, 0]
                dy = py + 0.5 - mean2d[i, 1]
                q = conic[i, 0] * dx * dx + 2.0 * conic[i, 1] * dx * dy + conic[i, 2] * dy * dy
                a = min(cfg.alpha_max, opac[i] * float(kernel_value(q, cfg)[1]))
                if a <= 0.0 or a < cfg.alpha_min:
                    continue
                Tn = T * (1.0 - a)
                if Tn < cfg.t_min:
                    break
                acc += rgb[i] * a * T
                T = Tn
            C[py, px] = acc
            Tout[py, px] = T
    return C, Tout
