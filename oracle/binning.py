"""Tile binning: the FP32 operation sequence that decides every integer
output, the intersection list, its (tile, depth) order and the tile ranges.

The paper does not describe binning (it keeps the 3DGS pipeline, Sec. 3.2 and
Sec. 4.1).  An FP64 oracle cannot reproduce FP32 integer decisions by luck, so
the rectangle of tiles a splat touches and its depth key are *defined* by the
FP32 sequence below: each arithmetic operation rounds to FP32
(round-to-nearest-even, no fused multiply-add), parentheses fix the order,
division and square root are correctly rounded.  NumPy float32 elementwise
operations are exactly that.

The support of the linear kernel with distribution alignment (Eq. 12) is the
ellipse D' < lambda; its axis-aligned bounding box has half-extents
lambda*sqrt(Sigma_2D,xx) and lambda*sqrt(Sigma_2D,yy).  Another kernel of the
family uses its extent lambda * s_f (config.py) in place of lambda.  A pixel (px, py) is
sampled at its centre (px + 0.5, py + 0.5).
"""
from __future__ import annotations

import numpy as np

from .config import extent

f32 = np.float32


def binning_fp32(means, scales, quats, viewmat, intrin, width, height, cfg):
    """FP32 binning of N splats in one camera.

    Returns (rect [N,4] int64 as (tx0, ty0, tx1, ty1) inclusive, ntiles [N]
    int64, depth_key [N] uint32).  Culled splats (non-finite, outside the
    near/far planes, or with an empty pixel range) get ntiles 0, rect zeros
    and depth_key 0xFFFFFFFF.
    """
    with np.errstate(all="ignore"):
        mu = np.asarray(means, f32)
        s = np.asarray(scales, f32)
        q = np.asarray(quats, f32)
        V = np.asarray(viewmat, f32)
        fx, fy, cx, cy = (f32(v) for v in np.asarray(intrin, f32))
        W, H = f32(width), f32(height)
        lam, eps, clip = f32(extent(cfg)), f32(cfg.eps2d), f32(cfg.clip)
        near, far = f32(cfg.near), f32(cfg.far)

        # normalised quaternion
        w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
        n2 = ((w * w + x * x) + y * y) + z * z
        r = np.sqrt(n2)
        w, x, y, z = w / r, x / r, y / r, z / r
        # rotation
        R = [[f32(1) - f32(2) * (y * y + z * z), f32(2) * (x * y - w * z), f32(2) * (x * z + w * y)],
             [f32(2) * (x * y + w * z), f32(1) - f32(2) * (x * x + z * z), f32(2) * (y * z - w * x)],
             [f32(2) * (x * z - w * y), f32(2) * (y * z + w * x), f32(1) - f32(2) * (x * x + y * y)]]
        # M = R diag(s), Sigma = M M^T
        M = [[R[rr][cc] * s[:, cc] for cc in range(3)] for rr in range(3)]
        Sig = [[(M[rr][0] * M[cc][0] + M[rr][1] * M[cc][1]) + M[rr][2] * M[cc][2]
                for cc in range(3)] for rr in range(3)]
        # camera-space centre
        t = [((V[rr, 0] * mu[:, 0] + V[rr, 1] * mu[:, 1]) + V[rr, 2] * mu[:, 2]) + V[rr, 3]
             for rr in range(3)]
        t0, t1, t2 = t
        # projected centre
        u = t0 / t2
        v = t1 / t2
        mx = fx * u + cx
        my = fy * v + cy
        # clipped tangents and the Jacobian
        limx = (clip * (f32(0.5) * W)) / fx
        limy = (clip * (f32(0.5) * H)) / fy
        uc = np.minimum(limx, np.maximum(-limx, u))
        vc = np.minimum(limy, np.maximum(-limy, v))
        J00 = fx / t2
        J02 = -((fx * uc) / t2)
        J11 = fy / t2
        J12 = -((fy * vc) / t2)
        T0 = [J00 * V[0, cc] + J02 * V[2, cc] for cc in range(3)]
        T1 = [J11 * V[1, cc] + J12 * V[2, cc] for cc in range(3)]
        P0 = [(T0[0] * Sig[0][cc] + T0[1] * Sig[1][cc]) + T0[2] * Sig[2][cc] for cc in range(3)]
        P1 = [(T1[0] * Sig[0][cc] + T1[1] * Sig[1][cc]) + T1[2] * Sig[2][cc] for cc in range(3)]
        a = ((P0[0] * T0[0] + P0[1] * T0[1]) + P0[2] * T0[2]) + eps
        c = ((P1[0] * T1[0] + P1[1] * T1[1]) + P1[2] * T1[2]) + eps
        rx = lam * np.sqrt(a)
        ry = lam * np.sqrt(c)
        half = f32(0.5)
        xlo = np.ceil((mx - rx) - half)
        xhi = np.floor((mx + rx) - half)
        ylo = np.ceil((my - ry) - half)
        yhi = np.floor((my + ry) - half)
        xlo = np.maximum(xlo, f32(0))
        ylo = np.maximum(ylo, f32(0))
        xhi = np.minimum(xhi, W - f32(1))
        yhi = np.minimum(yhi, H - f32(1))
        finite = (np.isfinite(t0) & np.isfinite(t1) & np.isfinite(t2) & np.isfinite(mx)
                  & np.isfinite(my) & np.isfinite(rx) & np.isfinite(ry))
        keep = finite & (t2 > near) & (t2 < far)
        keep &= (xlo <= xhi) & (ylo <= yhi)

    n = len(mu)
    rect = np.zeros((n, 4), np.int64)
    tw, th = int(cfg.tile_w), int(cfg.tile_h)
    rect[keep, 0] = xlo[keep].astype(np.int64) // tw
    rect[keep, 1] = ylo[keep].astype(np.int64) // th
    rect[keep, 2] = xhi[keep].astype(np.int64) // tw
    rect[keep, 3] = yhi[keep].astype(np.int64) // th
    ntiles = np.where(keep, (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1), 0)
    depth_key = np.where(keep, np.asarray(t2, f32).view(np.uint32), np.uint32(0xFFFFFFFF))
    return rect, ntiles.astype(np.int64), depth_key.astype(np.uint32)


def grid_size(width: int, height: int, cfg) -> tuple[int, int]:
    return (-(-int(width) // int(cfg.tile_w)), -(-int(height) // int(cfg.tile_h)))


def intersections(rect, ntiles, depth_key, pair_ids, tile_base, grid_x):
    """All (global tile, depth key, pair id) triples of one camera, unsorted.

    pair_ids are the global (camera, splat) pair indices of these splats,
    tile_base is the camera's first global tile id, grid_x its tiles per row."""
    out = []
    for i in np.nonzero(ntiles)[0]:
        tx0, ty0, tx1, ty1 = (int(v) for v in rect[i])
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                out.append((tile_base + ty * grid_x + tx, int(depth_key[i]), int(pair_ids[i])))
    return out


def sort_intersections(triples):
    """Lexicographic ascending order: tile, then depth key, then pair id."""
    return sorted(triples)


def intersections_array(rect, ntiles, depth_key, pair_ids, tile_base, grid_x):
    """Vectorised equivalent of ``intersections`` for large inputs: returns
    (gtile, depth_key, pair_id) int64 arrays in an unspecified order."""
    idx = np.nonzero(ntiles)[0]
    cnt = ntiles[idx]
    rep = np.repeat(idx, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(int(cnt.sum()), dtype=np.int64) - start
    wdt = rect[rep, 2] - rect[rep, 0] + 1
    tx = rect[rep, 0] + local % wdt
    ty = rect[rep, 1] + local // wdt
    return (tile_base + ty * grid_x + tx, depth_key[rep].astype(np.int64),
            np.asarray(pair_ids, np.int64)[rep])


def sort_arrays(gtile, dkey, pid):
    """Same order as ``sort_intersections`` via a library lexicographic sort."""
    order = np.lexsort((pid, dkey, gtile))
    return gtile[order], dkey[order], pid[order]


def tile_ranges(sorted_gtile, n_tiles_total):
    """offsets [T+1]: tile t owns sorted positions [off[t], off[t+1])."""
    counts = np.bincount(np.asarray(sorted_gtile, np.int64), minlength=n_tiles_total)
    off = np.zeros(n_tiles_total + 1, np.int64)
    off[1:] = np.cumsum(counts)
    return off


def tile_list(rect, ntiles, depth_key, gtile, lay):
    """One tile's list by its plain definition: the pairs of the tile's camera
    whose rectangle contains the tile, in (depth key, pair id) order."""
    c = int(np.searchsorted(lay.tile_off, gtile, side="right") - 1)
    gx = lay.grid[c][0]
    ty, tx = divmod(int(gtile - lay.tile_off[c]), gx)
    m0, m1 = int(lay.pair_off[c]), int(lay.pair_off[c + 1])
    r = rect[m0:m1]
    sel = (ntiles[m0:m1] > 0) & (r[:, 0] <= tx) & (tx <= r[:, 2]) & (r[:, 1] <= ty) & (ty <= r[:, 3])
    ids = m0 + np.nonzero(sel)[0]
    return ids[np.lexsort((ids, depth_key[ids].astype(np.int64)))]
