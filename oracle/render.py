"""Whole-path oracle driver: projection, binning, composite and reverse pass
over a batch of cameras that may view different scenes.

Indexing (shared with nothing but mirrored by the library's documented
layout): the (camera, splat) pairs are numbered camera-major, pair index
m = pair_off[c] + (local splat index); global tile ids are tile_off[c] +
ty * grid_x + tx; pixels are numbered camera-major, row-major inside a camera;
images are planar per camera, [3, H, W] blocks concatenated.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import binning, composite, projection


@dataclass
class Layout:
    pair_off: np.ndarray      # [C+1]
    tile_off: np.ndarray      # [C+1]
    pix_off: np.ndarray       # [C+1]
    grid: list                # [(gx, gy)] per camera
    splat_lo: np.ndarray      # [C] first global splat of the camera's scene
    splat_hi: np.ndarray      # [C]


def layout(scene_off, cams, cfg) -> Layout:
    C = cams.n
    pair_off = np.zeros(C + 1, np.int64)
    tile_off = np.zeros(C + 1, np.int64)
    pix_off = np.zeros(C + 1, np.int64)
    grid, lo, hi = [], np.zeros(C, np.int64), np.zeros(C, np.int64)
    for c in range(C):
        s = int(cams.scene_of_cam[c])
        lo[c], hi[c] = scene_off[s], scene_off[s + 1]
        gx, gy = binning.grid_size(cams.width[c], cams.height[c], cfg)
        grid.append((gx, gy))
        pair_off[c + 1] = pair_off[c] + (hi[c] - lo[c])
        tile_off[c + 1] = tile_off[c] + gx * gy
        pix_off[c + 1] = pix_off[c] + int(cams.width[c]) * int(cams.height[c])
    return Layout(pair_off, tile_off, pix_off, grid, lo, hi)


@dataclass
class Forward:
    cfg: object
    lay: Layout
    proj: list = field(default_factory=list)      # per camera projection dicts
    rect: np.ndarray = None                       # [M,4]
    ntiles: np.ndarray = None                     # [M]
    depth_key: np.ndarray = None                  # [M] uint32
    sorted_gtile: np.ndarray = None
    sorted_ids: np.ndarray = None                 # pair ids in (tile, depth, id) order
    ranges: np.ndarray = None                     # [T+1]
    image: np.ndarray = None                      # [sum 3HW]
    final_T: np.ndarray = None                    # [P]
    last: np.ndarray = None                       # [P]
    flag: np.ndarray = None                       # [P]
    jump: np.ndarray = None                       # [P] colour-jump bound of flagged pixels
    tiles_done: np.ndarray = None                 # [T] bool: composited
    tile_res: dict = field(default_factory=dict)  # gtile -> composite result (pairs)


def project_and_bin(scene, scene_off, cams, cfg):
    lay = layout(scene_off, cams, cfg)
    fw = Forward(cfg=cfg, lay=lay)
    rects, nts, dks, gts, dkk, pids = [], [], [], [], [], []
    for c in range(cams.n):
        lo, hi = lay.splat_lo[c], lay.splat_hi[c]
        sl = slice(lo, hi)
        p = projection.project(scene.means[sl], scene.scales[sl], scene.quats[sl],
                               scene.sh[sl], scene.sh_degree, cams.viewmat[c], cams.intrin[c],
                               cams.width[c], cams.height[c], cfg)
        fw.proj.append(p)
        rect, nt, dk = binning.binning_fp32(scene.means[sl], scene.scales[sl], scene.quats[sl],
                                            cams.viewmat[c], cams.intrin[c], cams.width[c],
                                            cams.height[c], cfg)
        rects.append(rect)
        nts.append(nt)
        dks.append(dk)
        pid = lay.pair_off[c] + np.arange(hi - lo, dtype=np.int64)
        g, d, i = binning.intersections_array(rect, nt, dk, pid, lay.tile_off[c], lay.grid[c][0])
        gts.append(g)
        dkk.append(d)
        pids.append(i)
    fw.rect = np.concatenate(rects)
    fw.ntiles = np.concatenate(nts)
    fw.depth_key = np.concatenate(dks)
    g, d, i = binning.sort_arrays(np.concatenate(gts), np.concatenate(dkk), np.concatenate(pids))
    fw.sorted_gtile, fw.sorted_ids = g, i
    fw.ranges = binning.tile_ranges(g, int(lay.tile_off[-1]))
    return fw


def _cam_of_tile(lay, gt):
    return int(np.searchsorted(lay.tile_off, gt, side="right") - 1)


def render_forward(scene, scene_off, cams, cfg, tiles=None, want_pairs=False):
    """Full forward.  ``tiles`` (optional iterable of global tile ids)
    restricts compositing to those tiles; other pixels stay unset (NaN)."""
    fw = project_and_bin(scene, scene_off, cams, cfg)
    lay = fw.lay
    P = int(lay.pix_off[-1])
    fw.image = np.full(3 * P, np.nan)
    fw.final_T = np.full(P, np.nan)
    fw.last = np.full(P, -1, np.int64)
    fw.flag = np.zeros(P, bool)
    fw.jump = np.zeros(P)
    T_total = int(lay.tile_off[-1])
    fw.tiles_done = np.zeros(T_total, bool)
    tiles = range(T_total) if tiles is None else tiles
    bg = np.asarray(cfg.bg, np.float64)
    for gt in tiles:
        gt = int(gt)
        c = _cam_of_tile(lay, gt)
        gx, _ = lay.grid[c]
        local = gt - int(lay.tile_off[c])
        ty, tx = divmod(local, gx)
        W, H = int(cams.width[c]), int(cams.height[c])
        px, py = composite._tile_pixels(tx, ty, W, H, cfg)
        ids = fw.sorted_ids[fw.ranges[gt]:fw.ranges[gt + 1]] - lay.pair_off[c]
        p = fw.proj[c]
        opac = np.asarray(scene.opacity[lay.splat_lo[c]:lay.splat_hi[c]], np.float64)
        res = composite.composite_tile(ids, px, py, p["mean2d"], p["conic"], opac, p["rgb"],
                                       cfg, want_pairs=want_pairs)
        pix = int(lay.pix_off[c]) + py * W + px
        img_base = 3 * int(lay.pix_off[c])
        for ch in range(3):
            fw.image[img_base + ch * W * H + py * W + px] = res["C"][:, ch] + res["T"] * bg[ch]
        fw.final_T[pix] = res["T"]
        fw.last[pix] = res["last"]
        fw.flag[pix] = res["flag"]
        fw.jump[pix] = res["jump"]
        fw.tiles_done[gt] = True
        if want_pairs:
            res["pix"] = pix
            fw.tile_res[gt] = res
    return fw


def render_backward(fw, scene, cams, dL_dimage, dL_dalpha=None):
    """Reverse pass of ``render_forward(..., want_pairs=True)`` over the tiles
    it composited.  dL_dimage has the image layout; dL_dalpha (optional, one
    value per pixel in the final_T layout) is the upstream gradient of the
    accumulated opacity 1 - T_final.  Returns a dict of gradients w.r.t.
    means [N,3], scales [N,3], quats [N,4], opacity [N], sh [N,K,3], plus the
    per-pair 2D gradients (for staged comparison) and mean2d_norm [M], the
    Euclidean norm of each pair's dL/d(projected centre)."""
    cfg, lay = fw.cfg, fw.lay
    N = scene.n
    K = scene.sh.shape[1]
    out = dict(means=np.zeros((N, 3)), scales=np.zeros((N, 3)), quats=np.zeros((N, 4)),
               opacity=np.zeros(N), sh=np.zeros((N, K, 3)))
    M = int(lay.pair_off[-1])
    g2 = dict(rgb=np.zeros((M, 3)), opacity=np.zeros(M), conic=np.zeros((M, 3)),
              mean2d=np.zeros((M, 2)))
    for c in range(cams.n):
        n_c = int(lay.splat_hi[c] - lay.splat_lo[c])
        p = fw.proj[c]
        opac = np.asarray(scene.opacity[lay.splat_lo[c]:lay.splat_hi[c]], np.float64)
        W, H = int(cams.width[c]), int(cams.height[c])
        acc = [np.zeros((n_c, 3)), np.zeros(n_c), np.zeros((n_c, 3)), np.zeros((n_c, 2))]
        img_base = 3 * int(lay.pix_off[c])
        for gt in range(int(lay.tile_off[c]), int(lay.tile_off[c + 1])):
            res = fw.tile_res.get(gt)
            if res is None:
                continue
            local = res["pix"] - int(lay.pix_off[c])
            G = np.stack([np.asarray(dL_dimage[img_base + ch * W * H + local], np.float64)
                          for ch in range(3)], axis=1)
            GA = None
            if dL_dalpha is not None:
                GA = np.asarray(dL_dalpha[int(lay.pix_off[c]) + local], np.float64)
            r = composite.reverse_tile(res, G, p["mean2d"], p["conic"], opac, p["rgb"], cfg, n_c,
                                       GA)
            for a, b in zip(acc, r):
                a += b
        m0, m1 = int(lay.pair_off[c]), int(lay.pair_off[c + 1])
        g2["rgb"][m0:m1], g2["opacity"][m0:m1] = acc[0], acc[1]
        g2["conic"][m0:m1], g2["mean2d"][m0:m1] = acc[2], acc[3]
        sl = slice(lay.splat_lo[c], lay.splat_hi[c])
        gm, gs, gq, gsh = projection.project_backward(p, scene.sh[sl], scene.sh_degree,
                                                      acc[3], acc[2], acc[0])
        out["means"][sl] += gm
        out["scales"][sl] += gs
        out["quats"][sl] += gq
        out["opacity"][sl] += acc[1]
        out["sh"][sl] += gsh
    out["pair"] = g2
    out["mean2d_norm"] = np.sqrt(np.sum(g2["mean2d"] ** 2, axis=1))
    return out
