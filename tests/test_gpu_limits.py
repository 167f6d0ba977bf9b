"""Parity at the limits the C ABI accepts:

  * one 16384 x 16384 view, the largest image: 1024 x 1024 tiles of 16 x 16,
    so tile ids take 20 bits and the tile sort three 8-bit passes, and pixel
    and plane offsets reach 8e8;
  * 65535 cameras, the most one call accepts, of 16 x 16 pixels (one tile
    each) around one scene: the camera tables and their searches at their
    largest.

As in the full-size tests, the FP64 oracle composites and differentiates a
seeded sample of tiles (each tile's list against its plain definition, the
composite, and the per-pair 2D gradients for an upstream gradient that is
non-zero on the sampled tiles only, every other pair receiving exactly
zero).  The GPU arrays are read back per sampled pixel and per sampled pair,
never whole.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import binning, composite, projection
from oracle.render import layout
from paper_2411_12440_amd import scenes
from tests.gpu_helpers import assert_close, cfg_pair, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sampled_tiles_parity(scene, off, cams, pick, seed, capacity, **cfg):
    """`pick(busy_tiles_by_camera, rng)` returns the (camera, global tile)
    samples."""
    import torch
    from paper_2411_12440_amd.rasterizer import Rasterizer, scene_to_device

    ocfg, gkw = cfg_pair(**cfg)
    sp = scene_to_device(scene)
    rast = Rasterizer(cams, off, capacity=capacity, sh_degree=scene.sh_degree, **gkw)
    rast.forward(sp)
    torch.cuda.synchronize()
    assert not rast.overflowed()
    L = rast.layout
    M, T, P = int(L.n_pairs), int(L.n_tiles), int(L.n_pixels)
    lay = layout(off, cams, ocfg)
    assert M == int(lay.pair_off[-1]) and T == int(lay.tile_off[-1]) and P == int(lay.pix_off[-1])
    base, rng_all = rast.lists()
    per_tile = (rng_all[:, 1:] - rng_all[:, :-1]).sum(axis=0)
    rs = np.random.default_rng(seed)
    samples = pick(per_tile, rs)
    say(f"  {M} pairs, {T} tiles, {P} pixels, {rast.n_isect()} intersections; "
        f"{len(samples)} sampled tiles")

    # the sampled cameras' binning and projection by the oracle
    rect = np.zeros((M, 4), np.int64)
    nt = np.zeros(M, np.int64)
    dk = np.zeros(M, np.uint32)
    sub = {}
    for c in sorted({c for c, _ in samples}):
        s = slice(int(lay.splat_lo[c]), int(lay.splat_hi[c]))
        m = slice(int(lay.pair_off[c]), int(lay.pair_off[c + 1]))
        W, H = int(cams.width[c]), int(cams.height[c])
        rect[m], nt[m], dk[m] = binning.binning_fp32(scene.means[s], scene.scales[s], scene.quats[s],
                                                     cams.viewmat[c], cams.intrin[c], W, H, ocfg)
        g_nt = rast.view("ntiles", torch.int32, m.stop - m.start, m.start).cpu().numpy()
        np.testing.assert_array_equal(g_nt.view(np.uint32).astype(np.int64), nt[m])
        sub[c] = projection.project(scene.means[s], scene.scales[s], scene.quats[s], scene.sh[s],
                                    scene.sh_degree, cams.viewmat[c], cams.intrin[c], W, H, ocfg)

    G = torch.zeros(3 * P, dtype=torch.float32, device="cuda")
    g_full = np.random.default_rng(seed + 1)
    tiles = []
    for c, gt in samples:
        W, H = int(cams.width[c]), int(cams.height[c])
        gx = lay.grid[c][0]
        ty, tx = divmod(gt - int(lay.tile_off[c]), gx)
        ref = binning.tile_list(rect, nt, dk, gt, lay)
        segs = [rast.view("vals", torch.int32, int(rng_all[q, gt + 1] - rng_all[q, gt]),
                          int(base[q] + rng_all[q, gt])).cpu().numpy().view(np.uint32)
                for q in range(len(base) - 1)]
        got = np.concatenate(segs).astype(np.int64)
        assert len(got) <= len(ref)
        np.testing.assert_array_equal(got, ref[:len(got)])
        loc = ref - int(lay.pair_off[c])
        p = sub[c]
        px, py = composite._tile_pixels(tx, ty, W, H, ocfg)
        opac = scene.opacity[int(lay.splat_lo[c]) + loc].astype(np.float64)
        res = composite.composite_tile(np.arange(len(loc)), px, py, p["mean2d"][loc],
                                       p["conic"][loc], opac, p["rgb"][loc], ocfg, want_pairs=True)
        assert len(got) >= res["last"].max()
        pix = int(lay.pix_off[c]) + py.astype(np.int64) * W + px
        pix_t = torch.from_numpy(pix).cuda()
        planes = [3 * int(lay.pix_off[c]) + ch * W * H + py.astype(np.int64) * W + px
                  for ch in range(3)]
        ok = ~res["flag"]
        np.testing.assert_array_equal(rast.last[pix_t].cpu().numpy()[ok], res["last"][ok])
        assert_close("final_T", rast.final_T[pix_t].cpu().numpy(), res["T"], mask=ok)
        for ch in range(3):
            ib = torch.from_numpy(planes[ch]).cuda()
            assert_close(f"image[{ch}]", rast.image[ib].cpu().numpy(), res["C"][:, ch], mask=ok)
            gv = g_full.normal(0.0, 1.0, size=len(px)).astype(np.float32) * ok
            G[ib] = torch.from_numpy(gv).cuda()
        tiles.append((c, gt, loc, res, px, py, planes))
    say(f"  {len(tiles)} sampled tiles equal (largest pixel index {max(int(t[6][2].max()) for t in tiles)})")

    rast.backward(sp, G)
    torch.cuda.synchronize()
    g2 = rast.view("grad2d", torch.float64, 9 * M).cpu().numpy().reshape(9, M)
    want = np.zeros((9, M))
    touched = np.zeros(M, bool)
    Gh = {}
    for c, gt, loc, res, px, py, planes in tiles:
        idx = np.concatenate(planes)
        Gh[gt] = G[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    for c in sub:
        mine = [t for t in tiles if t[0] == c]
        n_c = int(lay.pair_off[c + 1] - lay.pair_off[c])
        acc = [np.zeros((n_c, 3)), np.zeros(n_c), np.zeros((n_c, 3)), np.zeros((n_c, 2))]
        p = sub[c]
        for _, gt, loc, res, px, py, planes in mine:
            r2 = dict(res)
            if res["pairs"] is not None:
                r2["pairs"] = dict(res["pairs"], id=loc[res["pairs"]["id"]])
            Gt = Gh[gt].reshape(3, -1).T
            r = composite.reverse_tile(r2, Gt, p["mean2d"], p["conic"],
                                       scene.opacity[int(lay.splat_lo[c]):int(lay.splat_hi[c])]
                                       .astype(np.float64), p["rgb"], ocfg, n_c)
            for a, b in zip(acc, r):
                a += b
        m0 = int(lay.pair_off[c])
        sl = slice(m0, m0 + n_c)
        want[0:2, sl] = acc[3].T
        want[2:5, sl] = projection.cov2d_grad(p["conic"], acc[2]).T
        want[5, sl] = acc[1]
        want[6:9, sl] = acc[0].T
        for _, gt, loc, res, px, py, planes in mine:
            touched[m0 + loc] = True
    assert np.all(g2[:, ~touched] == 0.0)
    for name, rows in (("d_mean2d", slice(0, 2)), ("d_cov2d", slice(2, 5)),
                       ("d_opacity2d", slice(5, 6)), ("d_rgb", slice(6, 9))):
        assert_close(name, g2[rows, touched], want[rows, touched])


def test_largest_image():
    """One 16384 x 16384 view of 20,000 splats (SH1), AGS, 7 depth chunks; 16
    sampled tiles, the last tile with entries among them."""
    say("case: one 16384x16384 view, 20000 splats SH1, AGS, depth chunks 7")
    scene = scenes.make_scene(20000, 4401, -5.0, 0.6, 1)
    cams = scenes.front_camera(16384, 16384)

    def pick(per_tile, rs):
        busy = np.nonzero(per_tile > 0)[0]
        out = [(0, int(t)) for t in rs.choice(busy, 15, replace=False)]
        return out + [(0, int(busy[-1]))]

    _sampled_tiles_parity(scene, np.array([0, scene.n]), cams, pick, 4401, 1 << 24,
                          ags=True, depth_chunks=7)


def test_most_cameras():
    """65535 cameras of 16 x 16 pixels on a sphere around one scene of 48
    splats (SH2), AGS, 3 depth chunks; 16 sampled cameras, the first and the
    last with entries among them."""
    say("case: 65535 cameras of 16x16, 48 splats SH2, AGS, depth chunks 3")
    n = 65535
    scene = scenes.make_scene(48, 4402, -1.5, 0.4, 2)
    cams = scenes.sphere_cameras(n, 4.0, [(16, 16)] * n)

    def pick(per_tile, rs):
        busy = np.nonzero(per_tile > 0)[0]
        out = [int(t) for t in rs.choice(busy, 14, replace=False)] + [int(busy[0]), int(busy[-1])]
        return [(t, t) for t in out]     # one tile per camera: the tile id is the camera

    _sampled_tiles_parity(scene, np.array([0, scene.n]), cams, pick, 4402, 1 << 23,
                          ags=True, depth_chunks=3)
