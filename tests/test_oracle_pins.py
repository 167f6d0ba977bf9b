"""Pins of the FP64 oracle to facts that do not come from the oracle itself:
closed forms, invariants, brute force, library routines, finite differences
and an independent autograd transcription.  CPU only."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest
import scipy.special as sps

from oracle import RasterConfig, binning, composite, projection, render_forward, render_backward
from oracle.config import KERNELS
from oracle import sh as oracle_sh
from paper_2411_12440_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# helpers that build tiny inputs by hand
# --------------------------------------------------------------------------

def one_camera(W, H, dist=3.0):
    return scenes.front_camera(W, H, dist)


def manual_scene(means, scales, quats, opac, rgb):
    """SH degree 0 scene whose colour is given through a DC coefficient of 0
    plus 0.5 offset trick: rgb must be 0.5 for exactness (dc = 0)."""
    n = len(means)
    sh = np.zeros((n, 1, 3), np.float32)
    sh[:, 0, :] = (np.asarray(rgb, np.float64) - 0.5) / oracle_sh.Y00
    return scenes.Scene(np.asarray(means, np.float32), np.asarray(scales, np.float32),
                        np.asarray(quats, np.float32), np.asarray(opac, np.float32), sh, 0)


# --------------------------------------------------------------------------
# linear kernel (Eq. 10-12)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lam", [1.0, 2.5])
def test_linear_kernel_values(lam):
    cfg = RasterConfig(lambda_=lam, alpha_max=1.0)
    Ds = np.array([0.0, 0.25, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 10.0])
    px = Ds - 0.5                     # pixel centre at px + 0.5 = D, splat at origin
    py = np.full_like(px, -0.5)
    mean2d = np.zeros((1, 2))
    conic = np.array([[1.0, 0.0, 1.0]])    # identity: D' = |x - mu'|
    _, _, D, L, raw, alpha = composite._pair_terms(px, py, mean2d, conic, np.array([1.0]), cfg)
    np.testing.assert_array_equal(D[:, 0], Ds)
    expect = np.array([max(0.0, 1.0 - d / lam) for d in Ds])
    np.testing.assert_allclose(L[:, 0], expect, rtol=0, atol=1e-15)
    assert L[0, 0] == 1.0
    assert L[list(Ds).index(lam), 0] == 0.0
    assert np.all(L[Ds >= lam, 0] == 0.0)
    # slope -1/lambda inside the support
    inside = Ds < lam
    d1, d2 = Ds[inside][1], Ds[inside][2]
    l1, l2 = L[inside, 0][1], L[inside, 0][2]
    assert abs((l2 - l1) / (d2 - d1) + 1.0 / lam) < 1e-12


def test_kernel_lambda_one_is_eq10():
    """lambda = 1 reproduces max(0, 1 - D) exactly."""
    cfg = RasterConfig(lambda_=1.0, alpha_max=1.0)
    rng = np.random.default_rng(0)
    px, py = rng.uniform(-3, 3, 50), rng.uniform(-3, 3, 50)
    mean2d = np.zeros((1, 2))
    conic = np.array([[0.7, 0.2, 1.3]])
    _, _, D, L, _, _ = composite._pair_terms(px, py, mean2d, conic, np.array([1.0]), cfg)
    x, y = px + 0.5, py + 0.5
    D_ref = np.sqrt(0.7 * x * x + 0.4 * x * y + 1.3 * y * y)
    np.testing.assert_allclose(D[:, 0], D_ref, rtol=1e-14)
    np.testing.assert_allclose(L[:, 0], np.maximum(0.0, 1.0 - D_ref), atol=1e-14)


# --------------------------------------------------------------------------
# single isotropic splat on the optical axis: closed form
# --------------------------------------------------------------------------

def _iso_setup(s=0.05, o=0.8, W=64, H=64, lam=2.5, strict=False, dist=3.0, **kw):
    sc = manual_scene([[0, 0, 0]], [[s, s, s]], [[1, 0, 0, 0]], [o], [[0.5, 0.5, 0.5]])
    cams = one_camera(W, H, dist)
    cfg = (RasterConfig.strict if strict else RasterConfig)(lambda_=lam, **kw)
    f = float(cams.intrin[0, 0])
    sig2 = (f * float(np.float32(s)) / dist) ** 2 + cfg.eps2d
    return sc, cams, cfg, math.sqrt(sig2)


@pytest.mark.parametrize("lam", [1.0, 2.5])
def test_single_splat_closed_form(lam):
    sc, cams, cfg, sigma = _iso_setup(lam=lam)
    fw = render_forward(sc, np.array([0, 1]), cams, cfg)
    W = H = 64
    ys, xs = np.mgrid[0:H, 0:W]
    r = np.hypot(xs + 0.5 - W / 2, ys + 0.5 - H / 2)
    o = float(np.float32(0.8))
    a = np.minimum(cfg.alpha_max, o * np.maximum(0, 1 - r / (lam * sigma)))
    a = np.where(a >= cfg.alpha_min, a, 0.0)
    img = fw.image.reshape(3, H, W)
    for ch in range(3):
        np.testing.assert_allclose(img[ch], 0.5 * a, atol=1e-13)
    np.testing.assert_allclose(fw.final_T.reshape(H, W), 1.0 - a, atol=1e-13)
    # support pixel count ~ pi (lambda sigma)^2
    npx = np.count_nonzero(o * np.maximum(0, 1 - r / (lam * sigma)) > 0)
    assert abs(npx - math.pi * (lam * sigma) ** 2) < 2 * math.pi * lam * sigma + 4


def test_coverage_integral():
    """Sum over pixels of alpha -> o * (pi/3) lambda^2 sigma^2 (the volume of a
    cone of height o and radius lambda*sigma)."""
    sc, cams, cfg, sigma = _iso_setup(s=0.5, o=0.5, W=256, H=256, strict=True)
    fw = render_forward(sc, np.array([0, 1]), cams, cfg)
    total = (1.0 - fw.final_T).sum()
    expect = 0.5 * math.pi / 3.0 * cfg.lambda_ ** 2 * sigma ** 2
    assert sigma * cfg.lambda_ < 120
    assert abs(total / expect - 1) < 2e-4


# Sum over pixels of alpha for one isotropic splat against o * lambda^2 sigma^2
# times the kernel's 2D mass 2 pi int_0^s r f(r) dr up to its support cut s,
# in closed form: Gaussian 2 pi (1 - e^-4.5), Laplacian 2 pi (1 - e^-L (1 + L))
# with L = ln 255, raised cosine 2 pi (1/4 - 1/pi^2), quadratic pi / 2, linear
# pi / 3.  (lambda, scale) keep the support well inside the image; the
# tolerance covers the pixel sampling of the kernel's cusp or cut.
_LN255 = float(np.float32(math.log(255.0)))
FAMILY_MASS = {
    "linear": (2.5, 0.5, math.pi / 3, 2e-4),
    "gaussian": (1.0, 0.45, 2 * math.pi * (1 - math.exp(-4.5)), 2e-4),
    "laplacian": (1.0, 0.25, 2 * math.pi * (1 - math.exp(-_LN255) * (1 + _LN255)), 5e-4),
    "cosine": (2.5, 0.5, 2 * math.pi * (0.25 - 1 / math.pi ** 2), 1e-4),
    "quadratic": (6.0, 0.2, math.pi / 2, 1e-4),
}


@pytest.mark.parametrize("kernel", KERNELS)
def test_kernel_family_mass(kernel):
    lam, s, mass, tol = FAMILY_MASS[kernel]
    sc, cams, cfg, sigma = _iso_setup(s=s, o=0.5, W=256, H=256, lam=lam, strict=True,
                                      kernel=kernel)
    from oracle.config import extent
    assert extent(cfg) * sigma < 125          # support inside the image
    fw = render_forward(sc, np.array([0, 1]), cams, cfg)
    total = (1.0 - fw.final_T).sum()
    o = float(np.float32(0.5))
    expect = o * mass * cfg.lambda_ ** 2 * sigma ** 2
    assert abs(total / expect - 1) < tol, (total, expect)


def test_kernel_family_centre_and_cut():
    """At the splat's centre every kernel gives alpha = o; beyond the support
    cut none contributes, and inside it the Gaussian still does at its 3-sigma
    edge (alpha = o e^-4.5 > 1/255 for o = 0.8)."""
    for kernel in KERNELS:
        sc, cams, cfg, sigma = _iso_setup(s=0.3, o=0.8, W=65, H=65, lam=1.0, strict=False,
                                          kernel=kernel)
        fw = render_forward(sc, np.array([0, 1]), cams, cfg)
        img = fw.image.reshape(3, 65, 65)
        # the centre pixel of an odd image sits half a pixel from the splat centre
        assert abs(img[0, 32, 32] - 0.5 * min(cfg.alpha_max, float(np.float32(0.8)))) < 0.02
    sc, cams, cfg, sigma = _iso_setup(s=0.05, o=0.8, W=128, H=128, lam=1.0, kernel="gaussian")
    fw = render_forward(sc, np.array([0, 1]), cams, cfg)
    a = 1.0 - fw.final_T.reshape(128, 128)
    ys, xs = np.mgrid[0:128, 0:128]
    r = np.hypot(xs + 0.5 - 64, ys + 0.5 - 64) / sigma
    assert np.all(a[r > 3.0 + 1e-6] == 0.0)
    edge = (r > 2.9) & (r < 3.0 - 1e-6)
    assert edge.any() and np.all(a[edge] > 1.0 / 255.0)


def test_mass_matching_lambda():
    """Distribution alignment widens the linear kernel so that its coverage
    matches the Gaussian's: with the printed lambda values the 2D masses of
    f(D/lambda) are within a few percent of the Gaussian's 2 pi sigma^2."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        g = json.load(fh)
    lam = g["da_lambda"]
    gauss = 2 * math.pi
    lin = math.pi / 3 * lam["linear"] ** 2                  # cone volume
    # raised cosine 1/2 (1 + cos(pi r)) on r < 1, radial integral 2 pi int r f dr
    from scipy.integrate import quad
    cos_mass = 2 * math.pi * lam["cosine"] ** 2 * quad(lambda r: r * 0.5 * (1 + math.cos(math.pi * r)), 0, 1)[0]
    lap = 2 * math.pi * lam["laplacian"] ** 2 * quad(lambda r: r * math.exp(-r), 0, np.inf)[0]
    for m in (lin, cos_mass, lap):
        assert abs(m / gauss - 1) < 0.08
    # the linear kernel's exact match would be lambda = sqrt(6)
    assert abs(math.sqrt(6) - lam["linear"]) < 0.06


# --------------------------------------------------------------------------
# compositing invariants
# --------------------------------------------------------------------------

def test_two_splat_order_and_swap():
    W = H = 32
    cams = one_camera(W, H, 3.0)
    cfg = RasterConfig.strict()
    s = [[0.04] * 3, [0.06] * 3]
    sc = manual_scene([[0, 0, -0.5], [0, 0, 0.5]], s, [[1, 0, 0, 0]] * 2, [0.6, 0.7],
                      [[0.9, 0.1, 0.3], [0.2, 0.8, 0.4]])
    f = float(cams.intrin[0, 0])

    def alphas(scn):
        out = []
        for i in range(2):
            z = 3.0 + float(scn.means[i, 2])
            sig = math.sqrt((f * float(scn.scales[i, 0]) / z) ** 2 + cfg.eps2d)
            ys, xs = np.mgrid[0:H, 0:W]
            r = np.hypot(xs + 0.5 - W / 2, ys + 0.5 - H / 2)
            out.append(np.minimum(cfg.alpha_max, float(scn.opacity[i]) * np.maximum(0, 1 - r / (2.5 * sig))))
        return out

    rgb = [0.5 + oracle_sh.Y00 * sc.sh[i, 0].astype(np.float64) for i in range(2)]
    fw = render_forward(sc, np.array([0, 2]), cams, cfg)
    a1, a2 = alphas(sc)
    img = fw.image.reshape(3, H, W)
    for ch in range(3):
        np.testing.assert_allclose(img[ch], rgb[0][ch] * a1 + rgb[1][ch] * a2 * (1 - a1), atol=1e-12)
    # swap the depths: the second splat is now in front
    sc2 = manual_scene([[0, 0, 0.5], [0, 0, -0.5]], s, [[1, 0, 0, 0]] * 2, [0.6, 0.7],
                       [[0.9, 0.1, 0.3], [0.2, 0.8, 0.4]])
    fw2 = render_forward(sc2, np.array([0, 2]), cams, cfg)
    b1, b2 = alphas(sc2)
    img2 = fw2.image.reshape(3, H, W)
    for ch in range(3):
        np.testing.assert_allclose(img2[ch], rgb[1][ch] * b2 + rgb[0][ch] * b1 * (1 - b2), atol=1e-12)


@pytest.mark.parametrize("stop_after", [3, 4, 5])
def test_early_stop_closed_form(stop_after):
    """Five opaque isotropic splats stacked on the optical axis.  t_min is set
    so that splat ``stop_after`` + 1 would take T below it: that splat stops
    the pixel and is not added (Eq. 6 with the 3DGS stop rule)."""
    W = H = 16
    cams = one_camera(W, H, 3.0)
    z = [-0.4, -0.2, 0.0, 0.2, 0.4]
    cols = [[0.9, 0.1, 0.2], [0.1, 0.8, 0.3], [0.3, 0.3, 0.9], [0.7, 0.7, 0.1], [0.2, 0.5, 0.6]]
    sc = manual_scene([[0, 0, zz] for zz in z], [[1.0] * 3] * 5, [[1, 0, 0, 0]] * 5, [0.99] * 5, cols)
    f = float(cams.intrin[0, 0])
    px = py = 7
    r = math.hypot(px + 0.5 - W / 2, py + 0.5 - H / 2)
    rgb = [0.5 + oracle_sh.Y00 * sc.sh[i, 0].astype(np.float64) for i in range(5)]
    base = RasterConfig(alpha_max=0.999)
    a = []
    for i in range(5):
        sig = math.sqrt((f * float(sc.scales[i, 0]) / (3.0 + float(sc.means[i, 2]))) ** 2 + base.eps2d)
        a.append(min(base.alpha_max, float(sc.opacity[i]) * (1 - r / (base.lambda_ * sig))))
    assert all(0.85 < ai < 0.99 for ai in a)
    Ts = np.cumprod([1 - ai for ai in a])          # T after each splat
    tmin = 0.0 if stop_after == 5 else 1.2 * float(Ts[stop_after])
    cfg = RasterConfig(alpha_max=0.999, t_min=tmin)
    fw = render_forward(sc, np.array([0, 5]), cams, cfg)
    C = np.zeros(3)
    T = 1.0
    for i in range(stop_after):
        C += np.array(rgb[i]) * a[i] * T
        T *= 1 - a[i]
    pix = py * W + px
    img = fw.image.reshape(3, H * W)
    np.testing.assert_allclose(img[:, pix], C, rtol=1e-12)
    np.testing.assert_allclose(fw.final_T[pix], T, rtol=1e-12)
    assert fw.last[pix] == stop_after


def test_flagged_pixels_move_within_their_jump_bound():
    """A flagged pixel's decision may go the other way on another machine; the
    oracle's per-pixel jump bound must cover that.  Moving the alpha floor
    and the stop threshold by 0.99 of the flag margin either way flips the
    flagged decisions of sampled tiles of workload 2 (100k splats, 720p); every
    pixel's colour must then stay within jump * max|colour - background| of
    the unperturbed composite, and unflagged pixels must not move at all."""
    from oracle.composite import FLAG_REL
    sc, off, cams = scenes.workload(2)
    rng = np.random.default_rng(0)
    tiles = rng.choice(80 * 45, 60, replace=False)
    base_cfg = RasterConfig()
    fw = render_forward(sc, off, cams, base_cfg, tiles=tiles)
    done = ~np.isnan(fw.final_T)
    assert 0 < fw.flag[done].sum() < 0.01 * done.sum()
    rgb = np.concatenate([p["rgb"] for p in fw.proj])
    scale = float(np.max(np.abs(rgb)))
    img_done = np.concatenate([done] * 3)
    flag3 = np.concatenate([fw.flag] * 3)
    bound3 = np.concatenate([fw.jump] * 3) * scale
    moved = 0
    for fa, ft in [(1 - 0.99 * FLAG_REL, 1.0), (1 + 0.99 * FLAG_REL, 1.0),
                   (1.0, 1 - 0.99 * FLAG_REL), (1.0, 1 + 0.99 * FLAG_REL)]:
        cfg = RasterConfig(alpha_min=base_cfg.alpha_min * fa, t_min=base_cfg.t_min * ft)
        fp = render_forward(sc, off, cams, cfg, tiles=tiles)
        d = np.abs(fp.image - fw.image)
        assert np.all(d[img_done & ~flag3] == 0.0)
        assert np.all(d[img_done & flag3] <= bound3[img_done & flag3] * (1 + 1e-9) + 1e-15)
        moved += int(np.count_nonzero(d[img_done & flag3]))
    assert moved > 0       # the perturbations did flip decisions


def test_transmittance_telescopes_and_bounds():
    sc, off, cams = scenes.workload(1)
    cfg = RasterConfig()
    fw = render_forward(sc, off, cams, cfg, want_pairs=True)
    P = len(fw.final_T)
    wsum = np.zeros(P)
    for gt, res in fw.tile_res.items():
        pr = res["pairs"]
        if pr is None:
            continue
        np.add.at(wsum, res["pix"][pr["p"]], pr["alpha"] * pr["Tb"])
        # T non-increasing along each pixel's list
        order = np.lexsort((pr["k"], pr["p"]))
        p, Tb = pr["p"][order], pr["Tb"][order]
        same = p[1:] == p[:-1]
        assert np.all(Tb[1:][same] <= Tb[:-1][same])
    np.testing.assert_allclose(wsum + fw.final_T, 1.0, atol=1e-12)
    assert np.all(fw.final_T > 0) and np.all(fw.final_T <= 1)
    assert np.all(fw.final_T >= cfg.t_min)
    img = fw.image.reshape(3, -1)
    rgb = np.concatenate([p["rgb"] for p in fw.proj])
    lo, hi = rgb.min(), rgb.max()
    assert np.all(img >= lo * (1 - fw.final_T) - 1e-12)
    assert np.all(img <= hi * (1 - fw.final_T) + 1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("strict", [False, True])
def test_tiled_equals_bruteforce(seed, strict):
    """Bounded support: the tiled composite equals a plain per-pixel loop over
    every visible splat in depth order."""
    sc = scenes.make_scene(40, 300 + seed, -2.3, 0.5, 1)
    W, H = 40, 24
    cams = one_camera(W, H, 3.0)
    cfg = (RasterConfig.strict if strict else RasterConfig)(tile_w=16, tile_h=8)
    fw = render_forward(sc, np.array([0, sc.n]), cams, cfg)
    p = fw.proj[0]
    vis = np.nonzero(fw.ntiles)[0]
    order = vis[np.lexsort((vis, fw.depth_key[vis]))]
    C, T = composite.composite_bruteforce(W, H, order, p["mean2d"], p["conic"],
                                          sc.opacity.astype(np.float64), p["rgb"], cfg)
    img = fw.image.reshape(3, H, W)
    tol = 1e-12 if not strict else 1e-6
    for ch in range(3):
        np.testing.assert_allclose(img[ch], C[:, :, ch], atol=tol)
    np.testing.assert_allclose(fw.final_T.reshape(H, W), T, atol=tol)


# --------------------------------------------------------------------------
# binning, sort, ranges
# --------------------------------------------------------------------------

def test_sort_and_ranges_against_python():
    sc, off, cams = scenes.workload(1)
    cfg = RasterConfig()
    fw = render_forward(sc, off, cams, cfg, tiles=[])
    gx, gy = binning.grid_size(128, 128, cfg)
    trip = binning.intersections(fw.rect, fw.ntiles, fw.depth_key, np.arange(sc.n), 0, gx)
    ref = binning.sort_intersections(trip)
    assert [t[2] for t in ref] == list(fw.sorted_ids)
    assert [t[0] for t in ref] == list(fw.sorted_gtile)
    # ranges: brute-force membership by rectangle
    for t in range(gx * gy):
        ty, tx = divmod(t, gx)
        members = [i for i in range(sc.n) if fw.ntiles[i] and
                   fw.rect[i, 0] <= tx <= fw.rect[i, 2] and fw.rect[i, 1] <= ty <= fw.rect[i, 3]]
        lst = list(fw.sorted_ids[fw.ranges[t]:fw.ranges[t + 1]])
        assert sorted(lst) == members
        keys = [(int(fw.depth_key[i]), i) for i in lst]
        assert keys == sorted(keys)
    assert fw.ranges[-1] == len(fw.sorted_ids) == int(fw.ntiles.sum())


@pytest.mark.parametrize("case", ["workload1", "three_scenes_six_cameras"])
def test_tile_list_equals_the_sorted_lists(case):
    """binning.tile_list (one tile's list from its plain definition, the
    reference list of every sampled tile in the full-size GPU tests) equals
    the tile's range of the globally sorted intersections (pinned to Python's
    sorted() above), for every tile: one camera, and three scenes seen by six
    cameras of uneven, ragged sizes (camera lookup, tile offsets, pair
    offsets).  The tile shapes include a non-square one, so swapped tile
    coordinates cannot pass."""
    if case == "workload1":
        sc, off, cams = scenes.workload(1)
        cfgs = [RasterConfig()]
    else:
        scs = [scenes.make_scene(n, 900 + i, -3.0, 0.5, 0) for i, n in enumerate((300, 500, 200))]
        sc, off = scenes.concat_scenes(scs)
        res = [(96, 64), (130, 70), (64, 64), (200, 90), (50, 120), (128, 96)]
        cams = scenes.sphere_cameras(6, 4.0, res, scene_of_cam=[0, 1, 2, 0, 1, 2])
        cfgs = [RasterConfig(), RasterConfig(tile_w=32, tile_h=8)]
    for cfg in cfgs:
        fw = render_forward(sc, off, cams, cfg, tiles=[])
        T = int(fw.lay.tile_off[-1])
        nonempty = 0
        for t in range(T):
            want = fw.sorted_ids[fw.ranges[t]:fw.ranges[t + 1]]
            got = binning.tile_list(fw.rect, fw.ntiles, fw.depth_key, t, fw.lay)
            np.testing.assert_array_equal(got, want, err_msg=f"tile {t}")
            nonempty += len(want) > 0
        assert nonempty > T // 2


def test_binning_fp32_tracks_fp64():
    """The FP32 sequence agrees with the FP64 projection: centre to 1e-4 px,
    the Sigma_2D diagonal to 1e-5 relative, and the FP64 ellipse's bounding box
    reproduces the same tile rectangle except within rounding distance of a
    pixel-centre boundary."""
    sc, off, cams = scenes.workload(2, n_override=20000)
    cfg = RasterConfig()
    p = projection.project(sc.means, sc.scales, sc.quats, sc.sh, 3, cams.viewmat[0],
                           cams.intrin[0], 1280, 720, cfg)
    rect, nt, dk = binning.binning_fp32(sc.means, sc.scales, sc.quats, cams.viewmat[0],
                                        cams.intrin[0], 1280, 720, cfg)
    vis = nt > 0
    assert vis.sum() > 15000
    np.testing.assert_allclose(dk[vis].view(np.float32), p["t"][vis, 2], rtol=1e-6)
    rx = cfg.lambda_ * np.sqrt(p["cov2d"][:, 0])
    ry = cfg.lambda_ * np.sqrt(p["cov2d"][:, 2])
    mx, my = p["mean2d"][:, 0], p["mean2d"][:, 1]
    xlo = np.clip(np.ceil(mx - rx - 0.5), 0, 1279)
    xhi = np.clip(np.floor(mx + rx - 0.5), 0, 1279)
    ylo = np.clip(np.ceil(my - ry - 0.5), 0, 719)
    yhi = np.clip(np.floor(my + ry - 0.5), 0, 719)
    r64 = np.stack([xlo // 16, ylo // 16, xhi // 16, yhi // 16], 1)
    agree = np.all(r64[vis] == rect[vis], axis=1)
    assert agree.mean() > 0.999


@pytest.mark.parametrize("kernel", KERNELS)
def test_rects_cover_support(kernel):
    """Every pixel whose FP64 kernel value is above 1e-6 lies in the rect."""
    sc, off, cams = scenes.workload(1)
    cfg = RasterConfig(kernel=kernel)
    fw = render_forward(sc, off, cams, cfg, tiles=[])
    p = fw.proj[0]
    ys, xs = np.mgrid[0:128, 0:128]
    for i in np.nonzero(fw.ntiles)[0][:200]:
        _, _, D, L, _, _ = composite._pair_terms(xs.ravel().astype(float), ys.ravel().astype(float),
                                                 p["mean2d"][i:i + 1], p["conic"][i:i + 1],
                                                 np.array([1.0]), cfg)
        hit = L[:, 0] > 1e-6
        tx, ty = xs.ravel()[hit] // 16, ys.ravel()[hit] // 16
        assert np.all((tx >= fw.rect[i, 0]) & (tx <= fw.rect[i, 2]) &
                      (ty >= fw.rect[i, 1]) & (ty <= fw.rect[i, 3]))


# --------------------------------------------------------------------------
# projection
# --------------------------------------------------------------------------

def test_rotation_matrix():
    rng = np.random.default_rng(1)
    q = rng.normal(size=(100, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    R = projection.quat_to_rot(q)
    np.testing.assert_allclose(R @ np.swapaxes(R, 1, 2), np.broadcast_to(np.eye(3), R.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)
    c = math.cos(math.pi / 4)
    Rz = projection.quat_to_rot(np.array([[c, 0, 0, c]]))[0]
    np.testing.assert_allclose(Rz, [[0, -1, 0], [1, 0, 0], [0, 0, 1]], atol=1e-15)
    Rx = projection.quat_to_rot(np.array([[c, c, 0, 0]]))[0]
    np.testing.assert_allclose(Rx @ [0, 1, 0], [0, 0, 1], atol=1e-15)


def test_anisotropic_rotated_closed_form():
    """A splat on the optical axis with scale (s1, s2, s3) rotated 90 deg about
    z: Sigma_2D = (f/z)^2 diag(s2^2, s1^2) + eps."""
    c = math.cos(math.pi / 4)
    sc = manual_scene([[0, 0, 0]], [[0.02, 0.07, 0.03]], [[c, 0, 0, c]], [0.5], [[0.5] * 3])
    cams = one_camera(64, 64, 3.0)
    cfg = RasterConfig()
    p = projection.project(sc.means, sc.scales, sc.quats, sc.sh, 0, cams.viewmat[0], cams.intrin[0], 64, 64, cfg)
    f = float(cams.intrin[0, 0])
    s = sc.scales[0].astype(np.float64)
    qn = sc.quats[0].astype(np.float64)
    qn /= np.linalg.norm(qn)
    # rounding of the FP32 quaternion perturbs the rotation at ~1e-8
    np.testing.assert_allclose(p["cov2d"][0], [(f / 3) ** 2 * s[1] ** 2 + cfg.eps2d, 0.0,
                                               (f / 3) ** 2 * s[0] ** 2 + cfg.eps2d], rtol=1e-6, atol=1e-6)
    a, b, cc = p["cov2d"][0]
    np.testing.assert_allclose(p["conic"][0], np.array([cc, -b, a]) / (a * cc - b * b), rtol=1e-14)


def test_jacobian_against_finite_differences():
    """J of the oracle equals the central-difference Jacobian of the pinhole
    map, and Sigma_2D equals (J_fd W) Sigma (J_fd W)^T + eps I."""
    sc = scenes.make_scene(50, 77, -3.0, 0.5, 0)
    cams = one_camera(128, 96, 3.0)
    vm = cams.viewmat[0].astype(np.float64)
    vm[:, :3] = projection.quat_to_rot(np.array([[0.9, 0.1, -0.2, 0.15]]) /
                                       np.linalg.norm([0.9, 0.1, -0.2, 0.15]))[0]
    cfg = RasterConfig(clip=100.0)
    p = projection.project(sc.means, sc.scales, sc.quats, sc.sh, 0, vm, cams.intrin[0], 128, 96, cfg)
    fx, fy, cx, cy = cams.intrin[0].astype(np.float64)

    def pin(t):
        return np.array([fx * t[0] / t[2] + cx, fy * t[1] / t[2] + cy])

    for i in range(10):
        t = p["t"][i]
        Jfd = np.zeros((2, 3))
        for k in range(3):
            h = 1e-6 * max(1.0, abs(t[k]))
            e = np.zeros(3)
            e[k] = h
            Jfd[:, k] = (pin(t + e) - pin(t - e)) / (2 * h)
        np.testing.assert_allclose(p["J"][i], Jfd, rtol=1e-7, atol=1e-6)
        T = Jfd @ vm[:, :3]
        cov = T @ p["Sigma"][i] @ T.T
        np.testing.assert_allclose(p["cov2d"][i], [cov[0, 0] + cfg.eps2d, cov[0, 1], cov[1, 1] + cfg.eps2d],
                                   rtol=1e-6)
        lam = np.linalg.eigvalsh(np.array([[p["cov2d"][i, 0], p["cov2d"][i, 1]],
                                           [p["cov2d"][i, 1], p["cov2d"][i, 2]]]))
        assert lam.min() >= cfg.eps2d * (1 - 1e-12)


def _real_sh(l, m, theta, phi):
    """Real orthonormal SH from scipy's complex ones (Condon-Shortley phase)."""
    if m == 0:
        return sps.sph_harm_y(l, 0, theta, phi).real
    if m > 0:
        return math.sqrt(2) * (-1) ** m * sps.sph_harm_y(l, m, theta, phi).real
    return math.sqrt(2) * (-1) ** m * sps.sph_harm_y(l, -m, theta, phi).imag


def test_sh_basis_against_scipy():
    rng = np.random.default_rng(3)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = oracle_sh.basis(d, 3)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    for l in range(4):
        for m in range(-l, l + 1):
            k = l * l + l + m
            ref = _real_sh(l, m, theta, phi)
            ratio = Y[:, k] / np.where(np.abs(ref) > 1e-3, ref, np.nan)
            ratio = ratio[np.isfinite(ratio)]
            assert np.allclose(np.abs(ratio), 1.0, atol=1e-10), (l, m)
            assert np.allclose(ratio, ratio[0], atol=1e-10), (l, m)   # one sign per function


def test_sh_gradient_against_finite_differences():
    rng = np.random.default_rng(4)
    d = rng.normal(size=(20, 3))
    G = oracle_sh.basis_grad(d, 3)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd = (oracle_sh.basis(d + e, 3) - oracle_sh.basis(d - e, 3)) / (2 * h)
        np.testing.assert_allclose(G[:, :, j], fd, atol=1e-8)


# --------------------------------------------------------------------------
# reverse pass
# --------------------------------------------------------------------------

def general_camera(W, H):
    """A camera with fx != fy, an off-centre principal point and a rotated
    view, so that no symmetry of the front camera hides a mistake."""
    c = np.array([0.4, -0.3, -2.9])
    vm = scenes.look_at_origin(c)
    ang = 0.3
    roll = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    vm = roll @ vm
    f = scenes.focal_for(W)
    intr = np.array([[1.1 * f, 0.9 * f, 0.45 * W, 0.55 * H]], np.float32)
    return scenes.Cameras(vm[None].astype(np.float32), intr, np.array([W], np.int32),
                          np.array([H], np.int32))


def _tiny_grad_problem(seed, deg=1, n=12, W=28, H=20):
    sc = scenes.make_scene(n, 500 + seed, -2.2, 0.4, deg)
    cams = general_camera(W, H)
    G = scenes.upstream_grad(cams, 7100 + seed)
    return sc, cams, G


def _loss_and_grads(sc, cams, G, cfg):
    fw = render_forward(sc, np.array([0, sc.n]), cams, cfg, want_pairs=True)
    g = render_backward(fw, sc, cams, G)
    return float(np.dot(G.astype(np.float64), fw.image)), g


def _rms_close(a, b, rel):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    rms = math.sqrt(np.mean(b * b)) if b.size else 0.0
    return np.all(np.abs(a - b) <= rel * (np.abs(b) + rms))


@pytest.mark.parametrize("seed,clip,kernel",
                         [(0, 1.3, "linear"), (1, 1.3, "linear"), (2, 0.2, "linear"),
                          (3, 1.3, "gaussian"), (4, 1.3, "laplacian"), (5, 1.3, "cosine"),
                          (6, 1.3, "quadratic")])
def test_reverse_pass_against_finite_differences(seed, clip, kernel):
    """clip 0.2 clamps the Jacobian's tangent for several splats; the other
    kernels of the family are checked the same way (with their printed DA
    lambda where the paper gives one, 1 for the Gaussian)."""
    sc, cams, G = _tiny_grad_problem(seed)
    lam = {"linear": 2.5, "gaussian": 1.0, "laplacian": 1.0, "cosine": 2.5, "quadratic": 6.0}
    cfg = RasterConfig.strict(clip=clip, kernel=kernel, lambda_=lam[kernel])
    if clip < 1:
        fw = render_forward(sc, np.array([0, sc.n]), cams, cfg, tiles=[])
        assert (~fw.proj[0]["u_free"]).sum() >= 3
    _, g = _loss_and_grads(sc, cams, G, cfg)
    fields = dict(means=sc.means, scales=sc.scales, quats=sc.quats, opacity=sc.opacity, sh=sc.sh)
    for name, arr in fields.items():
        flat = arr.reshape(-1)
        fd = np.zeros(flat.size)
        for i in range(flat.size):
            h = 1e-6 * max(1.0, abs(float(flat[i])))
            vals = []
            for sgn in (+1, -1):
                pert = {k: v.astype(np.float64).copy() for k, v in fields.items()}
                pert[name].reshape(-1)[i] += sgn * h
                sc2 = scenes.Scene(pert["means"], pert["scales"], pert["quats"], pert["opacity"],
                                   pert["sh"], sc.sh_degree)
                fw = render_forward(sc2, np.array([0, sc.n]), cams, cfg)
                vals.append(float(np.dot(G.astype(np.float64), fw.image)))
            fd[i] = (vals[0] - vals[1]) / (2 * h)
        assert _rms_close(g[name].reshape(-1), fd, 1e-5), name


def test_alpha_channel_gradient_against_finite_differences():
    """Loss = G . image + GA . (1 - T_final): the accumulated-opacity term of
    the reverse pass against central differences of the forward pass."""
    sc, cams, G = _tiny_grad_problem(3)
    cfg = RasterConfig.strict()
    rng = np.random.default_rng(77)
    GA = rng.normal(size=int(cams.width[0]) * int(cams.height[0]))

    def loss(scene):
        fw = render_forward(scene, np.array([0, sc.n]), cams, cfg, want_pairs=True)
        return float(np.dot(G.astype(np.float64), fw.image) + np.dot(GA, 1.0 - fw.final_T)), fw

    _, fw = loss(sc)
    g = render_backward(fw, sc, cams, G, dL_dalpha=GA)
    g_img = render_backward(fw, sc, cams, G)
    assert not np.allclose(g["opacity"], g_img["opacity"])     # the term is not empty
    fields = dict(means=sc.means, scales=sc.scales, quats=sc.quats, opacity=sc.opacity, sh=sc.sh)
    for name in ("means", "opacity", "scales"):
        flat = fields[name].reshape(-1)
        fd = np.zeros(flat.size)
        for i in range(flat.size):
            h = 1e-6 * max(1.0, abs(float(flat[i])))
            vals = []
            for sgn in (+1, -1):
                pert = {k: v.astype(np.float64).copy() for k, v in fields.items()}
                pert[name].reshape(-1)[i] += sgn * h
                sc2 = scenes.Scene(pert["means"], pert["scales"], pert["quats"], pert["opacity"],
                                   pert["sh"], sc.sh_degree)
                vals.append(loss(sc2)[0])
            fd[i] = (vals[0] - vals[1]) / (2 * h)
        assert _rms_close(g[name].reshape(-1), fd, 1e-5), name


def test_mean2d_norm_is_the_norm_of_the_projected_centre_gradient():
    sc, cams, G = _tiny_grad_problem(4)
    cfg = RasterConfig.strict()
    fw = render_forward(sc, np.array([0, sc.n]), cams, cfg, want_pairs=True)
    g = render_backward(fw, sc, cams, G)
    gm = g["pair"]["mean2d"]
    np.testing.assert_allclose(g["mean2d_norm"], np.hypot(gm[:, 0], gm[:, 1]), rtol=1e-15)
    assert np.count_nonzero(g["mean2d_norm"]) >= 3


@pytest.mark.parametrize("ags,ags_arg,ags_scope",
                         [(False, 0, 0), (True, 0, 0), (True, 1, 0), (True, 0, 1), (True, 1, 1)])
@pytest.mark.parametrize("deg", [0, 3])
def test_reverse_pass_against_autograd(ags, ags_arg, ags_scope, deg):
    """The oracle's reverse pass against autograd of an independent untiled
    transcription (tests/torch_reference.py), AGS off and under each reading
    of its weight's argument and scope (Eq. 13-14)."""
    torch = pytest.importorskip("torch")
    from tests import torch_reference as tr
    sc, cams, G = _tiny_grad_problem(5 + deg, deg=deg, n=15)
    cfg = RasterConfig.strict(ags=ags, ags_arg=ags_arg, ags_scope=ags_scope)
    _, g = _loss_and_grads(sc, cams, G, cfg)
    W, H = int(cams.width[0]), int(cams.height[0])
    fw = render_forward(sc, np.array([0, sc.n]), cams, cfg, tiles=[])
    vis = np.nonzero(fw.ntiles)[0]
    order = torch.tensor(vis[np.lexsort((vis, fw.depth_key[vis]))])
    ps = [torch.tensor(a.astype(np.float64), requires_grad=True)
          for a in (sc.means, sc.scales, sc.quats, sc.opacity, sc.sh)]
    img = tr.render(*ps[:4], ps[4], deg, torch.tensor(cams.viewmat[0].astype(np.float64)),
                    [float(v) for v in cams.intrin[0].astype(np.float64)], W, H, order,
                    lam=cfg.lambda_, eps=cfg.eps2d, clip=cfg.clip, alpha_max=cfg.alpha_max,
                    ags=ags, ags_arg=ags_arg, ags_scope=ags_scope)
    loss = (img.reshape(-1) * torch.tensor(G.astype(np.float64))).sum()
    loss.backward()
    for name, p in zip(("means", "scales", "quats", "opacity", "sh"), ps):
        assert _rms_close(g[name], p.grad.numpy(), 1e-8), name


@pytest.mark.parametrize("ags,ags_arg,ags_scope",
                         [(False, 0, 0), (True, 0, 0), (True, 1, 0), (True, 0, 1), (True, 1, 1)])
def test_ags_single_splat_closed_form(ags, ags_arg, ags_scope):
    """One isotropic splat, D' = r / sigma (Eq. 11 with Sigma_2D = sigma^2 I):
    d C / d mean2d = rgb o (x - mu') / (lambda sigma r); AGS (Eq. 13-14)
    multiplies it by omega = exp(-D'^2) (raw distance, ags_arg 0) or
    exp(-(D'/lambda)^2) (ags_arg 1).  Scope 0 leaves the colour and opacity
    gradients unscaled (dC/do = rgb L', dC/drgb = o L'); scope 1 multiplies
    them by the same omega."""
    sc, cams, cfg, sigma = _iso_setup(s=0.3, o=0.8, W=32, H=32, strict=True, ags=ags,
                                      ags_arg=ags_arg, ags_scope=ags_scope)
    W = H = 32
    G = np.zeros(3 * W * H, np.float32)
    px, py = 19, 13
    G[0 * W * H + py * W + px] = 1.0        # red channel at one pixel
    fw = render_forward(sc, np.array([0, 1]), cams, cfg, want_pairs=True)
    g = render_backward(fw, sc, cams, G)
    dx, dy = px + 0.5 - W / 2, py + 0.5 - H / 2
    r = math.hypot(dx, dy)
    Dp = r / sigma
    o = float(np.float32(0.8))
    omega = 1.0
    if ags:
        omega = math.exp(-Dp * Dp) if ags_arg == 0 else math.exp(-(Dp / cfg.lambda_) ** 2)
    # the two readings of the weight differ by orders of magnitude here
    assert 0.02 < Dp / cfg.lambda_ < 0.9
    fac = 0.5 * o / (cfg.lambda_ * sigma * r) * omega
    np.testing.assert_allclose(g["pair"]["mean2d"][0], [fac * dx, fac * dy], rtol=1e-10)
    L = 1 - r / (cfg.lambda_ * sigma)
    sc_w = omega if ags_scope == 1 else 1.0
    np.testing.assert_allclose(g["pair"]["opacity"][0], 0.5 * L * sc_w, rtol=1e-10)
    np.testing.assert_allclose(g["pair"]["rgb"][0], [o * L * sc_w, 0, 0], rtol=1e-10)
