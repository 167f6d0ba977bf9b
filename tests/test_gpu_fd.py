"""The library's gradients against FP64 central finite differences of the
oracle's forward pass (not of the library's FP32 image): 50 splats with SH
degree 1 in a 64 x 64 view from a general camera (fx != fy, rotated, off-centre
principal point), strict mode (no skip or stop threshold, so the forward pass
is differentiable away from the kernel's kinks), AGS off.  A seeded sample
of the splat parameters is differenced; the bar is 1e-5 relative, floored at
the sample's RMS (central differences with a step of 1e-6 are accurate to
about 1e-9 here; the library's FP32 outputs add 6e-8)."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import RasterConfig, render_forward
from paper_2411_12440_amd import scenes
from tests.gpu_helpers import say
from tests.test_oracle_pins import general_camera

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("kernel,lam", [("linear", 2.5), ("gaussian", 1.0)])
def test_gradients_against_central_differences(kernel, lam):
    import torch
    from paper_2411_12440_amd.rasterizer import Rasterizer, scene_to_device
    say(f"fd: 50 splats SH1 64x64 general camera, strict, {kernel}")
    sc = scenes.make_scene(50, 808, -2.0, 0.4, 1)
    cams = general_camera(64, 64)
    G = scenes.upstream_grad(cams, 7808)
    cfg = RasterConfig.strict(kernel=kernel, lambda_=lam)
    off = np.array([0, sc.n])
    rast = Rasterizer(cams, off, sh_degree=1, kernel=kernel, lambda_=lam, alpha_min=0.0,
                      t_min=0.0)
    sp = scene_to_device(sc)
    rast.forward(sp)
    grads = rast.backward(sp, torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    gpu = dict(means=grads["means"].cpu().numpy().T, scales=grads["scales"].cpu().numpy().T,
               quats=grads["quats"].cpu().numpy().T, opacity=grads["opacity"].cpu().numpy(),
               sh=grads["sh"].cpu().numpy().transpose(2, 0, 1))
    fields = dict(means=sc.means, scales=sc.scales, quats=sc.quats, opacity=sc.opacity, sh=sc.sh)
    rng = np.random.default_rng(9)
    for name, arr in fields.items():
        flat = arr.reshape(-1)
        idx = rng.choice(flat.size, size=min(flat.size, 30), replace=False)
        fd = np.zeros(len(idx))
        for t, i in enumerate(idx):
            h = 1e-6 * max(1.0, abs(float(flat[i])))
            vals = []
            for sgn in (+1, -1):
                pert = {k: v.astype(np.float64).copy() for k, v in fields.items()}
                pert[name].reshape(-1)[i] += sgn * h
                sc2 = scenes.Scene(pert["means"], pert["scales"], pert["quats"], pert["opacity"],
                                   pert["sh"], sc.sh_degree)
                fw = render_forward(sc2, off, cams, cfg)
                vals.append(float(np.dot(G.astype(np.float64), fw.image)))
            fd[t] = (vals[0] - vals[1]) / (2 * h)
        got = gpu[name].reshape(-1)[idx].astype(np.float64)
        rms = math.sqrt(np.mean(fd * fd))
        ratio = np.abs(got - fd) / (np.abs(fd) + rms)
        say(f"  {name}: worst |gpu - fd| / (|fd| + rms) = {ratio.max():.2e}")
        assert np.all(ratio <= 1e-5), (name, float(ratio.max()))
        assert rms > 0, name


def _crop_lists(rect, nt, dk, tiles):
    """Per crop tile, the subset-local ids whose rectangle holds it, in
    (depth key, id) order: the tile lists of their plain definition."""
    out = {}
    for tx, ty in tiles:
        sel = (nt > 0) & (rect[:, 0] <= tx) & (tx <= rect[:, 2]) & (rect[:, 1] <= ty) & (ty <= rect[:, 3])
        ids = np.nonzero(sel)[0]
        out[(tx, ty)] = ids[np.lexsort((ids, dk[ids].astype(np.int64)))]
    return out


def test_multi_scene_crop_against_central_differences():
    """The uneven multi-scene workload (4 scenes, 3.7M splats): one camera of
    the 2M-splat scene rendered by the library with its benchmark settings
    (16x16 tiles, seven depth chunks; the default skip/stop thresholds; AGS
    off, since with AGS the result is not a gradient) and an upstream
    gradient that is non-zero on the central 64 x 64 crop only (and zero on
    the crop's flagged pixels, as in the parity tests).  50 random splats
    that contribute to the crop are differenced: FP64 central differences of
    the oracle's crop composite, re-projecting and re-binning the perturbed
    splat each time.  A sample whose perturbation moves the splat within a
    tile list (a change of blending order, where the image jumps) is skipped.
    Bar: 1e-5 relative, floored at the field sample's RMS."""
    import torch
    from oracle import binning, composite, projection
    from paper_2411_12440_amd.rasterizer import Rasterizer, scene_to_device
    scene, off, cams = scenes.workload(5)
    c = 56                                  # scene 3 (2M splats), 1600 x 1063
    s = int(cams.scene_of_cam[c])
    W, H = int(cams.width[c]), int(cams.height[c])
    say(f"fd: workload 5, camera {c} ({W}x{H}, scene {s}), central 64x64 crop, 50 splats")
    one = cams.subset([c])
    cfg = RasterConfig(ags=False)
    lo, hi = int(off[s]), int(off[s + 1])
    x0, y0 = (W // 2 - 32) // 16 * 16, (H // 2 - 32) // 16 * 16
    tiles = [(x0 // 16 + i, y0 // 16 + j) for j in range(4) for i in range(4)]
    # the splats whose lists reach the crop (no other splat can change it)
    rect, nt, dk = binning.binning_fp32(scene.means[lo:hi], scene.scales[lo:hi], scene.quats[lo:hi],
                                        one.viewmat[0], one.intrin[0], W, H, cfg)
    hit = (nt > 0) & (rect[:, 0] <= tiles[-1][0]) & (rect[:, 2] >= tiles[0][0]) & \
          (rect[:, 1] <= tiles[-1][1]) & (rect[:, 3] >= tiles[0][1])
    sub = lo + np.nonzero(hit)[0]
    rect, nt, dk = rect[hit], nt[hit], dk[hit]
    f64 = {k: np.asarray(getattr(scene, k)[sub], np.float64)
           for k in ("means", "scales", "quats", "opacity", "sh")}

    def proj(fields, idx=None):
        sl = slice(None) if idx is None else slice(idx, idx + 1)
        return projection.project(fields["means"][sl], fields["scales"][sl], fields["quats"][sl],
                                  fields["sh"][sl], 3, one.viewmat[0], one.intrin[0], W, H, cfg)

    base = proj(f64)
    lists = _crop_lists(rect, nt, dk, tiles)
    pix = {t: composite._tile_pixels(t[0], t[1], W, H, cfg) for t in tiles}

    def crop_loss(p, opac, lists_, which):
        tot = 0.0
        for t in which:
            px, py = pix[t]
            r = composite.composite_tile(lists_[t], px, py, p["mean2d"], p["conic"], opac, p["rgb"],
                                         cfg)
            tot += float(np.sum(Gc[t] * r["C"]))
        return tot

    # upstream gradient on the crop, zero on flagged pixels; the contributing splats
    G_full = scenes.upstream_grad(one, 7805)
    G = np.zeros_like(G_full)
    Gc, contrib = {}, set()
    for t in tiles:
        px, py = pix[t]
        r = composite.composite_tile(lists[t], px, py, base["mean2d"], base["conic"], f64["opacity"],
                                     base["rgb"], cfg, want_pairs=True)
        ok = ~r["flag"]
        g = np.stack([G_full[ch * W * H + py * W + px] for ch in range(3)], axis=1) * ok[:, None]
        Gc[t] = g.astype(np.float64)
        for ch in range(3):
            G[ch * W * H + py * W + px] = g[:, ch]
        if r["pairs"] is not None:
            contrib.update(int(i) for i in np.unique(r["pairs"]["id"]))
    pick = np.random.default_rng(55).choice(sorted(contrib), size=50, replace=False)

    rast = Rasterizer(one, off, capacity=1 << 25, sh_degree=3, depth_chunks=7, ags=False)
    sp = scene_to_device(scene)
    rast.forward(sp)
    grads = rast.backward(sp, torch.from_numpy(G.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    gpu = dict(means=grads["means"].cpu().numpy().T, scales=grads["scales"].cpu().numpy().T,
               quats=grads["quats"].cpu().numpy().T, opacity=grads["opacity"].cpu().numpy(),
               sh=grads["sh"].cpu().numpy().transpose(2, 0, 1))
    del rast, grads, sp

    rng = np.random.default_rng(56)
    skipped = 0
    for name in ("means", "scales", "quats", "opacity", "sh"):
        fd, got = [], []
        for i in pick:
            shape = f64[name].shape[1:]
            j = int(rng.integers(int(np.prod(shape)))) if shape else None
            x = f64[name][i].reshape(-1)[j] if shape else f64[name][i]
            h = 1e-6 * max(1.0, abs(float(x)))
            vals, moved = [], False
            for sgn in (+1, -1):
                fields = {k: v.copy() for k, v in f64.items()}
                if shape:
                    fields[name][i].reshape(-1)[j] += sgn * h
                else:
                    fields[name][i] += sgn * h
                p1 = proj(fields, i)
                p = dict(base)
                for k in ("mean2d", "conic", "rgb"):
                    p[k] = base[k].copy()
                    p[k][i] = p1[k][0]
                # re-bin the perturbed splat: its tiles and its place in each list
                r1, n1, d1 = binning.binning_fp32(fields["means"][i:i + 1], fields["scales"][i:i + 1],
                                                  fields["quats"][i:i + 1], one.viewmat[0],
                                                  one.intrin[0], W, H, cfg)
                rect2, nt2, dk2 = rect.copy(), nt.copy(), dk.copy()
                rect2[i], nt2[i], dk2[i] = r1[0], n1[0], d1[0]
                lists2 = _crop_lists(rect2, nt2, dk2, tiles)
                which = [t for t in tiles if i in lists[t] or i in lists2[t]]
                for t in which:
                    a, b = lists[t], lists2[t]
                    if len(a) != len(b) or not np.array_equal(a, b):
                        moved = True
                vals.append(crop_loss(p, fields["opacity"], lists2, which))
            if moved:
                skipped += 1
                continue
            fd.append((vals[0] - vals[1]) / (2 * h))
            g = gpu[name][sub[i]]
            got.append(float(g.reshape(-1)[j]) if shape else float(g))
        fd, got = np.array(fd), np.array(got)
        rms = math.sqrt(np.mean(fd * fd))
        ratio = np.abs(got - fd) / (np.abs(fd) + rms)
        say(f"  {name}: {len(fd)} samples, worst |gpu - fd| / (|fd| + rms) = {ratio.max():.2e}")
        assert rms > 0, name
        assert np.all(ratio <= 1e-5), (name, float(ratio.max()))
    assert skipped <= 25, skipped
