"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Integers bit-exact; colours and gradients within 1e-5
relative (normwise and RMS-floored per element); pixels whose skip/stop
decision lies within 1e-4 of a threshold are excluded from the element check
and bounded separately."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import render_backward, render_forward
from paper_2411_12440_amd import scenes
from tests.gpu_helpers import (assert_close, cfg_pair, compare_binning, compare_contributions,
                               compare_forward, compare_grads, compare_projection, gpu_arrays,
                               gpu_forward, pixel_flags_to_image, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grads_to_numpy(g):
    return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in g.items()}


def _run_fwd_bwd(scene, off, cams, gkw, G):
    import torch
    rast, sp = gpu_forward(scene, off, cams, gkw)
    g = gpu_arrays(rast)
    grads = rast.backward(sp, torch.from_numpy(G.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    return g, _grads_to_numpy(grads)


@pytest.mark.parametrize("chunks", [1, 5])
def test_workload1_forward(chunks):
    say(f"case: workload 1 (1k splats, SH0, 128x128) forward, depth chunks {chunks}")
    scene, off, cams = scenes.workload(1)
    ocfg, gkw = cfg_pair(depth_chunks=chunks)
    rast, _ = gpu_forward(scene, off, cams, gkw)
    g = gpu_arrays(rast)
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    compare_binning(g, fw)
    compare_projection(g, fw)
    compare_forward(g, fw, cams)
    compare_contributions(rast, fw)


@pytest.mark.parametrize("tw,th,batch", [(16, 16, 0), (16, 8, 64), (8, 8, 0), (32, 8, 128)])
def test_ragged_tile_shapes(tw, th, batch):
    say(f"case: ragged 150x100, tile {tw}x{th}, batch {batch}")
    scene = scenes.make_scene(1500, 4242, -3.0, 0.5, 1)
    cams = scenes.front_camera(150, 100)
    off = np.array([0, scene.n])
    ocfg, gkw = cfg_pair(tile_w=tw, tile_h=th, batch=batch)
    rast, _ = gpu_forward(scene, off, cams, gkw)
    g = gpu_arrays(rast)
    fw = render_forward(scene, off, cams, ocfg)
    compare_binning(g, fw)
    compare_forward(g, fw, cams)


# lambda 3 takes the AGS exponent of the D'^2 reading to 9 at the support's
# edge (the FP32 weight's relative error grows with the exponent)
@pytest.mark.parametrize("ags,ags_arg,ags_scope,strict,chunks,lam",
                         [(False, 0, 0, False, 1, 2.5), (True, 0, 0, False, 1, 2.5),
                          (True, 1, 0, True, 1, 2.5), (True, 0, 1, False, 1, 2.5),
                          (False, 0, 0, True, 1, 2.5), (True, 0, 0, False, 6, 2.5),
                          (False, 0, 0, True, 4, 2.5), (True, 0, 1, False, 3, 3.0),
                          (True, 0, 0, False, 1, 2.0)])
def test_forward_backward_small(ags, ags_arg, ags_scope, strict, chunks, lam):
    say(f"case: fwd+bwd 3000 splats SH3 200x120 ags={ags} arg={ags_arg} scope={ags_scope} "
        f"strict={strict} chunks={chunks} lambda={lam}")
    scene = scenes.make_scene(3000, 77, -3.0, 0.5, 3)
    cams = scenes.front_camera(200, 120)
    off = np.array([0, scene.n])
    ocfg, gkw = cfg_pair(ags=ags, ags_arg=ags_arg, ags_scope=ags_scope, strict=strict,
                         bg=(0.1, 0.2, 0.3), depth_chunks=chunks, lambda_=lam)
    G = scenes.upstream_grad(cams, 7002)
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    # zero the upstream gradient where a decision sits on a threshold
    G = G * ~pixel_flags_to_image(fw.flag, cams)
    g, grads = _run_fwd_bwd(scene, off, cams, gkw, G)
    compare_binning(g, fw)
    compare_forward(g, fw, cams)
    go = render_backward(fw, scene, cams, G)
    compare_grads(grads, go, scene)


# the appendix's kernel family, each with its printed alignment lambda (1 for
# the Gaussian), under complete lists and depth chunks, and two tile shapes
@pytest.mark.parametrize("kernel,lam,chunks,tw,th",
                         [("gaussian", 1.0, 1, 16, 16), ("gaussian", 1.0, 4, 16, 8),
                          ("laplacian", 1.0, 1, 16, 16), ("laplacian", 1.0, 3, 8, 8),
                          ("cosine", 2.5, 1, 16, 16), ("cosine", 2.5, 3, 32, 8),
                          ("quadratic", 6.0, 1, 16, 16), ("quadratic", 6.0, 4, 16, 8)])
def test_kernel_family_forward_backward(kernel, lam, chunks, tw, th):
    say(f"case: {kernel} lambda={lam} fwd+bwd 3000 splats SH3 200x120 chunks={chunks} "
        f"tile {tw}x{th}")
    scene = scenes.make_scene(3000, 78, -3.0, 0.5, 3)
    cams = scenes.front_camera(200, 120)
    off = np.array([0, scene.n])
    ocfg, gkw = cfg_pair(kernel=kernel, lambda_=lam, bg=(0.1, 0.2, 0.3), depth_chunks=chunks,
                         tile_w=tw, tile_h=th)
    G = scenes.upstream_grad(cams, 7012)
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    G = G * ~pixel_flags_to_image(fw.flag, cams)
    g, grads = _run_fwd_bwd(scene, off, cams, gkw, G)
    compare_binning(g, fw)
    compare_forward(g, fw, cams)
    go = render_backward(fw, scene, cams, G)
    compare_grads(grads, go, scene)


@pytest.mark.parametrize("chunks", [1, 3])
def test_multi_camera_multi_scene(chunks):
    say(f"case: 3 scenes, 6 cameras of uneven size, fwd+bwd, depth chunks {chunks}")
    scs = [scenes.make_scene(n, 900 + i, -3.0, 0.5, 2) for i, n in enumerate((700, 1200, 400))]
    scene, off = scenes.concat_scenes(scs)
    res = [(96, 64), (130, 70), (64, 64), (200, 90), (50, 120), (128, 96)]
    cams = scenes.sphere_cameras(6, 4.0, res, scene_of_cam=[0, 1, 2, 0, 1, 2])
    ocfg, gkw = cfg_pair(depth_chunks=chunks)
    G = scenes.upstream_grad(cams, 7003)
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    G = G * ~pixel_flags_to_image(fw.flag, cams)
    g, grads = _run_fwd_bwd(scene, off, cams, gkw, G)
    compare_binning(g, fw)
    compare_projection(g, fw)
    compare_forward(g, fw, cams)
    go = render_backward(fw, scene, cams, G)
    compare_grads(grads, go, scene)


@pytest.mark.parametrize("chunks,ratio", [(3, 0), (7, 0), (5, 3), (4, 8)])
def test_chunk_lists_are_prefixes_of_complete_lists(chunks, ratio):
    """Through the C ABI, the library against itself: with depth chunks each
    tile's list (its chunk segments in chunk order) is a prefix of the
    complete list that ls_bin_sort builds with one chunk, long enough to
    reach every pixel's last contributor, and the composite (image, final_T,
    last) is the same bit for bit."""
    from tests.gpu_helpers import gpu_arrays, gpu_forward, tile_lists
    say(f"case: chunk lists against complete lists, 3 scenes, 6 cameras, {chunks} chunks, "
        f"ratio {ratio}")
    # large splats (log-scale N(-1.5, 0.6)): about 40% of the pixels run out
    # of transmittance, so the chunks leave entries unbuilt
    scs = [scenes.make_scene(n, 920 + i, -1.5, 0.6, 1) for i, n in enumerate((900, 1500, 600))]
    scene, off = scenes.concat_scenes(scs)
    res = [(96, 64), (130, 70), (64, 64), (200, 90), (50, 120), (128, 96)]
    cams = scenes.sphere_cameras(6, 4.0, res, scene_of_cam=[0, 1, 2, 0, 1, 2])
    _, g1kw = cfg_pair(depth_chunks=1, ags=True)
    _, gkkw = cfg_pair(depth_chunks=chunks, ags=True, chunk_ratio=ratio)
    r1, _ = gpu_forward(scene, off, cams, g1kw)
    rk, _ = gpu_forward(scene, off, cams, gkkw)
    g1, gk = gpu_arrays(r1), gpu_arrays(rk)
    T = int(r1.layout.n_tiles)
    assert T == int(rk.layout.n_tiles) and len(gk["chunk_base"]) == chunks + 1
    L1, Lk = tile_lists(g1, T), tile_lists(gk, T)
    # the tile each pixel belongs to, to find its tile's longest reach
    pix_tile = []
    for c in range(cams.n):
        W, H = int(cams.width[c]), int(cams.height[c])
        gx = -(-W // 16)
        yy, xx = np.divmod(np.arange(W * H), W)
        pix_tile.append(int(sum(-(-int(cams.width[d]) // 16) * -(-int(cams.height[d]) // 16)
                                for d in range(c))) + (yy // 16) * gx + xx // 16)
    pix_tile = np.concatenate(pix_tile)
    reach = np.zeros(T, np.int64)
    np.maximum.at(reach, pix_tile, gk["last"])
    built = 0
    for t in range(T):
        assert len(Lk[t]) <= len(L1[t]), t
        np.testing.assert_array_equal(Lk[t], L1[t][:len(Lk[t])])
        assert len(Lk[t]) >= reach[t], t
        built += len(Lk[t])
    assert built == int(gk["chunk_base"][-1]) and built < int(g1["chunk_base"][-1])
    for k in ("image", "final_T", "last"):
        assert np.array_equal(g1[k], gk[k]), k
    say(f"  {built} of {int(g1['chunk_base'][-1])} entries built; composites equal")


@pytest.mark.parametrize("chunks,ratio", [(1, 0), (7, 0), (5, 3)])
def test_workload2_binning_and_sampled_tiles(chunks, ratio):
    """100k splats, SH3, 1280x720: binning bit-exact; composite and
    gradients compared on a seeded sample of tiles (upstream gradient zero
    elsewhere)."""
    say(f"case: workload 2 (100k splats, SH3, 1280x720), depth chunks {chunks}, ratio {ratio}")
    scene, off, cams = scenes.workload(2)
    ocfg, gkw = cfg_pair(ags=True, depth_chunks=chunks, chunk_ratio=ratio)
    rng = np.random.default_rng(11)
    T = 80 * 45
    tiles = np.sort(rng.choice(T, 40, replace=False))
    fw = render_forward(scene, off, cams, ocfg, tiles=tiles, want_pairs=True)
    G = scenes.upstream_grad(cams, 7002)
    ok = ~np.isnan(fw.final_T) & ~fw.flag
    G = G * pixel_flags_to_image(ok, cams)
    g, grads = _run_fwd_bwd(scene, off, cams, gkw, G)
    compare_binning(g, fw)
    compare_projection(g, fw)
    compare_forward(g, fw, cams)
    go = render_backward(fw, scene, cams, G)
    compare_grads(grads, go, scene)


@pytest.mark.parametrize("chunks", [1, 4])
def test_alpha_gradient_mean2d_norm_and_counts(chunks):
    """The accumulated-opacity upstream gradient, the per-pair norm of the
    projected-centre gradient and the per-tile contribution counts."""
    import torch
    say(f"case: dL/dalpha + mean2d_norm, 2500 splats SH2 176x112, depth chunks {chunks}")
    scene = scenes.make_scene(2500, 61, -3.0, 0.5, 2)
    cams = scenes.front_camera(176, 112)
    off = np.array([0, scene.n])
    ocfg, gkw = cfg_pair(ags=True, bg=(0.3, 0.1, 0.2), depth_chunks=chunks)
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    keep = ~fw.flag
    G = scenes.upstream_grad(cams, 7011) * pixel_flags_to_image(keep, cams)
    GA = np.random.default_rng(7012).normal(size=fw.final_T.size).astype(np.float32) * keep
    rast, sp = gpu_forward(scene, off, cams, gkw)
    compare_contributions(rast, fw)
    grads = rast.backward(sp, torch.from_numpy(G.astype(np.float32)).cuda(),
                          dL_dalpha=torch.from_numpy(GA).cuda(), mean2d_norm=True)
    torch.cuda.synchronize()
    got = _grads_to_numpy(grads)
    go = render_backward(fw, scene, cams, G, dL_dalpha=GA)
    compare_grads(got, go, scene)
    assert_close("mean2d_norm", got["mean2d_norm"], go["mean2d_norm"])
    # the alpha term changes the result (it is not silently ignored)
    g0 = render_backward(fw, scene, cams, G)
    assert np.linalg.norm(go["opacity"] - g0["opacity"]) > 1e-3 * np.linalg.norm(g0["opacity"])


def test_empty_and_culled():
    import torch
    say("case: every splat behind the camera; and an empty scene")
    scene = scenes.make_scene(500, 5, -3.0, 0.5, 0)
    scene.means[:, 2] = -5.0            # behind the camera at z = -3
    cams = scenes.front_camera(64, 48)
    off = np.array([0, scene.n])
    ocfg, gkw = cfg_pair(bg=(0.25, 0.5, 0.75))
    rast, _ = gpu_forward(scene, off, cams, gkw)
    g = gpu_arrays(rast)
    assert g["n_isect"] == 0 and np.all(g["ntiles"] == 0)
    img = g["image"].reshape(3, -1)
    np.testing.assert_array_equal(img[0], 0.25)
    np.testing.assert_array_equal(img[2], 0.75)
    assert np.all(g["final_T"] == 1.0) and np.all(g["last"] == 0)
    empty = scenes.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                         np.zeros((0, 4), np.float32), np.zeros(0, np.float32),
                         np.zeros((0, 1, 3), np.float32), 0)
    rast, sp = gpu_forward(empty, np.array([0, 0]), cams, gkw)
    g = gpu_arrays(rast)
    assert g["n_isect"] == 0
    np.testing.assert_array_equal(g["image"].reshape(3, -1)[1], 0.5)
    grads = rast.backward(sp, torch.ones(3 * 64 * 48, device="cuda"))
    torch.cuda.synchronize()


@pytest.mark.parametrize("chunks", [1, 4])
def test_capacity_overflow_is_reported(chunks):
    say(f"case: intersection capacity too small, depth chunks {chunks}")
    import torch
    from paper_2411_12440_amd.rasterizer import Rasterizer, scene_to_device
    scene, off, cams = scenes.workload(1)
    ocfg, gkw = cfg_pair(bg=(0.5, 0.5, 0.5), depth_chunks=chunks)
    rast = Rasterizer(cams, off, capacity=100, sh_degree=0, **gkw)
    sp = scene_to_device(scene)
    rast.forward(sp, check_capacity=False)
    torch.cuda.synchronize()
    fw = render_forward(scene, off, cams, ocfg)
    assert rast.n_isect() == len(fw.sorted_ids) > 100
    assert rast.overflowed()
    if chunks == 1:
        assert torch.all(rast.image == 0.5)
    # growing the capacity recovers the exact result
    rast.forward(sp, check_capacity=True)
    torch.cuda.synchronize()
    g = gpu_arrays(rast)
    compare_binning(g, fw)
    compare_forward(g, fw, cams)


@pytest.mark.parametrize("chunks", [1, 6])
def test_fullscreen_splats(chunks):
    """A few splats larger than the image (every tile) among small ones; the
    keygen load balancing must give every tile its entry."""
    say(f"case: full-screen splats, depth chunks {chunks}")
    scene = scenes.make_scene(800, 31, -3.0, 0.5, 0)
    scene.scales[:5] = 3.0
    cams = scenes.front_camera(160, 96)
    off = np.array([0, scene.n])
    ocfg, gkw = cfg_pair(depth_chunks=chunks)
    rast, _ = gpu_forward(scene, off, cams, gkw)
    g = gpu_arrays(rast)
    fw = render_forward(scene, off, cams, ocfg)
    assert fw.ntiles[:5].min() == 60
    compare_binning(g, fw)
    compare_forward(g, fw, cams)


def test_autograd_function():
    import torch
    from paper_2411_12440_amd.rasterizer import Rasterizer, render, scene_to_device
    say("case: torch.autograd.Function")
    scene = scenes.make_scene(1000, 8, -3.0, 0.5, 1)
    cams = scenes.front_camera(96, 80)
    off = np.array([0, scene.n])
    ocfg, gkw = cfg_pair(strict=True)
    sp = scene_to_device(scene)
    rast = Rasterizer(cams, off, sh_degree=1, **gkw)
    leaves = [sp[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]
    img = render(*leaves, rast)
    G = scenes.upstream_grad(cams, 7010)
    (img * torch.from_numpy(G).cuda()).sum().backward()
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    go = render_backward(fw, scene, cams, G)
    got = {k: l.grad.detach().cpu().numpy().astype(np.float64)
           for k, l in zip(("means", "scales", "quats", "opacity", "sh"), leaves)}
    compare_grads(got, go, scene)


def test_autograd_stale_forward_raises():
    """A second render through the same Rasterizer overwrites the workspace
    the first graph node's backward pass reads: that backward raises, and the
    second one (whose forward is current) still runs."""
    import torch
    from paper_2411_12440_amd.rasterizer import (Rasterizer, StaleForwardError, render,
                                                 scene_to_device)
    say("case: stale forward raises in backward")
    scene = scenes.make_scene(300, 9, -3.0, 0.5, 0)
    cams = scenes.front_camera(64, 48)
    rast = Rasterizer(cams, np.array([0, scene.n]), sh_degree=0)
    sp = scene_to_device(scene)
    leaves1 = [sp[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]
    leaves2 = [sp[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]
    img1 = render(*leaves1, rast)
    img2 = render(*leaves2, rast)
    with pytest.raises(StaleForwardError):
        img1.sum().backward()
    img2.sum().backward()
    torch.cuda.synchronize()
    assert all(l.grad is not None and torch.isfinite(l.grad).all() for l in leaves2)


@pytest.mark.parametrize("chunks", [1, 7])
def test_backward_sums_start_at_zero(chunks):
    """Every backward pass starts its per-pair sums from zero: three backward
    passes after one forward, and one after a second forward, give the same
    per-pair sums (up to the order of the FP64 atomics) and the oracle's
    gradients; a backward with a different upstream gradient in between
    gives its own sums and changes nothing for the ones after it."""
    import torch
    say(f"case: repeated backward passes after one forward, depth chunks {chunks}")
    scs = [scenes.make_scene(n, 930 + i, -3.0, 0.5, 1) for i, n in enumerate((900, 500))]
    scene, off = scenes.concat_scenes(scs)
    cams = scenes.sphere_cameras(3, 4.0, [(96, 80), (150, 70), (64, 64)], scene_of_cam=[0, 1, 0])
    ocfg, gkw = cfg_pair(depth_chunks=chunks, ags=True)
    G = scenes.upstream_grad(cams, 7021)
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    G = (G * ~pixel_flags_to_image(fw.flag, cams)).astype(np.float32)
    rast, sp = gpu_forward(scene, off, cams, gkw)
    Gd = torch.from_numpy(G).cuda()
    M = int(rast.layout.n_pairs)

    def sums():
        torch.cuda.synchronize()
        return rast.view("grad2d", torch.float64, 9 * M).cpu().numpy().reshape(9, M).copy()

    first = _grads_to_numpy(rast.backward(sp, Gd))
    ref = sums()
    scale = np.abs(ref).max()
    assert scale > 0
    for rep in range(2):
        rast.backward(sp, Gd)
        assert np.abs(sums() - ref).max() <= 1e-12 * scale, rep
    # a different upstream gradient (twice the first: exact in FP32, and every
    # FP64 term of the sums scales by 2 exactly)
    rast.backward(sp, 2.0 * Gd)
    assert np.abs(sums() - 2.0 * ref).max() <= 2e-12 * scale
    rast.forward(sp)
    torch.cuda.synchronize()
    last = _grads_to_numpy(rast.backward(sp, Gd))
    assert np.abs(sums() - ref).max() <= 1e-12 * scale
    go = render_backward(fw, scene, cams, G)
    compare_grads(first, go, scene)
    compare_grads(last, go, scene)


@pytest.mark.parametrize("chunks,ratio", [(1, 0), (3, 0), (5, 3)])
def test_deterministic_backward(chunks, ratio):
    """Deterministic mode: two backward passes give bitwise-equal splat
    gradients; the per-pair 2D gradients and the image of the batched call
    equal, bit for bit, those of each camera rendered alone; and the
    gradients meet the oracle bar."""
    import torch
    from paper_2411_12440_amd.rasterizer import Rasterizer
    say(f"case: deterministic backward, 3 scenes, 6 cameras, depth chunks {chunks}, ratio {ratio}")
    scs = [scenes.make_scene(n, 910 + i, -3.0, 0.5, 2) for i, n in enumerate((700, 1200, 400))]
    scene, off = scenes.concat_scenes(scs)
    res = [(96, 64), (130, 70), (64, 64), (200, 90), (50, 120), (128, 96)]
    cams = scenes.sphere_cameras(6, 4.0, res, scene_of_cam=[0, 1, 2, 0, 1, 2])
    ocfg, gkw = cfg_pair(depth_chunks=chunks, deterministic=True, ags=True, chunk_ratio=ratio)
    G = scenes.upstream_grad(cams, 7013)
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    G = (G * ~pixel_flags_to_image(fw.flag, cams)).astype(np.float32)
    rast, sp = gpu_forward(scene, off, cams, gkw)
    Gd = torch.from_numpy(G).cuda()
    M = int(rast.layout.n_pairs)
    runs = []
    for _ in range(2):
        gr = rast.backward(sp, Gd)
        torch.cuda.synchronize()
        runs.append(({k: v.cpu().numpy() for k, v in gr.items()},
                     rast.view("grad2d", torch.float64, 9 * M).cpu().numpy().reshape(9, M)))
    for k in runs[0][0]:
        assert np.array_equal(runs[0][0][k], runs[1][0][k]), k
    assert np.array_equal(runs[0][1], runs[1][1])
    go = render_backward(fw, scene, cams, G)
    compare_grads(_grads_to_numpy(rast.backward(sp, Gd)), go, scene)
    image = rast.image.cpu().numpy()
    g2d = runs[0][1]
    pix = 0
    for c in range(cams.n):
        one = cams.subset([c])
        r1 = Rasterizer(one, off, sh_degree=scene.sh_degree, **gkw)
        r1.forward(sp)
        W, H = int(cams.width[c]), int(cams.height[c])
        n = W * H
        r1.backward(sp, Gd[3 * pix: 3 * (pix + n)].contiguous())
        torch.cuda.synchronize()
        assert np.array_equal(r1.image.cpu().numpy(), image[3 * pix: 3 * (pix + n)]), c
        m1 = int(r1.layout.n_pairs)
        one2d = r1.view("grad2d", torch.float64, 9 * m1).cpu().numpy().reshape(9, m1)
        p0 = int(fw.lay.pair_off[c])
        assert np.array_equal(one2d, g2d[:, p0:p0 + m1]), c
        pix += n


def test_non_finite_splats_are_culled():
    """Splats with a non-finite centre, scale or rotation touch no tile on
    either side; the rest of the scene renders and differentiates as usual,
    and the culled splats receive exactly zero gradient."""
    say("case: non-finite centres, scales and rotations among 400 splats")
    scene = scenes.make_scene(400, 321, -3.0, 0.5, 1)
    bad = np.array([0, 1, 2, 3, 4, 5])
    scene.means[0, 0] = np.nan
    scene.means[1, 2] = np.inf
    scene.means[2, 1] = -np.inf
    scene.scales[3, 1] = np.inf
    scene.quats[4, :] = np.nan
    scene.scales[5, 0] = np.nan
    cams = scenes.front_camera(96, 64)
    off = np.array([0, scene.n])
    ocfg, gkw = cfg_pair()
    G = scenes.upstream_grad(cams, 7321)
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    G = G * ~pixel_flags_to_image(fw.flag, cams)
    g, grads = _run_fwd_bwd(scene, off, cams, gkw, G)
    assert np.all(g["ntiles"][bad] == 0) and np.all(fw.ntiles[bad] == 0)
    assert np.count_nonzero(g["ntiles"]) > 200
    compare_binning(g, fw)
    compare_forward(g, fw, cams)
    assert np.all(np.isfinite(g["image"]))
    go = render_backward(fw, scene, cams, G)
    ok = np.ones(scene.n, bool)
    ok[bad] = False
    for k, v in grads.items():
        rows = v.T if v.ndim == 2 else (v.transpose(2, 0, 1) if v.ndim == 3 else v)
        ref = go[k]
        assert np.all(rows[bad] == 0.0), k
        assert_close(f"d_{k}", rows[ok].astype(np.float64), ref[ok])
