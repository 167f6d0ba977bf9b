"""Seeded random configurations of small scenes: for each seed the scene
size, splat-size distribution, SH degree, camera set (one to four cameras of
random size, one or two scenes), tile shape, LDS batch, depth chunks and their ratio, kernel,
AGS reading, strictness, background and the deterministic flag are drawn,
and the library is compared with the oracle at the usual bars (binning
integers bit-exact, composite and gradients within 1e-5), together with the
densification statistics of the same backward pass."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import render_backward, render_forward
from paper_2411_12440_amd import scenes
from tests.gpu_helpers import (cfg_pair, compare_binning, compare_forward, compare_grads,
                               gpu_forward, pixel_flags_to_image, say)

pytestmark = pytest.mark.gpu

TILES = [(16, 16), (16, 8), (8, 8), (32, 8)]
KERNELS = [("linear", 2.5), ("linear", 1.0), ("gaussian", 1.0), ("laplacian", 1.0),
           ("cosine", 2.5), ("quadratic", 6.0)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def draw_case(seed):
    r = np.random.Generator(np.random.PCG64(40_000 + seed))
    kernel, lam = KERNELS[int(r.integers(len(KERNELS)))]
    ags = kernel == "linear" and bool(r.integers(2))
    tw, th = TILES[int(r.integers(len(TILES)))]
    cap = tw * th // 2 if tw * th >= 128 else tw * th    # forward threads per tile
    batches = [b for b in (0, 64, 128) if b <= cap]
    case = dict(
        n_scenes=int(r.integers(1, 3)),
        n=[int(r.integers(1, 900)) for _ in range(2)],
        log_scale=float(r.uniform(-4.0, -2.0)),
        sh=int(r.integers(0, 4)),
        cams=int(r.integers(1, 5)),
        res=[(int(r.integers(8, 180)), int(r.integers(8, 140))) for _ in range(4)],
        kw=dict(kernel=kernel, lambda_=lam, ags=ags, ags_arg=int(r.integers(2)),
                ags_scope=int(r.integers(2)), strict=bool(r.integers(2)),
                tile_w=tw, tile_h=th, batch=int(r.choice(batches)),
                depth_chunks=int(r.choice([1, 1, 2, 3, 5])),
                bg=tuple(float(x) for x in r.uniform(0, 1, 3)),
                deterministic=bool(r.integers(2))),
    )
    # the chunk boundary ratio from a stream of its own, so the other draws
    # stay those of the earlier cases
    r2 = np.random.Generator(np.random.PCG64(50_000 + seed))
    case["kw"]["chunk_ratio"] = int(r2.choice([0, 2, 3, 4, 8]))
    return case


@pytest.mark.parametrize("seed", range(48))
def test_random_configuration(seed):
    import torch
    c = draw_case(seed)
    say(f"random case {seed}: {c}")
    scs = [scenes.make_scene(c["n"][i], 4100 + 7 * seed + i, c["log_scale"], 0.5, c["sh"])
           for i in range(c["n_scenes"])]
    scene, off = scenes.concat_scenes(scs)
    res = c["res"][:c["cams"]]
    scene_of_cam = [i % c["n_scenes"] for i in range(c["cams"])]
    cams = scenes.sphere_cameras(c["cams"], 4.0, res, scene_of_cam=scene_of_cam)
    ocfg, gkw = cfg_pair(**c["kw"])
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    G = scenes.upstream_grad(cams, 9100 + seed)
    G = (G * ~pixel_flags_to_image(fw.flag, cams)).astype(np.float32)
    rast, sp = gpu_forward(scene, off, cams, gkw)
    from tests.gpu_helpers import gpu_arrays
    g = gpu_arrays(rast)
    compare_binning(g, fw)
    compare_forward(g, fw, cams)
    grads = rast.backward(sp, torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    go = render_backward(fw, scene, cams, G)
    compare_grads({k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()}, go, scene)
    # densification statistics of the same backward pass
    from paper_2411_12440_amd import binding as B
    from tests.test_gpu_train import _oracle_stats, _within_ulp
    from oracle import densify as odens
    N = scene.n
    acc_t = [torch.zeros(N, dtype=torch.float32, device="cuda"),
             torch.zeros(N, dtype=torch.int32, device="cuda"),
             torch.zeros(N, dtype=torch.float32, device="cuda")]
    B.ls_densify_stats(rast.cfg, rast.cams, rast.ws, rast.capacity, B.densify_acc(*acc_t))
    torch.cuda.synchronize()
    oacc = _oracle_stats(fw, go, cams, ocfg, odens.new_acc(N))
    assert np.array_equal(acc_t[1].cpu().numpy(), oacc["count"])
    _within_ulp(acc_t[2].cpu().numpy(), oacc["max_extent"], 2, "max_extent")
    from tests.gpu_helpers import assert_close
    assert_close("densify grad", acc_t[0].cpu().numpy().astype(np.float64), oacc["grad"])
