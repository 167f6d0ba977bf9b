"""The autotuner on the GPU: it times every candidate through a captured
graph, caches the fastest, and the configuration it picks is checked against
the FP64 oracle (tile shape changes the binning, so the oracle runs with the
chosen shape)."""
from __future__ import annotations

import json

import numpy as np
import pytest

from oracle import render_backward, render_forward
from paper_2411_12440_amd import scenes
from tests.gpu_helpers import (cfg_pair, compare_binning, compare_forward, compare_grads,
                               gpu_arrays, gpu_forward, pixel_flags_to_image, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_autotuner_choice_is_exact(tmp_path):
    import torch
    from paper_2411_12440_amd.autotune import Autotuner
    from paper_2411_12440_amd.rasterizer import scene_to_device
    say("case: autotune 3 candidates on 4000 splats SH1, 2 views")
    scene = scenes.make_scene(4000, 812, -3.0, 0.5, 1)
    cams = scenes.sphere_cameras(2, 4.0, [(200, 120), (150, 100)])
    off = np.array([0, scene.n])
    sp = scene_to_device(scene)
    dL = torch.from_numpy(scenes.upstream_grad(cams, 7031).astype(np.float32)).cuda()
    cands = [dict(tile_w=16, tile_h=16, batch=0, depth_chunks=1),
             dict(tile_w=16, tile_h=8, batch=0, depth_chunks=3),
             dict(tile_w=8, tile_h=8, batch=0, depth_chunks=1)]
    path = tmp_path / "tune.json"
    best = Autotuner(str(path)).choose(cams, off, sp, dL, 1, candidates=cands, steps=2, ags=True)
    assert best in cands
    (entry,) = json.loads(path.read_text()).values()
    assert len(entry["results"]) == 3 and all(r["ms"] > 0 for r in entry["results"])
    say(f"  timings {[r['ms'] for r in entry['results']]}, chose {best}")
    # the chosen settings against the oracle
    ocfg, gkw = cfg_pair(ags=True, tile_w=best["tile_w"], tile_h=best["tile_h"],
                         batch=best["batch"], depth_chunks=best["depth_chunks"])
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    G = scenes.upstream_grad(cams, 7031) * pixel_flags_to_image(~fw.flag, cams)
    rast, sp2 = gpu_forward(scene, off, cams, gkw)
    g = gpu_arrays(rast)
    compare_binning(g, fw)
    compare_forward(g, fw, cams)
    grads = rast.backward(sp2, torch.from_numpy(G.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    got = {k: v.double().cpu().numpy() for k, v in grads.items()}
    compare_grads(got, render_backward(fw, scene, cams, G), scene)
