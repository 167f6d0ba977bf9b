"""The batched call sequence captured into a HIP graph: every replay (with
eager work and host synchronisation between replays, and an input changed in
place) must give the eager result: images, final transmittance and `last`
bit for bit (the forward uses no atomics), gradients to float-atomic
reordering; and the eager result must match the FP64 oracle."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import render_backward, render_forward
from paper_2411_12440_amd import scenes
from tests.gpu_helpers import (assert_close, cfg_pair, compare_forward, compare_grads,
                               gpu_arrays, pixel_flags_to_image, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _snapshot(rast, grads):
    out = dict(image=rast.image.clone(), final_T=rast.final_T.clone(), last=rast.last.clone())
    out.update({"g_" + k: v.clone() for k, v in grads.items()})
    return out


def _same(a, b, tag):
    import torch
    for k in ("image", "final_T", "last"):
        assert torch.equal(a[k], b[k]), f"{tag}: {k} differs"
    for k in a:
        if k.startswith("g_"):
            x, y = a[k].double().cpu().numpy(), b[k].double().cpu().numpy()
            scale = np.linalg.norm(y) + 1e-30
            assert np.linalg.norm(x - y) <= 1e-6 * scale, f"{tag}: {k}"


@pytest.mark.parametrize("chunks", [1, 3])
def test_graph_replay_matches_eager(chunks):
    import torch
    from paper_2411_12440_amd.rasterizer import Rasterizer, StepGraph, scene_to_device
    say(f"case: HIP graph of the batched step, 2 scenes x 5 cameras, depth chunks {chunks}")
    scs = [scenes.make_scene(n, 300 + i, -3.0, 0.5, 2) for i, n in enumerate((900, 1400))]
    scene, off = scenes.concat_scenes(scs)
    res = [(96, 64), (130, 70), (64, 64), (200, 90), (128, 96)]
    cams = scenes.sphere_cameras(5, 4.0, res, scene_of_cam=[0, 1, 0, 1, 1])
    ocfg, gkw = cfg_pair(ags=True, depth_chunks=chunks)
    fw = render_forward(scene, off, cams, ocfg, want_pairs=True)
    keep = pixel_flags_to_image(~fw.flag, cams)
    G1 = scenes.upstream_grad(cams, 7021) * keep
    G2 = scenes.upstream_grad(cams, 7022) * keep

    sp = scene_to_device(scene)
    rast = Rasterizer(cams, off, capacity=1 << 16, sh_degree=2, **gkw)
    rast.forward(sp)                    # sizes the workspace (host check)
    torch.cuda.synchronize()
    grads = {k: torch.empty_like(v) for k, v in sp.items()}
    dL = torch.from_numpy(G1.astype(np.float32)).cuda()

    def eager():
        rast.project(sp)
        rast.bin_sort()
        rast.rasterize_fwd()
        rast.rasterize_bwd(sp, dL, grads)
        torch.cuda.synchronize()
        return _snapshot(rast, grads)

    ref1 = eager()
    # the eager result is the oracle's
    g = gpu_arrays(rast)
    compare_forward(g, fw, cams)
    got = {k: v.double().cpu().numpy() for k, v in grads.items()}
    compare_grads(got, render_backward(fw, scene, cams, G1), scene)

    graph = StepGraph(rast, sp, dL, grads)
    for rep in range(3):
        for t in (rast.image, rast.final_T, grads["means"], grads["sh"]):
            t.fill_(-7.0)                   # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert not rast.overflowed()
        _same(_snapshot(rast, grads), ref1, f"replay {rep}")
        ref_again = eager()                 # eager calls on the same workspace in between
        _same(ref_again, ref1, f"eager after replay {rep}")
    # an input changed in place is seen by the next replay
    dL.copy_(torch.from_numpy(G2.astype(np.float32)))
    ref2 = eager()
    graph.replay()
    torch.cuda.synchronize()
    _same(_snapshot(rast, grads), ref2, "replay with new upstream gradient")
    got = {k: v.double().cpu().numpy() for k, v in grads.items()}
    compare_grads(got, render_backward(fw, scene, cams, G2), scene)
    say("  replays equal the eager results")
