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


def test_training_stages_in_a_graph():
    """The loss, an Adam step and the densification decision captured into
    one HIP graph: each replay (eager work and a host synchronisation between
    replays) gives the eager results.  The image gradient, Adam and the
    decision use no float atomics (bit for bit); the per-camera loss sums do
    (to 1e-14)."""
    import torch
    from paper_2411_12440_amd import binding as B
    say("case: loss + Adam + densification decision captured in a graph")
    widths, heights = [64, 37, 90], [48, 53, 30]
    img, tgt = scenes.image_pair(widths, heights, seed=61)
    cams = B.CamerasHost(None, None, np.array(widths), np.array(heights), np.zeros(3),
                         np.array([0, 0]))
    ti, tt = torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda()
    lws = torch.empty(B.ls_loss_workspace_size(cams), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(62)
    n = 10007
    p0 = torch.from_numpy(rng.normal(size=n).astype(np.float32)).cuda()
    g0 = torch.from_numpy(rng.normal(size=n).astype(np.float32)).cuda()
    scales = torch.from_numpy(np.exp(rng.normal(-5, 1.5, (3, n))).astype(np.float32)).cuda()
    opac = torch.from_numpy(rng.uniform(0, 0.1, n).astype(np.float32)).cuda()
    acc_g = torch.from_numpy((rng.uniform(0, 1e-3, n)).astype(np.float32)).cuda()
    acc_c = torch.from_numpy(rng.integers(0, 4, n).astype(np.int32)).cuda()
    acc_e = torch.from_numpy(rng.uniform(0, 0.3, n).astype(np.float32)).cuda()
    acc = B.densify_acc(acc_g, acc_c, acc_e)
    prm = B.densify_params(0.05, grow2d=True, prune_big=True)

    def fresh():
        return dict(dimg=torch.zeros_like(ti), loss=torch.zeros(3, dtype=torch.float64, device="cuda"),
                    p=p0.clone(), m=torch.zeros_like(p0), v=torch.zeros_like(p0),
                    action=torch.zeros(n, dtype=torch.uint8, device="cuda"),
                    counts=torch.zeros(3, dtype=torch.int64, device="cuda"))

    def stages(o, stream=None):
        B.ls_loss(cams, ti, tt, o["dimg"], o["loss"], lws, stream)
        B.ls_adam(B.adam_params(0.01, 3), o["p"], g0, o["m"], o["v"], stream)
        B.ls_densify_select(prm, n, scales, opac, acc, o["action"], o["counts"], stream)

    ref = fresh()
    stages(ref)
    torch.cuda.synchronize()
    cap = fresh()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        stages(cap, side.cuda_stream)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        stages(cap, torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        for k in ("p", "m", "v"):      # Adam updates in place: start each replay from the state
            cap[k].copy_(fresh()[k])  # the eager reference started from
        cap["dimg"].zero_()
        cap["action"].zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()     # eager work between replays
        for k in ("dimg", "p", "m", "v", "action", "counts"):
            assert torch.equal(cap[k], ref[k]), f"replay {rep}: {k} differs"
        assert torch.allclose(cap["loss"], ref["loss"], rtol=1e-14, atol=0), f"replay {rep}: loss"


def test_adam_steps_replayed_from_a_graph():
    """ls_adam_device_step and the step increment captured together: three
    replays are three successive Adam steps (t = 1, 2, 3), as eager ls_adam
    calls give them (within 1 FP32 ulp: host and device form the bias
    corrections separately)."""
    import torch
    from paper_2411_12440_amd import binding as B
    say("case: Adam with a device-side step count replayed from a graph")
    rng = np.random.default_rng(71)
    n = 20011
    p0 = rng.normal(size=n).astype(np.float32)
    grads = [rng.normal(size=n).astype(np.float32) for _ in range(3)]
    # eager reference
    pe, me, ve = (torch.from_numpy(a).cuda() for a in (p0, np.zeros(n, np.float32),
                                                       np.zeros(n, np.float32)))
    for t in range(1, 4):
        B.ls_adam(B.adam_params(0.01, t), pe, torch.from_numpy(grads[t - 1]).cuda(), me, ve)
    torch.cuda.synchronize()
    # graph: the gradient buffer is refilled in place before each replay
    pg, mg, vg = (torch.from_numpy(a).cuda() for a in (p0, np.zeros(n, np.float32),
                                                       np.zeros(n, np.float32)))
    gbuf = torch.zeros(n, dtype=torch.float32, device="cuda")
    step = torch.ones(1, dtype=torch.int64, device="cuda")
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):      # warm the allocator off the capture stream
        tmp = step + 0
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        B.ls_adam_device_step(B.adam_params(0.01, 0), step, pg, gbuf, mg, vg,
                              torch.cuda.current_stream().cuda_stream)
        step.add_(1)
    for t in range(1, 4):
        gbuf.copy_(torch.from_numpy(grads[t - 1]).cuda())
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
    assert int(step.item()) == 4
    for name, a, b in (("param", pg, pe), ("m", mg, me), ("v", vg, ve)):
        x, y = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(x - y) <= 2.0 ** -23 * np.abs(y) + 1e-38), name
    del tmp
