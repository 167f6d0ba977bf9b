"""The 2D pattern-fitting workload (paper_2411_12440_amd/fit2d.py) on the GPU:
one iteration's loss and gradients with respect to the optimised variables
against the oracle composition (projection, binning, composite, loss,
reverse pass and the activations' chain rule, all FP64 on the CPU), and a
short fit that must raise the PSNR."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import RasterConfig, render_backward, render_forward
from oracle import loss as oloss
from paper_2411_12440_amd import scenes
from tests.gpu_helpers import assert_close, pixel_flags_to_image, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("kernel", ["linear", "gaussian", "linear_ags"])
def test_fit_iteration_matches_oracle(kernel):
    import torch
    from paper_2411_12440_amd import binding as B
    from paper_2411_12440_amd.fit2d import LAMBDA, PatternFit
    W, H = 64, 48
    say(f"fit2d iteration: {kernel} {W}x{H}")
    target = scenes.pattern("circles", 3, W, H, seed=3)
    s0 = scenes.plane_splats(300, W, H, seed=4)
    fit = PatternFit(target, s0, kernel=kernel)
    # the oracle's splats: the same raw float32 variables, activated in FP64
    raw_s = np.log(s0.scales).astype(np.float32)
    raw_o = np.log(s0.opacity / (1.0 - s0.opacity)).astype(np.float32)
    act = scenes.Scene(s0.means, np.exp(raw_s.astype(np.float64)).astype(np.float32), s0.quats,
                       (1.0 / (1.0 + np.exp(-raw_o.astype(np.float64)))).astype(np.float32),
                       s0.sh, 0)
    ocfg = RasterConfig(lambda_=LAMBDA[kernel], kernel="linear" if kernel == "linear_ags" else kernel,
                        ags=kernel == "linear_ags")
    off = np.array([0, act.n])
    fw = render_forward(act, off, fit.cams, ocfg, want_pairs=True)
    Lo, Go, _ = oloss.loss_one(fw.image.reshape(3, H, W), target.astype(np.float64))
    keep = ~pixel_flags_to_image(fw.flag, fit.cams)
    go = render_backward(fw, act, fit.cams, Go.reshape(-1) * keep)

    # the library's iteration, with the same pixels' upstream gradient zeroed
    sp = fit.activated()
    fit.rast.forward(sp)
    B.ls_loss(fit.rast.cams, fit.rast.image, fit.target, fit.dimg, fit.lossv, fit.lws)
    assert abs(float(fit.lossv.item()) - Lo) < 1e-5 * Lo
    fit.dimg *= torch.from_numpy(keep.astype(np.float32)).cuda()
    g = fit.rast.backward(sp, fit.dimg)
    torch.cuda.synchronize()
    img = fit.rast.image.cpu().numpy().astype(np.float64)
    assert_close("fit2d image", img[np.tile(keep, 1)], fw.image[keep])
    s_act = act.scales.astype(np.float64)
    o_act = act.opacity.astype(np.float64)
    gs = g["scales"].cpu().numpy().T.astype(np.float64) * sp["scales"].cpu().numpy().T
    gop = g["opacity"].cpu().numpy().astype(np.float64)
    gop = gop * (sp["opacity"].cpu().numpy() * (1.0 - sp["opacity"].cpu().numpy()))
    assert_close("d/d log-scale", gs[:, :2], (go["scales"] * s_act)[:, :2])
    assert_close("d/d logit-opacity", gop, go["opacity"] * o_act * (1.0 - o_act))
    assert_close("d/d centre", g["means"].cpu().numpy().T[:, :2].astype(np.float64),
                 go["means"][:, :2])
    assert_close("d/d quaternion", g["quats"].cpu().numpy().T.astype(np.float64), go["quats"])
    assert_close("d/d colour", g["sh"].cpu().numpy().transpose(2, 0, 1).astype(np.float64),
                 go["sh"])


@pytest.mark.parametrize("kernel", ["linear", "gaussian"])
def test_fit_raises_psnr(kernel):
    from paper_2411_12440_amd.fit2d import PatternFit
    say(f"fit2d short fit: {kernel}")
    target = scenes.pattern("stripes", 2, 64, 64, seed=9)
    fit = PatternFit(target, scenes.plane_splats(1024, 64, 64, seed=10), kernel=kernel)
    fit.step()
    p0 = fit.psnr()
    curve = fit.fit(400, log_every=100)
    assert curve[-1][1] > p0 + 3.0, (p0, curve)
    assert all(np.isfinite(c[2]) for c in curve)


@pytest.mark.parametrize("kernel", ["linear", "linear_ags"])
def test_graph_iterations_match_eager(kernel):
    """The iteration captured in a HIP graph against eager iterations: before
    each of three replays the eager fit takes the graph fit's variables and
    Adam moments, and both take one step.  With the deterministic backward
    the gradients are bitwise equal, so the variables and moments may differ
    only by the bias corrections, which the graph forms on the device from
    its own step count (within a few FP32 ulp); the losses agree to the
    rounding of their FP64 sums."""
    import torch
    from paper_2411_12440_amd.fit2d import PatternFit
    W, H = 64, 48
    say(f"fit2d graph replays against eager iterations: {kernel} {W}x{H}")
    target = scenes.pattern("stripes", 4, W, H, seed=5)
    s0 = scenes.plane_splats(400, W, H, seed=6)
    eager = PatternFit(target, s0, kernel=kernel, deterministic=True)
    graph = PatternFit(target, s0, kernel=kernel, deterministic=True, graph=True)
    for it in range(3):
        for k in eager.raw:
            eager.raw[k].copy_(graph.raw[k])
        for k in eager.state:
            for a, b in zip(eager.state[k], graph.state[k]):
                a.copy_(b)
        eager.step_count = graph.step_count
        eager.step()
        graph.step()
        torch.cuda.synchronize()
        le, lg = float(eager.lossv.item()), float(graph.lossv.item())
        assert abs(le - lg) <= 1e-12 * abs(le), (it, le, lg)
        for k in eager.raw:
            x = graph.raw[k].cpu().numpy().astype(np.float64)
            y = eager.raw[k].cpu().numpy().astype(np.float64)
            assert np.all(np.abs(x - y) <= 2.0 ** -21 * np.abs(y) + 1e-9), (it, k)
        for k in eager.state:
            for a, b, nm in zip(graph.state[k], eager.state[k], ("m", "v")):
                x, y = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
                assert np.all(np.abs(x - y) <= 2.0 ** -21 * np.abs(y) + 1e-20), (it, k, nm)
    assert graph.step_count == 3 and int(graph._step_dev.item()) == 4
    assert not graph.rast.overflowed()

