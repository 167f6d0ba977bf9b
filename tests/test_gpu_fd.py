"""The library's gradients against FP64 central finite differences of the
oracle's forward pass (not of the library's FP32 image): 50 splats with SH
degree 1 in a 64 x 64 view from a general camera (fx != fy, rotated, off-centre
principal point), strict mode (no skip or stop threshold, so the forward pass
is differentiable away from the kernel's kinks), AGS off.  A seeded sample
of the splat parameters is differenced; the bar is 5e-5 relative, floored at
the sample's RMS: the library's 1e-5 agreement with the oracle plus the
oracle's own 1e-5 agreement with the differences."""
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
        err = np.abs(got - fd)
        assert np.all(err <= 5e-5 * (np.abs(fd) + rms)), (name, float((err / (np.abs(fd) + rms)).max()))
        assert rms > 0, name
