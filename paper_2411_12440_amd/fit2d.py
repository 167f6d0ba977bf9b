"""2D pattern fitting with the kernel family (the kernel study of the paper's
discussion section and its appendix, Fig. 4): flat splats on the plane z = 0,
seen by a front camera, are fitted to a generated two-colour pattern with the
paper's training loss and Adam, and the PSNR is recorded over the iterations.

Each iteration runs the library end to end: project, bin_sort,
rasterize_fwd, the L1/L2/SSIM loss and its image gradient, rasterize_bwd and
one Adam step per parameter group.  With ``graph=True`` the whole iteration
(the activations and their chain rule included, Adam reading its step count
from device memory) is captured once in a HIP graph and replayed, so the
loop issues one launch per iteration and never waits for the host.  The optimised variables are the
in-plane centre, the log of the two in-plane scales (the z scale stays at 1%
of the initial in-plane scale), the quaternion, the logit of the opacity and
the degree-0 colour coefficient; the activations exp and sigmoid and their
derivatives are elementwise tensor operations between the library calls.
The number of splats is fixed (no densification), so every kernel gets the
same budget; the learning rates are the 3DGS ones, held constant.

    python -m paper_2411_12440_amd.fit2d [--size 256] [--splats 4096]
        [--iters 3000] [--freqs 4 16 32] [--graph] [--out results.json]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import binding as B
from . import scenes
from .rasterizer import Rasterizer

# kernel -> DA factor of the appendix (the Gaussian's is 1); "linear_ags" is
# the linear kernel with adaptive gradient scaling (the paper's full method)
# under the D'^2 reading of its weight, "linear_ags_n" under the D'^2 / lambda^2
# reading
LAMBDA = dict(linear=2.5, linear_ags=2.5, linear_ags_n=2.5, gaussian=1.0, laplacian=1.0,
              cosine=2.5, quadratic=6.0)
# 3DGS learning rates (centres scaled by the half-width of the visible plane)
LR = dict(means=1.6e-4, scales=5e-3, quats=1e-3, opacity=5e-2, sh=2.5e-3)


class PatternFit:
    """Splats on a plane fitted to ``target`` [3, H, W] (float32)."""

    def __init__(self, target: np.ndarray, scene0, kernel: str = "linear", ags: bool = False,
                 lambda_: float | None = None, device="cuda", graph: bool = False,
                 deterministic: bool = False):
        self.dev = torch.device(device)
        _, H, W = target.shape
        self.n = scene0.n
        self.cams = scenes.front_camera(W, H)
        lam = LAMBDA[kernel] if lambda_ is None else lambda_
        ags_arg = 0
        if kernel.startswith("linear_ags"):
            ags, ags_arg = True, 1 if kernel == "linear_ags_n" else 0
            kernel = "linear"
        self.rast = Rasterizer(self.cams, np.array([0, self.n]), device=self.dev,
                               kernel=kernel, lambda_=lam, ags=ags, ags_arg=ags_arg,
                               sh_degree=0, deterministic=deterministic)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(self.dev)
        self.raw = dict(means=t(scene0.means.T), scales=t(np.log(scene0.scales).T),
                        quats=t(scene0.quats.T),
                        opacity=t(np.log(scene0.opacity / (1.0 - scene0.opacity))),
                        sh=t(np.asarray(scene0.sh, np.float32).transpose(1, 2, 0)))
        # optimised slices: the x, y rows of the centres and of the log-scales
        self.opt = dict(means=self.raw["means"][:2], scales=self.raw["scales"][:2],
                        quats=self.raw["quats"], opacity=self.raw["opacity"], sh=self.raw["sh"])
        self.state = {k: (torch.zeros_like(v), torch.zeros_like(v)) for k, v in self.opt.items()}
        hw = 3.0 * math.tan(math.radians(30.0))
        self.lr = dict(LR, means=LR["means"] * hw)
        self.target = t(target.reshape(-1))
        self.lws = torch.empty(B.ls_loss_workspace_size(self.rast.cams), dtype=torch.uint8,
                               device=self.dev)
        self.dimg = torch.empty_like(self.target)
        self.lossv = torch.empty(1, dtype=torch.float64, device=self.dev)
        self.step_count = 0
        self.graph = None
        if graph:
            self.capture()

    def activated(self) -> dict:
        r = self.raw
        return dict(means=r["means"], scales=torch.exp(r["scales"]), quats=r["quats"],
                    opacity=torch.sigmoid(r["opacity"]), sh=r["sh"])

    def gradients(self):
        """Render, loss and backward of the current parameters: returns the
        activated splats and the gradients with respect to the optimised
        (raw) variables, full arrays."""
        sp = self.activated()
        self.rast.forward(sp)
        B.ls_loss(self.rast.cams, self.rast.image, self.target, self.dimg, self.lossv, self.lws)
        g = self.rast.backward(sp, self.dimg)
        g["scales"] = g["scales"] * sp["scales"]
        g["opacity"] = g["opacity"] * sp["opacity"] * (1.0 - sp["opacity"])
        return sp, g

    # -- one iteration captured in a HIP graph ---------------------------------
    def capture(self):
        """Capture the whole iteration in a HIP graph; step() then replays
        it.  The lists of the current parameters size the workspace first;
        a replay whose lists outgrow it raises the rasterizer's overflow
        flag (checked by fit())."""
        self.rast.forward(self.activated())
        torch.cuda.synchronize(self.dev)
        r = self.raw
        self._sp = dict(means=r["means"], scales=torch.empty_like(r["scales"]), quats=r["quats"],
                        opacity=torch.empty_like(r["opacity"]), sh=r["sh"])
        self._g = {k: torch.empty_like(v) for k, v in self._sp.items()}
        self._step_dev = torch.full((1,), self.step_count + 1, dtype=torch.int64,
                                    device=self.dev)
        side = torch.cuda.Stream(device=self.dev)
        side.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(side):            # one gradient pass off the capture stream
            self._graph_gradients()
        torch.cuda.current_stream(self.dev).wait_stream(side)
        torch.cuda.synchronize(self.dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._graph_gradients()
            self._graph_adam()

    def _graph_gradients(self):
        sp, g, r = self._sp, self._g, self.raw
        st = torch.cuda.current_stream(self.dev).cuda_stream
        torch.exp(r["scales"], out=sp["scales"])
        torch.sigmoid(r["opacity"], out=sp["opacity"])
        self.rast.project(sp)
        self.rast.bin_sort()
        self.rast.rasterize_fwd()
        B.ls_loss(self.rast.cams, self.rast.image, self.target, self.dimg, self.lossv, self.lws, st)
        self.rast.rasterize_bwd(sp, self.dimg, g)
        # the chain rule in the eager path's operation order (same rounding)
        g["scales"].mul_(sp["scales"])
        g["opacity"].mul_(sp["opacity"]).mul_(1.0 - sp["opacity"])

    def _graph_adam(self):
        g = self._g
        st = torch.cuda.current_stream(self.dev).cuda_stream
        grads = dict(means=g["means"][:2], scales=g["scales"][:2], quats=g["quats"],
                     opacity=g["opacity"], sh=g["sh"])
        for k, p in self.opt.items():
            m, v = self.state[k]
            B.ls_adam_device_step(B.adam_params(self.lr[k], 0), self._step_dev, p, grads[k], m, v,
                                  st)
        self._step_dev.add_(1)

    def step(self):
        if self.graph is not None:
            self.graph.replay()
            self.step_count += 1
            return
        _, g = self.gradients()
        self.step_count += 1
        grads = dict(means=g["means"][:2], scales=g["scales"][:2], quats=g["quats"],
                     opacity=g["opacity"], sh=g["sh"])
        for k, p in self.opt.items():
            m, v = self.state[k]
            B.ls_adam(B.adam_params(self.lr[k], self.step_count), p, grads[k].contiguous(), m, v)

    def psnr(self) -> float:
        """PSNR of the image the last iteration rendered (data range 1)."""
        mse = torch.mean((self.rast.image - self.target) ** 2).item()
        return 10.0 * math.log10(1.0 / max(mse, 1e-20))

    def fit(self, iters: int, log_every: int = 100) -> list[tuple[int, float, float]]:
        """[(iteration, PSNR, loss)] after every ``log_every`` iterations."""
        curve = []
        for it in range(1, iters + 1):
            self.step()
            if it % log_every == 0 or it == iters:
                if self.graph is not None and self.rast.overflowed():
                    raise RuntimeError("tile lists outgrew the workspace captured in the graph")
                curve.append((it, round(self.psnr(), 3), round(float(self.lossv.item()), 6)))
        return curve


def run_study(size=256, splats=4096, iters=3000, freqs=(4, 16, 32), kernels=None,
              patterns=scenes.PATTERNS, log_every=600, seed=0, graph=False):
    kernels = kernels or ["gaussian", "laplacian", "cosine", "quadratic", "linear", "linear_ags",
                          "linear_ags_n"]
    rows = []
    for pi, kind in enumerate(patterns):
        for f in freqs:
            target = scenes.pattern(kind, f, size, size, seed=500 + pi)
            for kname in kernels:
                fit = PatternFit(target, scenes.plane_splats(splats, size, size, seed=600 + seed),
                                 kernel=kname, graph=graph)
                torch.cuda.synchronize()
                t0 = time.time()
                curve = fit.fit(iters, log_every)
                torch.cuda.synchronize()
                dt = time.time() - t0
                rows.append(dict(pattern=kind, freq=f, kernel=kname, psnr=curve[-1][1],
                                 curve=curve, iters_per_s=round(iters / dt, 1)))
                print(f"{kind:8s} f={f:3d} {kname:10s} PSNR {curve[-1][1]:7.3f} dB "
                      f"({iters / dt:.0f} it/s)", file=sys.stderr, flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--splats", type=int, default=4096)
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--freqs", type=int, nargs="+", default=[4, 16, 32])
    ap.add_argument("--kernels", nargs="+", default=None)
    ap.add_argument("--graph", action="store_true",
                    help="replay each iteration from a captured HIP graph")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rows = run_study(a.size, a.splats, a.iters, tuple(a.freqs), a.kernels, graph=a.graph)
    js = json.dumps(dict(size=a.size, splats=a.splats, iters=a.iters, graph=a.graph, rows=rows))
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(js + "\n")
    print(js)


if __name__ == "__main__":
    main()
