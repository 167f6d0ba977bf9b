"""PyTorch-facing wrapper around liblsplat.

PyTorch supplies device memory (the workspace and the outputs are torch
tensors) and the stream; every stage runs in the library's HIP kernels through
the ctypes binding.  Splat attributes use the library's planar layout:
means/scales [3, N], quats [4, N], opacity [N], sh [K, 3, N] (float32, cuda).
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def scene_to_device(scene, device="cuda"):
    """numpy Scene ([N, d] arrays) -> dict of planar float32 device tensors."""
    def planar(a):
        return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32).T)).to(device)
    sh = np.asarray(scene.sh, np.float32)                       # [N, K, 3]
    return dict(means=planar(scene.means), scales=planar(scene.scales), quats=planar(scene.quats),
                opacity=torch.from_numpy(np.ascontiguousarray(scene.opacity, np.float32)).to(device),
                sh=torch.from_numpy(np.ascontiguousarray(sh.transpose(1, 2, 0))).to(device))


class Rasterizer:
    """Holds the camera set, the settings and a workspace sized for an
    intersection capacity.

    ``forward`` runs project -> bin_sort -> rasterize_fwd.  With
    ``check_capacity`` (default) it reads the overflow flag back and, if the
    lists did not fit, grows the workspace and runs again; without it nothing
    synchronises and an overflow leaves an incomplete composite
    (``overflowed()`` tells).
    """

    def __init__(self, cams, scene_splat_off, device="cuda", capacity=None, **cfg):
        self.device = torch.device(device)
        self.cfg = B.make_config(**cfg)
        self.cams_np = cams
        vm = torch.from_numpy(np.ascontiguousarray(cams.viewmat, np.float32)).to(self.device)
        it = torch.from_numpy(np.ascontiguousarray(cams.intrin, np.float32)).to(self.device)
        self.cams = B.CamerasHost(vm, it, cams.width, cams.height, cams.scene_of_cam,
                                  scene_splat_off)
        self.capacity = 0
        self.ws = None
        self.layout = None
        self.image = self.final_T = self.last = None
        # bumped by every call that overwrites what a backward pass reads (the
        # projections, lists, final transmittance, `last`) and by a regrown
        # workspace; RenderFunction checks it
        self.generation = 0
        self._alloc(int(capacity) if capacity is not None else 1 << 20)

    # -- memory ---------------------------------------------------------------
    def _alloc(self, capacity: int):
        self.generation += 1
        nbytes = B.ls_workspace_size(self.cfg, self.cams, capacity)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.capacity = capacity
        self.layout = B.ls_workspace_layout(self.cfg, self.cams, capacity)
        P = int(self.layout.n_pixels)
        if self.image is None:
            self.image = torch.empty(3 * P, dtype=torch.float32, device=self.device)
            self.final_T = torch.empty(P, dtype=torch.float32, device=self.device)
            self.last = torch.empty(P, dtype=torch.int32, device=self.device)

    def view(self, name: str, dtype, count: int, offset_elems: int = 0) -> torch.Tensor:
        """Typed view of one workspace array (see ls_layout)."""
        off = getattr(self.layout, name)
        esz = torch.tensor([], dtype=dtype).element_size()
        return self.ws[off + offset_elems * esz: off + (offset_elems + count) * esz].view(dtype)

    def n_isect(self) -> int:
        """Intersections of the complete tile lists."""
        return int(self.view("n_isect", torch.int64, 1).item())

    def n_built(self) -> int:
        """Entries actually built (all chunks)."""
        K = int(self.layout.n_chunks)
        return int(self.view("chunk_base", torch.int64, 1, K).item())

    def overflowed(self) -> bool:
        return int(self.view("flags", torch.int32, 1).item()) != 0

    def lists(self):
        """Per-chunk (chunk_base, ranges [T+1]) as numpy arrays (for tests)."""
        K, T = int(self.layout.n_chunks), int(self.layout.n_tiles)
        base = self.view("chunk_base", torch.int64, K + 1).cpu().numpy()
        rng = self.view("ranges", torch.int64, K * (T + 1)).cpu().numpy().reshape(K, T + 1)
        return base, rng

    # -- stages -----------------------------------------------------------------
    def _splats(self, sp):
        n = int(sp["opacity"].shape[0])
        return B.splats_struct(n, sp["means"], sp["scales"], sp["quats"], sp["opacity"], sp["sh"])

    def project(self, sp, stream=None):
        self.generation += 1
        B.ls_project(self.cfg, self._splats(sp), self.cams, self.ws, self.capacity,
                     self._stream(stream))

    def bin_sort(self, stream=None):
        self.generation += 1
        B.ls_bin_sort(self.cfg, self.cams, self.ws, self.capacity, self._stream(stream))

    def rasterize_fwd(self, stream=None):
        self.generation += 1
        B.ls_rasterize_fwd(self.cfg, self.cams, self.ws, self.capacity, self.image,
                           self.final_T, self.last, self._stream(stream))

    def rasterize_bwd(self, sp, dL_dimage, grads, stream=None, dL_dalpha=None):
        """grads: dict of output tensors (means, scales, quats, opacity, sh and,
        optionally, mean2d_norm [M])."""
        g = B.grads_struct(grads["means"], grads["scales"], grads["quats"], grads["opacity"],
                           grads["sh"], grads.get("mean2d_norm"))
        B.ls_rasterize_bwd(self.cfg, self._splats(sp), self.cams, self.ws, self.capacity,
                           self.final_T, self.last, dL_dimage.contiguous(),
                           None if dL_dalpha is None else dL_dalpha.contiguous(), g,
                           self._stream(stream))

    def _stream(self, stream):
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return stream.cuda_stream

    # -- composite calls ---------------------------------------------------------
    def forward(self, sp, check_capacity=True, stream=None):
        """project -> bin_sort -> rasterize_fwd.  With check_capacity, a run
        whose lists did not fit is repeated with a larger workspace (the
        complete-list count n_isect bounds what any run can need)."""
        while True:
            self.project(sp, stream)
            self.bin_sort(stream)
            self.rasterize_fwd(stream)
            if not check_capacity or not self.overflowed():
                break
            n = self.n_isect()
            grow = min(n, max(2 * self.capacity, 1 << 20))
            self._alloc(int(grow) + 1024)
        return self.image, self.final_T, self.last

    def backward(self, sp, dL_dimage, stream=None, dL_dalpha=None, mean2d_norm=False):
        grads = {k: torch.empty_like(v) for k, v in sp.items()}
        if mean2d_norm:
            grads["mean2d_norm"] = torch.empty(int(self.layout.n_pairs), dtype=torch.float32,
                                               device=self.device)
        self.rasterize_bwd(sp, dL_dimage, grads, stream, dL_dalpha)
        return grads

    def contributions(self) -> int:
        """(pixel, splat) pairs that contributed in the last forward call."""
        T = int(self.layout.n_tiles)
        return int(self.view("tile_contrib", torch.int32, T).to(torch.int64).sum().item())


class StepGraph:
    """One full pass over every camera (project -> bin_sort -> rasterize_fwd
    -> rasterize_bwd) captured once into a HIP graph and replayed.

    The graph holds the addresses of the splat tensors, the upstream
    gradient(s), the gradient outputs and the rasterizer's workspace: update
    inputs in place (``copy_``) between replays.  Nothing in the captured
    sequence synchronises with the host, so a replay whose lists outgrow the
    workspace only raises the overflow flag: check ``rast.overflowed()`` when
    the scene changes, and capture again after growing the workspace.
    """

    def __init__(self, rast: Rasterizer, sp, dL_dimage, grads, dL_dalpha=None):
        self.rast, self.sp, self.dL_dimage, self.grads = rast, sp, dL_dimage, grads
        self.dL_dalpha = dL_dalpha
        dev = rast.device
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):            # one eager pass off the capture stream
            self._step()
        torch.cuda.current_stream(dev).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step()

    def _step(self):
        r = self.rast
        r.project(self.sp)
        r.bin_sort()
        r.rasterize_fwd()
        r.rasterize_bwd(self.sp, self.dL_dimage, self.grads, dL_dalpha=self.dL_dalpha)

    def replay(self):
        self.graph.replay()


class StaleForwardError(RuntimeError):
    """The rasterizer ran another forward pass (or regrew its workspace)
    after the one a backward pass belongs to."""


def check_generation(rast, generation: int):
    if rast.generation != generation:
        raise StaleForwardError(
            "the Rasterizer's workspace was overwritten by a later forward pass (generation "
            f"{rast.generation}, this graph node's is {generation}); a Rasterizer holds the "
            "state of one forward pass at a time: run backward before the next render through "
            "it, or use one Rasterizer per live graph node")


class RenderFunction(torch.autograd.Function):
    """image = render(means, scales, quats, opacity, sh) through a Rasterizer;
    the backward pass is the library's hand-written reverse pass.  The
    Rasterizer's workspace holds one forward pass: a backward pass whose
    forward was followed by another render through the same Rasterizer
    raises StaleForwardError instead of returning wrong gradients."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacity, sh, rast: Rasterizer):
        sp = dict(means=means.contiguous(), scales=scales.contiguous(), quats=quats.contiguous(),
                  opacity=opacity.contiguous(), sh=sh.contiguous())
        image, _, _ = rast.forward(sp)
        ctx.rast = rast
        ctx.sp = sp
        ctx.generation = rast.generation
        return image.clone()

    @staticmethod
    def backward(ctx, dL_dimage):
        check_generation(ctx.rast, ctx.generation)
        g = ctx.rast.backward(ctx.sp, dL_dimage.contiguous())
        return g["means"], g["scales"], g["quats"], g["opacity"], g["sh"], None


def render(means, scales, quats, opacity, sh, rast: Rasterizer):
    return RenderFunction.apply(means, scales, quats, opacity, sh, rast)
