"""Seeded synthetic scenes and cameras (input generation only).

This module draws splat parameters and builds camera matrices.  It holds no
step of the rendering method itself: no projection, kernel, binning or
compositing arithmetic.  Both the HIP path and the CPU oracle consume the
FP32 arrays it returns, byte for byte.

Splat parameters follow the paper's primitive (Sec. 3.1, Eq. 1-2): a centre,
per-axis scale and a rotation quaternion build the covariance; each splat also
has an opacity and a colour (Eq. 6).  Colour is stored as real spherical
harmonics coefficients of degree 0..3 in the layout ``sh[N, K, 3]`` with
``K = (degree + 1)**2``.

Distributions (drawn in this order from ``numpy.random.Generator(PCG64(seed))``,
in float64 and then cast to float32):
  1. means        U[-1, 1]^3
  2. log-scales   N(mu_s, sigma_s) per axis; scales = exp(log-scales)
  3. quaternions  g / |g| with g ~ N(0, I_4)  (uniform on S^3), order (w, x, y, z)
  4. opacity      sigmoid(N(0, 1))
  5. colour DC    SH degree 0: colour ~ U[0, 1]^3, stored as the DC coefficient
                  that the degree-0 band maps back to that colour;
                  higher degrees: DC coefficient ~ U[0, 1]^3
  6. other bands  N(0, 0.1) (degree > 0 only)

Cameras use OpenCV axes (x right, y down, z forward) and a horizontal field
of view of 60 degrees: fx = fy = W / (2 tan 30deg), cx = W/2, cy = H/2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Degree-0 real spherical-harmonic constant 1/(2 sqrt(pi)); used only to map a
# drawn colour to the coefficient that encodes it.
_SH_DC = 0.5 / math.sqrt(math.pi)

RESOLUTIONS = ((640, 480), (1280, 720), (1600, 1063), (1920, 1080))


@dataclass
class Scene:
    means: np.ndarray      # [N, 3] float32
    scales: np.ndarray     # [N, 3] float32, > 0
    quats: np.ndarray      # [N, 4] float32, (w, x, y, z), unit norm up to rounding
    opacity: np.ndarray    # [N]    float32, in (0, 1)
    sh: np.ndarray         # [N, K, 3] float32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


@dataclass
class Cameras:
    viewmat: np.ndarray    # [C, 3, 4] float32 world -> camera (rotation | translation)
    intrin: np.ndarray     # [C, 4] float32 (fx, fy, cx, cy)
    width: np.ndarray      # [C] int32
    height: np.ndarray     # [C] int32
    scene_of_cam: np.ndarray = field(default=None)  # [C] int32

    def __post_init__(self):
        if self.scene_of_cam is None:
            self.scene_of_cam = np.zeros(len(self.width), np.int32)

    @property
    def n(self) -> int:
        return int(self.width.shape[0])

    def subset(self, idx) -> "Cameras":
        idx = np.atleast_1d(np.asarray(idx))
        return Cameras(self.viewmat[idx].copy(), self.intrin[idx].copy(),
                       self.width[idx].copy(), self.height[idx].copy(),
                       self.scene_of_cam[idx].copy())


def make_scene(n: int, seed: int, log_scale_mean: float = -3.0,
               log_scale_std: float = 0.5, sh_degree: int = 0,
               rgb_dc: bool | None = None) -> Scene:
    """Draw ``n`` splats.  ``rgb_dc`` (default: True for degree 0) draws the
    colour itself uniformly in [0,1] and stores its DC coefficient."""
    if rgb_dc is None:
        rgb_dc = sh_degree == 0
    g = np.random.Generator(np.random.PCG64(seed))
    means = g.uniform(-1.0, 1.0, size=(n, 3))
    log_scales = g.normal(log_scale_mean, log_scale_std, size=(n, 3))
    q = g.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opacity = 1.0 / (1.0 + np.exp(-g.normal(0.0, 1.0, size=n)))
    k = (sh_degree + 1) ** 2
    sh = np.zeros((n, k, 3))
    dc = g.uniform(0.0, 1.0, size=(n, 3))
    sh[:, 0, :] = (dc - 0.5) / _SH_DC if rgb_dc else dc
    if k > 1:
        sh[:, 1:, :] = g.normal(0.0, 0.1, size=(n, k - 1, 3))
    return Scene(means.astype(np.float32), np.exp(log_scales).astype(np.float32),
                 q.astype(np.float32), opacity.astype(np.float32),
                 sh.astype(np.float32), sh_degree)


def concat_scenes(scenes: list[Scene]) -> tuple[Scene, np.ndarray]:
    """Concatenate scenes (same SH degree); returns the scene and the int64
    splat offsets ``[S + 1]``."""
    deg = scenes[0].sh_degree
    assert all(s.sh_degree == deg for s in scenes)
    off = np.zeros(len(scenes) + 1, np.int64)
    off[1:] = np.cumsum([s.n for s in scenes])
    cat = Scene(np.concatenate([s.means for s in scenes]),
                np.concatenate([s.scales for s in scenes]),
                np.concatenate([s.quats for s in scenes]),
                np.concatenate([s.opacity for s in scenes]),
                np.concatenate([s.sh for s in scenes]), deg)
    return cat, off


def focal_for(width: int) -> float:
    return width / (2.0 * math.tan(math.radians(30.0)))


def _intrin(w: int, h: int) -> list[float]:
    f = focal_for(w)
    return [f, f, w / 2.0, h / 2.0]


def front_camera(width: int, height: int, distance: float = 3.0) -> Cameras:
    """Camera at (0, 0, -distance) looking at the origin along +z."""
    vm = np.zeros((1, 3, 4))
    vm[0, :, :3] = np.eye(3)
    vm[0, 2, 3] = distance
    return Cameras(vm.astype(np.float32), np.array([_intrin(width, height)], np.float32),
                   np.array([width], np.int32), np.array([height], np.int32))


def look_at_origin(center: np.ndarray) -> np.ndarray:
    """[3, 4] world->camera matrix whose rows are (right, down, forward)."""
    c = np.asarray(center, np.float64)
    fwd = -c / np.linalg.norm(c)
    down_hint = np.array([0.0, 1.0, 0.0])
    if abs(fwd @ down_hint) > 0.99:
        down_hint = np.array([1.0, 0.0, 0.0])
    right = np.cross(down_hint, fwd)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    rot = np.stack([right, down, fwd])
    out = np.zeros((3, 4))
    out[:, :3] = rot
    out[:, 3] = -rot @ c
    return out


def sphere_cameras(n: int, radius: float, resolutions: list[tuple[int, int]],
                   scene_of_cam=None) -> Cameras:
    """``n`` cameras on a Fibonacci sphere of ``radius`` looking at the origin."""
    vms, intr, ws, hs = [], [], [], []
    golden = math.pi * (1.0 + math.sqrt(5.0))
    for i in range(n):
        z = 1.0 - 2.0 * (i + 0.5) / n
        rho = math.sqrt(max(0.0, 1.0 - z * z))
        az = golden * (i + 0.5)
        c = radius * np.array([rho * math.cos(az), rho * math.sin(az), z])
        vms.append(look_at_origin(c))
        w, h = resolutions[i]
        intr.append(_intrin(w, h))
        ws.append(w)
        hs.append(h)
    soc = np.zeros(n, np.int32) if scene_of_cam is None else np.asarray(scene_of_cam, np.int32)
    return Cameras(np.array(vms, np.float32), np.array(intr, np.float32),
                   np.array(ws, np.int32), np.array(hs, np.int32), soc)


def mixed_resolutions(count: int, seed: int) -> list[tuple[int, int]]:
    """A seeded permutation of the four resolutions, each repeated count/4 times."""
    assert count % len(RESOLUTIONS) == 0
    base = [r for r in RESOLUTIONS for _ in range(count // len(RESOLUTIONS))]
    g = np.random.Generator(np.random.PCG64(seed))
    perm = g.permutation(len(base))
    return [base[i] for i in perm]


def upstream_grad(cams: Cameras, seed: int) -> np.ndarray:
    """dL/dimage ~ N(0, 1), float32, planar per camera: concatenation over
    cameras of [3, H, W] blocks."""
    g = np.random.Generator(np.random.PCG64(seed))
    total = int(sum(3 * int(w) * int(h) for w, h in zip(cams.width, cams.height)))
    return g.normal(0.0, 1.0, size=total).astype(np.float32)


def image_pair(widths, heights, seed: int, noise: float | None = 0.1):
    """A rendered image and its target photograph for the training loss,
    float32, planar per camera like ``upstream_grad``.  Per camera and
    channel the target is 0.5 + 0.25 sin(a x + b y + phi) (a, b ~ U[-0.3, 0.3],
    phi ~ U[0, 2 pi]) plus U[-0.25, 0.25] texture; the render is the target
    plus N(0, noise), clipped to [0, 1].  noise=None: both images are
    independent U[0, 1] (no structure shared)."""
    g = np.random.Generator(np.random.PCG64(seed))
    imgs, tgts = [], []
    for w, h in zip(widths, heights):
        w, h = int(w), int(h)
        if noise is None:
            imgs.append(g.uniform(0.0, 1.0, 3 * w * h))
            tgts.append(g.uniform(0.0, 1.0, 3 * w * h))
            continue
        yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
        t = np.empty((3, h, w))
        for ch in range(3):
            a, b = g.uniform(-0.3, 0.3, 2)
            phi = g.uniform(0.0, 2.0 * math.pi)
            t[ch] = 0.5 + 0.25 * np.sin(a * xx + b * yy + phi) + g.uniform(-0.25, 0.25, (h, w))
        r = np.clip(t + g.normal(0.0, noise, t.shape), 0.0, 1.0)
        imgs.append(r.ravel())
        tgts.append(t.ravel())
    return (np.concatenate(imgs).astype(np.float32), np.concatenate(tgts).astype(np.float32))


PATTERNS = ("stripes", "checker", "circles")


def pattern(kind: str, freq: int, width: int, height: int, seed: int) -> np.ndarray:
    """A two-colour test pattern [3, H, W] float32 with hard edges: vertical
    stripes with ``freq`` cycles across the width, a checkerboard of squares
    W / (2 freq) pixels wide, or concentric rings with ``freq`` cycles from
    the centre to the half-width.  Pixel (x, y) is sampled at its centre;
    the two colours are U[0, 1]^3 from ``seed``."""
    g = np.random.Generator(np.random.PCG64(seed))
    c0, c1 = g.uniform(0.0, 1.0, 3), g.uniform(0.0, 1.0, 3)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64) + 0.5
    band = 2.0 * freq / width
    if kind == "stripes":
        sel = np.floor(band * xx).astype(np.int64) % 2
    elif kind == "checker":
        sel = (np.floor(band * xx).astype(np.int64) + np.floor(band * yy).astype(np.int64)) % 2
    elif kind == "circles":
        r = np.hypot(xx - width / 2.0, yy - height / 2.0)
        sel = np.floor(2.0 * band * r).astype(np.int64) % 2
    else:
        raise ValueError(f"unknown pattern {kind!r}")
    img = np.where(sel[None] == 0, c0[:, None, None], c1[:, None, None])
    return img.astype(np.float32)


def plane_splats(n: int, width: int, height: int, seed: int, distance: float = 3.0) -> Scene:
    """``n`` flat splats on the plane z = 0 seen by ``front_camera(width,
    height, distance)``: centres uniform over the visible rectangle, equal
    in-plane scales sqrt(area / n) / 2 (z scale 1% of that), a rotation about
    z uniform in [0, pi), opacity 0.5, colour U[0, 1]^3 (SH degree 0)."""
    g = np.random.Generator(np.random.PCG64(seed))
    hw = distance * math.tan(math.radians(30.0))
    hh = hw * height / width
    means = np.zeros((n, 3))
    means[:, 0] = g.uniform(-hw, hw, n)
    means[:, 1] = g.uniform(-hh, hh, n)
    s0 = 0.5 * math.sqrt(4.0 * hw * hh / n)
    scales = np.tile([s0, s0, 0.01 * s0], (n, 1))
    th = g.uniform(0.0, math.pi, n)
    quats = np.stack([np.cos(th / 2), np.zeros(n), np.zeros(n), np.sin(th / 2)], axis=1)
    colour = g.uniform(0.0, 1.0, (n, 3))
    sh = ((colour - 0.5) / _SH_DC)[:, None, :]
    return Scene(means.astype(np.float32), scales.astype(np.float32), quats.astype(np.float32),
                 np.full(n, 0.5, np.float32), sh.astype(np.float32), 0)


# ---------------------------------------------------------------------------
# The five workloads.  Seeds: scene k -> 1000 + k, extra scene s -> 5000 + s,
# upstream gradient -> 7000 + k, resolution permutation -> 9000 + k.
# ---------------------------------------------------------------------------

def workload(k: int, seed_offset: int = 0, n_override: int | None = None):
    """Return (scene, scene_splat_off [S+1] int64, cameras) for workload ``k``.

    1: 1,000 splats, SH0, log-scale N(-3, .5), one 128x128 front camera.
    2: 100,000 splats, SH3, log-scale N(-3, .5), one 1280x720 front camera.
    3: 1,000,000 splats, SH3, 16 sphere cameras (r = 4) at mixed resolutions.
    4: 3,200,000 splats, SH3, log-scale N(-4, 1), one 1920x1080 front camera.
       ``workload(40)`` gives the same scene with 8 sphere cameras at 1920x1080.
    5: 4 scenes (200k, 500k, 1M, 2M), SH3, 64 cameras (16 per scene), mixed
       resolutions.
    ``n_override`` shrinks the splat count (tests), keeping the distributions.
    """
    seed = 1000 + (4 if k == 40 else k) + seed_offset
    if k == 1:
        sc = make_scene(n_override or 1000, seed, -3.0, 0.5, 0)
        return sc, np.array([0, sc.n], np.int64), front_camera(128, 128)
    if k == 2:
        sc = make_scene(n_override or 100_000, seed, -3.0, 0.5, 3)
        return sc, np.array([0, sc.n], np.int64), front_camera(1280, 720)
    if k == 3:
        sc = make_scene(n_override or 1_000_000, seed, -3.0, 0.5, 3)
        cams = sphere_cameras(16, 4.0, mixed_resolutions(16, 9000 + 3))
        return sc, np.array([0, sc.n], np.int64), cams
    if k in (4, 40):
        sc = make_scene(n_override or 3_200_000, seed, -4.0, 1.0, 3)
        if k == 4:
            cams = front_camera(1920, 1080)
        else:
            cams = sphere_cameras(8, 4.0, [(1920, 1080)] * 8)
        return sc, np.array([0, sc.n], np.int64), cams
    if k == 5:
        sizes = (200_000, 500_000, 1_000_000, 2_000_000)
        if n_override:
            sizes = tuple(max(1, (s * n_override) // 2_000_000) for s in sizes)
        scenes = [make_scene(s, 5000 + i + seed_offset, -3.0, 0.5, 3) for i, s in enumerate(sizes)]
        sc, off = concat_scenes(scenes)
        res = mixed_resolutions(64, 9000 + 5)
        soc = np.repeat(np.arange(4, dtype=np.int32), 16)
        cams = sphere_cameras(64, 4.0, res, soc)
        return sc, off, cams
    raise ValueError(f"unknown workload {k}")
