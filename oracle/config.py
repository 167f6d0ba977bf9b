"""Oracle settings.  Every real value is held as the FP32 number the GPU side
receives, and is upcast exactly when used in FP64 arithmetic.

lambda_   distribution-alignment factor of Eq. 12 (Sec. 3.3.1); the paper uses
          2.5, and 1.0 gives the plain linear kernel of Eq. 10.
ags       adaptive gradient scaling of Eq. 13-14 (Sec. 3.3.2) in the reverse pass.
ags_arg   0: omega = exp(-D'^2) with the raw 2D Mahalanobis distance D' (the
          literal reading of Eq. 13); 1: omega = exp(-(D'/lambda)^2).
ags_scope 0: omega scales only the gradient that flows through the kernel value
          L' into the geometry (Eq. 14 scales grad L'); 1: omega scales every
          gradient of the (pixel, splat) pair.
kernel    the attenuation f(D) of the generalised kernel E(x) = f(D(x)) (appendix,
          "Generalizing the 3DGS Kernel Function"), evaluated at the aligned
          distance D'/lambda (the DA of Eq. 12 applied to every kernel):
            linear     max(0, 1 - D)            (the paper's kernel, Eq. 10)
            gaussian   exp(-D^2 / 2)
            laplacian  exp(-D)
            cosine     (1 + cos(pi D)) / 2 for D <= 1, else 0
            quadratic  max(0, 1 - D^2)
          A splat's support is D'/lambda < s_f with s_f = 1 for the kernels that
          reach 0 at D = 1, 3 for the Gaussian (the 3-sigma cut of 3DGS) and
          ln 255 for the Laplacian (beyond it alpha < 1/255); the binning
          rectangle bounds the ellipse D' = lambda * s_f (the `extent`).
The paper leaves the rest unstated (it keeps 3DGS's blending, Sec. 3.2); the
defaults are the usual 3DGS ones: skip a splat whose alpha is below 1/255,
clamp alpha at 0.99, stop before a splat that would take transmittance below
1e-4, dilate the 2D covariance by 0.3 px^2, clip the Jacobian's tangent at
1.3x the half field of view, near/far planes 0.01 / 1e10.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _f32(x) -> float:
    return float(np.float32(x))


KERNELS = ("linear", "gaussian", "laplacian", "cosine", "quadratic")

# support radius in aligned distance D'/lambda, as the FP32 number both sides use
SUPPORT = {"linear": _f32(1.0), "gaussian": _f32(3.0), "laplacian": _f32(np.log(255.0)),
           "cosine": _f32(1.0), "quadratic": _f32(1.0)}


def extent(cfg) -> float:
    """FP32 lambda * s_f: the binning half-extent factor and the support radius
    in D' (the composite keeps a pair only while D'^2 < extent^2)."""
    return float(np.float32(np.float32(cfg.lambda_) * np.float32(SUPPORT[cfg.kernel])))


@dataclass
class RasterConfig:
    lambda_: float = 2.5
    ags: bool = False
    ags_arg: int = 0
    ags_scope: int = 0
    eps2d: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    near: float = 0.01
    far: float = 1e10
    clip: float = 1.3
    tile_w: int = 16
    tile_h: int = 16
    bg: tuple = (0.0, 0.0, 0.0)
    kernel: str = "linear"

    def __post_init__(self):
        if self.kernel not in KERNELS:
            raise ValueError(f"unknown kernel {self.kernel!r}")
        if self.ags and self.kernel != "linear":
            raise ValueError("adaptive gradient scaling (Eq. 13-14) is defined for the linear kernel")
        for name in ("lambda_", "eps2d", "alpha_min", "alpha_max", "t_min",
                     "near", "far", "clip"):
            setattr(self, name, _f32(getattr(self, name)))
        self.bg = tuple(_f32(b) for b in self.bg)

    @classmethod
    def strict(cls, **kw) -> "RasterConfig":
        """No alpha floor and no early stop: the composite is a continuous
        function of the parameters except at the alpha clamp."""
        kw.setdefault("alpha_min", 0.0)
        kw.setdefault("t_min", 0.0)
        return cls(**kw)
