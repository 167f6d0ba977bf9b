"""FP64 CPU oracle for the 3D Linear Splatting tile rasterizer.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or
links anything in this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path:
the two meet only at the seeded FP32 input arrays.

What it computes, and where the paper fixes it:
  * projection of each splat (Sec. 3.1, Eq. 2-4): covariance from rotation
    and scale, EWA projection with the local affine Jacobian, 2D covariance;
  * the linear kernel with distribution alignment (Sec. 3.2 Eq. 10-11,
    Sec. 3.3.1 Eq. 12): L' = max(0, 1 - D'/lambda);
  * front-to-back alpha compositing (Sec. 3.1, Eq. 6), unchanged by the
    method (Sec. 3.2);
  * the reverse pass of that composite, with the adaptive gradient scaling
    of Sec. 3.3.2 (Eq. 13-14) as an option.
Tile binning and the (tile, depth) sort are not described by the paper; the
oracle defines them by an explicit FP32 operation sequence (binning.py) so
that integer outputs can be compared bit for bit.

Every function here is plain and slow on purpose.  Modules:
  config      settings (thresholds, lambda, AGS flags) as FP32 values
  sh          real spherical harmonics basis, degree <= 3
  projection  FP64 projection and its reverse pass
  binning     FP32 binning sequence, intersection list, sort, tile ranges
  composite   tiled composite (forward + reverse) and brute-force composite
  render      whole-path driver over cameras and scenes
  loss        the training loss (L1, L2, SSIM; implementation section) and its
              gradient with respect to the rendered image
  adam        one Adam step (FP64)
  densify     densification statistics and the grow / prune decision with
              the 3DLS thresholds
"""
from .config import RasterConfig  # noqa: F401
from .render import render_forward, render_backward  # noqa: F401
