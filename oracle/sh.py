"""Real spherical harmonics up to degree 3 for the view-dependent colour.

The paper only says each splat has a colour c_i (Eq. 6); it keeps the 3DGS
framework (Sec. 3.2, Sec. 4.1), whose colour is a degree <= 3 real SH
expansion evaluated at the unit direction from the camera centre to the splat
centre, offset by 0.5 and clamped at 0.  The basis below is written from the
closed forms of the normalised real harmonics, with the sign of each function
following the 3DGS convention (several odd-m functions carry a minus sign).
Index k = l*l + l + m orders the functions by degree l and order m.
"""
from __future__ import annotations

import math

import numpy as np

PI = math.pi
Y00 = 0.5 * math.sqrt(1.0 / PI)
Y1 = math.sqrt(3.0 / (4.0 * PI))
Y2a = 0.5 * math.sqrt(15.0 / PI)        # xy, yz, xz
Y2b = 0.25 * math.sqrt(5.0 / PI)        # 2z^2 - x^2 - y^2
Y2c = 0.25 * math.sqrt(15.0 / PI)       # x^2 - y^2
Y3a = 0.25 * math.sqrt(35.0 / (2 * PI)) # y(3x^2 - y^2), x(x^2 - 3y^2)
Y3b = 0.5 * math.sqrt(105.0 / PI)       # xyz
Y3c = 0.25 * math.sqrt(21.0 / (2 * PI)) # y(4z^2-x^2-y^2), x(4z^2-x^2-y^2)
Y3d = 0.25 * math.sqrt(7.0 / PI)        # z(2z^2 - 3x^2 - 3y^2)
Y3e = 0.25 * math.sqrt(105.0 / PI)      # z(x^2 - y^2)


def basis(d: np.ndarray, degree: int) -> np.ndarray:
    """Y[..., k] for unit directions d[..., 3]; k < (degree+1)^2."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = [np.full_like(x, Y00)]
    if degree >= 1:
        out += [-Y1 * y, Y1 * z, -Y1 * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [Y2a * x * y, -Y2a * y * z, Y2b * (2 * zz - xx - yy),
                -Y2a * x * z, Y2c * (xx - yy)]
    if degree >= 3:
        out += [-Y3a * y * (3 * xx - yy), Y3b * x * y * z,
                -Y3c * y * (4 * zz - xx - yy), Y3d * z * (2 * zz - 3 * xx - 3 * yy),
                -Y3c * x * (4 * zz - xx - yy), Y3e * z * (xx - yy),
                -Y3a * x * (xx - 3 * yy)]
    return np.stack(out, axis=-1)


def basis_grad(d: np.ndarray, degree: int) -> np.ndarray:
    """dY_k/dd of the polynomial forms above: [..., k, 3]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    zero = np.zeros_like(x)
    rows = [(zero, zero, zero)]
    if degree >= 1:
        rows += [(zero, -Y1 + zero, zero), (zero, zero, Y1 + zero), (-Y1 + zero, zero, zero)]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        rows += [(Y2a * y, Y2a * x, zero),
                 (zero, -Y2a * z, -Y2a * y),
                 (-2 * Y2b * x, -2 * Y2b * y, 4 * Y2b * z),
                 (-Y2a * z, zero, -Y2a * x),
                 (2 * Y2c * x, -2 * Y2c * y, zero)]
    if degree >= 3:
        rows += [(-Y3a * 6 * x * y, -Y3a * (3 * xx - 3 * yy), zero),
                 (Y3b * y * z, Y3b * x * z, Y3b * x * y),
                 (Y3c * 2 * x * y, -Y3c * (4 * zz - xx - 3 * yy), -Y3c * 8 * y * z),
                 (-Y3d * 6 * x * z, -Y3d * 6 * y * z, Y3d * (6 * zz - 3 * xx - 3 * yy)),
                 (-Y3c * (4 * zz - 3 * xx - yy), Y3c * 2 * x * y, -Y3c * 8 * x * z),
                 (Y3e * 2 * x * z, -Y3e * 2 * y * z, Y3e * (xx - yy)),
                 (-Y3a * (3 * xx - 3 * yy), Y3a * 6 * x * y, zero)]
    return np.stack([np.stack(r, axis=-1) for r in rows], axis=-2)
