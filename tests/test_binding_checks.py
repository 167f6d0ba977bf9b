"""The ctypes binding checks every tensor before its pointer reaches the
library (element type, contiguity, element count, device), and the autograd
wrapper refuses a backward pass whose forward state was overwritten.  CPU
only: every check fires before anything touches a GPU."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def _B():
    from paper_2411_12440_amd import binding as B
    return B


def test_tensor_checks_in_order():
    B = _B()
    good = torch.zeros(12, dtype=torch.float32)
    with pytest.raises(TypeError, match="float32"):
        B._dev(torch.zeros(12, dtype=torch.float64), "x", "f32", 12)
    with pytest.raises(ValueError, match="contiguous"):
        B._dev(torch.zeros(4, 6, dtype=torch.float32).t(), "x", "f32", 24)
    with pytest.raises(ValueError, match="elements"):
        B._dev(good, "x", "f32", 13)
    with pytest.raises(TypeError, match="GPU"):
        B._dev(good, "x", "f32", 12)            # right type and size, but host memory
    with pytest.raises(TypeError, match="torch tensor"):
        B._dev(np.zeros(12, np.float32), "x", "f32", 12)
    with pytest.raises(ValueError, match="required"):
        B._dev(None, "x", "f32", 12)
    assert B._dev(None, "x", "f32", 12, optional=True) == 0


def test_entry_points_check_before_calling():
    B = _B()
    cams = B.CamerasHost(None, None, np.array([40, 7]), np.array([30, 5]), np.zeros(2),
                         np.array([0, 0]))
    assert cams.n_pixels == 40 * 30 + 7 * 5
    P3 = 3 * cams.n_pixels
    f32 = torch.zeros(P3, dtype=torch.float32)
    loss = torch.zeros(2, dtype=torch.float64)
    # a float64 upstream gradient, a row-major image and a short target are refused
    with pytest.raises(TypeError, match="float32"):
        B.ls_loss(cams, f32, f32, f32.double(), loss, torch.zeros(8, dtype=torch.uint8))
    with pytest.raises(ValueError, match="elements"):
        B.ls_loss_noalloc(cams, f32, f32[:-1], f32, loss)
    with pytest.raises(TypeError, match="float64"):
        B.ls_loss_noalloc(cams, f32, f32, f32, loss.float())
    # splat arrays: [N, 3] row-major data has the right count but a transposed
    # view of it is not contiguous; a wrong count is refused
    n = 5
    means = torch.zeros(n, 3).t()
    with pytest.raises(ValueError, match="contiguous"):
        B.splats_struct(n, means, torch.zeros(3 * n), torch.zeros(4 * n), torch.zeros(n),
                        torch.zeros(3 * n))
    with pytest.raises(ValueError, match="elements"):
        B.splats_struct(n, torch.zeros(3 * n), torch.zeros(3 * n), torch.zeros(3 * n),
                        torch.zeros(n), torch.zeros(3 * n))
    # Adam: the four arrays must agree
    with pytest.raises(ValueError, match="elements"):
        B.ls_adam(B.adam_params(0.1, 1), torch.zeros(8), torch.zeros(7), torch.zeros(8),
                  torch.zeros(8))
    with pytest.raises(TypeError, match="int64"):
        B.ls_adam_device_step(B.adam_params(0.1, 0), torch.zeros(1, dtype=torch.int32),
                              torch.zeros(8), torch.zeros(8), torch.zeros(8), torch.zeros(8))


def test_stale_forward_is_refused():
    from paper_2411_12440_amd.rasterizer import StaleForwardError, check_generation

    class Stub:
        generation = 3

    check_generation(Stub, 3)
    with pytest.raises(StaleForwardError):
        check_generation(Stub, 2)
