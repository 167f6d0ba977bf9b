"""ctypes binding of liblsplat (include/lsplat.h): argument marshalling only.

Every function here takes torch tensors already on the GPU (or host arrays for
the h_* camera fields), builds the C structs and calls the entry point of the
same name.  No step of the rasterizer runs in Python; if the shared library is
missing the import of this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsplat.so")

LS_OK = 0
_STATUS = {0: "LS_OK", -1: "LS_ERR_INVALID_ARG", -2: "LS_ERR_CAPACITY", -3: "LS_ERR_HIP",
           -4: "LS_ERR_UNSUPPORTED", -5: "LS_ERR_WORKSPACE"}


class LsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("lambda_", C.c_float), ("eps2d", C.c_float), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("t_min", C.c_float), ("near_z", C.c_float),
                ("far_z", C.c_float), ("clip", C.c_float), ("bg", C.c_float * 3),
                ("ags", C.c_int32), ("ags_arg", C.c_int32), ("ags_scope", C.c_int32),
                ("sh_degree", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("batch", C.c_int32), ("depth_chunks", C.c_int32), ("kernel", C.c_int32),
                ("deterministic", C.c_int32), ("chunk_ratio", C.c_int32)]


KERNELS = {"linear": 0, "gaussian": 1, "laplacian": 2, "cosine": 3, "quadratic": 4}


class Splats(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("mean2d_norm", C.c_void_p)]


class Cams(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("n_scenes", C.c_int32), ("viewmat", C.c_void_p),
                ("intrin", C.c_void_p), ("h_width", C.c_void_p), ("h_height", C.c_void_p),
                ("h_scene_of_cam", C.c_void_p), ("h_scene_splat_off", C.c_void_p)]


class Layout(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("n_tiles", C.c_int64), ("n_pixels", C.c_int64),
                ("capacity", C.c_int64), ("n_chunks", C.c_int64), ("total_bytes", C.c_size_t),
                ("cams", C.c_size_t), ("proj", C.c_size_t), ("rect", C.c_size_t),
                ("ntiles", C.c_size_t), ("depth_key", C.c_size_t), ("order", C.c_size_t),
                ("isect_off", C.c_size_t), ("keys", C.c_size_t), ("vals", C.c_size_t),
                ("ranges", C.c_size_t), ("n_isect", C.c_size_t), ("chunk_base", C.c_size_t),
                ("chunk_n", C.c_size_t), ("flags", C.c_size_t), ("grad2d", C.c_size_t),
                ("tile_contrib", C.c_size_t), ("scratch", C.c_size_t)]


class AdamParams(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("step", C.c_int64)]


class DensifyAcc(C.Structure):
    _fields_ = [("grad", C.c_void_p), ("count", C.c_void_p), ("max_extent", C.c_void_p)]


class DensifyParams(C.Structure):
    _fields_ = [("grad_threshold", C.c_double), ("grow_scale2d", C.c_double),
                ("grow_scale3d", C.c_double), ("prune_scale2d", C.c_double),
                ("prune_scale3d", C.c_double), ("prune_opacity", C.c_double),
                ("scene_scale", C.c_double), ("grow2d", C.c_int32), ("prune_big", C.c_int32)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double)]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2411_12440_amd.build` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    sig = {
        "ls_version": ([], C.c_int),
        "ls_last_error": ([], C.c_char_p),
        "ls_workspace_size": ([P(Config), P(Cams), C.c_int64, P(C.c_size_t)], C.c_int),
        "ls_workspace_layout": ([P(Config), P(Cams), C.c_int64, P(Layout)], C.c_int),
        "ls_project": ([P(Config), P(Splats), P(Cams), C.c_void_p, C.c_size_t, C.c_int64,
                        C.c_void_p], C.c_int),
        "ls_bin_sort": ([P(Config), P(Cams), C.c_void_p, C.c_size_t, C.c_int64, C.c_void_p],
                        C.c_int),
        "ls_rasterize_fwd": ([P(Config), P(Cams), C.c_void_p, C.c_size_t, C.c_int64, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
        "ls_rasterize_bwd": ([P(Config), P(Splats), P(Cams), C.c_void_p, C.c_size_t, C.c_int64,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, P(Grads), C.c_void_p],
                             C.c_int),
        "ls_loss_workspace_size": ([P(Cams), P(C.c_size_t)], C.c_int),
        "ls_loss": ([P(Cams), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                     C.c_size_t, C.c_void_p], C.c_int),
        "ls_loss_noalloc": ([P(Cams), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
                            C.c_int),
        "ls_adam": ([P(AdamParams), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                     C.c_void_p], C.c_int),
        "ls_adam_device_step": ([P(AdamParams), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
        "ls_densify_stats": ([P(Config), P(Cams), C.c_void_p, C.c_size_t, C.c_int64,
                              P(DensifyAcc), C.c_void_p], C.c_int),
        "ls_densify_select": ([P(DensifyParams), C.c_int64, C.c_void_p, C.c_void_p,
                               P(DensifyAcc), C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
        "ls_profile_enable": ([C.c_int], C.c_int),
        "ls_profile_read": ([P(KernelTime), C.c_int, P(C.c_int), C.c_int], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


LIB = _load()
EXPORTS = ("ls_version", "ls_last_error", "ls_workspace_size", "ls_workspace_layout",
           "ls_project", "ls_bin_sort", "ls_rasterize_fwd", "ls_rasterize_bwd",
           "ls_loss_workspace_size", "ls_loss", "ls_loss_noalloc", "ls_adam", "ls_adam_device_step", "ls_densify_stats",
           "ls_densify_select", "ls_profile_enable", "ls_profile_read")


def _check(st: int):
    if st != LS_OK:
        raise LsError(st, LIB.ls_last_error().decode())


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


_DTYPES = {}


def _dtype(name):
    # torch is imported lazily so that the CPU-side ABI checks need no GPU
    if not _DTYPES:
        import torch
        _DTYPES.update(f32=torch.float32, f64=torch.float64, i32=torch.int32, i64=torch.int64,
                       u8=torch.uint8)
    return _DTYPES[name]


def _meta(t, what: str, dtype: str, numel=None, optional=False) -> bool:
    """Check what the C side assumes of tensor ``t`` apart from its device:
    the element type, a contiguous layout and the element count the entry
    point will read or write.  Raises TypeError or ValueError instead of
    handing the library a pointer it would misread.  False for an absent
    optional tensor."""
    if t is None:
        if optional:
            return False
        raise ValueError(f"{what} is required")
    if not hasattr(t, "data_ptr") or not hasattr(t, "dtype"):
        raise TypeError(f"{what} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != _dtype(dtype):
        raise TypeError(f"{what} must be {_dtype(dtype)}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if numel is not None and t.numel() != int(numel):
        raise ValueError(f"{what} has {t.numel()} elements, expected {int(numel)}")
    return True


def _devs(*specs) -> list[int]:
    """Pointers of several tensors, each spec (tensor, what, dtype[, numel[,
    optional]]): every argument's type and size is checked before any
    argument's device, so that a wrong argument is reported as such."""
    present = [_meta(*sp) for sp in specs]
    out = []
    for sp, have in zip(specs, present):
        t = sp[0]
        if have and not t.is_cuda:
            raise TypeError(f"{sp[1]} must be on a GPU (device {t.device})")
        out.append(int(t.data_ptr()) if have else 0)
    return out


def _dev(t, what: str, dtype: str, numel=None, optional=False) -> int:
    """Device pointer of one tensor after the checks of _meta and that its
    memory is on a GPU."""
    return _devs((t, what, dtype, numel, optional))[0]


def _ws(t, what="workspace") -> int:
    return _dev(t, what, "u8")


def _stream(stream) -> int:
    return 0 if stream is None else int(stream)


class CamerasHost:
    """Camera metadata: host arrays kept alive for the C struct, plus device
    tensors for viewmat / intrin."""

    def __init__(self, viewmat, intrin, width, height, scene_of_cam, scene_splat_off):
        self.viewmat = viewmat        # device float32 [C,3,4] contiguous
        self.intrin = intrin          # device float32 [C,4]
        self.h_width = np.ascontiguousarray(width, np.int32)
        self.h_height = np.ascontiguousarray(height, np.int32)
        self.h_scene = np.ascontiguousarray(scene_of_cam, np.int32)
        self.h_off = np.ascontiguousarray(scene_splat_off, np.int64)
        n = len(self.h_width)
        # device camera matrices are optional: the loss reads only the sizes
        self.c = Cams(n, len(self.h_off) - 1,
                      _dev(viewmat, "viewmat [C,3,4]", "f32", 12 * n, optional=True),
                      _dev(intrin, "intrin [C,4]", "f32", 4 * n, optional=True),
                      self.h_width.ctypes.data, self.h_height.ctypes.data,
                      self.h_scene.ctypes.data, self.h_off.ctypes.data)

    @property
    def n_pixels(self) -> int:
        return int(np.sum(self.h_width.astype(np.int64) * self.h_height.astype(np.int64)))

    @property
    def n_splats(self) -> int:
        return int(self.h_off[-1]) if len(self.h_off) else 0

    def require_matrices(self):
        if self.viewmat is None or self.intrin is None:
            raise ValueError("these cameras carry no device viewmat/intrin")


def make_config(lambda_=2.5, eps2d=0.3, alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4,
                near=0.01, far=1e10, clip=1.3, bg=(0.0, 0.0, 0.0), ags=False, ags_arg=0,
                ags_scope=0, sh_degree=0, tile_w=16, tile_h=16, batch=0,
                depth_chunks=1, kernel="linear", deterministic=False, chunk_ratio=0) -> Config:
    cfg = Config()
    cfg.lambda_, cfg.eps2d, cfg.alpha_min, cfg.alpha_max, cfg.t_min = lambda_, eps2d, alpha_min, alpha_max, t_min
    cfg.near_z, cfg.far_z, cfg.clip = near, far, clip
    for i in range(3):
        cfg.bg[i] = bg[i]
    cfg.ags, cfg.ags_arg, cfg.ags_scope = int(ags), ags_arg, ags_scope
    cfg.sh_degree, cfg.tile_w, cfg.tile_h, cfg.batch = sh_degree, tile_w, tile_h, batch
    cfg.depth_chunks = depth_chunks
    cfg.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    cfg.deterministic = int(deterministic)
    cfg.chunk_ratio = int(chunk_ratio)
    return cfg


def _sh_bands(sh, n: int, what: str) -> int:
    K = sh.numel() // (3 * n) if n > 0 else 0
    if n > 0 and (sh.numel() != 3 * n * K or K not in (1, 4, 9, 16)):
        raise ValueError(f"{what} has {sh.numel()} elements, expected K*3*{n} with K in 1, 4, 9, 16")
    return K


def splats_struct(n, means, scales, quats, opacity, sh) -> Splats:
    """Planar float32 device arrays: means/scales [3,n], quats [4,n],
    opacity [n], sh [K,3,n]."""
    ptrs = _devs((means, "means [3,n]", "f32", 3 * n), (scales, "scales [3,n]", "f32", 3 * n),
                 (quats, "quats [4,n]", "f32", 4 * n), (opacity, "opacity [n]", "f32", n),
                 (sh, "sh [K,3,n]", "f32"))
    bands = _sh_bands(sh, n, "sh [K,3,n]")
    st = Splats(n, *ptrs)
    st.bands = bands
    return st


def grads_struct(means, scales, quats, opacity, sh, mean2d_norm=None) -> Grads:
    """Gradient outputs; their sizes are checked against the splats and
    cameras when ls_rasterize_bwd is called."""
    g = Grads(*_devs((means, "grad means", "f32"), (scales, "grad scales", "f32"),
                     (quats, "grad quats", "f32"), (opacity, "grad opacity", "f32"),
                     (sh, "grad sh", "f32"), (mean2d_norm, "mean2d_norm", "f32", None, True)))
    g.sizes = (means.numel(), scales.numel(), quats.numel(), opacity.numel(), sh.numel(),
               None if mean2d_norm is None else mean2d_norm.numel())
    return g


def _check_splats(cfg: Config, splats: Splats, cams: CamerasHost):
    if splats.n != cams.n_splats:
        raise ValueError(f"splats.n = {splats.n}, the cameras' scenes hold {cams.n_splats}")
    K = (cfg.sh_degree + 1) ** 2
    if splats.n > 0 and getattr(splats, "bands", K) != K:
        raise ValueError(f"sh holds {splats.bands} bands per channel, sh_degree "
                         f"{cfg.sh_degree} needs {K}")


def _n_pairs(cams: CamerasHost) -> int:
    sizes = np.diff(cams.h_off)
    return int(np.sum(sizes[cams.h_scene])) if len(cams.h_scene) else 0


def ls_version() -> int:
    return LIB.ls_version()


def ls_workspace_size(cfg: Config, cams: CamerasHost, capacity: int) -> int:
    out = C.c_size_t(0)
    _check(LIB.ls_workspace_size(C.byref(cfg), C.byref(cams.c), capacity, C.byref(out)))
    return out.value


def ls_workspace_layout(cfg: Config, cams: CamerasHost, capacity: int) -> Layout:
    out = Layout()
    _check(LIB.ls_workspace_layout(C.byref(cfg), C.byref(cams.c), capacity, C.byref(out)))
    return out


def ls_project(cfg, splats: Splats, cams: CamerasHost, ws, capacity, stream=None):
    cams.require_matrices()
    _check_splats(cfg, splats, cams)
    _check(LIB.ls_project(C.byref(cfg), C.byref(splats), C.byref(cams.c), _ws(ws), ws.numel(),
                          capacity, _stream(stream)))


def ls_bin_sort(cfg, cams: CamerasHost, ws, capacity, stream=None):
    _check(LIB.ls_bin_sort(C.byref(cfg), C.byref(cams.c), _ws(ws), ws.numel(), capacity,
                           _stream(stream)))


def ls_rasterize_fwd(cfg, cams: CamerasHost, ws, capacity, image, final_T, last, stream=None):
    P = cams.n_pixels
    ptrs = _devs((ws, "workspace", "u8"), (image, "image", "f32", 3 * P),
                 (final_T, "final_T", "f32", P), (last, "last", "i32", P))
    _check(LIB.ls_rasterize_fwd(C.byref(cfg), C.byref(cams.c), ptrs[0], ws.numel(), capacity,
                                *ptrs[1:], _stream(stream)))


def ls_rasterize_bwd(cfg, splats: Splats, cams: CamerasHost, ws, capacity, final_T, last,
                     dL_dimage, dL_dalpha, grads: Grads, stream=None):
    P, n = cams.n_pixels, splats.n
    _check_splats(cfg, splats, cams)
    want = (3 * n, 3 * n, 4 * n, n, (cfg.sh_degree + 1) ** 2 * 3 * n, _n_pairs(cams))
    names = ("grad means", "grad scales", "grad quats", "grad opacity", "grad sh", "mean2d_norm")
    for name, have, need in zip(names, getattr(grads, "sizes", want), want):
        if have is not None and have != need:
            raise ValueError(f"{name} has {have} elements, expected {need}")
    ptrs = _devs((ws, "workspace", "u8"), (final_T, "final_T", "f32", P), (last, "last", "i32", P),
                 (dL_dimage, "dL_dimage", "f32", 3 * P), (dL_dalpha, "dL_dalpha", "f32", P, True))
    _check(LIB.ls_rasterize_bwd(C.byref(cfg), C.byref(splats), C.byref(cams.c), ptrs[0],
                                ws.numel(), capacity, *ptrs[1:], C.byref(grads), _stream(stream)))


def ls_loss_workspace_size(cams: CamerasHost) -> int:
    out = C.c_size_t(0)
    _check(LIB.ls_loss_workspace_size(C.byref(cams.c), C.byref(out)))
    return out.value


def _loss_ptrs(cams: CamerasHost, image, target, dL_dimage, loss):
    P3 = 3 * cams.n_pixels
    return _devs((image, "image", "f32", P3), (target, "target", "f32", P3),
                 (dL_dimage, "dL_dimage", "f32", P3), (loss, "loss", "f64", int(cams.c.n_cams)))


def ls_loss(cams: CamerasHost, image, target, dL_dimage, loss, ws, stream=None):
    _meta(ws, "workspace", "u8")
    _check(LIB.ls_loss(C.byref(cams.c), *_loss_ptrs(cams, image, target, dL_dimage, loss),
                       _ws(ws), ws.numel(), _stream(stream)))


# bytes of the static scratch behind ls_loss_noalloc (LS_LOSS_NOALLOC_SCRATCH_BYTES)
LOSS_NOALLOC_SCRATCH_BYTES = 144 << 20


def ls_loss_noalloc(cams: CamerasHost, image, target, dL_dimage, loss, stream=None):
    _check(LIB.ls_loss_noalloc(C.byref(cams.c), *_loss_ptrs(cams, image, target, dL_dimage, loss),
                               _stream(stream)))


def adam_params(lr, step, beta1=0.9, beta2=0.999, eps=1e-15) -> AdamParams:
    return AdamParams(lr, beta1, beta2, eps, step)


def _adam_ptrs(param, grad, m, v):
    n = param.numel()
    return n, _devs(*[(t, name, "f32", n) for t, name in
                      ((param, "param"), (grad, "grad"), (m, "m"), (v, "v"))])


def ls_adam(prm: AdamParams, param, grad, m, v, stream=None):
    n, ptrs = _adam_ptrs(param, grad, m, v)
    _check(LIB.ls_adam(C.byref(prm), n, *ptrs, _stream(stream)))


def ls_adam_device_step(prm: AdamParams, step_dev, param, grad, m, v, stream=None):
    _meta(step_dev, "step_dev", "i64", 1)
    n, ptrs = _adam_ptrs(param, grad, m, v)
    _check(LIB.ls_adam_device_step(C.byref(prm), _dev(step_dev, "step_dev", "i64", 1), n, *ptrs,
                                   _stream(stream)))


def densify_acc(grad, count, max_extent) -> DensifyAcc:
    """Per-splat accumulators: grad float32 [n], count int32 [n], max_extent
    float32 [n]."""
    n = grad.numel()
    acc = DensifyAcc(*_devs((grad, "acc grad", "f32", n), (count, "acc count", "i32", n),
                            (max_extent, "acc max_extent", "f32", n)))
    acc.n = n
    return acc


# thresholds of the paper's densification table, in the order of the
# DensifyParams fields: gradient, 2D grow, 3D grow, 2D prune, 3D prune, opacity
THRESH_3DLS = (0.0002, 0.05, 0.006, 0.15, 0.4, 0.025)
THRESH_3DGS = (0.0002, 0.05, 0.01, 0.15, 0.1, 0.005)


def densify_params(scene_scale, thresholds=THRESH_3DLS, grow2d=False,
                   prune_big=False) -> DensifyParams:
    return DensifyParams(*thresholds, scene_scale, int(grow2d), int(prune_big))


def _check_acc(acc: DensifyAcc, n: int):
    if getattr(acc, "n", n) != n:
        raise ValueError(f"densification accumulators hold {acc.n} splats, expected {n}")


def ls_densify_stats(cfg, cams: CamerasHost, ws, capacity, acc: DensifyAcc, stream=None):
    _check_acc(acc, cams.n_splats)
    _check(LIB.ls_densify_stats(C.byref(cfg), C.byref(cams.c), _ws(ws), ws.numel(), capacity,
                                C.byref(acc), _stream(stream)))


def ls_densify_select(prm: DensifyParams, n, scales, opacity, acc: DensifyAcc, action,
                      counts=None, stream=None):
    opt = n == 0   # nothing is read or written for zero splats
    if not opt:
        _check_acc(acc, n)
    sc, op, act, cnt = _devs((scales, "scales", "f32", 3 * n, opt), (opacity, "opacity", "f32", n, opt),
                             (action, "action", "u8", n, opt), (counts, "counts", "i64", 3, True))
    _check(LIB.ls_densify_select(C.byref(prm), n, sc, op, C.byref(acc), act, cnt, _stream(stream)))


def ls_profile_enable(on: bool = True):
    _check(LIB.ls_profile_enable(1 if on else 0))


def ls_profile_read(reset: bool = True) -> list[tuple[str, int, float]]:
    """[(kernel, launches, total_ms)] longest first; waits for the events."""
    cap = 64
    arr = (KernelTime * cap)()
    n = C.c_int(0)
    _check(LIB.ls_profile_read(arr, cap, C.byref(n), 1 if reset else 0))
    return [(arr[i].name.decode(), int(arr[i].launches), float(arr[i].total_ms))
            for i in range(min(n.value, cap))]
