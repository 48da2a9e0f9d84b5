"""Python binding of librz.so (the C ABI in include/rz.h).

Argument marshalling only: torch supplies device memory and the stream, and
every step of the rasterizer runs in the library's HIP kernels.  There is no
fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librz.so")

RZ_OK = 0
RZ_EINVAL = -1
RZ_EDEPTHRANGE = -2
RZ_EHIP = -3
RZ_EOVERFLOW = -4
RZ_EBUDGET = -5
RZ_ESTATE = -6
RZ_KEEP_KEYS = 1
RZ_STATUS_HQ_OVERFLOW = 1
DEPTH_LINEAR = 0
DEPTH_SCALE = 1

CLEAR_DEPTH = 0xFFFFFFFFFF000000


class RzError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(what)


c_void_p, c_int32, c_int64, c_uint32, c_double = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                                  ctypes.c_uint32, ctypes.c_double)


class rz_points(ctypes.Structure):
    _fields_ = [("x", c_void_p), ("y", c_void_p), ("z", c_void_p), ("rgb", c_void_p),
                ("n", c_int64)]


class rz_view(ctypes.Structure):
    _fields_ = [("vp", c_double * 16), ("near_", c_double), ("far_", c_double),
                ("width", c_int32), ("height", c_int32)]


class rz_depth_map(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("scale", c_double)]


class rz_hq_params(ctypes.Structure):
    _fields_ = [("eps_num", c_uint32), ("eps_den", c_uint32)]


class rz_launch(ctypes.Structure):
    _fields_ = [("block", c_int32), ("ppt", c_int32), ("early_out", c_int32),
                ("xcd_remap", c_int32), ("bin", c_int32)]


P = ctypes.POINTER
SIGNATURES = {
    "rasterize_atomicmin": ([P(rz_points), P(rz_view), P(rz_depth_map), c_uint32, c_void_p,
                             c_void_p, c_uint32, c_void_p], ctypes.c_int),
    "rasterize_hq_splat": ([P(rz_points), P(rz_view), P(rz_depth_map), P(rz_hq_params), c_uint32,
                            c_void_p, c_void_p, c_void_p, c_void_p, c_uint32, c_void_p],
                           ctypes.c_int),
    "rz_clear": ([c_void_p, c_void_p, c_int64, c_uint32, c_void_p], ctypes.c_int),
    "rz_hq_accumulate": ([P(rz_points), P(rz_view), P(rz_depth_map), P(rz_hq_params), c_void_p,
                          c_void_p, c_void_p], ctypes.c_int),
    "rz_resolve_min": ([c_void_p, c_int64, c_uint32, c_void_p, c_void_p], ctypes.c_int),
    "rz_resolve_hq": ([c_void_p, c_void_p, c_int64, c_uint32, c_void_p, c_void_p, c_void_p],
                      ctypes.c_int),
    "rz_set_launch": ([P(rz_launch)], ctypes.c_int),
    "rz_get_launch": ([P(rz_launch)], ctypes.c_int),
    "rz_error_string": ([ctypes.c_int], ctypes.c_char_p),
    "rz_last_hip_error": ([], ctypes.c_int),
    "rz_version": ([], ctypes.c_int),
}

_lock = threading.Lock()
_lib = None


def load(path: str = LIB_PATH):
    """Load librz.so (after torch, so that both share torch's HIP runtime)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise RzError(RZ_EINVAL, f"{path} is not built; run "
                              "`python -m paper_1908_02681_amd.build`")
            import torch  # noqa: F401  (loads the HIP runtime the library binds to)
            lib = ctypes.CDLL(path)
            for name, (args, res) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = res
            _lib = lib
    return _lib


def error_string(code: int) -> str:
    return load().rz_error_string(int(code)).decode()


def _check(rc: int, what: str):
    if rc != RZ_OK:
        lib = load()
        extra = f", hipError {lib.rz_last_hip_error()}" if rc == RZ_EHIP else ""
        raise RzError(rc, f"{what}: {error_string(rc)} ({rc}{extra})")


# --------------------------------------------------------------------------
# marshalling helpers
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _require_gpu(*tensors):
    torch = _torch()
    if not torch.cuda.is_available():
        raise RzError(RZ_EHIP, "no HIP device available: the rasterizer runs on the GPU only")
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise RzError(RZ_EINVAL, "buffers must be device (cuda) tensors")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class Points:
    """Device point planes: x, y, z float32 and rgb (int32 storage of the
    R | G << 8 | B << 16 word)."""
    x: object
    y: object
    z: object
    rgb: object

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @classmethod
    def from_numpy(cls, x, y, z, rgb, device="cuda"):
        torch = _torch()
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        c = torch.from_numpy(np.ascontiguousarray(rgb, np.uint32).view(np.int32)).to(device)
        return cls(f(x), f(y), f(z), c)

    @classmethod
    def from_cloud(cls, cloud, device="cuda"):
        return cls.from_numpy(cloud.x, cloud.y, cloud.z, cloud.rgb, device)

    def struct(self) -> rz_points:
        torch = _torch()
        for t, dt in ((self.x, torch.float32), (self.y, torch.float32), (self.z, torch.float32),
                      (self.rgb, torch.int32)):
            if t.dtype != dt or t.dim() != 1 or not t.is_contiguous() or t.shape[0] != self.n:
                raise RzError(RZ_EINVAL, "point planes must be contiguous 1-D tensors of "
                              "float32 (x, y, z) and int32 (rgb) with equal length")
        return rz_points(self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr(),
                         self.rgb.data_ptr(), self.n)


def view_struct(view) -> rz_view:
    """From any object with vp (4x4), near, far, width, height."""
    vp = np.ascontiguousarray(view.vp, np.float64).reshape(16)
    return rz_view((c_double * 16)(*vp.tolist()), float(view.near), float(view.far),
                   int(view.width), int(view.height))


def depth_struct(kind=DEPTH_LINEAR, scale=0.0) -> rz_depth_map:
    return rz_depth_map(int(kind), float(scale))


def _npix(view):
    return int(view.width) * int(view.height)


def new_framebuffer(view, background=0, hq=False, stream=None):
    """Device fb (int64 storage of uint64 keys) in the cleared state, and for
    the splatting path the zeroed accumulator (2 words per pixel)."""
    torch = _torch()
    _require_gpu()
    n = _npix(view)
    fb = torch.empty(n, dtype=torch.int64, device="cuda")
    acc = torch.empty(2 * n, dtype=torch.int64, device="cuda") if hq else None
    clear(fb, acc, n, background, stream)
    return fb, acc


def clear(fb, acc, npix, background=0, stream=None):
    _require_gpu(fb, acc)
    _check(load().rz_clear(_ptr(fb), _ptr(acc), int(npix), int(background) & 0xFFFFFFFF,
                           _stream(stream)), "rz_clear")


def resolve_min(fb, npix, background=0, img=None, stream=None):
    torch = _torch()
    _require_gpu(fb, img)
    if img is None:
        img = torch.empty(int(npix), dtype=torch.int32, device="cuda")
    _check(load().rz_resolve_min(_ptr(fb), int(npix), int(background) & 0xFFFFFFFF, _ptr(img),
                                 _stream(stream)), "rz_resolve_min")
    return img


def resolve_hq(fb, acc, npix, background=0, img=None, status=None, stream=None):
    torch = _torch()
    _require_gpu(fb, acc, img, status)
    if img is None:
        img = torch.empty(int(npix), dtype=torch.int32, device="cuda")
    _check(load().rz_resolve_hq(_ptr(fb), _ptr(acc), int(npix), int(background) & 0xFFFFFFFF,
                                _ptr(img), _ptr(status), _stream(stream)), "rz_resolve_hq")
    return img


def rasterize_atomicmin(points: Points, view, depth=None, background=0, fb=None, img=None,
                        keep_keys=False, stream=None):
    """Section 2.1 on the GPU.  Returns (fb, img); fb is left cleared unless
    keep_keys (then it holds the keys and img is None)."""
    torch = _torch()
    _require_gpu(points.x, fb, img)
    if fb is None:
        fb, _ = new_framebuffer(view, background, stream=stream)
    if img is None and not keep_keys:
        img = torch.empty(_npix(view), dtype=torch.int32, device="cuda")
    ps, vs = points.struct(), view_struct(view)
    ds = depth if isinstance(depth, rz_depth_map) else depth_struct(*(depth or (DEPTH_LINEAR, 0.0)))
    rc = load().rasterize_atomicmin(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds),
                                    int(background) & 0xFFFFFFFF, _ptr(fb),
                                    None if keep_keys else _ptr(img),
                                    RZ_KEEP_KEYS if keep_keys else 0, _stream(stream))
    _check(rc, "rasterize_atomicmin")
    return fb, (None if keep_keys else img)


def rasterize_hq_splat(points: Points, view, depth=None, eps=(1, 100), background=0, fb=None,
                       acc=None, img=None, status=None, keep_keys=False, stream=None):
    """Section 2.2 on the GPU.  Returns (fb, acc, img, status)."""
    torch = _torch()
    _require_gpu(points.x, fb, acc, img, status)
    if fb is None or acc is None:
        fb, acc = new_framebuffer(view, background, hq=True, stream=stream)
    if img is None and not keep_keys:
        img = torch.empty(_npix(view), dtype=torch.int32, device="cuda")
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ps, vs = points.struct(), view_struct(view)
    ds = depth if isinstance(depth, rz_depth_map) else depth_struct(*(depth or (DEPTH_LINEAR, 0.0)))
    hq = rz_hq_params(int(eps[0]), int(eps[1]))
    rc = load().rasterize_hq_splat(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds),
                                   ctypes.byref(hq), int(background) & 0xFFFFFFFF, _ptr(fb),
                                   _ptr(acc), None if keep_keys else _ptr(img), _ptr(status),
                                   RZ_KEEP_KEYS if keep_keys else 0, _stream(stream))
    _check(rc, "rasterize_hq_splat")
    return fb, acc, (None if keep_keys else img), status


def hq_accumulate(points: Points, view, fb, acc, depth=None, eps=(1, 100), stream=None):
    """Second splatting pass alone; fb holds the finished depth pass."""
    _require_gpu(points.x, fb, acc)
    ps, vs = points.struct(), view_struct(view)
    ds = depth if isinstance(depth, rz_depth_map) else depth_struct(*(depth or (DEPTH_LINEAR, 0.0)))
    hq = rz_hq_params(int(eps[0]), int(eps[1]))
    _check(load().rz_hq_accumulate(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds),
                                   ctypes.byref(hq), _ptr(fb), _ptr(acc), _stream(stream)),
           "rz_hq_accumulate")
    return acc


def set_launch(block=256, ppt=16, early_out=1, xcd_remap=1, bin=1):
    """Launch shape of the point kernels (defaults = the library's)."""
    _check(load().rz_set_launch(ctypes.byref(rz_launch(block, ppt, early_out, xcd_remap, bin))),
           "rz_set_launch")


def get_launch() -> dict:
    l = rz_launch()
    _check(load().rz_get_launch(ctypes.byref(l)), "rz_get_launch")
    return {f: getattr(l, f) for f, _ in rz_launch._fields_}


# --------------------------------------------------------------------------
# host-side views of results
# --------------------------------------------------------------------------

def to_u64(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def to_u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def unpack_acc(acc) -> np.ndarray:
    """(npix, 4) exact sums R, G, B, count from the packed accumulator."""
    a = to_u64(acc).reshape(-1, 2)
    lo = np.uint64(0xFFFFFFFF)
    return np.stack([a[:, 0] & lo, a[:, 0] >> np.uint64(32), a[:, 1] & lo,
                     a[:, 1] >> np.uint64(32)], axis=1)
