"""ctypes front end of the plain C oracle (rz_oracle.c).

TEST INFRASTRUCTURE: imported only by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  It builds the oracle with gcc on first use
(-O2 -ffp-contract=off, no fast-math: every float operation is one IEEE
operation) and exposes numpy-level calls.  It imports nothing from the
product package and the product never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "rz_oracle.c")
LIB = os.path.join(_HERE, "librz_oracle.so")
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
          "-shared", "-Wall", "-Wextra", "-Werror"]

LINEAR = 0
SCALE = 1
PIECEWISE = 2
GL24 = 3        # depth pass only: 24-bit window depth of the perspective matrix
F32REV = 4      # depth pass only: reversed single-precision depth

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle library (plain gcc, single file)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


def configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    P = ctypes.c_void_p
    i64, i32, u32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    cam = [P, f64, f64, i32, i32, i32, f64, i32, P, P]
    lib.rzo_depth_constants.argtypes = cam + [P, P, P]
    lib.rzo_fragments.argtypes = [P, P, P, i64] + cam + [P, P]
    lib.rzo_clear.argtypes = [P, i64, u32]
    lib.rzo_clear.restype = None
    lib.rzo_raster_min.argtypes = [P, P, P, P, i64] + cam + [i32, P]
    lib.rzo_resolve_min.argtypes = [P, i64, u32, P]
    lib.rzo_resolve_min.restype = None
    lib.rzo_hq_accumulate.argtypes = [P, P, P, P, i64] + cam + [i32, u32, u32, P, P]
    lib.rzo_hq_resolve.argtypes = [P, P, i64, u32, P]
    lib.rzo_hq_resolve.restype = None
    lib.rzo_merge_min.argtypes = [P, P, i64]
    lib.rzo_merge_min.restype = None
    lib.rzo_merge_sum.argtypes = [P, P, i64]
    lib.rzo_merge_sum.restype = None
    return lib


def _load():
    """The oracle library; RZ_ORACLE_LIB names another build of the same
    source to load instead (the sanitizer tests use an instrumented one)."""
    global _lib
    with _lock:
        if _lib is None:
            other = os.environ.get("RZ_ORACLE_LIB")
            if not other:
                build()
            _lib = configure(ctypes.CDLL(other or LIB))
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def _u32(a):
    return np.ascontiguousarray(a, np.uint32)


_KEEP = []


def _cam_args(vp, near, far, width, height, kind, scale):
    """kind LINEAR / SCALE with a number scale, or PIECEWISE with
    scale = ((start_0, values_per_unit_0), (start_1, ...), ...)."""
    vp = np.ascontiguousarray(vp, np.float64).reshape(16)
    if int(kind) == PIECEWISE:
        rng = np.asarray(scale, np.float64).reshape(-1, 2)
        rb, rs = np.ascontiguousarray(rng[:, 0]), np.ascontiguousarray(rng[:, 1])
        _KEEP[:] = [rb, rs]
        return vp, [_ptr(vp), float(near), float(far), int(width), int(height), int(kind), 0.0,
                    int(rb.size), _ptr(rb), _ptr(rs)]
    return vp, [_ptr(vp), float(near), float(far), int(width), int(height), int(kind),
                float(scale), 0, None, None]


def depth_constants(vp, near, far, width, height, kind=LINEAR, scale=0.0):
    """(o, s, z0) of the depth map."""
    lib = _load()
    vp, cam = _cam_args(vp, near, far, width, height, kind, scale)
    o, s, z0 = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint64()
    if lib.rzo_depth_constants(*cam, ctypes.byref(o), ctypes.byref(s), ctypes.byref(z0)):
        raise ValueError("invalid camera or depth map")
    return o.value, s.value, z0.value


def fragments(x, y, z, vp, near, far, width, height, kind=LINEAR, scale=0.0):
    """Per-point (pixel index or -1, 40-bit depth)."""
    lib = _load()
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.shape[0]
    pix = np.empty(n, np.int64)
    q = np.empty(n, np.uint64)
    vp, cam = _cam_args(vp, near, far, width, height, kind, scale)
    if lib.rzo_fragments(_ptr(x), _ptr(y), _ptr(z), n, *cam, _ptr(pix), _ptr(q)):
        raise ValueError("invalid camera or depth map")
    return pix, q


def clear_value(bg: int = 0) -> int:
    fb = np.empty(1, np.uint64)
    _load().rzo_clear(_ptr(fb), 1, int(bg) & 0xFFFFFFFF)
    return int(fb[0])


def raster_min(x, y, z, rgb, vp, near, far, width, height, kind=LINEAR, scale=0.0,
               bg=0, fb=None, point_size=1):
    """Depth pass: the per-pixel minimum key (unresolved framebuffer)."""
    lib = _load()
    x, y, z, rgb = _f32(x), _f32(y), _f32(z), _u32(rgb)
    npix = int(width) * int(height)
    if fb is None:
        fb = np.empty(npix, np.uint64)
        lib.rzo_clear(_ptr(fb), npix, int(bg) & 0xFFFFFFFF)
    vp, cam = _cam_args(vp, near, far, width, height, kind, scale)
    if lib.rzo_raster_min(_ptr(x), _ptr(y), _ptr(z), _ptr(rgb), x.shape[0], *cam,
                          int(point_size), _ptr(fb)):
        raise ValueError("invalid camera or depth map")
    return fb


def resolve_min(fb, bg=0):
    """Image of a framebuffer; fb is cleared in place."""
    img = np.empty(fb.shape[0], np.uint32)
    _load().rzo_resolve_min(_ptr(fb), fb.shape[0], int(bg) & 0xFFFFFFFF, _ptr(img))
    return img


def render_atomicmin(x, y, z, rgb, vp, near, far, width, height, kind=LINEAR,
                     scale=0.0, bg=0, point_size=1):
    """Both steps of section 2.1. Returns (keys, image)."""
    fb = raster_min(x, y, z, rgb, vp, near, far, width, height, kind, scale, bg,
                    point_size=point_size)
    keys = fb.copy()
    img = resolve_min(fb, bg)
    return keys, img


def hq_accumulate(x, y, z, rgb, vp, near, far, width, height, fb, kind=LINEAR,
                  scale=0.0, eps=(1, 100), sums=None, point_size=1):
    """Second splatting pass: exact (R, G, B, count) per pixel."""
    lib = _load()
    x, y, z, rgb = _f32(x), _f32(y), _f32(z), _u32(rgb)
    npix = int(width) * int(height)
    if sums is None:
        sums = np.zeros((npix, 4), np.uint64)
    vp, cam = _cam_args(vp, near, far, width, height, kind, scale)
    rc = lib.rzo_hq_accumulate(_ptr(x), _ptr(y), _ptr(z), _ptr(rgb), x.shape[0], *cam,
                               int(point_size), int(eps[0]), int(eps[1]), _ptr(fb), _ptr(sums))
    if rc:
        raise ValueError(f"hq accumulate failed ({rc})")
    return sums


def hq_resolve(sums, fb, bg=0):
    img = np.empty(fb.shape[0], np.uint32)
    _load().rzo_hq_resolve(_ptr(sums), _ptr(fb), fb.shape[0], int(bg) & 0xFFFFFFFF, _ptr(img))
    return img


def render_hq(x, y, z, rgb, vp, near, far, width, height, kind=LINEAR, scale=0.0,
              eps=(1, 100), bg=0, point_size=1):
    """All three passes of section 2.2. Returns (keys, sums[npix, 4], image)."""
    fb = raster_min(x, y, z, rgb, vp, near, far, width, height, kind, scale, bg,
                    point_size=point_size)
    keys = fb.copy()
    sums = hq_accumulate(x, y, z, rgb, vp, near, far, width, height, fb, kind, scale, eps,
                         point_size=point_size)
    out = sums.copy()
    img = hq_resolve(sums, fb, bg)
    return keys, out, img


def merge_min(dst, src):
    """Sort-last composition of depth passes: dst = min(dst, src) per pixel."""
    assert dst.dtype == np.uint64 and src.dtype == np.uint64 and dst.shape == src.shape
    _load().rzo_merge_min(_ptr(dst), _ptr(np.ascontiguousarray(src)), dst.shape[0])
    return dst


def merge_sum(dst, src):
    """Sort-last composition of splat sums ((npix, 4) exact words): dst += src."""
    assert dst.dtype == np.uint64 and src.dtype == np.uint64 and dst.shape == src.shape
    _load().rzo_merge_sum(_ptr(dst), _ptr(np.ascontiguousarray(src)), dst.shape[0])
    return dst
