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
RZ_EIO = -7
RZ_KEEP_KEYS = 1
RZ_STATUS_HQ_OVERFLOW = 1
RZ_CHECK_ESTIMATE_ONLY = 1
RZ_NOALLOC_SCRATCH_BYTES = 64 << 20
DEPTH_LINEAR = 0
DEPTH_SCALE = 1
DEPTH_PIECEWISE = 2
DEPTH_GL24 = 3      # depth pass only: 24-bit window depth of the perspective matrix
DEPTH_F32REV = 4    # depth pass only: reversed single-precision depth

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


RZ_MAX_RANGES = 8


class rz_depth_map(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("scale", c_double), ("nranges", c_int32),
                ("range_start", c_double * RZ_MAX_RANGES), ("range_scale", c_double * RZ_MAX_RANGES)]


class rz_hq_params(ctypes.Structure):
    _fields_ = [("eps_num", c_uint32), ("eps_den", c_uint32)]


class rz_launch(ctypes.Structure):
    _fields_ = [("block", c_int32), ("ppt", c_int32), ("early_out", c_int32),
                ("xcd_remap", c_int32), ("bin", c_int32)]


class rz_batch_view(ctypes.Structure):
    _fields_ = [("view", rz_view), ("depth", rz_depth_map), ("mode", c_int32),
                ("hq", rz_hq_params), ("background", c_uint32), ("fb", c_void_p),
                ("acc", c_void_p), ("img", c_void_p)]


class rz_batch_opts(ctypes.Structure):
    _fields_ = [("views_per_group", c_int32), ("launch", rz_launch), ("use_graph", c_int32),
                ("status", c_void_p)]


class rz_tune_entry(ctypes.Structure):
    _fields_ = [("views_per_group", c_int32), ("depth", rz_launch), ("accum", rz_launch),
                ("ms", ctypes.c_float)]


class rz_server_opts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("streams", c_int32), ("max_inflight", c_int32),
                ("dry_run", c_int32), ("dry_run_us", c_int32), ("work_cap", c_int64),
                ("merge_views", c_int32), ("pad", c_int32), ("exclusive_work", c_int64)]


class rz_request(ctypes.Structure):
    _fields_ = [("cloud", c_int32), ("mode", c_int32), ("view", rz_view), ("depth", rz_depth_map),
                ("hq", rz_hq_params), ("background", c_uint32), ("flags", c_uint32),
                ("img", c_void_p), ("after", c_void_p)]


class rz_request_status(ctypes.Structure):
    _fields_ = [("state", c_int32), ("error", c_int32), ("hq_status", c_uint32),
                ("stream", c_uint32), ("group", c_int32), ("pad", c_int32),
                ("t_submit_us", c_double), ("t_admit_us", c_double), ("t_done_us", c_double)]


class rz_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("peak_inflight", c_int32), ("queued", c_int32), ("inflight", c_int32),
                ("pad", c_int32), ("merged_launches", ctypes.c_uint64),
                ("merged_requests", ctypes.c_uint64), ("chained_requests", ctypes.c_uint64)]


P = ctypes.POINTER
SIGNATURES = {
    "rasterize_atomicmin": ([P(rz_points), P(rz_view), P(rz_depth_map), c_uint32, c_void_p,
                             c_void_p, c_uint32, c_void_p], ctypes.c_int),
    "rasterize_hq_splat": ([P(rz_points), P(rz_view), P(rz_depth_map), P(rz_hq_params), c_uint32,
                            c_void_p, c_void_p, c_void_p, c_void_p, c_uint32, c_void_p],
                           ctypes.c_int),
    "rz_sorted_workspace_bytes": ([c_int64, c_int32, c_int32], c_int64),
    "rasterize_sorted": ([P(rz_points), P(rz_view), P(rz_depth_map), P(rz_hq_params), c_uint32,
                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_uint32,
                          c_void_p], ctypes.c_int),
    "rasterize_sorted_noalloc": ([P(rz_points), P(rz_view), P(rz_depth_map), P(rz_hq_params),
                                  c_uint32, c_void_p, c_void_p, c_void_p, c_void_p, c_uint32,
                                  c_void_p], ctypes.c_int),
    "rasterize_points": ([P(rz_points), P(rz_view), P(rz_depth_map), P(rz_hq_params), c_int32,
                          c_uint32, c_void_p, c_void_p, c_void_p, c_void_p, c_uint32, c_void_p],
                         ctypes.c_int),
    "rz_merge_min": ([c_void_p, c_void_p, c_int64, c_void_p], ctypes.c_int),
    "rz_merge_sum": ([c_void_p, c_void_p, c_int64, c_void_p], ctypes.c_int),
    "rz_check_reciprocal": ([c_uint32, c_int64, c_void_p, c_uint32, c_void_p], ctypes.c_int),
    "rz_reciprocal": ([c_void_p, c_void_p, c_int64, c_void_p], ctypes.c_int),
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
    "rz_batch_plan": ([P(rz_points), P(rz_batch_view), c_int32, P(rz_batch_opts), P(c_void_p)],
                      ctypes.c_int),
    "rz_batch_capture": ([c_void_p], ctypes.c_int),
    "rz_batch_run": ([c_void_p, c_void_p], ctypes.c_int),
    "rz_batch_autotune": ([c_void_p, c_void_p, c_int32, P(rz_batch_opts), P(ctypes.c_float)],
                          ctypes.c_int),
    "rz_batch_get_opts": ([c_void_p, P(rz_batch_opts)], ctypes.c_int),
    "rz_batch_autotune_cached": ([c_void_p, c_void_p, c_int32, ctypes.c_char_p, P(rz_batch_opts),
                                  P(ctypes.c_float), P(c_int32), ctypes.c_char_p, c_int32],
                                 ctypes.c_int),
    "rz_order_class_host": ([c_void_p, c_void_p, c_void_p, c_int64], ctypes.c_int),
    "rz_tune_cache_lookup": ([ctypes.c_char_p, ctypes.c_char_p, P(rz_tune_entry)], ctypes.c_int),
    "rz_tune_cache_store": ([ctypes.c_char_p, ctypes.c_char_p, P(rz_tune_entry)], ctypes.c_int),
    "rz_batch_destroy": ([c_void_p], ctypes.c_int),
    "rz_server_create": ([P(rz_server_opts), P(c_void_p)], ctypes.c_int),
    "rz_server_add_cloud": ([c_void_p, P(rz_points), P(c_int32)], ctypes.c_int),
    "rz_server_submit": ([c_void_p, P(rz_request), P(ctypes.c_uint64)], ctypes.c_int),
    "rz_server_poll": ([c_void_p, ctypes.c_uint64, P(rz_request_status)], ctypes.c_int),
    "rz_server_drain": ([c_void_p, c_double], ctypes.c_int),
    "rz_server_get_stats": ([c_void_p, P(rz_server_stats)], ctypes.c_int),
    "rz_server_destroy": ([c_void_p, c_double], ctypes.c_int),
}

RZ_REQ_QUEUED, RZ_REQ_RUNNING, RZ_REQ_DONE, RZ_REQ_FAILED = 0, 1, 2, 3
RZ_REQ_INJECT_FAILURE = 1

RZ_MODE_ATOMICMIN = 0
RZ_MODE_HQ = 1

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


def _fits(what, t, nbytes):
    """The library writes nbytes from t's address: t must be a contiguous
    device tensor holding at least that many bytes."""
    if t is None:
        return
    if not t.is_contiguous() or t.numel() * t.element_size() < nbytes:
        raise RzError(RZ_EINVAL, f"{what}: needs a contiguous device tensor of at least "
                      f"{nbytes} bytes, got {t.numel() * t.element_size()} "
                      f"({'contiguous' if t.is_contiguous() else 'not contiguous'})")


def _fits_view(npix, fb=None, acc=None, img=None, status=None):
    """Framebuffer (8 B), splat sums (16 B) and image (4 B) per pixel, and a
    4-byte status word."""
    _fits("fb", fb, 8 * npix)
    _fits("acc", acc, 16 * npix)
    _fits("img", img, 4 * npix)
    _fits("status", status, 4)


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
    """LINEAR / SCALE (scale a number) or PIECEWISE with
    scale = ((start_0, values_per_unit_0), (start_1, values_per_unit_1), ...)."""
    d = rz_depth_map()
    d.kind = int(kind)
    if int(kind) == DEPTH_PIECEWISE:
        r = list(scale)
        d.nranges = len(r)
        for k, (b, sc) in enumerate(r[:RZ_MAX_RANGES]):
            d.range_start[k] = float(b)
            d.range_scale[k] = float(sc)
    else:
        d.scale = float(scale)
    return d


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
    _fits_view(int(npix), fb, acc)
    _check(load().rz_clear(_ptr(fb), _ptr(acc), int(npix), int(background) & 0xFFFFFFFF,
                           _stream(stream)), "rz_clear")


def resolve_min(fb, npix, background=0, img=None, stream=None):
    torch = _torch()
    _require_gpu(fb, img)
    if img is None:
        img = torch.empty(int(npix), dtype=torch.int32, device="cuda")
    _fits_view(int(npix), fb, img=img)
    _check(load().rz_resolve_min(_ptr(fb), int(npix), int(background) & 0xFFFFFFFF, _ptr(img),
                                 _stream(stream)), "rz_resolve_min")
    return img


def resolve_hq(fb, acc, npix, background=0, img=None, status=None, stream=None):
    """Third splatting pass.  status (one int32, zero) receives the overflow
    bit; one is allocated when None."""
    torch = _torch()
    _require_gpu(fb, acc, img, status)
    if img is None:
        img = torch.empty(int(npix), dtype=torch.int32, device="cuda")
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
    _fits_view(int(npix), fb, acc, img, status)
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
    _fits_view(_npix(view), fb, img=img)
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
    _fits_view(_npix(view), fb, acc, img, status)
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
    _fits_view(_npix(view), fb, acc)
    ps, vs = points.struct(), view_struct(view)
    ds = depth if isinstance(depth, rz_depth_map) else depth_struct(*(depth or (DEPTH_LINEAR, 0.0)))
    hq = rz_hq_params(int(eps[0]), int(eps[1]))
    _check(load().rz_hq_accumulate(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds),
                                   ctypes.byref(hq), _ptr(fb), _ptr(acc), _stream(stream)),
           "rz_hq_accumulate")
    return acc


def rasterize_points(points: Points, view, depth=None, hq=False, eps=(1, 100), point_size=1,
                     background=0, fb=None, acc=None, img=None, status=None, keep_keys=False,
                     stream=None):
    """Points of point_size x point_size pixels and every depth encoding
    (float encodings: depth pass only).  Returns (fb, acc, img, status); acc
    and status are None without hq."""
    torch = _torch()
    _require_gpu(points.x, fb, acc, img, status)
    if fb is None or (hq and acc is None):
        fb, acc = new_framebuffer(view, background, hq=hq, stream=stream)
    if img is None and not keep_keys:
        img = torch.empty(_npix(view), dtype=torch.int32, device="cuda")
    if hq and status is None:
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
    _fits_view(_npix(view), fb, acc if hq else None, None if keep_keys else img,
               status if hq else None)
    ps, vs = points.struct(), view_struct(view)
    ds = depth if isinstance(depth, rz_depth_map) else depth_struct(*(depth or (DEPTH_LINEAR, 0.0)))
    hp = ctypes.byref(rz_hq_params(int(eps[0]), int(eps[1]))) if hq else None
    rc = load().rasterize_points(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds), hp,
                                 int(point_size), int(background) & 0xFFFFFFFF, _ptr(fb),
                                 _ptr(acc) if hq else None, None if keep_keys else _ptr(img),
                                 _ptr(status) if hq else None,
                                 RZ_KEEP_KEYS if keep_keys else 0, _stream(stream))
    _check(rc, "rasterize_points")
    return fb, (acc if hq else None), (None if keep_keys else img), (status if hq else None)


def sorted_workspace_bytes(n: int, width: int, height: int) -> int:
    """Workspace the screen-sorted path needs for n points at width x height."""
    b = load().rz_sorted_workspace_bytes(int(n), int(width), int(height))
    if b < 0:
        raise RzError(RZ_EINVAL, "rz_sorted_workspace_bytes: invalid size")
    return b


def new_workspace(n: int, width: int, height: int):
    """Device workspace (256-byte aligned) for rasterize_sorted."""
    torch = _torch()
    nbytes = max(sorted_workspace_bytes(n, width, height), 256)
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def rasterize_sorted(points: Points, view, depth=None, hq=False, eps=(1, 100), background=0,
                     fb=None, acc=None, img=None, status=None, workspace=None, keep_keys=False,
                     stream=None):
    """Screen-sorted rendering: the images of rasterize_atomicmin (hq=False)
    or rasterize_hq_splat (hq=True), bit for bit, through a counting sort of
    the fragments by screen tile.  Returns (fb, acc, img, status); acc and
    status are None without hq."""
    torch = _torch()
    _require_gpu(points.x, fb, acc, img, status, workspace)
    if fb is None or (hq and acc is None):
        fb, acc = new_framebuffer(view, background, hq=hq, stream=stream)
    if img is None and not keep_keys:
        img = torch.empty(_npix(view), dtype=torch.int32, device="cuda")
    if hq and status is None:
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
    if workspace is None:
        workspace = new_workspace(points.n, view.width, view.height)
    _fits_view(_npix(view), fb, acc if hq else None, None if keep_keys else img,
               status if hq else None)
    _fits("workspace", workspace, 0)
    ps, vs = points.struct(), view_struct(view)
    ds = depth if isinstance(depth, rz_depth_map) else depth_struct(*(depth or (DEPTH_LINEAR, 0.0)))
    hp = ctypes.byref(rz_hq_params(int(eps[0]), int(eps[1]))) if hq else None
    rc = load().rasterize_sorted(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds), hp,
                                 int(background) & 0xFFFFFFFF, _ptr(fb),
                                 _ptr(acc) if hq else None, None if keep_keys else _ptr(img),
                                 _ptr(status) if hq else None, _ptr(workspace),
                                 workspace.numel() * workspace.element_size(),
                                 RZ_KEEP_KEYS if keep_keys else 0, _stream(stream))
    _check(rc, "rasterize_sorted")
    return fb, (acc if hq else None), (None if keep_keys else img), (status if hq else None)


def rasterize_sorted_noalloc(points: Points, view, fb, img, depth=None, hq=False, eps=(1, 100),
                             background=0, acc=None, status=None, keep_keys=False, stream=None):
    """rasterize_sorted with the library's static device scratch in place of
    a workspace: the C call allocates nothing.  The caller passes every
    buffer (fb cleared; with hq also acc zeroed and a zeroed status word).
    Calls that overlap on one device race on the shared scratch."""
    _require_gpu(points.x, fb, acc, img, status)
    _fits_view(_npix(view), fb, acc if hq else None, None if keep_keys else img,
               status if hq else None)
    ps, vs = points.struct(), view_struct(view)
    ds = depth if isinstance(depth, rz_depth_map) else depth_struct(*(depth or (DEPTH_LINEAR, 0.0)))
    hp = ctypes.byref(rz_hq_params(int(eps[0]), int(eps[1]))) if hq else None
    rc = load().rasterize_sorted_noalloc(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds), hp,
                                         int(background) & 0xFFFFFFFF, _ptr(fb),
                                         _ptr(acc) if hq else None,
                                         None if keep_keys else _ptr(img),
                                         _ptr(status) if hq else None,
                                         RZ_KEEP_KEYS if keep_keys else 0, _stream(stream))
    _check(rc, "rasterize_sorted_noalloc")
    return fb, (acc if hq else None), (None if keep_keys else img), (status if hq else None)


def merge_min(dst, src, npix=None, stream=None):
    """Sort-last composition of depth passes: dst = min(dst, src) per pixel."""
    _require_gpu(dst, src)
    n = dst.numel() if npix is None else int(npix)
    _fits("dst", dst, 8 * n)
    _fits("src", src, 8 * n)
    _check(load().rz_merge_min(_ptr(dst), _ptr(src), n, _stream(stream)), "rz_merge_min")
    return dst


def merge_sum(dst, src, npix=None, stream=None):
    """Sort-last composition of packed splat sums (2 words per pixel)."""
    _require_gpu(dst, src)
    n = dst.numel() // 2 if npix is None else int(npix)
    _fits("dst", dst, 16 * n)
    _fits("src", src, 16 * n)
    _check(load().rz_merge_sum(_ptr(dst), _ptr(src), n, _stream(stream)), "rz_merge_sum")
    return dst


def check_reciprocal(first_bits=0, count=1 << 32, estimate_only=False, stream=None):
    """Number of positive float patterns in [first_bits, first_bits + count)
    whose reciprocal, as the kernels compute it (or only its corrected
    estimate), differs from 1.0f / w; a one-element device tensor."""
    torch = _torch()
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    flags = RZ_CHECK_ESTIMATE_ONLY if estimate_only else 0
    _check(load().rz_check_reciprocal(int(first_bits), int(count), _ptr(out), flags,
                                      _stream(stream)), "rz_check_reciprocal")
    return out


def reciprocal(w, out=None, stream=None):
    """The kernels' 1 / w applied to a float32 device tensor."""
    torch = _torch()
    _require_gpu(w, out)
    if w.dtype != torch.float32 or not w.is_contiguous():
        raise RzError(RZ_EINVAL, "w must be a contiguous float32 device tensor")
    if out is None:
        out = torch.empty_like(w)
    _fits("out", out, 4 * w.numel())
    _check(load().rz_reciprocal(_ptr(w), _ptr(out), w.numel(), _stream(stream)), "rz_reciprocal")
    return out


def set_launch(block=64, ppt=16, early_out=1, xcd_remap=0, bin=2):
    """Launch shape of both point passes of the one-view calls."""
    _check(load().rz_set_launch(ctypes.byref(rz_launch(block, ppt, early_out, xcd_remap, bin))),
           "rz_set_launch")


def reset_launch():
    """Back to the library's default launch shapes (they differ between the
    depth and the splat pass)."""
    _check(load().rz_set_launch(None), "rz_set_launch")


def get_launch() -> dict:
    l = rz_launch()
    _check(load().rz_get_launch(ctypes.byref(l)), "rz_get_launch")
    return {f: getattr(l, f) for f, _ in rz_launch._fields_}


def order_class(x, y, z) -> str:
    """Point order class of host float32 arrays ("ordered" or "shuffled"), as
    the batch autotune cache keys it (rz_order_class_host)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, z)]
    n = arrs[0].size
    if any(a.size != n for a in arrs):
        raise RzError(RZ_EINVAL, "x, y and z must have the same length")
    rc = load().rz_order_class_host(*(a.ctypes.data_as(c_void_p) for a in arrs), n)
    if rc < 0:
        _check(rc, "rz_order_class_host")
    return "ordered" if rc == 0 else "shuffled"


def _entry_dict(e: rz_tune_entry) -> dict:
    return {"views_per_group": e.views_per_group,
            "depth": {f: getattr(e.depth, f) for f, _ in rz_launch._fields_},
            "accum": {f: getattr(e.accum, f) for f, _ in rz_launch._fields_},
            "ms": float(e.ms)}


def tune_cache_lookup(path, key):
    """The cached entry for `key` as a dict, or None (rz_tune_cache_lookup)."""
    e = rz_tune_entry()
    rc = load().rz_tune_cache_lookup(os.fsencode(path), key.encode(), ctypes.byref(e))
    if rc < 0:
        _check(rc, "rz_tune_cache_lookup")
    return _entry_dict(e) if rc == 1 else None


def tune_cache_store(path, key, views_per_group, depth, accum, ms):
    """Stores one entry (depth / accum: dicts of rz_launch fields)."""
    e = rz_tune_entry(views_per_group, rz_launch(**depth), rz_launch(**accum), ms)
    _check(load().rz_tune_cache_store(os.fsencode(path), key.encode(), ctypes.byref(e)),
           "rz_tune_cache_store")


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


# --------------------------------------------------------------------------
# batched multi-view rendering
# --------------------------------------------------------------------------

def _opts_dict(o: rz_batch_opts) -> dict:
    return {"views_per_group": o.views_per_group, "use_graph": o.use_graph,
            **{f: getattr(o.launch, f) for f, _ in rz_launch._fields_}}


class Batch:
    """Many views of one resident cloud (rz_batch_* in include/rz.h).

    views: objects with vp, near, far, width, height; modes: RZ_MODE_* per
    view; depth: one depth map for all views, or a list with one per view.  Allocates (torch) and clears each view's fb / acc / img once; the
    library owns only its view table and graph.  Every run renders all views
    and leaves fb/acc cleared again."""

    def __init__(self, points: Points, views, modes, depth=None, eps=(1, 100), backgrounds=None,
                 views_per_group=0, launch=None, use_graph=False, status=None):
        torch = _torch()
        _require_gpu(points.x, status)
        self.points = points
        self.views = list(views)
        self.modes = [int(m) for m in modes]
        n = len(self.views)
        if len(self.modes) != n:
            raise RzError(RZ_EINVAL, "one mode per view")
        bgs = [0] * n if backgrounds is None else [int(b) for b in backgrounds]
        self.backgrounds = bgs
        self.fbs, self.accs, self.imgs = [], [], []
        arr = (rz_batch_view * n)()

        def as_struct(d):
            return d if isinstance(d, rz_depth_map) else depth_struct(*(d or (DEPTH_LINEAR, 0.0)))
        per_view = isinstance(depth, list)
        if per_view and len(depth) != n:
            raise RzError(RZ_EINVAL, "one depth map per view")
        ds_all = [as_struct(d) for d in depth] if per_view else [as_struct(depth)] * n
        for i, (v, m) in enumerate(zip(self.views, self.modes)):
            ds = ds_all[i]
            fb, acc = new_framebuffer(v, bgs[i], hq=(m == RZ_MODE_HQ))
            img = torch.empty(_npix(v), dtype=torch.int32, device="cuda")
            self.fbs.append(fb)
            self.accs.append(acc)
            self.imgs.append(img)
            arr[i] = rz_batch_view(view_struct(v), ds, m, rz_hq_params(int(eps[0]), int(eps[1])),
                                   bgs[i] & 0xFFFFFFFF, fb.data_ptr(),
                                   acc.data_ptr() if acc is not None else None, img.data_ptr())
        if status is None and RZ_MODE_HQ in self.modes:
            status = torch.zeros(1, dtype=torch.int32, device="cuda")   # overflow bit
        self.status = status
        opts = rz_batch_opts()
        opts.views_per_group = int(views_per_group)
        if launch is not None:
            opts.launch = rz_launch(*launch) if not isinstance(launch, dict) else rz_launch(
                **{k: launch[k] for k, _ in rz_launch._fields_})
        opts.use_graph = 1 if use_graph else 0
        _fits("status", status, 4)
        opts.status = status.data_ptr() if status is not None else None
        self._ps = points.struct()
        self._arr = arr
        h = c_void_p()
        torch.cuda.synchronize()
        _check(load().rz_batch_plan(ctypes.byref(self._ps), arr, n, ctypes.byref(opts),
                                    ctypes.byref(h)), "rz_batch_plan")
        self._h = h

    def run(self, stream=None):
        _check(load().rz_batch_run(self._h, _stream(stream)), "rz_batch_run")

    def capture(self):
        _check(load().rz_batch_capture(self._h), "rz_batch_capture")

    def autotune(self, reps=3, stream=None):
        o = rz_batch_opts()
        ms = ctypes.c_float()
        _check(load().rz_batch_autotune(self._h, _stream(stream), int(reps), ctypes.byref(o),
                                        ctypes.byref(ms)), "rz_batch_autotune")
        return _opts_dict(o), float(ms.value)

    def autotune_cached(self, path, reps=3, stream=None):
        """autotune() through the cache file at `path` (rz_batch_autotune_cached):
        returns (options, ms, hit, key)."""
        o = rz_batch_opts()
        ms = ctypes.c_float()
        hit = c_int32()
        key = ctypes.create_string_buffer(160)
        _check(load().rz_batch_autotune_cached(self._h, _stream(stream), int(reps),
                                               os.fsencode(path), ctypes.byref(o),
                                               ctypes.byref(ms), ctypes.byref(hit), key, 160),
               "rz_batch_autotune_cached")
        return _opts_dict(o), float(ms.value), bool(hit.value), key.value.decode()

    def opts(self) -> dict:
        o = rz_batch_opts()
        _check(load().rz_batch_get_opts(self._h, ctypes.byref(o)), "rz_batch_get_opts")
        return _opts_dict(o)

    def images(self):
        return [to_u32(i) for i in self.imgs]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(load().rz_batch_destroy(self._h), "rz_batch_destroy")
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------

class Server:
    """Continuous-batching render server (rz_server_* in include/rz.h).

    Clouds stay resident (the caller keeps the Points alive); each request
    renders one view into a caller-owned device image.  dry_run=True runs
    the scheduler without any device work (requests take dry_run_us)."""

    def __init__(self, budget_bytes, streams=4, max_inflight=0, dry_run=False, dry_run_us=0,
                 work_cap=0, merge_views=0, exclusive_work=0):
        if not dry_run:
            _require_gpu()
        o = rz_server_opts(int(budget_bytes), int(streams), int(max_inflight), 1 if dry_run else 0,
                           int(dry_run_us), int(work_cap), int(merge_views), 0,
                           int(exclusive_work))
        h = c_void_p()
        _check(load().rz_server_create(ctypes.byref(o), ctypes.byref(h)), "rz_server_create")
        self._h = h
        self._clouds = []
        self.dry_run = dry_run

    def add_cloud(self, points) -> int:
        ps = points.struct() if isinstance(points, Points) else points
        cid = c_int32()
        _check(load().rz_server_add_cloud(self._h, ctypes.byref(ps), ctypes.byref(cid)),
               "rz_server_add_cloud")
        self._clouds.append(points)
        return cid.value

    def submit(self, cloud, view, mode, img=None, depth=None, eps=(1, 100), background=0,
               inject_failure=False, after="current") -> int:
        """Queue one request.  after: the stream whose queued work (e.g. the
        fill of img) the request waits for; "current" = torch's current
        stream, None = no wait (the caller has synchronised)."""
        _fits("img", img, 4 * _npix(view))
        ds = depth if isinstance(depth, rz_depth_map) else depth_struct(*(depth or (DEPTH_LINEAR, 0.0)))
        if self.dry_run or after is None:
            after_p = None
        elif isinstance(after, str):
            after_p = _stream(None).value
        else:
            after_p = after.cuda_stream
        r = rz_request(int(cloud), int(mode), view_struct(view), ds,
                       rz_hq_params(int(eps[0]), int(eps[1])), int(background) & 0xFFFFFFFF,
                       RZ_REQ_INJECT_FAILURE if inject_failure else 0,
                       img.data_ptr() if img is not None else None, after_p)
        t = ctypes.c_uint64()
        _check(load().rz_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)),
               "rz_server_submit")
        return t.value

    def poll(self, ticket) -> dict:
        st = rz_request_status()
        _check(load().rz_server_poll(self._h, int(ticket), ctypes.byref(st)), "rz_server_poll")
        return {f: getattr(st, f) for f, _ in rz_request_status._fields_ if f != "pad"}

    def drain(self, timeout_s=60.0):
        _check(load().rz_server_drain(self._h, float(timeout_s)), "rz_server_drain")

    def stats(self) -> dict:
        st = rz_server_stats()
        _check(load().rz_server_get_stats(self._h, ctypes.byref(st)), "rz_server_get_stats")
        return {f: getattr(st, f) for f, _ in rz_server_stats._fields_ if f != "pad"}

    def close(self, timeout_s=600.0):
        """Waits up to timeout_s for the submitted requests, then frees the
        server; RzError(RZ_ESTATE) if requests are still running then (the
        server stays open)."""
        if getattr(self, "_h", None) and self._h.value:
            _check(load().rz_server_destroy(self._h, float(timeout_s)), "rz_server_destroy")
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
