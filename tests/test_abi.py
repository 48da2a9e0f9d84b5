"""The C-ABI library loads, exports every function include/rz.h declares, and
rejects bad arguments with the documented codes before touching a device
(no GPU needed: validation runs on the host before any HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


@pytest.fixture(scope="module")
def rz():
    from paper_1908_02681_amd import build, rz as binding
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    binding.load()
    return binding


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                             text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("rasterize_atomicmin", "rasterize_hq_splat", "rz_clear", "rz_resolve_min",
              "rz_resolve_hq", "rz_error_string", "rasterize_sorted", "rz_sorted_workspace_bytes",
              "rasterize_points", "rz_merge_min", "rz_merge_sum", "rz_check_reciprocal"):
        assert n in names


def test_library_exports_every_declared_symbol(rz):
    lib = ctypes.CDLL(rz.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header(rz):
    assert set(declared_functions()) <= set(rz.SIGNATURES)


def test_error_strings(rz):
    assert rz.error_string(0) == "ok"
    for code in (rz.RZ_EINVAL, rz.RZ_EDEPTHRANGE, rz.RZ_EHIP, rz.RZ_EOVERFLOW, rz.RZ_EBUDGET,
                 rz.RZ_ESTATE):
        assert rz.error_string(code) not in ("ok", "unknown error")
    assert rz.error_string(12345) == "unknown error"
    assert rz.load().rz_version() >= 100


class _View:
    def __init__(self, near=0.5, far=100.0, w=64, h=48, vp=None):
        self.vp = np.eye(4) if vp is None else vp
        self.near, self.far, self.width, self.height = near, far, w, h


def _call_min(rz, pts=None, view=None, depth=(0, 0.0), fb=1, img=1, flags=0):
    lib = rz.load()
    ps = pts if pts is not None else rz.rz_points(1, 1, 1, 1, 10)
    vs = rz.view_struct(view or _View())
    ds = rz.depth_struct(*depth)
    return lib.rasterize_atomicmin(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds), 0,
                                   fb and ctypes.c_void_p(fb), img and ctypes.c_void_p(img),
                                   flags, None)


def test_argument_validation(rz):
    E = rz
    lib = rz.load()
    assert _call_min(rz, pts=rz.rz_points(0, 1, 1, 1, 10)) == E.RZ_EINVAL        # null plane
    assert _call_min(rz, pts=rz.rz_points(1, 1, 1, 1, -1)) == E.RZ_EINVAL        # n < 0
    assert _call_min(rz, pts=rz.rz_points(1, 1, 1, 1, 2 ** 32)) == E.RZ_EINVAL   # n too large
    assert _call_min(rz, view=_View(w=0)) == E.RZ_EINVAL
    assert _call_min(rz, view=_View(h=40000)) == E.RZ_EINVAL
    assert _call_min(rz, view=_View(near=0.0)) == E.RZ_EINVAL
    assert _call_min(rz, view=_View(near=2.0, far=1.0)) == E.RZ_EINVAL
    bad = np.eye(4)
    bad[0, 0] = np.nan
    assert _call_min(rz, view=_View(vp=bad)) == E.RZ_EINVAL
    assert _call_min(rz, depth=(7, 0.0)) == E.RZ_EINVAL                            # unknown map
    assert _call_min(rz, depth=(1, -1.0)) == E.RZ_EINVAL                           # scale <= 0
    # millimetres up to 1e9 m fit 40 bits; 1.1e9 m do not (section 2.1)
    assert _call_min(rz, view=_View(far=1.2e9), depth=(1, 1000.0)) == E.RZ_EDEPTHRANGE
    # piecewise: starts must increase, the first must not lie beyond near,
    # and the last range must reach far inside 40 bits
    pw = ((0.0, 1e9), (10.0, 1e6), (1e4, 1e3))
    assert _call_min(rz, view=_View(near=0.5), depth=(2, ((1.0, 1e3),))) == E.RZ_EINVAL
    assert _call_min(rz, view=_View(far=5.0), depth=(2, ((0.0, 1e3), (0.0, 1e3)))) == E.RZ_EINVAL
    assert _call_min(rz, view=_View(far=5.0), depth=(2, ((0.0, -1.0),))) == E.RZ_EINVAL
    assert _call_min(rz, view=_View(far=5.0), depth=(2, ())) == E.RZ_EINVAL
    assert _call_min(rz, view=_View(far=2e9), depth=(2, pw)) == E.RZ_EDEPTHRANGE
    assert _call_min(rz, fb=0) == E.RZ_EINVAL
    assert _call_min(rz, img=0) == E.RZ_EINVAL                                     # img needed
    assert _call_min(rz, flags=2) == E.RZ_EINVAL
    # hq: eps limits
    ps, vs, ds = rz.rz_points(1, 1, 1, 1, 10), rz.view_struct(_View()), rz.depth_struct()
    for num, den, code in ((1, 0, E.RZ_EINVAL), (1, 2 ** 21, E.RZ_EINVAL),
                           (2 ** 21, 1, E.RZ_EINVAL)):
        hq = rz.rz_hq_params(num, den)
        assert lib.rasterize_hq_splat(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds),
                                      ctypes.byref(hq), 0, ctypes.c_void_p(1), ctypes.c_void_p(1),
                                      ctypes.c_void_p(1), None, 0, None) == code
    # eps test would overflow: huge near/far ratio makes z0 enormous
    vz = rz.view_struct(_View(near=1e6, far=1e6 + 1e-3))
    hq = rz.rz_hq_params(2 ** 20, 1)
    assert lib.rasterize_hq_splat(ctypes.byref(ps), ctypes.byref(vz), ctypes.byref(ds),
                                  ctypes.byref(hq), 0, ctypes.c_void_p(1), ctypes.c_void_p(1),
                                  ctypes.c_void_p(1), None, 0, None) == E.RZ_EDEPTHRANGE
    assert lib.rz_clear(None, None, 5, 0, None) == E.RZ_EINVAL
    assert lib.rz_clear(None, None, -1, 0, None) == E.RZ_EINVAL
    assert lib.rz_resolve_min(ctypes.c_void_p(1), 4, 0, None, None) == E.RZ_EINVAL
    assert lib.rz_resolve_hq(ctypes.c_void_p(1), None, 4, 0, ctypes.c_void_p(1), None,
                             None) == E.RZ_EINVAL


def test_splat_resolve_requires_a_status_word(rz):
    """Every call that resolves splat sums refuses a NULL status word (the
    only place an overflowed count is reported, section 2.2's sums being
    packed); with RZ_KEEP_KEYS nothing is resolved and NULL is accepted as
    far as validation goes (it fails later only on the fake pointers, which
    these calls never reach)."""
    lib = rz.load()
    ps, vs, ds = rz.rz_points(1, 1, 1, 1, 10), rz.view_struct(_View()), rz.depth_struct()
    hq = rz.rz_hq_params(1, 100)
    one = ctypes.c_void_p(16)
    b = ctypes.byref
    assert lib.rasterize_hq_splat(b(ps), b(vs), b(ds), b(hq), 0, one, one, one, None, 0,
                                  None) == rz.RZ_EINVAL
    assert lib.rasterize_points(b(ps), b(vs), b(ds), b(hq), 2, 0, one, one, one, None, 0,
                                None) == rz.RZ_EINVAL
    assert lib.rasterize_sorted(b(ps), b(vs), b(ds), b(hq), 0, one, one, one, None, one,
                                1 << 40, 0, None) == rz.RZ_EINVAL
    assert lib.rz_resolve_hq(one, one, 4, 0, one, None, None) == rz.RZ_EINVAL
    assert lib.rz_resolve_hq(one, one, 0, 0, one, None, None) == rz.RZ_EINVAL
    # the depth-only forms need no status word (they fail here on the
    # missing image instead, which shows they got past the status check)
    assert lib.rasterize_points(b(ps), b(vs), b(ds), None, 2, 0, one, None, None, None, 0,
                                None) == rz.RZ_EINVAL
    # a batch with a splatting view needs opts.status
    views = (rz.rz_batch_view * 2)(
        rz.rz_batch_view(vs, ds, rz.RZ_MODE_ATOMICMIN, hq, 0, 16, None, 48),
        rz.rz_batch_view(vs, ds, rz.RZ_MODE_HQ, hq, 0, 80, 96, 112))
    opts = rz.rz_batch_opts()
    h = ctypes.c_void_p()
    assert lib.rz_batch_plan(b(ps), views, 2, b(opts), b(h)) == rz.RZ_EINVAL
    assert not h.value


def test_sorted_path_validation(rz):
    """Workspace sizes and the checks made before any launch."""
    lib = rz.load()
    assert lib.rz_sorted_workspace_bytes(-1, 64, 48) == -1
    assert lib.rz_sorted_workspace_bytes(10, 0, 48) == -1
    small = lib.rz_sorted_workspace_bytes(0, 64, 48)
    big = lib.rz_sorted_workspace_bytes(1_000_000, 64, 48)
    assert small >= 0 and small % 256 == 0 and big % 256 == 0
    assert big >= small + 10 * 1_000_000      # an 8-byte key + 2-byte pixel per point
    ps, ds = rz.rz_points(1, 1, 1, 1, 10), rz.depth_struct()
    need = lib.rz_sorted_workspace_bytes(10, 64, 48)

    def call(view=None, ws=256 * 4096, ws_bytes=None, hq=None, fb=1, acc=1, img=1):
        vs = rz.view_struct(view or _View())
        return lib.rasterize_sorted(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds),
                                    hq and ctypes.byref(hq), 0, fb and ctypes.c_void_p(fb),
                                    acc and ctypes.c_void_p(acc), img and ctypes.c_void_p(img),
                                    None, ws and ctypes.c_void_p(ws),
                                    need if ws_bytes is None else ws_bytes, 0, None)
    E = rz.RZ_EINVAL
    assert call(view=_View(w=4352, h=4096)) == E            # 68 x 64 buckets > 4096
    assert lib.rz_sorted_workspace_bytes(10, 4352, 4096) == -1
    assert lib.rz_sorted_workspace_bytes(10, 4096, 4096) > 0
    assert call(ws=0) == E                                   # no workspace
    assert call(ws=256 * 4096 + 8) == E                      # not 256-byte aligned
    assert call(ws_bytes=need - 1) == E                      # too small
    assert call(hq=rz.rz_hq_params(1, 100), acc=0) == E      # splatting needs acc
    assert call(hq=rz.rz_hq_params(1, 0)) == E
    assert call(fb=0) == E and call(img=0) == E


def test_points_and_float_depth_validation(rz):
    """Checks of rasterize_points and of the float depth encodings made
    before any launch."""
    lib = rz.load()
    ps = rz.rz_points(1, 1, 1, 1, 10)
    vs = rz.view_struct(_View())
    E = rz.RZ_EINVAL

    def call(k=2, depth=(0, 0.0), hq=None, acc=1):
        ds = rz.depth_struct(*depth)
        return lib.rasterize_points(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds),
                                    hq and ctypes.byref(hq), k, 0, ctypes.c_void_p(1),
                                    acc and ctypes.c_void_p(acc), ctypes.c_void_p(1), None, 0,
                                    None)
    assert call(k=0) == E and call(k=17) == E
    assert call(hq=rz.rz_hq_params(1, 100), acc=0) == E
    for kind in (rz.DEPTH_GL24, rz.DEPTH_F32REV):
        assert call(depth=(kind, 0.0), hq=rz.rz_hq_params(1, 100)) == E   # depth pass only
        ds = rz.depth_struct(kind, 0.0)
        hq = rz.rz_hq_params(1, 100)
        assert lib.rasterize_hq_splat(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds),
                                      ctypes.byref(hq), 0, ctypes.c_void_p(1), ctypes.c_void_p(1),
                                      ctypes.c_void_p(1), None, 0, None) == E
        assert lib.rasterize_sorted(ctypes.byref(ps), ctypes.byref(vs), ctypes.byref(ds), None, 0,
                                    ctypes.c_void_p(1), None, ctypes.c_void_p(1), None,
                                    ctypes.c_void_p(256 * 4096), 1 << 30, 0, None) == E
    assert call(depth=(5, 0.0)) == E                                        # unknown kind


def test_merge_validation(rz):
    lib = rz.load()
    E = rz.RZ_EINVAL
    P = ctypes.c_void_p
    for fn in (lib.rz_merge_min, lib.rz_merge_sum):
        assert fn(P(256), P(1 << 20), -1, None) == E
        assert fn(P(256), P(1 << 20), 0, None) == rz.RZ_OK       # nothing to do
        assert fn(None, P(1 << 20), 4, None) == E
        assert fn(P(256 + 8), P(1 << 20), 4, None) == E          # not 16-byte aligned
        assert fn(P(4096), P(4096 + 16), 4, None) == E           # overlapping


def test_reciprocal_check_validation(rz):
    lib = rz.load()
    E = rz.RZ_EINVAL
    P = ctypes.c_void_p
    assert lib.rz_check_reciprocal(0, -1, P(256), 0, None) == E
    assert lib.rz_check_reciprocal(1, 1 << 32, P(256), 0, None) == E       # past 2^32 patterns
    assert lib.rz_check_reciprocal(0xFFFFFFFF, 2, P(256), 0, None) == E
    assert lib.rz_check_reciprocal(0, 16, None, 0, None) == E
    assert lib.rz_check_reciprocal(0, 16, P(256 + 4), 0, None) == E       # not 8-byte aligned
    assert lib.rz_check_reciprocal(0, 16, P(256), 2, None) == E            # unknown flag
    assert lib.rz_check_reciprocal(0, 0, P(256), rz.RZ_CHECK_ESTIMATE_ONLY, None) == rz.RZ_OK


def test_noalloc_sorted_validation(rz):
    """The allocation-free sorted call refuses, before any device call, a
    cloud whose workspace would not fit its static scratch, and bad sizes."""
    lib = rz.load()
    b = ctypes.byref
    vs, ds = rz.view_struct(_View(w=1920, h=1080)), rz.depth_struct()
    one = ctypes.c_void_p(16)
    big = rz.rz_points(16, 16, 16, 16, 10_000_000)
    assert rz.sorted_workspace_bytes(big.n, 1920, 1080) > rz.RZ_NOALLOC_SCRATCH_BYTES
    assert lib.rasterize_sorted_noalloc(b(big), b(vs), b(ds), None, 0, one, None, one, None, 0,
                                        None) == rz.RZ_EBUDGET
    assert lib.rasterize_sorted_noalloc(None, b(vs), b(ds), None, 0, one, None, one, None, 0,
                                        None) == rz.RZ_EINVAL
    huge = rz.view_struct(_View(w=20000, h=20000))    # too many screen buckets
    small = rz.rz_points(16, 16, 16, 16, 10)
    assert lib.rasterize_sorted_noalloc(b(small), b(huge), b(ds), None, 0, one, None, one, None,
                                        0, None) == rz.RZ_EINVAL


def test_reciprocal_values_validation(rz):
    lib = rz.load()
    assert lib.rz_reciprocal(None, None, -1, None) == rz.RZ_EINVAL
    assert lib.rz_reciprocal(None, ctypes.c_void_p(16), 4, None) == rz.RZ_EINVAL
    assert lib.rz_reciprocal(ctypes.c_void_p(16), None, 4, None) == rz.RZ_EINVAL
    assert lib.rz_reciprocal(None, None, 0, None) == rz.RZ_OK


def test_launch_shape_validation(rz):
    lib = rz.load()
    before = rz.get_launch()
    for bad in ((96, 8, 1, 1, 0), (256, 6, 1, 1, 0), (256, 8, 2, 1, 0), (256, 8, 1, 5, 0),
                (256, 8, 1, 1, 4), (256, 8, 1, 1, -1)):
        assert lib.rz_set_launch(ctypes.byref(rz.rz_launch(*bad))) == rz.RZ_EINVAL
    assert rz.get_launch() == before
    rz.set_launch(128, 4, 0, 0)
    assert rz.get_launch()["block"] == 128 and rz.get_launch()["ppt"] == 4
    rz.set_launch(256, 4, 1, 0, 3)   # the small per-wave tile
    assert rz.get_launch()["bin"] == 3
    rz.set_launch(**before)
    rz.reset_launch()
    assert rz.get_launch() == {"block": 64, "ppt": 16, "early_out": 1, "xcd_remap": 0, "bin": 2}


def test_binding_refuses_without_gpu(rz):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(rz.RzError):
        rz.new_framebuffer(_View())


def test_batch_plan_validation(rz):
    """rz_batch_plan rejects bad batches before it allocates anything."""
    lib = rz.load()
    ps = rz.rz_points(1, 1, 1, 1, 10)

    def view(mode=0, fb=16, acc=32, img=48, w=64):
        return rz.rz_batch_view(rz.view_struct(_View(w=w)), rz.depth_struct(), mode,
                                rz.rz_hq_params(1, 100), 0, fb, acc, img)

    def plan(views, k=0, block=0):
        arr = (rz.rz_batch_view * max(1, len(views)))(*views)
        opts = rz.rz_batch_opts()
        opts.views_per_group = k
        opts.launch.block = block
        if block:
            opts.launch.ppt = 8
        h = ctypes.c_void_p()
        return lib.rz_batch_plan(ctypes.byref(ps), arr, len(views), ctypes.byref(opts),
                                 ctypes.byref(h))

    assert plan([]) == rz.RZ_EINVAL
    assert plan([view(mode=2)]) == rz.RZ_EINVAL
    assert plan([view(fb=0)]) == rz.RZ_EINVAL
    assert plan([view(mode=1, acc=0)]) == rz.RZ_EINVAL
    assert plan([view(), view(fb=16, img=80)]) == rz.RZ_EINVAL        # shared fb
    assert plan([view(), view(fb=96, img=48)]) == rz.RZ_EINVAL        # shared img
    assert plan([view(w=0)]) == rz.RZ_EINVAL
    assert plan([view()], k=9) == rz.RZ_EINVAL
    assert plan([view()], block=96) == rz.RZ_EINVAL
    for fn in ("rz_batch_run", "rz_batch_capture", "rz_batch_destroy"):
        args = (None, None) if fn == "rz_batch_run" else (None,)
        assert getattr(lib, fn)(*args) == rz.RZ_EINVAL


def test_launch_shape_is_never_torn(rz):
    """rz_set_launch and rz_get_launch from several threads at once (ctypes
    drops the GIL around each call): every read returns one of the shapes
    written, never a mix of two."""
    import threading
    shapes = [(256, 4, 0, 1, 0), (64, 16, 1, 0, 2), (512, 8, 1, 1, 1)]
    allowed = {s for s in shapes}
    bad = []

    def writer(shape):
        for _ in range(3000):
            rz.set_launch(*shape)

    def reader():
        for _ in range(3000):
            g = rz.get_launch()
            t = (g["block"], g["ppt"], g["early_out"], g["xcd_remap"], g["bin"])
            if t not in allowed:
                bad.append(t)

    rz.set_launch(*shapes[0])
    threads = [threading.Thread(target=writer, args=(s,)) for s in shapes]
    threads += [threading.Thread(target=reader) for _ in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    rz.reset_launch()
    assert not bad, bad[:3]


def test_binding_checks_buffer_sizes(rz):
    """The binding refuses a buffer too small or not contiguous for what the
    library will write into it (the C ABI takes bare pointers)."""
    import torch
    npix = 6
    rz._fits_view(npix, torch.empty(npix, dtype=torch.int64), torch.empty(2 * npix, dtype=torch.int64),
                  torch.empty(npix, dtype=torch.int32), torch.empty(1, dtype=torch.int32))
    for kw in ({"fb": torch.empty(npix - 1, dtype=torch.int64)},
               {"acc": torch.empty(2 * npix - 1, dtype=torch.int64)},
               {"img": torch.empty(npix, dtype=torch.int16)},
               {"status": torch.empty(0, dtype=torch.int32)},
               {"fb": torch.empty(2 * npix, dtype=torch.int64)[::2]}):
        with pytest.raises(rz.RzError):
            rz._fits_view(npix, **kw)
