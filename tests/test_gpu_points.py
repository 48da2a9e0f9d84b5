"""rasterize_points vs the oracle, bit for bit: points of k x k pixels (both
methods, every integer depth map) and the float depth encodings of a
graphics depth buffer (depth pass), with the 1 mm at 1 km precision case."""
import sys

import numpy as np
import pytest

from paper_1908_02681_amd import gen

pytestmark = pytest.mark.gpu

GL24, F32REV = 3, 4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1908_02681_amd import rz as binding
    binding.load()
    return binding


def gpu_keys(rz, pts, view, depth, hq, k, eps=(1, 100), bg=0):
    import torch
    fb, acc = rz.new_framebuffer(view, bg, hq=hq)
    rz.rasterize_points(pts, view, depth, hq, eps, k, bg, fb=fb, acc=acc, keep_keys=True)
    keys = rz.to_u64(fb)
    sums = rz.unpack_acc(acc) if hq else None
    torch.cuda.synchronize()
    _, _, img, st = rz.rasterize_points(pts, view, depth, hq, eps, k, bg)
    torch.cuda.synchronize()
    if hq:
        assert int(st.item()) == 0
    return keys, sums, rz.to_u32(img)


def check(rz, oracle, cloud, view, depth=(0, 0.0), k=1, hq=True, eps=(1, 100), bg=0, label=""):
    say(f"[points] {label} n={cloud.n} {view.width}x{view.height} k={k} depth={depth}")
    pts = rz.Points.from_cloud(cloud)
    args = (cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near, view.far, view.width,
            view.height, depth[0], depth[1])
    want_k, want_img = oracle.render_atomicmin(*args, bg=bg, point_size=k)
    keys, _, img = gpu_keys(rz, pts, view, depth, False, k, eps, bg)
    assert np.array_equal(keys, want_k), f"{label}: keys differ at {np.flatnonzero(keys != want_k)[:8]}"
    assert np.array_equal(img, want_img)
    if hq:
        hk, hs, himg = oracle.render_hq(*args, eps=eps, bg=bg, point_size=k)
        k2, s2, i2 = gpu_keys(rz, pts, view, depth, True, k, eps, bg)
        assert np.array_equal(k2, hk)
        assert np.array_equal(s2, hs), f"{label}: sums differ at {np.flatnonzero((s2 != hs).any(1))[:8]}"
        assert np.array_equal(i2, himg)
    return keys


@pytest.mark.parametrize("k", [1, 2, 3, 4, 7])
def test_point_sizes_spheres(rz, oracle, k):
    cloud, _ = gen.config1(n=200_000)
    view = gen.make_view((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, 321, 203, 0.01, 10.0)
    check(rz, oracle, cloud, view, k=k, bg=0x102030, label="spheres")


@pytest.mark.parametrize("size,k", [((1, 1), 3), ((3, 2), 5), ((1, 7), 4), ((7, 1), 2)])
def test_points_larger_than_the_screen(rz, oracle, size, k):
    """k x k squares clipped on every side by a screen of a few pixels."""
    cloud, _ = gen.config1(n=20_000)
    view = gen.make_view((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, *size, 0.01, 10.0)
    check(rz, oracle, cloud, view, k=k, bg=0x0A0B0C, label=f"tiny {size}")


@pytest.mark.parametrize("k", [2, 5])
def test_point_sizes_terrain(rz, oracle, k):
    cloud = gen.terrain(500_000, 51, extent=100.0, amplitude=10.0, wavelength=40.0)
    view = gen.orbit_views(1, 12, [(200, 150)], extent=100.0, rmin=60.0, rmax=120.0, near=0.5,
                           far=400.0)[0]
    check(rz, oracle, cloud, view, k=k, label="terrain")


def test_point_size_piecewise_and_scale(rz, oracle):
    cloud, view = gen.config1(n=100_000)
    pw = (2, ((0.0, 1.0e9), (2.0, 1.0e7), (3.0, 1.0e4)))
    check(rz, oracle, cloud, view, depth=pw, k=3, label="piecewise")
    check(rz, oracle, cloud, view, depth=(1, 1.0e6), k=2, eps=(3, 100), label="scale")


@pytest.mark.parametrize("kind", [GL24, F32REV])
@pytest.mark.parametrize("k", [1, 3])
def test_float_depth_encodings(rz, oracle, kind, k):
    cloud, _ = gen.config1(n=300_000)
    view = gen.make_view((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, 256, 192, 0.01, 10.0)
    check(rz, oracle, cloud, view, depth=(kind, 0.0), k=k, hq=False, label=f"kind {kind}")
    terrain = gen.terrain(400_000, 52, extent=100.0, amplitude=10.0, wavelength=40.0)
    tv = gen.orbit_views(1, 13, [(160, 120)], extent=100.0, rmin=60.0, rmax=120.0, near=0.5,
                         far=400.0)[0]
    check(rz, oracle, terrain, tv, depth=(kind, 0.0), k=k, hq=False, label=f"terrain kind {kind}")


def test_atomicmin_call_takes_float_encodings(rz, oracle):
    import torch
    cloud, view = gen.config1(n=100_000)
    pts = rz.Points.from_cloud(cloud)
    for kind in (GL24, F32REV):
        _, img = rz.rasterize_atomicmin(pts, view, (kind, 0.0))
        torch.cuda.synchronize()
        _, want = oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp,
                                          view.near, view.far, view.width, view.height, kind)
        assert np.array_equal(rz.to_u32(img), want)


def test_float_depth_every_launch_shape(rz, oracle):
    """One-pixel float encodings take the depth pass's tile kernel at the
    default launch shape and the general point kernel at any other; both
    give the oracle's keys."""
    import torch
    cloud, view = gen.config1(n=150_000)
    pts = rz.Points.from_cloud(cloud)
    try:
        for shape in ((64, 16, 1, 0, 2), (256, 8, 1, 0, 2), (64, 16, 1, 0, 1), (128, 16, 1, 1, 2)):
            rz.set_launch(*shape)
            for kind in (GL24, F32REV):
                fb, _ = rz.new_framebuffer(view, 0)
                rz.rasterize_atomicmin(pts, view, (kind, 0.0), fb=fb, keep_keys=True)
                torch.cuda.synchronize()
                want = oracle.raster_min(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near,
                                         view.far, view.width, view.height, kind)
                assert np.array_equal(rz.to_u64(fb), want), (shape, kind)
    finally:
        rz.reset_launch()


def test_one_millimetre_at_one_kilometre(rz, oracle):
    """The precision case of the oracle pins on the GPU: the 40-bit map and
    the reversed float depth show the nearer surface everywhere, the 24-bit
    window depth lets the farther one through."""
    rng = np.random.default_rng(3)
    n, W, H = 20000, 64, 64
    v = gen.make_view((0, 0, 1000.0), (0, 0, 0), (0, 1, 0), 1.0, W, H, 0.5, 4000.0)
    x = rng.uniform(-8, 8, n).astype(np.float32)
    y = rng.uniform(-8, 8, n).astype(np.float32)
    front = np.arange(n) % 2 == 0
    z = np.where(front, np.float32(0.0), np.float32(-0.001)).astype(np.float32)
    rgb = np.where(front, 0x00FF00, 0x0000FF).astype(np.uint32)
    cloud = gen.Cloud(x, y, z, rgb)
    px = oracle.fragments(x[front], y[front], z[front], v.vp, v.near, v.far, W, H)[0]
    px = np.unique(px[px >= 0])
    shown = {}
    for kind in (0, F32REV, GL24):
        keys = check(rz, oracle, cloud, v, depth=(kind, 0.0), k=1, hq=False, label=f"1mm {kind}")
        shown[kind] = ((keys[px] & np.uint64(0xFFFFFF)) == 0x00FF00).mean()
    say(f"[points] nearer surface shown: {shown}")
    assert shown[0] == 1.0 and shown[F32REV] == 1.0 and shown[GL24] < 0.2


def test_full_size_terrain(rz, oracle):
    """The 50M-point terrain at 1920x1080, every pixel: points of 2 x 2
    pixels (depth and splat frames) and the 24-bit window depth."""
    cloud, view = gen.config2()
    check(rz, oracle, cloud, view, k=2, label="50M terrain, point size 2")
    check(rz, oracle, cloud, view, depth=(GL24, 0.0), k=1, hq=False, label="50M terrain, gl24")


@pytest.mark.parametrize("n", [0, 1, 1023, 1025])
def test_ragged_and_unaligned(rz, oracle, n):
    cloud, view = gen.config1(n=max(n, 2) + 1)
    c = gen.Cloud(cloud.x[1:n + 1], cloud.y[1:n + 1], cloud.z[1:n + 1], cloud.rgb[1:n + 1])
    check(rz, oracle, c, view, k=3, label=f"n={n}")
    full = rz.Points.from_cloud(cloud)
    pts = rz.Points(full.x[1:n + 1], full.y[1:n + 1], full.z[1:n + 1], full.rgb[1:n + 1])
    keys, _, _ = gpu_keys(rz, pts, view, (0, 0.0), False, 3)
    want = oracle.raster_min(c.x, c.y, c.z, c.rgb, view.vp, view.near, view.far, view.width,
                             view.height, point_size=3)
    assert np.array_equal(keys, want)
