"""Screen-sorted path vs the oracle, bit for bit: keys, splat sums and images
for shuffled and ordered clouds, screens that are not multiples of the tile
size, the largest screen the tile limit allows, tiles split into many slices,
piecewise depth maps, empty and fully culled inputs, and the count limit."""
import sys

import numpy as np
import pytest

from paper_1908_02681_amd import gen

pytestmark = pytest.mark.gpu


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


def sorted_keys(rz, pts, view, depth=None, hq=False, eps=(1, 100), bg=0):
    """Keys (and sums) left by the sorted path, then its resolved image."""
    import torch
    fb, acc = rz.new_framebuffer(view, bg, hq=hq)
    ws = rz.new_workspace(pts.n, view.width, view.height)
    ws.fill_(0x5A)   # contents on entry must not matter
    rz.rasterize_sorted(pts, view, depth, hq, eps, bg, fb=fb, acc=acc, workspace=ws,
                        keep_keys=True)
    keys = rz.to_u64(fb)
    sums = rz.unpack_acc(acc) if hq else None
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    npix = view.width * view.height
    img = (rz.resolve_hq(fb, acc, npix, bg, status=status) if hq else
           rz.resolve_min(fb, npix, bg))
    torch.cuda.synchronize()
    return keys, sums, rz.to_u32(img)


def check(rz, oracle, cloud, view, depth=(0, 0.0), eps=(1, 100), bg=0, label=""):
    import torch
    say(f"[sorted] {label} n={cloud.n} {view.width}x{view.height} depth={depth}")
    pts = rz.Points.from_cloud(cloud)
    ok_keys, ok_img = oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp,
                                              view.near, view.far, view.width, view.height,
                                              depth[0], depth[1], bg)
    keys, _, img = sorted_keys(rz, pts, view, depth, False, eps, bg)
    assert np.array_equal(keys, ok_keys), f"{label}: keys differ at {np.flatnonzero(keys != ok_keys)[:10]}"
    assert np.array_equal(img, ok_img)
    hk, hs, himg = oracle.render_hq(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near,
                                    view.far, view.width, view.height, depth[0], depth[1], eps, bg)
    k2, s2, i2 = sorted_keys(rz, pts, view, depth, True, eps, bg)
    assert np.array_equal(k2, hk)
    assert np.array_equal(s2, hs), f"{label}: sums differ at {np.flatnonzero((s2 != hs).any(1))[:10]}"
    assert np.array_equal(i2, himg)
    # the one-call form (resolve included) gives the same images
    _, _, a, _ = rz.rasterize_sorted(pts, view, depth, False, eps, bg)
    _, _, b, st = rz.rasterize_sorted(pts, view, depth, True, eps, bg)
    torch.cuda.synchronize()
    assert np.array_equal(rz.to_u32(a), ok_img) and np.array_equal(rz.to_u32(b), himg)
    assert int(st.item()) == 0
    return keys, s2


@pytest.mark.parametrize("size", [(97, 61), (1, 1), (33, 257), (640, 360), (32, 32)])
def test_shuffled_spheres(rz, oracle, size):
    cloud, view = gen.config1(n=300_000)
    view = gen.make_view((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, *size, 0.01, 10.0)
    check(rz, oracle, gen.shuffle(cloud, 4), view, bg=0x123456, label=f"spheres {size}")


def test_ordered_terrain(rz, oracle):
    """Morton order: long runs of fragments in one tile."""
    cloud = gen.terrain(2_000_000, 41, extent=100.0, amplitude=10.0, wavelength=40.0)
    view = gen.orbit_views(1, 7, [(320, 200)], extent=100.0, rmin=60.0, rmax=120.0, near=0.5,
                           far=400.0)[0]
    check(rz, oracle, cloud, view, label="terrain ordered")


@pytest.mark.parametrize("size", [(3840, 2160), (4096, 4096)])
def test_largest_screens(rz, oracle, size):
    """4096x4096 is 64 x 64 buckets of 64 x 64 pixels, the limit (pass A's
    16 KiB histogram and pass C's bucket offsets)."""
    cloud = gen.shuffle(gen.terrain(1_000_000, 42, extent=100.0, amplitude=10.0,
                                    wavelength=40.0), 2)
    view = gen.orbit_views(1, 8, [size], extent=100.0, rmin=60.0, rmax=120.0, near=0.5,
                           far=400.0)[0]
    check(rz, oracle, cloud, view, label=f"{size[0]}x{size[1]}")


def test_tile_limit(rz):
    import torch
    pts = rz.Points.from_cloud(gen.config1(n=1000)[0])
    view = gen.make_view((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, 4352, 4096, 0.01,
                         10.0)   # 68 x 64 buckets > 4096
    assert rz.load().rz_sorted_workspace_bytes(1000, 4352, 4096) == -1
    with pytest.raises(rz.RzError):
        rz.rasterize_sorted(pts, view, workspace=torch.empty(1 << 20, dtype=torch.uint8,
                                                             device="cuda"))


def test_many_slices(rz, oracle):
    """2M fragments on a 64x48 screen (one bucket): its entries are split
    over many chunks whose partial results merge in the global atomics."""
    cloud, _ = gen.config1(n=2_000_000)
    view = gen.make_view((0.5, 0.5, 2.0), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, 64, 48, 0.01, 10.0)
    check(rz, oracle, gen.shuffle(cloud, 5), view, label="many slices")


@pytest.mark.parametrize("which", ["spheres", "terrain"])
def test_piecewise(rz, oracle, which):
    pw = (2, ((0.0, 1.0e9), (2.0, 1.0e6), (50.0, 1.0e4)))
    if which == "spheres":
        cloud, view = gen.config1(n=200_000)
        pw = (2, ((0.0, 1.0e9), (2.0, 1.0e7), (3.0, 1.0e4)))
    else:
        cloud = gen.terrain(500_000, 43, extent=100.0, amplitude=10.0, wavelength=40.0)
        view = gen.orbit_views(1, 9, [(200, 150)], extent=100.0, rmin=60.0, rmax=120.0,
                               near=0.5, far=400.0)[0]
    check(rz, oracle, gen.shuffle(cloud, 6), view, depth=pw, label=f"piecewise {which}")


def test_scale_map_and_eps(rz, oracle):
    cloud, view = gen.config1(n=100_000)
    check(rz, oracle, gen.shuffle(cloud, 7), view, depth=(1, 1.0e6), eps=(3, 100), bg=0xFFFFFF,
          label="scale map eps 3%")


@pytest.mark.parametrize("n", [0, 1, 2047, 2048 * 1024 + 3])
def test_ragged_counts(rz, oracle, n):
    cloud, view = gen.config1(n=max(n, 1))
    cloud = gen.Cloud(cloud.x[:n], cloud.y[:n], cloud.z[:n], cloud.rgb[:n])
    check(rz, oracle, cloud, view, label=f"n={n}")


def test_all_culled(rz, oracle):
    cloud, view = gen.config1(n=10_000)
    behind = gen.Cloud(cloud.x, cloud.y, cloud.z + 100.0, cloud.rgb)   # behind the camera
    keys, _ = check(rz, oracle, behind, view, label="culled")
    assert (keys == np.uint64(oracle.clear_value(0))).all()


def test_unaligned_planes(rz, oracle):
    cloud, view = gen.config1(n=50_001)
    cl = gen.shuffle(cloud, 8)
    ok_keys, _ = oracle.render_atomicmin(cl.x[1:], cl.y[1:], cl.z[1:], cl.rgb[1:], view.vp,
                                         view.near, view.far, view.width, view.height)
    full = rz.Points.from_cloud(cl)
    pts = rz.Points(full.x[1:], full.y[1:], full.z[1:], full.rgb[1:])
    assert pts.x.data_ptr() % 16 != 0
    keys, _, _ = sorted_keys(rz, pts, view)
    assert np.array_equal(keys, ok_keys)


def test_shuffled_terrain_full_size(rz, oracle):
    """The 50M-point terrain, shuffled, at 1920x1080: every pixel, both modes."""
    cloud, view = gen.config2()
    keys, sums = check(rz, oracle, gen.shuffle(cloud, 1), view, label="50M shuffled 1920x1080")
    assert (keys != np.uint64(oracle.clear_value(0))).mean() > 0.3
    assert sums[:, 3].max() > 10


def test_count_limit(rz):
    """One pixel, 16843010 fragments in 64 slices of one tile: the partial
    sums merge exactly and the overflow status is set."""
    import torch
    n = 16_843_010
    view = gen.View(np.diag([1.0, 1.0, 0.0, 0.0]) + np.array(
        [[0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, -1.0, 0]]), 1.0, 100.0, 2, 2)
    pts = rz.Points(torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"),
                    torch.full((n,), -10.0, device="cuda"),
                    torch.full((n,), 0x00FF00, dtype=torch.int32, device="cuda"))
    fb, acc, _, _ = rz.rasterize_sorted(pts, view, hq=True, keep_keys=True)
    s = rz.unpack_acc(acc)
    assert s[3, 3] == n and s[3, 1] == (255 * n) % (1 << 32) and s[3, 0] == 0 and s[3, 2] == 0
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    rz.resolve_hq(fb, acc, 4, 0, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & rz.RZ_STATUS_HQ_OVERFLOW


LAYOUTS = {   # bucket (64x64 tile of a 640x360 screen, 10 x 6 of them) -> entries
    "sparse": {0: 3, 10: 100_000, 31: 1, 59: 777},
    "511 entries": {5: 200, 40: 311},
    "512 entries": {5: 200, 40: 312},
    "513 entries": {5: 200, 40: 313},
    "one bucket": {59: 3 * 512 + 1},
    "every other": {b: 1000 + b for b in range(0, 60, 2)},
}


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_shares_across_buckets(rz, oracle, layout):
    """Equal shares of the sorted entries per workgroup of the depth pass:
    totals around a multiple of the workgroup count, shares that cross runs
    of empty buckets, one bucket holding most entries, and depth-culled
    points (on screen, past far) among the entries."""
    W, H = 640, 360
    rng = np.random.default_rng(2024)
    xs, ys, ds = [], [], []
    for b, c in LAYOUTS[layout].items():
        tx, ty = b % 10, b // 10
        px = rng.integers(tx * 64, min(W, tx * 64 + 64), c)
        py = rng.integers(ty * 64, min(H, ty * 64 + 64), c)
        d = rng.uniform(1.0, 3.9, c)
        d[: c // 20] = 5.0   # past far: an entry with the key ~0
        xs.append(px)
        ys.append(py)
        ds.append(d)
    px, py, d = np.concatenate(xs), np.concatenate(ys), np.concatenate(ds)
    perm = rng.permutation(len(d))
    px, py, d = px[perm], py[perm], d[perm]
    cx = (2 * px + 1) / W - 1.0
    cy = (2 * py + 1) / H - 1.0
    cloud = gen.Cloud((cx * d).astype(np.float32), (cy * d).astype(np.float32),
                      (-d).astype(np.float32),
                      rng.integers(0, 1 << 24, len(d)).astype(np.uint32))
    # clip w = -z and x, y unscaled: (c * D, c' * D, -D) lands on NDC (c, c')
    vp = np.diag([1.0, 1.0, 0.0, 0.0]) + np.array(
        [[0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, -1.0, 0]])
    check(rz, oracle, cloud, gen.View(vp, 0.5, 4.0, W, H), label=layout)
