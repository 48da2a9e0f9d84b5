"""GPU path vs CPU oracle, bit for bit (framebuffer keys, splat sums and
images are integers).  Runs through the C ABI via the Python binding."""
import json
import os
import sys

import numpy as np
import pytest

from paper_1908_02681_amd import gen

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1908_02681_amd import rz as binding
    binding.load()
    yield binding
    binding.reset_launch()


def gpu_min(rz, pts, view, depth=None, bg=0):
    """(keys, image) from the GPU: keys via RZ_KEEP_KEYS, image via a full call."""
    import torch
    fb, _ = rz.new_framebuffer(view, bg)
    fb, _ = rz.rasterize_atomicmin(pts, view, depth, bg, fb=fb, keep_keys=True)
    keys = rz.to_u64(fb)
    img = rz.resolve_min(fb, view.width * view.height, bg)
    torch.cuda.synchronize()
    cleared = rz.to_u64(fb)
    return keys, rz.to_u32(img), cleared


def gpu_hq(rz, pts, view, depth=None, eps=(1, 100), bg=0):
    import torch
    fb, acc = rz.new_framebuffer(view, bg, hq=True)
    rz.rasterize_hq_splat(pts, view, depth, eps, bg, fb=fb, acc=acc, keep_keys=True)
    keys = rz.to_u64(fb)
    sums = rz.unpack_acc(acc)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    img = rz.resolve_hq(fb, acc, view.width * view.height, bg, status=status)
    torch.cuda.synchronize()
    return keys, sums, rz.to_u32(img), rz.to_u64(fb), rz.to_u64(acc), int(status.item())


def full_call(rz, pts, view, depth=None, eps=(1, 100), bg=0):
    """Images of the one-call forms (resolve included)."""
    import torch
    _, img = rz.rasterize_atomicmin(pts, view, depth, bg)
    fb, acc, himg, status = rz.rasterize_hq_splat(pts, view, depth, eps, bg)
    torch.cuda.synchronize()
    return rz.to_u32(img), rz.to_u32(himg), rz.to_u64(fb), rz.to_u64(acc), int(status.item())


def check_scene(rz, oracle, cloud, view, depth=(0, 0.0), eps=(1, 100), bg=0, label=""):
    say(f"[parity] {label} n={cloud.n} {view.width}x{view.height} depth={depth} eps={eps}")
    pts = rz.Points.from_cloud(cloud)
    ok_keys, ok_img = oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp,
                                              view.near, view.far, view.width, view.height,
                                              depth[0], depth[1], bg)
    keys, img, cleared = gpu_min(rz, pts, view, depth, bg)
    assert np.array_equal(keys, ok_keys), f"{label}: keys differ at {np.flatnonzero(keys != ok_keys)[:10]}"
    assert np.array_equal(img, ok_img)
    assert (cleared == np.uint64(oracle.clear_value(bg))).all()
    hk, hs, himg = oracle.render_hq(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near,
                                    view.far, view.width, view.height, depth[0], depth[1], eps, bg)
    k2, s2, i2, fb_after, acc_after, status = gpu_hq(rz, pts, view, depth, eps, bg)
    assert np.array_equal(k2, hk)
    assert np.array_equal(s2, hs), f"{label}: sums differ at {np.flatnonzero((s2 != hs).any(1))[:10]}"
    assert np.array_equal(i2, himg)
    assert (fb_after == np.uint64(oracle.clear_value(bg))).all() and (acc_after == 0).all()
    assert status == 0
    a, b, fb3, acc3, st3 = full_call(rz, pts, view, depth, eps, bg)
    assert np.array_equal(a, ok_img) and np.array_equal(b, himg)
    assert (fb3 == np.uint64(oracle.clear_value(bg))).all() and (acc3 == 0).all() and st3 == 0
    return ok_keys, hs


# --------------------------------------------------------------------------

def test_hand_cases_on_gpu(rz, oracle):
    with open(os.path.join(GOLD, "hand_cases.json")) as f:
        g = json.load(f)
    view = gen.View(np.array(g["vp"], np.float64), g["near"], g["far"], g["width"], g["height"])
    for c in g["cases"]:
        say(f"[hand] {c['name']}")
        a = np.array([[r[0], r[1], r[2]] for r in c["points"]], np.float32)
        rgb = np.array([int(r[3], 16) for r in c["points"]], np.uint32)
        cloud = gen.Cloud(a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy(), rgb)
        pts = rz.Points.from_cloud(cloud)
        keys, img, _ = gpu_min(rz, pts, view, (1, g["scale"]))
        if "key" in c:
            assert int(keys[c["pixel"]]) == int(c["key"], 16)
            assert int(img[c["pixel"]]) == int(c["image"], 16)
        if "sums" in c:
            _, sums, himg, *_ = gpu_hq(rz, pts, view, (1, g["scale"]), tuple(c["eps"]))
            assert sums[c["pixel"]].tolist() == c["sums"]
            assert int(himg[c["pixel"]]) == int(c["hq_image"], 16)


def test_config1_spheres(rz, oracle):
    cloud, view = gen.config1()
    check_scene(rz, oracle, cloud, view, label="1M spheres 1024x768")


PAPER_RANGES = ((0.0, 1.0e9), (10.0, 1.0e6), (1.0e4, 1.0e3))   # nm, um, mm (section 2.1)


@pytest.mark.parametrize("which", ["spheres", "terrain"])
def test_piecewise_depth_map(rz, oracle, which):
    if which == "spheres":
        cloud, view = gen.config1(n=400_000)
    else:
        cloud = gen.terrain(2_000_000, 6)
        view = gen.terrain_view(640, 360)
    check_scene(rz, oracle, cloud, view, depth=(2, PAPER_RANGES), label=f"piecewise {which}")


def test_piecewise_window_across_ranges(rz, oracle):
    """Fragments straddling the 10 m range boundary: the GPU's window test in
    linear depth equals the oracle's (hand-worked values in the oracle pins)."""
    rng = np.random.default_rng(4)
    n = 20000
    z = -rng.uniform(9.9, 10.1, n).astype(np.float32)
    x = (rng.integers(0, 4, n) * 0.5 - 0.75).astype(np.float32)
    y = (rng.integers(0, 4, n) * 0.5 - 0.75).astype(np.float32)
    vp = np.zeros((4, 4))
    vp[0, 0] = vp[1, 1] = 10.0
    vp[3, 2] = -1.0
    cloud = gen.Cloud(x * 1.0, y * 1.0, z, rng.integers(0, 1 << 24, n, dtype=np.uint32))
    view = gen.View(vp, 0.25, 1.0e7, 8, 8)
    check_scene(rz, oracle, cloud, view, depth=(2, PAPER_RANGES), label="window across ranges")


def test_background_and_scale_map(rz, oracle):
    cloud, view = gen.config1(n=300_000)
    check_scene(rz, oracle, cloud, view, depth=(1, 1000.0), bg=0x3A2B1C, label="mm map, bg")


def test_window_with_large_depth_offset(rz, oracle):
    """A thin depth range far from the camera (near 10 km, far 10 km + 1 m)
    puts the linear map's offset z0 = floor(near * s) above 2^52, where the
    accumulate kernels skip their double-precision pre-test of the eps
    window and use the integer test alone; dense enough that many pixels
    average several fragments."""
    rng = np.random.default_rng(21)
    n = 400_000
    W, H = 96, 64
    view = gen.make_view((0, 0, 10000.5), (0, 0, 0), (0, 1, 0), 0.5, W, H, 10000.0, 10001.0)
    o, s, z0 = oracle.depth_constants(view.vp, view.near, view.far, W, H)
    assert z0 >= 2 ** 52
    x = rng.uniform(-45, 45, n).astype(np.float32)
    y = rng.uniform(-30, 30, n).astype(np.float32)
    z = rng.uniform(-0.45, 0.45, n).astype(np.float32)
    rgb = rng.integers(0, 1 << 24, n, dtype=np.uint32)
    _, sums = check_scene(rz, oracle, gen.Cloud(x, y, z, rgb), view, eps=(1, 100000),
                          label="z0 above 2^52")
    assert (sums[:, 3] > 1).sum() > W * H // 4


@pytest.mark.parametrize("n", [0, 1, 3, 63, 1000, 4097, 2048 * 8 + 5, 123_457])
def test_ragged_sizes(rz, oracle, n):
    cloud = gen.terrain(max(n, 1), 5, extent=50.0, amplitude=5.0, wavelength=20.0)
    cloud = cloud.take(np.arange(n))
    view = gen.terrain_view(97, 61, extent=50.0, distance=60.0, near=0.5, far=400.0)
    check_scene(rz, oracle, cloud, view, label=f"ragged n={n}")


LAUNCHES = [(b, p, e, x, n) for b in (64, 256, 512) for p in (4, 8, 16) for e in (0, 1)
            for x in (0, 1) for n in (0, 1, 2, 3)]


def test_every_launch_shape_is_bit_identical(rz, oracle):
    cloud = gen.terrain(200_003, 9, extent=100.0, amplitude=10.0, wavelength=40.0)
    view = gen.terrain_view(160, 120, extent=100.0, distance=120.0, near=0.5, far=400.0)
    ok_keys, _ = oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near,
                                         view.far, view.width, view.height)
    _, ok_sums, ok_img = oracle.render_hq(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near,
                                          view.far, view.width, view.height)
    pts = rz.Points.from_cloud(cloud)
    try:
        for b, p, e, x, n in LAUNCHES:
            say(f"[launch] block={b} ppt={p} early={e} xcd={x} bin={n}")
            rz.set_launch(b, p, e, x, n)
            keys, _, _ = gpu_min(rz, pts, view)
            assert np.array_equal(keys, ok_keys)
            _, sums, img, *_ = gpu_hq(rz, pts, view)
            assert np.array_equal(sums, ok_sums) and np.array_equal(img, ok_img)
    finally:
        rz.reset_launch()


@pytest.mark.parametrize("bin_", [0, 1, 2, 3])
def test_tile_fallback_and_sparse_screens(rz, oracle, bin_):
    """Workgroups whose fragments span more than one LDS tile (random points
    over a wide screen) take the direct path; both give the oracle's bits."""
    rng = np.random.default_rng(12)
    n = 300_000
    cloud = gen.Cloud(rng.uniform(-1, 1, n).astype(np.float32), rng.uniform(-1, 1, n).astype(np.float32),
                      rng.uniform(0, 1, n).astype(np.float32),
                      rng.integers(0, 1 << 24, n, dtype=np.uint32))
    vp = np.eye(4)
    vp[3, :] = [0, 0, 0.5, 1.0]
    view = gen.View(vp, 0.9, 2.0, 1500, 900)
    try:
        rz.set_launch(bin=bin_)
        check_scene(rz, oracle, cloud, view, label=f"wide random bin={bin_}")
        # a Morton terrain clipped by the screen edge: tiles at the border
        t = gen.terrain(400_000, 8, extent=100.0, amplitude=10.0, wavelength=40.0)
        v2 = gen.terrain_view(300, 200, extent=100.0, distance=60.0, near=0.5, far=400.0)
        check_scene(rz, oracle, t, v2, label=f"clipped terrain bin={bin_}")
    finally:
        rz.reset_launch()


@pytest.mark.parametrize("size", [(1, 1), (1, 7), (7, 1), (3, 2)])
def test_tiny_screens(rz, oracle, size):
    """Screens of one pixel, one column and one row: every wave's fragments
    pile onto a few pixels, in tiles one pixel wide or high; under every
    merge mode (direct atomics, workgroup tiles, wave tiles)."""
    cloud, _ = gen.config1(n=20_000)
    view = gen.make_view((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, *size, 0.01, 10.0)
    try:
        for bin_ in (3, 2, 1, 0):
            rz.set_launch(bin=bin_)
            check_scene(rz, oracle, cloud, view, bg=0x0A0B0C, label=f"tiny {size} bin={bin_}")
    finally:
        rz.reset_launch()


def test_binding_refuses_small_buffers(rz):
    """Each call refuses an fb, acc or img shorter than the view before
    anything is enqueued.  The short buffers are slices of full-size ones, so
    nothing could be written outside an allocation either way."""
    import torch
    cloud, view = gen.config1(n=1000)
    view = gen.View(view.vp, view.near, view.far, 64, 32)
    pts = rz.Points.from_cloud(cloud)
    fb, acc = rz.new_framebuffer(view, hq=True)
    img = torch.empty(64 * 32, dtype=torch.int32, device="cuda")
    short_fb, short_acc, short_img = fb[:-1], acc[:-1], img[:-1]
    calls = [
        lambda: rz.rasterize_atomicmin(pts, view, fb=short_fb, img=img),
        lambda: rz.rasterize_atomicmin(pts, view, fb=fb, img=short_img),
        lambda: rz.rasterize_hq_splat(pts, view, fb=fb, acc=short_acc, img=img),
        lambda: rz.rasterize_points(pts, view, hq=True, point_size=3, fb=fb, acc=short_acc, img=img),
        lambda: rz.rasterize_sorted(pts, view, fb=short_fb, img=img),
        lambda: rz.resolve_min(short_fb, 64 * 32, img=img),
        lambda: rz.clear(fb, short_acc, 64 * 32),
        lambda: rz.merge_min(fb, short_fb, 64 * 32),
    ]
    for i, call in enumerate(calls):
        with pytest.raises(rz.RzError):
            call()
    torch.cuda.synchronize()
    # nothing ran: the buffers are still cleared
    assert (rz.to_u64(fb) == np.uint64(0xFFFFFFFFFF000000)).all() and (rz.to_u64(acc) == 0).all()


def test_unaligned_planes_take_the_scalar_path(rz, oracle):
    import torch
    cloud = gen.terrain(50_001, 4, extent=50.0, amplitude=5.0, wavelength=20.0)
    view = gen.terrain_view(80, 60, extent=50.0, distance=60.0, near=0.5, far=400.0)
    ok_keys, ok_img = oracle.render_atomicmin(cloud.x[1:], cloud.y[1:], cloud.z[1:], cloud.rgb[1:],
                                              view.vp, view.near, view.far, view.width, view.height)
    full = rz.Points.from_cloud(cloud)
    pts = rz.Points(full.x[1:], full.y[1:], full.z[1:], full.rgb[1:])
    assert pts.x.data_ptr() % 16 != 0
    keys, img, _ = gpu_min(rz, pts, view)
    assert np.array_equal(keys, ok_keys) and np.array_equal(img, ok_img)


def test_degenerate_points(rz, oracle):
    """NaN, infinities, points behind the camera and outside [near, far),
    points exactly on the window edges."""
    rng = np.random.default_rng(0)
    n = 5000
    W, H = 32, 16
    vp = np.eye(4)
    vp[2, :] = 0
    vp[3, :] = [0, 0, 0.25, 1.0]
    x = rng.choice(np.array([-1, -0.5, 0, 0.5, 1, np.nan, np.inf, -np.inf, 0.9999999], np.float32), n)
    y = rng.choice(np.array([-1, -0.25, 0, 0.75, 1, np.nan, 0.5], np.float32), n)
    z = rng.uniform(-12, 12, n).astype(np.float32)
    z[::17] = np.nan
    rgb = rng.integers(0, 2 ** 32, n, dtype=np.uint32)   # high byte must be ignored
    cloud = gen.Cloud(x, y, z, rgb)
    view = gen.View(vp, 0.5, 3.0, W, H)
    check_scene(rz, oracle, cloud, view, label="degenerate")


def test_reciprocal_is_the_ieee_quotient(rz):
    """The projection's 1 / w, as compiled into the library, equals the
    IEEE quotient 1.0f / w for every positive float, denormals and +inf
    included (about a millisecond of GPU time).  The corrected estimate on
    its own is exact on [2^-126, 2^126), where the kernels use it alone,
    and not below it, so the check does count what differs."""
    import torch
    say("[parity] reciprocal over every positive float")
    normal = (0x00800000, 0x7E800000 - 0x00800000)   # [2^-126, 2^126)
    counts = {
        "all positive": rz.check_reciprocal(1, 0x7F800000),
        "negative patterns": rz.check_reciprocal(0x80000000, 1 << 31),
        "estimate, normal range": rz.check_reciprocal(*normal, estimate_only=True),
        "estimate, denormals": rz.check_reciprocal(1, 0x007FFFFF, estimate_only=True),
    }
    torch.cuda.synchronize()
    counts = {k: int(v.item()) for k, v in counts.items()}
    say(f"[parity] reciprocal mismatches: {counts}")
    assert counts["all positive"] == 0 and counts["estimate, normal range"] == 0
    assert counts["negative patterns"] == 0          # not counted by definition
    assert counts["estimate, denormals"] > 0


@pytest.mark.parametrize("lo,hi", [(124.5, 127.99), (-129.5, -124.5)])
def test_extreme_clip_w(rz, oracle, lo, hi):
    """Clip w from about 2^-129 (denormal) to just below 2^128, straddling
    2^-126 and 2^126, where the kernels switch from the Newton-corrected
    reciprocal to the IEEE division; every wave mixes both kinds of lanes.
    Both passes and the point-size kernel match the oracle bit for bit."""
    import torch
    rng = np.random.default_rng(11)
    n, W, H = 20000, 24, 16
    vp = np.zeros((4, 4))
    vp[0, 1] = vp[1, 2] = vp[3, 0] = 1.0          # clip = (y, z, 0, x)
    w = np.exp2(rng.uniform(lo, hi, n)).astype(np.float32)
    fmax = float(np.finfo(np.float32).max)
    y = np.clip(w * rng.uniform(-1.1, 1.1, n), -fmax, fmax).astype(np.float32)
    z = np.clip(w * rng.uniform(-1.1, 1.1, n), -fmax, fmax).astype(np.float32)
    rgb = rng.integers(0, 1 << 24, n, dtype=np.uint32)
    view = gen.View(vp, 2.0 ** (lo - 1), 2.0 ** (hi + 1), W, H)
    cloud = gen.Cloud(w, y, z, rgb)
    pix, _ = oracle.fragments(w, y, z, vp, view.near, view.far, W, H)
    big, tiny = w >= np.float32(2.0 ** 126), w < np.float32(2.0 ** -126)
    edge = big if lo > 0 else tiny
    say(f"[parity] extreme w {lo}..{hi}: {int((pix[edge] >= 0).sum())} visible in the division range")
    assert (pix[edge] >= 0).sum() > 1000 and (pix[~edge] >= 0).sum() > 1000
    keys, _ = check_scene(rz, oracle, cloud, view, label=f"extreme w {lo}..{hi}")
    assert (keys != np.uint64(oracle.clear_value(0))).sum() > W * H // 2
    pts = rz.Points.from_cloud(cloud)
    fb, _ = rz.new_framebuffer(view, 0)
    rz.rasterize_points(pts, view, None, False, (1, 100), 2, 0, fb=fb, keep_keys=True)
    got = rz.to_u64(fb)
    torch.cuda.synchronize()
    want, _ = oracle.render_atomicmin(w, y, z, rgb, vp, view.near, view.far, W, H, point_size=2)
    assert np.array_equal(got, want)


def test_largest_screen(rz, oracle):
    """The largest screen the interface accepts, 32768 x 32768 (8 GiB of
    keys): a 300k-point cloud spread over it.  Every touched pixel holds the
    minimum key of its fragments (from the oracle's per-point fragments) and
    shows its colour after the resolve; no other pixel is written, and the
    resolve leaves the whole framebuffer cleared."""
    import torch
    rng = np.random.default_rng(31)
    n, side, bg = 300_000, 32768, 0x0A0B0C
    view = gen.make_view((0.0, 0.0, 5.0), (0.0, 0.0, 0.0), (0, 1, 0), 60.0, side, side, 0.1, 100.0)
    x = rng.uniform(-3.2, 3.2, n).astype(np.float32)
    y = rng.uniform(-3.2, 3.2, n).astype(np.float32)
    z = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    z[: n // 3] = z[n // 3: 2 * (n // 3)]               # repeated depths for the colour tie rule
    x[: n // 3] = x[n // 3: 2 * (n // 3)]
    y[: n // 3] = y[n // 3: 2 * (n // 3)]
    rgb = rng.integers(0, 1 << 24, n, dtype=np.uint32)
    pix, q = oracle.fragments(x, y, z, view.vp, view.near, view.far, side, side)
    keep = pix >= 0
    assert keep.mean() > 0.5 and (pix[keep] >= side * side // 2).any()
    keys = (q[keep] << np.uint64(24)) | (rgb[keep].astype(np.uint64) & np.uint64(0xFFFFFF))
    order = np.lexsort((keys, pix[keep]))
    p_sorted, k_sorted = pix[keep][order], keys[order]
    first = np.r_[True, p_sorted[1:] != p_sorted[:-1]]
    want_pix, want_key = p_sorted[first], k_sorted[first]
    say(f"[parity] {side}x{side}: {len(want_pix)} touched pixels")
    pts = rz.Points.from_cloud(gen.Cloud(x, y, z, rgb))
    fb, _ = rz.new_framebuffer(view, bg)
    rz.rasterize_atomicmin(pts, view, background=bg, fb=fb, keep_keys=True)
    idx = torch.from_numpy(want_pix).cuda()
    got = fb[idx].cpu().numpy().view(np.uint64)
    clear = int(np.uint64(oracle.clear_value(bg)).view(np.int64))
    written = int((fb != clear).sum().item())
    img = rz.resolve_min(fb, side * side, bg)
    colours = img[idx].cpu().numpy().view(np.uint32)
    still = int((fb != clear).sum().item())
    torch.cuda.synchronize()
    assert np.array_equal(got, want_key)
    assert written == len(want_pix)
    assert np.array_equal(colours, (want_key & np.uint64(0xFFFFFF)).astype(np.uint32))
    assert still == 0
    del fb, img
    torch.cuda.empty_cache()


def test_large_screen_splatting(rz, oracle):
    """8192 x 8192 (64M pixels), both methods against the oracle at every
    pixel, with a dense cluster so that pixels average several fragments."""
    rng = np.random.default_rng(32)
    n, side = 1_000_000, 8192
    view = gen.make_view((0.0, 0.0, 5.0), (0.0, 0.0, 0.0), (0, 1, 0), 60.0, side, side, 0.1, 100.0)
    x = rng.uniform(-3.2, 3.2, n).astype(np.float32)
    y = rng.uniform(-3.2, 3.2, n).astype(np.float32)
    z = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    x[: n // 2] = rng.normal(0, 0.01, n // 2).astype(np.float32)
    y[: n // 2] = rng.normal(0, 0.01, n // 2).astype(np.float32)
    rgb = rng.integers(0, 1 << 24, n, dtype=np.uint32)
    _, sums = check_scene(rz, oracle, gen.Cloud(x, y, z, rgb), view, bg=0x203040,
                          label="8192x8192")
    assert (sums[:, 3] > 1).sum() > 1000


def test_config2_terrain_full_size(rz, oracle):
    """The 50M-point Morton terrain at 1920x1080, every pixel, both modes."""
    cloud, view = gen.config2()
    keys, sums = check_scene(rz, oracle, cloud, view, label="50M terrain 1920x1080")
    # the workload is non-trivial: most of the screen is covered, many
    # fragments per pixel fall in the 1% window
    assert (keys != np.uint64(oracle.clear_value(0))).mean() > 0.3
    assert sums[:, 3].max() > 10


def test_config2_shuffled_sample(rz, oracle):
    cloud, view = gen.config2(n=8_000_000)
    check_scene(rz, oracle, gen.shuffle(cloud, 1), view, label="8M terrain shuffled")


def test_repeated_calls_reuse_cleared_buffers(rz, oracle):
    import torch
    cloud, view = gen.config1(n=200_000)
    pts = rz.Points.from_cloud(cloud)
    fb, acc = rz.new_framebuffer(view, 7, hq=True)
    outs = []
    for _ in range(3):
        _, img = rz.rasterize_atomicmin(pts, view, background=7, fb=fb)
        _, _, himg, _ = rz.rasterize_hq_splat(pts, view, background=7, fb=fb, acc=acc)
        torch.cuda.synchronize()
        outs.append((rz.to_u32(img), rz.to_u32(himg)))
    for a, b in outs[1:]:
        assert np.array_equal(a, outs[0][0]) and np.array_equal(b, outs[0][1])


def test_hq_count_limit(rz, oracle):
    """Largest exact splat count: 16843009 white fragments in one pixel sum to
    2^32 - 1 per channel; one more sets the overflow status."""
    import torch
    view = gen.View(np.diag([1.0, 1.0, 0.0, 0.0]) + np.array(
        [[0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, -1.0, 0]]), 1.0, 100.0, 2, 2)
    for n, over in ((16_843_009, False), (16_843_010, True)):
        say(f"[count] n={n}")
        pts = rz.Points(torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"),
                        torch.full((n,), -10.0, device="cuda"),
                        torch.full((n,), 0xFFFFFF, dtype=torch.int32, device="cuda"))
        fb, acc, img, status = rz.rasterize_hq_splat(pts, view)
        torch.cuda.synchronize()
        st = int(status.item())
        if over:
            assert st & rz.RZ_STATUS_HQ_OVERFLOW
        else:
            assert st == 0
            assert rz.to_u32(img)[3] == 0xFFFFFF
        del pts


@pytest.mark.parametrize("shape", [(64, 8, 3), (64, 8, 2), (128, 4, 3), (64, 16, 2)])
@pytest.mark.parametrize("rgb", [0xFFFFFF, 0xFF00FF, 0x00FF00])
def test_splat_sums_at_the_tile_word_limit(rz, shape, rgb):
    """Every point in one pixel with the same colour: with at most 8 points
    per thread each wave adds 512 fragments into one packed tile word
    (R | G << 17 | B << 34 | count << 51), the most a field can hold without
    carrying; 16 points per thread take the two-word tile.  The accumulator
    must hold exactly n times each channel and the count n (a carry would
    show in the next field: G for a magenta cloud, R and B for a green one)."""
    import torch
    view = gen.View(np.diag([1.0, 1.0, 0.0, 0.0]) + np.array(
        [[0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, -1.0, 0]]), 1.0, 100.0, 2, 2)
    n = 5 * 64 * 16 * 8 + 77   # several workgroups of every shape and a ragged tail
    block, ppt, binm = shape
    say(f"[tile word] shape={shape} rgb={rgb:06x} n={n}")
    pts = rz.Points(torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"),
                    torch.full((n,), -10.0, device="cuda"),
                    torch.full((n,), rgb, dtype=torch.int32, device="cuda"))
    rz.set_launch(block, ppt, 1, 0, binm)
    try:
        fb, acc, _, _ = rz.rasterize_hq_splat(pts, view, keep_keys=True)
        torch.cuda.synchronize()
    finally:
        rz.reset_launch()
    sums = rz.unpack_acc(acc)
    hit = np.flatnonzero(sums[:, 3])
    assert hit.size == 1
    want = [n * (rgb & 0xFF), n * ((rgb >> 8) & 0xFF), n * ((rgb >> 16) & 0xFF), n]
    assert sums[hit[0]].tolist() == want


def _sparse_sums_equal(rz, acc, want_sums):
    """The packed device sums against the oracle's exact sums, read back only
    at the pixels the oracle accepted fragments in; every other pixel of acc
    must hold zero (its count word is zero exactly when nothing was added)."""
    import torch
    nz = np.flatnonzero(want_sums[:, 3])
    pairs = acc.view(-1, 2)
    got = rz.unpack_acc(pairs[torch.from_numpy(nz).to("cuda")].reshape(-1))
    others = int((pairs[:, 1] != 0).sum().item()) - nz.size
    return np.array_equal(got, want_sums[nz]) and others == 0


@pytest.mark.parametrize("offset", [0.0, 3.0e5])
def test_rounding_edge_sets(rz, oracle, offset):
    """The point sets on which the fused and the unfused projection readings
    disagree (500 points within 10^-4 pixel of a pixel corner of a
    15000 x 12000 screen; the same scene 3·10^5 units from the origin, where
    the depth row's terms cancel): keys and splat sums of the depth pass,
    the splat pass and the point-size kernels equal the oracle's, whose
    rounding is pinned step by step against the IEEE definition."""
    import torch
    from tests.edge_scenes import rounding_edge_scene
    v, x, y, z, rgb = rounding_edge_scene(offset)
    W, H = v.width, v.height
    pts = rz.Points.from_numpy(x, y, z, rgb)
    args = (x, y, z, rgb, v.vp, v.near, v.far, W, H)
    pix, _ = oracle.fragments(x, y, z, v.vp, v.near, v.far, W, H)
    assert (pix >= 0).sum() > 300
    say(f"[edge] offset {offset}: atomicMin")
    want_k, _ = oracle.render_atomicmin(*args)
    fb, _ = rz.new_framebuffer(v, 0)
    rz.rasterize_atomicmin(pts, v, fb=fb, keep_keys=True)
    torch.cuda.synchronize()
    assert np.array_equal(rz.to_u64(fb), want_k), "depth pass keys"
    say(f"[edge] offset {offset}: splatting")
    hk, hs, _ = oracle.render_hq(*args)
    assert np.array_equal(hk, want_k)
    fb, acc = rz.new_framebuffer(v, 0, hq=True)
    rz.rasterize_hq_splat(pts, v, fb=fb, acc=acc, keep_keys=True)
    torch.cuda.synchronize()
    assert np.array_equal(rz.to_u64(fb), hk), "splat depth pass keys"
    assert _sparse_sums_equal(rz, acc, hs), "splat sums"
    del hs
    for k in (1, 2):
        say(f"[edge] offset {offset}: point size {k}")
        pk, _ = oracle.render_atomicmin(*args, point_size=k)
        fb, acc = rz.new_framebuffer(v, 0, hq=True)
        rz.rasterize_points(pts, v, point_size=k, fb=fb, keep_keys=True)
        torch.cuda.synchronize()
        assert np.array_equal(rz.to_u64(fb), pk), f"point size {k} keys"
        _, phs, _ = oracle.render_hq(*args, point_size=k)
        rz.clear(fb, None, W * H)
        rz.rasterize_points(pts, v, hq=True, point_size=k, fb=fb, acc=acc, keep_keys=True)
        torch.cuda.synchronize()
        assert _sparse_sums_equal(rz, acc, phs), f"point size {k} sums"
        del fb, acc, phs
        torch.cuda.empty_cache()


def test_reciprocal_matches_host_quotient(rz):
    """The kernels' 1 / w copied back and compared with the host's own IEEE
    single-precision quotient (numpy on the CPU, which does not flush
    denormals): 4096 random significands in every binade from the
    denormals to 2^127, plus the patterns at the ends of the estimate's
    range (2^-126, 2^126) and at the extremes.  Unlike the device self-check
    above, this does not rely on the device's own division."""
    import torch
    say("[parity] reciprocal against the host quotient")
    rng = np.random.default_rng(21)
    exps = np.arange(0, 255, dtype=np.uint32)
    bits = (exps[:, None] << np.uint32(23)) | rng.integers(0, 1 << 23, size=(255, 4096),
                                                           dtype=np.uint32)
    edges = np.array([1, 2, 0x007FFFFF, 0x00800000, 0x00800001, 0x3F7FFFFF, 0x3F800000,
                      0x3F800001, 0x7E7FFFFF, 0x7E800000, 0x7E800001, 0x7F7FFFFF, 0x7F800000],
                     np.uint32)
    bits = np.concatenate([bits.ravel(), edges])
    bits = bits[bits != 0]
    w = bits.view(np.float32)
    with np.errstate(divide="ignore", over="ignore", under="ignore"):
        want = (np.float32(1.0) / w).view(np.uint32)
    got = rz.reciprocal(torch.from_numpy(w.copy()).to("cuda"))
    torch.cuda.synchronize()
    got = rz.to_u32(got)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, [(hex(int(bits[i])), hex(int(got[i])), hex(int(want[i])))
                           for i in bad[:8]]


@pytest.mark.parametrize("seed,kind,scale,eps,offset", [
    (1, 0, 0.0, (1, 100), 0.0), (3, 1, 1000.0, (1, 100), 0.0), (2, 0, 0.0, (3, 100), 0.0),
    (4, 0, 0.0, (1, 100), 3.0e4)])
def test_window_edge_probes(rz, oracle, seed, kind, scale, eps, offset):
    """Points placed within a few float steps of pixels' splat window edges
    (section 2.2) and of the near and far planes, where the accumulate
    pass's double-precision pre-test meets its integer test on ties: splat
    sums and images equal the oracle's, with the points in pixel order
    (each wave's points in a small rectangle: the per-wave LDS tile) and in
    random order (rectangles too large for the tile: global atomics)."""
    from tests.edge_scenes import window_edge_scene
    sc = window_edge_scene(oracle, seed, kind, scale, eps, offset)
    v = sc["view"]
    pts = np.concatenate([sc["base"], sc["probes"]])
    rgb = np.concatenate([sc["rgb"], np.full(len(sc["probes"]), 0x010203, np.uint32)])
    pix, _ = oracle.fragments(pts[:, 0], pts[:, 1], pts[:, 2], v.vp, v.near, v.far, v.width,
                              v.height, kind, scale)
    order = np.argsort(np.where(pix < 0, 1 << 40, pix), kind="stable")
    for label, idx in (("pixel order", order),
                       ("random order", np.random.default_rng(seed).permutation(len(pts)))):
        cloud = gen.Cloud(pts[idx, 0].copy(), pts[idx, 1].copy(), pts[idx, 2].copy(), rgb[idx])
        check_scene(rz, oracle, cloud, v, depth=(kind, scale), eps=eps,
                    label=f"window edges, {label}")
