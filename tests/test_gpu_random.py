"""Seeded random scenes against the oracle, bit for bit: cloud shape (blobs,
box, plane, spherical shell, stacks of duplicate positions), size (empty to
250k, ragged), point order, camera, resolution (1x1 to 801x599), depth map
(linear, scale, piecewise; the float encodings for points of any size), eps,
background, launch shape and path (direct, screen-sorted), point size (1 to
16 pixels), and batches of up to 20 views with mixed methods, depth maps and
group sizes.  Keys, exact splat sums and images are compared; each case names
its seed and parameters first."""
import sys

import numpy as np
import pytest

from paper_1908_02681_amd import gen

pytestmark = pytest.mark.gpu

CASES = 200
Q40 = float((1 << 40) - 2)


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


SIZES = [0, 1, 63, 64, 65, 1000, 4097, 30_000, 120_000, 250_000]


def random_cloud(rng, sizes=SIZES):
    n = int(rng.choice(sizes))
    kind = str(rng.choice(["blobs", "box", "plane", "shell", "dups"]))
    if kind == "blobs":
        centres = rng.uniform(-1, 1, (int(rng.integers(1, 9)), 3))
        pick = rng.integers(0, len(centres), n)
        p = centres[pick] + rng.normal(0, float(rng.uniform(0.01, 0.3)), (n, 3))
    elif kind == "box":
        p = rng.uniform(-1, 1, (n, 3))
    elif kind == "plane":
        u, v = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        a, b = rng.normal(size=3), rng.normal(size=3)
        p = u[:, None] * a + v[:, None] * b
    elif kind == "shell":
        d = rng.normal(size=(n, 3))
        p = d / np.maximum(np.linalg.norm(d, axis=1, keepdims=True), 1e-9) * rng.uniform(0.3, 1)
    else:   # many points on few positions, colours differing: ties on the key's depth
        base = rng.uniform(-1, 1, (max(1, n // 50), 3))
        p = base[rng.integers(0, len(base), n)]
    p = p.astype(np.float32)
    rgb = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)   # bits 24-31 ignored
    order = str(rng.choice(["as made", "shuffled", "sorted by x"]))
    if order == "shuffled":
        perm = rng.permutation(n)
        p, rgb = p[perm], rgb[perm]
    elif order == "sorted by x":
        perm = np.argsort(p[:, 0], kind="stable")
        p, rgb = p[perm], rgb[perm]
    cloud = gen.Cloud(np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
                      np.ascontiguousarray(p[:, 2]), rgb)
    return cloud, f"{kind} n={n} {order}"


def random_view(rng):
    w = int(rng.choice([1, 2, 7, 64, 333, 640, 801]))
    h = int(rng.choice([1, 3, 48, 240, 480, 599]))
    d = rng.normal(size=3)
    eye = d / np.linalg.norm(d) * rng.uniform(1.5, 6.0)
    target = rng.uniform(-0.3, 0.3, 3)
    up = (0.0, 1.0, 0.0) if abs(d[1] / np.linalg.norm(d)) < 0.95 else (1.0, 0.0, 0.0)
    dist = float(np.linalg.norm(eye - target))
    if rng.random() < 0.75:   # the cloud (within about 1.7 of the origin) between near and far
        near = float(rng.uniform(0.01, max(0.02, dist - 1.8)))
        far = float((dist + 1.8) * 10 ** rng.uniform(0, 2))
    else:                     # near and far anywhere: clipping by depth
        near = float(10 ** rng.uniform(-2, 0))
        far = float(near * 10 ** rng.uniform(1, 3))
    fovy = float(rng.uniform(20, 100))
    return gen.make_view(eye, target, up, fovy, w, h, near, far), f"{w}x{h} near={near:.3g} far={far:.3g}"


def random_depth(rng, view, kind=None):
    kind = int(rng.integers(0, 3)) if kind is None else kind
    if kind in (0, 3, 4):   # linear, or the float encodings (no map parameters)
        return (kind, 0.0)
    if kind == 1:
        return (1, float(rng.uniform(0.05, 1.0) * Q40 / view.far))
    # piecewise: up to three ranges from 0, breakpoints inside (near, far),
    # each range spanning at most 2^38 quanta
    nr = int(rng.integers(1, 4))
    cuts = np.sort(rng.uniform(view.near, view.far, nr - 1))
    starts = [0.0] + [float(c) for c in cuts]
    ends = starts[1:] + [view.far]
    ranges = tuple((s, float(rng.uniform(0.1, 1.0) * 2.0 ** 38 / max(e - s, 1e-6)))
                   for s, e in zip(starts, ends))
    return (2, ranges)


def gpu_frames(rz, pts, view, depth, eps, bg, path, ws):
    """Keys, exact sums and both images of one call each (raw buffers kept,
    then resolved)."""
    import torch
    npix = view.width * view.height
    fb, acc = rz.new_framebuffer(view, bg, hq=True)
    if path == "sorted":
        rz.rasterize_sorted(pts, view, depth, False, eps, bg, fb=fb, acc=acc, workspace=ws,
                            keep_keys=True)
    else:
        rz.rasterize_atomicmin(pts, view, depth, bg, fb=fb, keep_keys=True)
    keys = rz.to_u64(fb)
    img = rz.to_u32(rz.resolve_min(fb, npix, bg))
    if path == "sorted":
        rz.rasterize_sorted(pts, view, depth, True, eps, bg, fb=fb, acc=acc, workspace=ws,
                            keep_keys=True)
    else:
        rz.rasterize_hq_splat(pts, view, depth, eps, bg, fb=fb, acc=acc, keep_keys=True)
    hkeys = rz.to_u64(fb)
    sums = rz.unpack_acc(acc)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    himg = rz.to_u32(rz.resolve_hq(fb, acc, npix, bg, status=status))
    torch.cuda.synchronize()
    cleared = rz.to_u64(fb)
    return keys, img, hkeys, sums, himg, int(status.item()), cleared, rz.to_u64(acc)


@pytest.mark.parametrize("seed", range(CASES))
def test_random_scene(rz, oracle, seed):
    rng = np.random.default_rng([1908, seed])
    cloud, what = random_cloud(rng)
    view, cam = random_view(rng)
    depth = random_depth(rng, view)
    den = int(rng.choice([1, 7, 100, 1000, 1 << 20]))
    eps = (int(rng.choice([0, 1, 3, den])), den)
    bg = int(rng.integers(0, 1 << 32))
    shape = (int(rng.choice([64, 256, 512])), int(rng.choice([4, 8, 16])),
             int(rng.integers(0, 2)), int(rng.integers(0, 2)), int(rng.integers(0, 4)))
    buckets = ((view.width + 63) // 64) * ((view.height + 63) // 64)
    path = str(rng.choice(["direct", "sorted"])) if buckets <= 4096 else "direct"
    say(f"[random] seed={seed} {what} {cam} depth={depth[0]} eps={eps} bg={bg:#x} "
        f"launch={shape} path={path}")
    want_keys, want_img = oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp,
                                                  view.near, view.far, view.width, view.height,
                                                  depth[0], depth[1], bg)
    hk, want_sums, want_himg = oracle.render_hq(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp,
                                                view.near, view.far, view.width, view.height,
                                                depth[0], depth[1], eps, bg)
    assert np.array_equal(hk, want_keys)
    pts = rz.Points.from_cloud(cloud)
    ws = rz.new_workspace(cloud.n, view.width, view.height) if path == "sorted" else None
    rz.set_launch(*shape)
    try:
        keys, img, hkeys, sums, himg, status, cleared, acc = gpu_frames(rz, pts, view, depth,
                                                                        eps, bg, path, ws)
    finally:
        rz.reset_launch()
    assert np.array_equal(keys, want_keys), f"keys differ at {np.flatnonzero(keys != want_keys)[:8]}"
    assert np.array_equal(img, want_img)
    assert np.array_equal(hkeys, want_keys)
    assert np.array_equal(sums, want_sums), f"sums differ at {np.flatnonzero((sums != want_sums).any(1))[:8]}"
    assert np.array_equal(himg, want_himg)
    assert status == 0
    assert (cleared == np.uint64(oracle.clear_value(bg))).all() and (acc == 0).all()


POINT_CASES = 80


@pytest.mark.parametrize("seed", range(POINT_CASES))
def test_random_points(rz, oracle, seed):
    """rasterize_points: squares of k x k pixels, every depth encoding."""
    import torch
    rng = np.random.default_rng([1909, seed])
    cloud, what = random_cloud(rng, [0, 1, 65, 1000, 4097, 30_000, 60_000])
    view, cam = random_view(rng)
    k = int(rng.choice([1, 2, 3, 4, 5, 7, 11, 16]))
    enc = int(rng.integers(0, 5))   # linear, scale, piecewise, 24-bit window, reversed float
    depth = random_depth(rng, view, enc)
    hq = enc < 3 and bool(rng.random() < 0.7)
    den = int(rng.choice([1, 7, 100, 1000]))
    eps = (int(rng.choice([0, 1, 3, den])), den)
    bg = int(rng.integers(0, 1 << 32))
    say(f"[random points] seed={seed} {what} {cam} k={k} depth={depth[0]} hq={hq} eps={eps}")
    args = (cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near, view.far, view.width,
            view.height, depth[0], depth[1])
    pts = rz.Points.from_cloud(cloud)
    want_keys, want_img = oracle.render_atomicmin(*args, bg=bg, point_size=k)
    fb, acc = rz.new_framebuffer(view, bg, hq=False)
    rz.rasterize_points(pts, view, depth, False, eps, k, bg, fb=fb, keep_keys=True)
    keys = rz.to_u64(fb)
    _, _, img, _ = rz.rasterize_points(pts, view, depth, False, eps, k, bg)
    torch.cuda.synchronize()
    assert np.array_equal(keys, want_keys), f"keys differ at {np.flatnonzero(keys != want_keys)[:8]}"
    assert np.array_equal(rz.to_u32(img), want_img)
    if hq:
        hk, want_sums, want_himg = oracle.render_hq(*args, eps=eps, bg=bg, point_size=k)
        fb, acc = rz.new_framebuffer(view, bg, hq=True)
        rz.rasterize_points(pts, view, depth, True, eps, k, bg, fb=fb, acc=acc, keep_keys=True)
        hkeys, sums = rz.to_u64(fb), rz.unpack_acc(acc)
        _, _, himg, st = rz.rasterize_points(pts, view, depth, True, eps, k, bg)
        torch.cuda.synchronize()
        assert np.array_equal(hkeys, hk)
        assert np.array_equal(sums, want_sums)
        assert np.array_equal(rz.to_u32(himg), want_himg) and int(st.item()) == 0


BATCH_CASES = 30


@pytest.mark.parametrize("seed", range(BATCH_CASES))
def test_random_batch(rz, oracle, seed):
    """rz_batch_*: up to 20 random views of one cloud, mixed methods, depth
    maps and backgrounds, random group size, launch shape and graph use; two
    runs, each image against the oracle's."""
    import torch
    rng = np.random.default_rng([1910, seed])
    cloud, what = random_cloud(rng, [1, 65, 4097, 30_000, 120_000])
    nv = int(rng.integers(1, 21))
    views, modes, depths, bgs = [], [], [], []
    for _ in range(nv):
        v, _ = random_view(rng)
        views.append(v)
        modes.append(int(rng.integers(0, 2)))
        depths.append(random_depth(rng, v))
        bgs.append(int(rng.integers(0, 1 << 32)))
    den = int(rng.choice([1, 7, 100, 1000]))
    eps = (int(rng.choice([0, 1, 3, den])), den)
    k = int(rng.integers(0, 9))   # 0: the library's choice
    shape = (int(rng.choice([64, 128, 256, 512])), int(rng.choice([4, 8, 16])),
             int(rng.integers(0, 2)), int(rng.integers(0, 2)), int(rng.integers(0, 4)))
    graph = bool(rng.random() < 0.5)
    say(f"[random batch] seed={seed} {what} views={nv} modes={modes} eps={eps} k={k} "
        f"launch={shape} graph={graph}")
    pts = rz.Points.from_cloud(cloud)
    b = rz.Batch(pts, views, modes, depth=depths, eps=eps, backgrounds=bgs, views_per_group=k,
                 launch=shape, use_graph=graph)
    want = []
    for v, m, d, bg in zip(views, modes, depths, bgs):
        args = (cloud.x, cloud.y, cloud.z, cloud.rgb, v.vp, v.near, v.far, v.width, v.height,
                d[0], d[1])
        want.append(oracle.render_hq(*args, eps=eps, bg=bg)[2] if m == 1
                    else oracle.render_atomicmin(*args, bg=bg)[1])
    for run in range(2):
        b.run()
        torch.cuda.synchronize()
        for i, (img, w) in enumerate(zip(b.imgs, want)):
            assert np.array_equal(rz.to_u32(img), w), f"run {run} view {i} differs"


SERVE_CASES = 40


@pytest.mark.parametrize("seed", range(SERVE_CASES))
def test_random_serving(rz, oracle, seed):
    """rz_server_*: random clouds and requests (views, methods, integer depth
    maps, eps, backgrounds) under random budgets, streams, work caps,
    exclusive sizes and request merging; every image against the oracle."""
    import torch
    rng = np.random.default_rng([1911, seed])
    clouds = [random_cloud(rng, [1, 65, 4097, 30_000, 120_000])[0]
              for _ in range(int(rng.integers(1, 5)))]
    nreq = int(rng.integers(5, 61))
    reqs = []
    for _ in range(nreq):
        c = int(rng.integers(0, len(clouds)))
        v, _ = random_view(rng)
        reqs.append((c, v, int(rng.integers(0, 2)), random_depth(rng, v),
                     int(rng.integers(0, 1 << 32))))
    den = int(rng.choice([1, 7, 100, 1000]))
    eps = (int(rng.choice([0, 1, 3, den])), den)
    biggest = 2 * max(cl.n for cl in clouds)
    opts = dict(budget_bytes=int(rng.choice([16, 64, 512])) << 20,
                streams=int(rng.choice([1, 2, 4, 8])),
                work_cap=int(rng.choice([0, biggest, max(1, biggest // 3)])),
                merge_views=int(rng.choice([0, 0, 2, 8])),
                exclusive_work=int(rng.choice([0, 0, max(1, biggest // 2)])))
    say(f"[random serve] seed={seed} clouds={[cl.n for cl in clouds]} requests={nreq} "
        f"eps={eps} {opts}")
    pts = [rz.Points.from_cloud(cl) for cl in clouds]
    s = rz.Server(**opts)
    try:
        ids = [s.add_cloud(p) for p in pts]
        imgs, tickets = [], []
        for c, v, m, d, bg in reqs:
            img = torch.full((v.width * v.height,), -1, dtype=torch.int32, device="cuda")
            imgs.append(img)
            tickets.append(s.submit(ids[c], v, m, img=img, depth=d, eps=eps, background=bg))
        s.drain(120)
        st = [s.poll(t) for t in tickets]
        stats = s.stats()
    finally:
        s.close()
    assert stats["completed"] == nreq and stats["failed"] == 0
    assert stats["peak_bytes"] <= opts["budget_bytes"]
    for i, ((c, v, m, d, bg), img, x) in enumerate(zip(reqs, imgs, st)):
        assert x["state"] == rz.RZ_REQ_DONE and x["error"] == 0, f"request {i}: {x}"
        cl = clouds[c]
        args = (cl.x, cl.y, cl.z, cl.rgb, v.vp, v.near, v.far, v.width, v.height, d[0], d[1])
        want = (oracle.render_hq(*args, eps, bg)[2] if m == 1
                else oracle.render_atomicmin(*args, bg)[1])
        assert np.array_equal(rz.to_u32(img), want), f"request {i} differs"
