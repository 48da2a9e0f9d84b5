"""Batched multi-view rendering: every view of a batch is bit-identical to the
oracle and to its one-view call, with and without a captured graph, for any
group size and launch shape, before and after autotuning."""
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
    yield binding
    binding.reset_launch()


SIZES = [(64, 48), (160, 120), (97, 61), (200, 150), (33, 257)]


@pytest.fixture(scope="module")
def scene():
    cloud = gen.terrain(600_000, 21, extent=100.0, amplitude=10.0, wavelength=40.0)
    views = gen.orbit_views(11, 5, SIZES, extent=100.0, rmin=60.0, rmax=120.0, near=0.5, far=400.0)
    rng = np.random.default_rng(3)
    modes = rng.integers(0, 2, len(views)).tolist()
    modes[0], modes[1] = 0, 1
    bgs = rng.integers(0, 1 << 24, len(views)).tolist()
    return cloud, views, modes, bgs


@pytest.fixture(scope="module")
def expected(scene, oracle):
    cloud, views, modes, bgs = scene
    out = []
    for v, m, bg in zip(views, modes, bgs):
        if m == 0:
            _, img = oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, v.vp, v.near,
                                             v.far, v.width, v.height, bg=bg)
        else:
            _, _, img = oracle.render_hq(cloud.x, cloud.y, cloud.z, cloud.rgb, v.vp, v.near,
                                         v.far, v.width, v.height, bg=bg)
        out.append(img)
    return out


def check_images(rz, batch, expected, label):
    import torch
    torch.cuda.synchronize()
    for i, (got, want) in enumerate(zip(batch.images(), expected)):
        assert np.array_equal(got, want), f"{label}: view {i} differs"
    for fb, acc, bg in zip(batch.fbs, batch.accs, batch.backgrounds):
        assert (rz.to_u64(fb) == np.uint64(0xFFFFFFFFFF000000 | (bg & 0xFFFFFF))).all()
        if acc is not None:
            assert (rz.to_u64(acc) == 0).all()


def test_batch_matches_oracle(rz, scene, expected):
    cloud, views, modes, bgs = scene
    pts = rz.Points.from_cloud(cloud)
    b = rz.Batch(pts, views, modes, backgrounds=bgs)
    b.run()
    check_images(rz, b, expected, "plain batch")
    b.run()   # the buffers are cleared again: a second run gives the same bits
    check_images(rz, b, expected, "second run")
    b.close()


def test_one_view_calls_match(rz, scene, expected):
    import torch
    cloud, views, modes, bgs = scene
    pts = rz.Points.from_cloud(cloud)
    for v, m, bg, want in zip(views, modes, bgs, expected):
        if m == 0:
            _, img = rz.rasterize_atomicmin(pts, v, background=bg)
        else:
            _, _, img, _ = rz.rasterize_hq_splat(pts, v, background=bg)
        torch.cuda.synchronize()
        assert np.array_equal(rz.to_u32(img), want)


@pytest.mark.parametrize("k", [1, 3, 8])
@pytest.mark.parametrize("launch", [(256, 4, 1, 1, 1), (512, 8, 1, 0, 1), (128, 16, 1, 1, 0),
                                    (256, 8, 1, 1, 2), (512, 16, 1, 0, 2), (256, 4, 1, 0, 3),
                                    (64, 16, 1, 1, 3)])
def test_group_sizes_and_shapes(rz, scene, expected, k, launch):
    cloud, views, modes, bgs = scene
    say(f"[batch] K={k} launch={launch}")
    pts = rz.Points.from_cloud(cloud)
    b = rz.Batch(pts, views, modes, backgrounds=bgs, views_per_group=k, launch=launch)
    b.run()
    check_images(rz, b, expected, f"K={k} {launch}")
    b.close()


def test_graph_replays_match_eager(rz, scene, expected):
    """The captured graph holds kernels only (no memset nodes); every replay,
    with unrelated eager GPU work and synchronisations in between, gives the
    eager result."""
    import torch
    cloud, views, modes, bgs = scene
    pts = rz.Points.from_cloud(cloud)
    b = rz.Batch(pts, views, modes, backgrounds=bgs, use_graph=True)
    scratch = torch.zeros(1 << 20, device="cuda")
    for r in range(4):
        say(f"[graph] replay {r}")
        b.run()
        check_images(rz, b, expected, f"replay {r}")
        scratch.add_(1.0)
        torch.cuda.synchronize()
        assert float(scratch[0].item()) == r + 1
    b.close()


def test_autotune_keeps_bits(rz, scene, expected):
    cloud, views, modes, bgs = scene
    pts = rz.Points.from_cloud(cloud)
    b = rz.Batch(pts, views, modes, backgrounds=bgs, use_graph=True)
    opts, ms = b.autotune(reps=2)
    say(f"[autotune] chosen {opts} {ms:.3f} ms")
    assert 1 <= opts["views_per_group"] <= 8 and opts["use_graph"] == 1 and ms > 0
    assert b.opts() == opts
    b.run()
    check_images(rz, b, expected, "after autotune")
    b.close()


def test_autotune_cache_round_trip(rz, scene, expected, tmp_path):
    """The first cached autotune searches and stores its choice under the
    batch's key; a second batch of the same class finds it, checks it against
    the default options' checksum and uses it; both render the oracle's bits."""
    cloud, views, modes, bgs = scene
    path = str(tmp_path / "tune.txt")
    pts = rz.Points.from_cloud(cloud)
    b = rz.Batch(pts, views, modes, backgrounds=bgs, use_graph=True)
    opts, ms, hit, key = b.autotune_cached(path, reps=1)
    say(f"[tune-cache] miss: {key} -> {opts} {ms:.3f} ms")
    assert not hit and ms > 0
    words = key.split(" ")
    assert len(words) == 6 and words[5] == "ordered" and words[3] == f"v{len(views)}"
    assert words[1] == f"n{round(np.log2(cloud.n))}"
    ent = rz.tune_cache_lookup(path, key)
    assert ent is not None and ent["views_per_group"] == opts["views_per_group"]
    assert ent["depth"] == {f: opts[f] for f in ("block", "ppt", "early_out", "xcd_remap", "bin")}
    b.run()
    check_images(rz, b, expected, "after the cached search")
    b.close()
    b2 = rz.Batch(pts, views, modes, backgrounds=bgs, use_graph=True)
    opts2, ms2, hit2, key2 = b2.autotune_cached(path, reps=1)
    say(f"[tune-cache] hit={hit2}: {opts2} {ms2:.3f} ms")
    assert hit2 and key2 == key and opts2 == opts and ms2 > 0
    b2.run()
    check_images(rz, b2, expected, "with the cached options")
    b2.close()
    # the same cloud shuffled: another order class, so another key (a miss)
    perm = np.random.default_rng(9).permutation(cloud.n)
    sh = rz.Points.from_numpy(cloud.x[perm], cloud.y[perm], cloud.z[perm], cloud.rgb[perm])
    b3 = rz.Batch(sh, views, modes, backgrounds=bgs)
    _, _, hit3, key3 = b3.autotune_cached(path, reps=1)
    assert not hit3 and key3.endswith(" shuffled") and key3.split(" ")[:5] == words[:5]
    b3.run()
    check_images(rz, b3, expected, "shuffled, after the cached search")
    b3.close()


def test_batch_status_flags_overflow(rz):
    """The fused resolve reports splat counts beyond the exact range like the
    one-view call does."""
    import torch
    n = 16_843_010
    view = gen.View(np.diag([1.0, 1.0, 0.0, 0.0]) + np.array(
        [[0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, -1.0, 0]]), 1.0, 100.0, 2, 2)
    pts = rz.Points(torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"),
                    torch.full((n,), -10.0, device="cuda"),
                    torch.full((n,), 0x00FF00, dtype=torch.int32, device="cuda"))
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    b = rz.Batch(pts, [view, view], [1, 0], status=status)
    b.run()
    torch.cuda.synchronize()
    assert int(status.item()) & rz.RZ_STATUS_HQ_OVERFLOW
    assert b.images()[1][3] == 0x00FF00
    b.close()


def test_batch_mixed_depth_maps(rz, oracle, scene):
    """Linear and piecewise views in one batch (one splatting kernel serves
    both kinds): each view equals its oracle image."""
    import torch
    cloud, views, modes, bgs = scene
    pw = (2, ((0.0, 1.0e9), (10.0, 1.0e6), (1.0e4, 1.0e3)))
    lin = (0, 0.0)
    depths = [pw if i % 2 else lin for i in range(len(views))]
    ms = [1, 1, 0, 1, 1, 0, 1, 1, 0, 1, 1][:len(views)]
    pts = rz.Points.from_cloud(cloud)
    b = rz.Batch(pts, views, ms, depth=depths, backgrounds=bgs)
    b.run()
    torch.cuda.synchronize()
    for got, v, m, bg, dm in zip(b.images(), views, ms, bgs, depths):
        if m == 0:
            _, want = oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, v.vp, v.near,
                                              v.far, v.width, v.height, dm[0], dm[1], bg)
        else:
            _, _, want = oracle.render_hq(cloud.x, cloud.y, cloud.z, cloud.rgb, v.vp, v.near,
                                          v.far, v.width, v.height, dm[0], dm[1], bg=bg)
        assert np.array_equal(got, want)
    b.close()


def test_batch_full_size(rz, oracle):
    """The batched multi-view workload at its full size (100M Morton-ordered
    terrain points resident, 64 orbit views at 256x256 to 1920x1080, modes
    drawn 50/50), in the default and in the autotuned launch shapes: every
    view's image equals its one-view call bit for bit, and one view of every
    (method, resolution) pair equals the oracle's whole image."""
    import torch
    sizes = [(256, 256), (640, 480), (1280, 720), (1920, 1080)]
    say("[batch-full] generating 100M terrain points")
    cloud = gen.terrain(100_000_000, gen.CONFIG_SEEDS[4])
    views = gen.orbit_views(64, gen.CONFIG_SEEDS[4], sizes)
    modes = np.random.default_rng([gen.CONFIG_SEEDS[4], 7]).integers(0, 2, 64).tolist()
    # the first view of each (method, resolution), checked against the oracle
    picks = {}
    for i in range(64):
        picks.setdefault((modes[i], views[i].width), i)
    assert len(picks) == 2 * len(sizes)
    want = {}
    for (m, _), i in sorted(picks.items()):
        v = views[i]
        say(f"[batch-full] oracle view {i} {v.width}x{v.height} mode {m}")
        if m == 0:
            _, want[i] = oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, v.vp,
                                                 v.near, v.far, v.width, v.height)
        else:
            _, _, want[i] = oracle.render_hq(cloud.x, cloud.y, cloud.z, cloud.rgb, v.vp, v.near,
                                             v.far, v.width, v.height)
    pts = rz.Points.from_cloud(cloud)
    del cloud
    say("[batch-full] one-view calls")
    plain = []
    for v, m in zip(views, modes):
        img = (rz.rasterize_atomicmin(pts, v)[1] if m == 0 else rz.rasterize_hq_splat(pts, v)[2])
        plain.append(img)
    torch.cuda.synchronize()
    for i in want:
        assert np.array_equal(rz.to_u32(plain[i]), want[i]), f"one-view call, view {i}"
    b = rz.Batch(pts, views, modes, use_graph=True)
    try:
        for label in ("default", "autotuned"):
            if label == "autotuned":
                say("[batch-full] autotune")
                b.autotune(reps=1)
            say(f"[batch-full] batch run, {label} shapes")
            b.run()
            torch.cuda.synchronize()
            for i, (got, ref) in enumerate(zip(b.imgs, plain)):
                assert torch.equal(got, ref), f"{label}: view {i} differs from its one-view call"
            for i in want:
                assert np.array_equal(rz.to_u32(b.imgs[i]), want[i]), f"{label}: view {i}"
    finally:
        b.close()
    say("[batch-full] done")
