"""Sort-last composition on the GPU: a cloud split into parts, each part
rendered into its own full framebuffer, merged with rz_merge_min (depth) and
rz_merge_sum (splat sums against the merged depth) equals the one-call
render and the oracle, bit for bit."""
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


def shards(rz, pts, k):
    n = pts.n
    cut = [n * i // k for i in range(k + 1)]
    return [rz.Points(pts.x[a:b], pts.y[a:b], pts.z[a:b], pts.rgb[a:b])
            for a, b in zip(cut[:-1], cut[1:])]


def sort_last(rz, pts, view, k, bg=0):
    """Depth keys, packed sums and image composed from k parts."""
    import torch
    npix = view.width * view.height
    parts = shards(rz, pts, k)
    fbs = []
    for part in parts:
        fb, _ = rz.new_framebuffer(view, bg)
        rz.rasterize_atomicmin(part, view, background=bg, fb=fb, keep_keys=True)
        fbs.append(fb)
    merged = fbs[0]
    for fb in fbs[1:]:
        rz.merge_min(merged, fb, npix)
    keys = rz.to_u64(merged)
    acc = torch.zeros(2 * npix, dtype=torch.int64, device="cuda")
    for part in parts:
        a = torch.zeros(2 * npix, dtype=torch.int64, device="cuda")
        rz.hq_accumulate(part, view, merged, a)
        rz.merge_sum(acc, a, npix)
    sums = rz.unpack_acc(acc)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    img = rz.resolve_hq(merged, acc, npix, bg, status=status)
    torch.cuda.synchronize()
    return keys, sums, rz.to_u32(img)


@pytest.mark.parametrize("k,size", [(2, (97, 61)), (4, (320, 200)), (7, (33, 257))])
def test_sort_last_matches_oracle(rz, oracle, k, size):
    cloud = gen.terrain(1_000_003, 61, extent=100.0, amplitude=10.0, wavelength=40.0)
    view = gen.orbit_views(1, 14, [size], extent=100.0, rmin=60.0, rmax=120.0, near=0.5,
                           far=400.0)[0]
    say(f"[merge] k={k} {size}")
    pts = rz.Points.from_cloud(cloud)
    keys, sums, img = sort_last(rz, pts, view, k, bg=0x445566)
    args = (cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near, view.far, view.width,
            view.height)
    ok_keys, ok_sums, ok_img = oracle.render_hq(*args, bg=0x445566)
    assert np.array_equal(keys, ok_keys)
    assert np.array_equal(sums, ok_sums)
    assert np.array_equal(img, ok_img)


def test_sort_last_full_size(rz):
    """The 50M terrain at 1920x1080 in 8 parts equals the one-call frames."""
    import torch
    cloud, view = gen.config2()
    pts = rz.Points.from_cloud(cloud)
    keys, sums, img = sort_last(rz, pts, view, 8)
    fb, acc, want, _ = rz.rasterize_hq_splat(pts, view, keep_keys=True)
    torch.cuda.synchronize()
    assert np.array_equal(keys, rz.to_u64(fb)) and np.array_equal(sums, rz.unpack_acc(acc))
    _, _, want, _ = rz.rasterize_hq_splat(pts, view)
    torch.cuda.synchronize()
    assert np.array_equal(img, rz.to_u32(want))


def test_merge_min_odd_sizes(rz):
    import torch
    rng = np.random.default_rng(5)
    for n in (1, 2, 3, 511, 513, 100_001):
        a = rng.integers(0, 2 ** 63, n, dtype=np.int64)
        b = rng.integers(0, 2 ** 63, n, dtype=np.int64)
        da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        rz.merge_min(da, db, n)
        s = torch.from_numpy(np.stack([a, b], 1).reshape(-1)).cuda()
        t = torch.from_numpy(np.stack([b, a], 1).reshape(-1)).cuda()
        rz.merge_sum(s, t, n)
        torch.cuda.synchronize()
        assert np.array_equal(rz.to_u64(da), np.minimum(a.view(np.uint64), b.view(np.uint64)))
        assert np.array_equal(rz.to_u64(s), (np.stack([a, b], 1).reshape(-1).view(np.uint64) +
                                             np.stack([b, a], 1).reshape(-1).view(np.uint64)))
