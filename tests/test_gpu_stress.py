"""The 300M-point stress cloud (250M terrain points + 20 dense spheres) at full
size: 2560x1440 and 640x360 (about 1300 points per pixel), both methods,
Morton-ordered and shuffled, direct and screen-sorted paths: every key, every
splat sum and every pixel against the oracle.  The oracle's result does not
depend on point order, so one oracle frame per resolution and method serves
both orders."""
import sys
import time

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


def frame(rz, pts, v, path, hq, ws=None):
    """One frame with the raw result kept: (keys, unpacked sums or None,
    resolved image).  The resolve then runs on the same buffers."""
    import torch
    npix = v.width * v.height
    fb, acc = rz.new_framebuffer(v, 0, hq=hq)
    if path == "direct" and not hq:
        rz.rasterize_atomicmin(pts, v, fb=fb, keep_keys=True)
    elif path == "direct":
        rz.rasterize_hq_splat(pts, v, fb=fb, acc=acc, keep_keys=True)
    else:
        rz.rasterize_sorted(pts, v, hq=hq, fb=fb, acc=acc, workspace=ws, keep_keys=True)
    torch.cuda.synchronize()
    keys = rz.to_u64(fb)
    sums = rz.unpack_acc(acc) if hq else None
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    img = (rz.resolve_hq(fb, acc, npix, 0, status=status) if hq
           else rz.resolve_min(fb, npix, 0))
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    return keys, sums, rz.to_u32(img)


def test_stress_cloud_full_size(rz, oracle, stress_cloud):
    """Keys, splat sums (exact R, G, B and count per pixel) and images of
    every (order, path, resolution, method) against the oracle's."""
    import torch
    t0 = time.time()
    say("[stress] generating 300M points (Morton order)")
    cloud, views = stress_cloud
    say(f"[stress] generated n={cloud.n} in {time.time() - t0:.0f} s")
    want = {}
    for v in views:
        keys, img = oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, v.vp, v.near,
                                            v.far, v.width, v.height)
        hkeys, sums, himg = oracle.render_hq(cloud.x, cloud.y, cloud.z, cloud.rgb, v.vp, v.near,
                                             v.far, v.width, v.height)
        assert np.array_equal(keys, hkeys)       # the splat depth pass is the same pass
        want[v.width] = (keys, img, sums, himg)
        say(f"[stress] oracle {v.width}x{v.height} done")
        assert (sums[:, 3] > 0).mean() > 0.3
    assert want[640][2][:, 3].max() > 100   # 640x360: many fragments per pixel in the window
    for order in ("morton", "shuffled"):
        if order == "shuffled":
            cloud = gen.shuffle(cloud, 3)
            say("[stress] shuffled")
        pts = rz.Points.from_cloud(cloud)
        for v in views:
            keys, img, sums, himg = want[v.width]
            paths = ("direct", "sorted") if order == "shuffled" else ("direct",)
            for path in paths:
                say(f"[stress] {order} {path} {v.width}x{v.height}")
                ws = rz.new_workspace(pts.n, v.width, v.height) if path == "sorted" else None
                k1, _, i1 = frame(rz, pts, v, path, False, ws)
                assert np.array_equal(k1, keys), f"{order} {path} atomicMin keys"
                assert np.array_equal(i1, img), f"{order} {path} atomicMin image"
                k2, s2, i2 = frame(rz, pts, v, path, True, ws)
                assert np.array_equal(k2, keys), f"{order} {path} splat depth pass keys"
                bad = np.flatnonzero((s2 != sums).any(1))
                assert bad.size == 0, f"{order} {path} sums differ at {bad[:8]}"
                assert np.array_equal(i2, himg), f"{order} {path} HQ image"
                del ws
        del pts
        torch.cuda.empty_cache()
    say(f"[stress] done in {time.time() - t0:.0f} s")
