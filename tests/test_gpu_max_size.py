"""Past 2^31 points: 2^31 + 2^20 + 77 points (34 GB of planes), and the
largest cloud the interface accepts, 2^32 - 512 points (69 GB), on a 1024x1024
screen with about 2050 or 4096 layers of points per pixel, through the direct
and the screen-sorted paths, both methods.  Every point index, chunk base and
sorted position beyond the 32-bit signed range is exercised, up to the last
unsigned 32-bit position the sorted path uses.

Point i lies on the centre ray of pixel p = i mod P (P = 1024 * 1024) at depth
1 + (i div P) / 2000, with a colour hashed from i.  The oracle checks the keys
and the exact splat sums of 2050 sampled pixels from all their points (read
back from the device planes, so both sides see the same inputs); every pixel
must hold a layer-0 key and the count of accepted layers the sampled pixels
show."""
import sys

import numpy as np
import pytest

from paper_1908_02681_amd import gen

pytestmark = pytest.mark.gpu

W = H = 1024
P = W * H
SIZES = [(1 << 31) + (1 << 20) + 77, (1 << 32) - 512]   # the second: kMaxPoints


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


def view():
    # clip w = -z and x, y unscaled: a point (c * D, c' * D, -D) lands on the
    # NDC point (c, c') at depth D
    vp = np.diag([1.0, 1.0, 0.0, 0.0]) + np.array(
        [[0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, -1.0, 0]])
    return gen.View(vp, 0.5, 4.0, W, H)


@pytest.fixture(scope="module", params=SIZES, ids=["2^31+", "2^32-512"])
def planes(rz, request):
    import torch
    N = request.param
    torch.cuda.empty_cache()
    say(f"[max] generating {N} points on the device")
    x = torch.empty(N, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    c = torch.empty(N, dtype=torch.int32, device="cuda")
    step = 1 << 26
    for s in range(0, N, step):
        i = torch.arange(s, min(N, s + step), dtype=torch.int64, device="cuda")
        p = i % P
        d = (i // P).to(torch.float32) * 0.0005 + 1.0
        cx = ((2 * (p % W) + 1).to(torch.float32) / W) - 1.0
        cy = ((2 * (p // W) + 1).to(torch.float32) / H) - 1.0
        x[s:s + i.numel()] = cx * d
        y[s:s + i.numel()] = cy * d
        z[s:s + i.numel()] = -d
        c[s:s + i.numel()] = (i * 40503 + (i >> 13)).bitwise_and(0xFFFFFF).to(torch.int32)
        del i, p, d, cx, cy
    torch.cuda.synchronize()
    yield rz.Points(x, y, z, c)
    del x, y, z, c
    torch.cuda.empty_cache()


def sampled_points(pts, pix):
    """Every point of the given pixels, read back from the device planes."""
    import torch
    idx = np.concatenate([np.arange(p, pts.n, P, dtype=np.int64) for p in pix])
    t = torch.from_numpy(idx).to("cuda")
    out = [pts.x[t].cpu().numpy(), pts.y[t].cpu().numpy(), pts.z[t].cpu().numpy(),
           pts.rgb[t].cpu().numpy().view(np.uint32)]
    del t
    return out


def run(rz, pts, v, path, hq, ws=None):
    import torch
    fb, acc = rz.new_framebuffer(v, 0, hq=hq)
    say(f"[max] {path} {'hq' if hq else 'atomicmin'}")
    if path == "direct" and not hq:
        rz.rasterize_atomicmin(pts, v, fb=fb, keep_keys=True)
    elif path == "direct":
        rz.rasterize_hq_splat(pts, v, fb=fb, acc=acc, keep_keys=True)
    else:
        rz.rasterize_sorted(pts, v, hq=hq, fb=fb, acc=acc, workspace=ws, keep_keys=True)
    torch.cuda.synchronize()
    keys = rz.to_u64(fb)
    sums = rz.unpack_acc(acc) if hq else None
    del fb, acc
    return keys, sums


@pytest.mark.parametrize("path", ["direct", "sorted"])
def test_past_two_to_the_31_points(rz, oracle, planes, path):
    import torch
    v = view()
    rng = np.random.default_rng(31)
    pix = np.unique(np.concatenate([[0, 76, 77, P - 1], rng.integers(0, P, 2046)]))
    sx, sy, sz, sc = sampled_points(planes, pix)
    want_keys, want_sums, _ = oracle.render_hq(sx, sy, sz, sc, v.vp, v.near, v.far, W, H)
    ws = rz.new_workspace(planes.n, W, H) if path == "sorted" else None
    keys, _ = run(rz, planes, v, path, False, ws)
    hkeys, sums = run(rz, planes, v, path, True, ws)
    del ws
    torch.cuda.empty_cache()
    # the sampled pixels, key for key and sum for sum
    assert np.array_equal(keys[pix], want_keys[pix])
    assert np.array_equal(hkeys[pix], want_keys[pix])
    assert np.array_equal(sums[pix], want_sums[pix])
    # every pixel: its nearest point is on layer 0, at the depth of the
    # sampled pixels' layer-0 keys, and the splat pass accepted as many
    # layers as at the sampled pixels
    q0 = want_keys[pix[0]] >> np.uint64(24)
    assert (keys >> np.uint64(24) == q0).all()
    accepted = want_sums[pix, 3]
    assert (accepted == accepted[0]).all() and accepted[0] > 1
    assert (sums[:, 3] == accepted[0]).all()
