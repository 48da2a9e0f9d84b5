"""The allocation-free entry point rasterize_sorted_noalloc (static device
scratch) against rasterize_sorted with a caller workspace: keys, splat sums
and images equal bit for bit, on two calls in a row, the second with a
smaller cloud and screen, so that the second runs over what the first left
in the shared scratch.  Called through the C ABI (ctypes binding)."""
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


def _with_workspace(rz, pts, view, hq):
    import torch
    fb, acc = rz.new_framebuffer(view, 0, hq=True)
    rz.rasterize_sorted(pts, view, hq=hq, fb=fb, acc=acc, keep_keys=True)
    torch.cuda.synchronize()
    keys, sums = rz.to_u64(fb), rz.unpack_acc(acc)
    _, _, img, st = rz.rasterize_sorted(pts, view, hq=hq)
    torch.cuda.synchronize()
    return keys, sums, rz.to_u32(img), (int(st.item()) if hq else 0)


def _without(rz, pts, view, hq):
    import torch
    npix = view.width * view.height
    fb, acc = rz.new_framebuffer(view, 0, hq=True)
    img = torch.empty(npix, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    rz.rasterize_sorted_noalloc(pts, view, fb, None, hq=hq, acc=acc, status=st, keep_keys=True)
    torch.cuda.synchronize()
    keys, sums = rz.to_u64(fb), rz.unpack_acc(acc)
    fb, acc = rz.new_framebuffer(view, 0, hq=True)
    rz.rasterize_sorted_noalloc(pts, view, fb, img, hq=hq, acc=acc, status=st)
    torch.cuda.synchronize()
    return keys, sums, rz.to_u32(img), int(st.item())


@pytest.mark.parametrize("hq", [False, True])
def test_noalloc_matches_workspace_call(rz, hq):
    import torch
    cases = [(gen.shuffle(gen.terrain(2_000_000, 41), 5), gen.terrain_view(1280, 720)),
             (gen.config1(n=300_000)[0], gen.config1()[1])]
    cases[1][1].width, cases[1][1].height = 640, 360
    for k, (cloud, view) in enumerate(cases):
        need = rz.sorted_workspace_bytes(cloud.n, view.width, view.height)
        assert need <= rz.RZ_NOALLOC_SCRATCH_BYTES
        say(f"[noalloc] call {k}: n={cloud.n} {view.width}x{view.height} hq={hq} "
            f"scratch {need >> 20} MiB")
        pts = rz.Points.from_cloud(cloud)
        want = _with_workspace(rz, pts, view, hq)
        got = _without(rz, pts, view, hq)
        assert np.array_equal(got[0], want[0]), "keys"
        if hq:
            assert np.array_equal(got[1], want[1]), "sums"
        assert np.array_equal(got[2], want[2]), "image"
        assert got[3] == 0 and want[3] == 0
        del pts
        torch.cuda.empty_cache()


def test_noalloc_refuses_what_does_not_fit(rz):
    """A cloud whose workspace exceeds the static scratch is refused with
    RZ_EBUDGET before anything runs."""
    import torch
    view = gen.terrain_view(1920, 1080)
    n = 8_000_000
    assert rz.sorted_workspace_bytes(n, view.width, view.height) > rz.RZ_NOALLOC_SCRATCH_BYTES
    z = torch.zeros(n, dtype=torch.float32, device="cuda")
    pts = rz.Points(z, z, z, torch.zeros(n, dtype=torch.int32, device="cuda"))
    fb, _ = rz.new_framebuffer(view, 0)
    img = torch.empty(view.width * view.height, dtype=torch.int32, device="cuda")
    with pytest.raises(rz.RzError) as e:
        rz.rasterize_sorted_noalloc(pts, view, fb, img)
    assert e.value.code == rz.RZ_EBUDGET
