"""Render server on the GPU: every request's image is bit-identical alone and
in the mix (mixed clouds, resolutions, methods, overlapping streams, a tight
memory budget), and an injected failure leaves the other requests intact."""
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


SIZES = [(64, 48), (256, 256), (320, 200), (97, 61)]


@pytest.fixture(scope="module")
def world(rz):
    clouds = [gen.config1(n=200_000)[0],
              gen.terrain(1_000_000, 31, extent=100.0, amplitude=10.0, wavelength=40.0),
              gen.terrain(3_000_003, 32, extent=100.0, amplitude=10.0, wavelength=40.0)]
    pts = [rz.Points.from_cloud(c) for c in clouds]
    rng = np.random.default_rng(9)
    reqs = []
    for i in range(30):
        c = int(rng.integers(0, 3))
        if c == 0:
            v = gen.make_view((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 60.0,
                              *SIZES[i % len(SIZES)], 0.01, 10.0)
        else:
            v = gen.orbit_views(1, 100 + i, [SIZES[i % len(SIZES)]], extent=100.0, rmin=60.0,
                                rmax=150.0, near=0.5, far=400.0)[0]
        reqs.append((c, v, int(rng.integers(0, 2)), int(rng.integers(0, 1 << 24))))
    return clouds, pts, reqs


@pytest.fixture(scope="module")
def alone(rz, world):
    """Each request rendered by itself with the one-view calls."""
    import torch
    clouds, pts, reqs = world
    out = []
    for c, v, m, bg in reqs:
        if m == 0:
            _, img = rz.rasterize_atomicmin(pts[c], v, background=bg)
        else:
            _, _, img, _ = rz.rasterize_hq_splat(pts[c], v, background=bg)
        torch.cuda.synchronize()
        out.append(rz.to_u32(img))
    return out


def serve(rz, pts, reqs, budget, streams, fail=()):
    import torch
    s = rz.Server(budget, streams=streams)
    ids = [s.add_cloud(p) for p in pts]
    imgs, tickets = [], []
    for i, (c, v, m, bg) in enumerate(reqs):
        img = torch.full((v.width * v.height,), -1, dtype=torch.int32, device="cuda")
        imgs.append(img)
        tickets.append(s.submit(ids[c], v, m, img=img, background=bg, inject_failure=i in fail))
    s.drain(120)
    st = [s.poll(t) for t in tickets]
    stats = s.stats()
    s.close()
    return [rz.to_u32(i) for i in imgs], st, stats


def test_small_requests_match_oracle(rz, oracle, world, alone):
    clouds, pts, reqs = world
    for (c, v, m, bg), img in list(zip(reqs, alone))[:6]:
        cl = clouds[c]
        if m == 0:
            _, want = oracle.render_atomicmin(cl.x, cl.y, cl.z, cl.rgb, v.vp, v.near, v.far,
                                              v.width, v.height, bg=bg)
        else:
            _, _, want = oracle.render_hq(cl.x, cl.y, cl.z, cl.rgb, v.vp, v.near, v.far, v.width,
                                          v.height, bg=bg)
        assert np.array_equal(img, want)


@pytest.mark.parametrize("budget_mb,streams", [(512, 4), (2, 2), (64, 16)])
def test_mix_equals_alone(rz, world, alone, budget_mb, streams):
    clouds, pts, reqs = world
    say(f"[serve] budget {budget_mb} MiB, {streams} streams")
    imgs, st, stats = serve(rz, pts, reqs, budget_mb << 20, streams)
    assert all(x["state"] == rz.RZ_REQ_DONE and x["error"] == 0 for x in st)
    for i, (got, want) in enumerate(zip(imgs, alone)):
        assert np.array_equal(got, want), f"request {i} differs in the mix"
    assert stats["completed"] == len(reqs) and stats["peak_bytes"] <= budget_mb << 20
    if budget_mb >= 64:
        assert stats["peak_inflight"] > 1      # the requests did overlap


def test_failed_request_is_isolated(rz, world, alone):
    clouds, pts, reqs = world
    fail = {3, 11, 12}
    imgs, st, stats = serve(rz, pts, reqs, 256 << 20, 4, fail=fail)
    for i, (x, got, want) in enumerate(zip(st, imgs, alone)):
        if i in fail:
            assert x["state"] == rz.RZ_REQ_FAILED and x["error"] == rz.RZ_EHIP
            assert (got == 0xFFFFFFFF).all()          # never touched
        else:
            assert x["state"] == rz.RZ_REQ_DONE and np.array_equal(got, want)
    assert stats["failed"] == len(fail)


def test_served_splat_overflow_is_an_error(rz):
    """A pixel with more splat fragments than the packed sums hold exactly
    (16,843,010 white points in one pixel; section 2.2's sums) fails its
    request with RZ_EOVERFLOW instead of returning unspecified colours as
    done; one fragment fewer is served normally."""
    import torch
    view = gen.View(np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 0, 0], [0, 0, -1.0, 0]]),
                    1.0, 100.0, 2, 2)
    s = rz.Server(64 << 20, streams=2)
    try:
        for n, over in ((16_843_009, False), (16_843_010, True)):
            say(f"[serve] count limit n={n}")
            pts = rz.Points(torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"),
                            torch.full((n,), -10.0, device="cuda"),
                            torch.full((n,), 0xFFFFFF, dtype=torch.int32, device="cuda"))
            cid = s.add_cloud(pts)
            img = torch.zeros(4, dtype=torch.int32, device="cuda")
            t = s.submit(cid, view, rz.RZ_MODE_HQ, img=img)
            s.drain(60)
            st = s.poll(t)
            if over:
                assert st["state"] == rz.RZ_REQ_FAILED and st["error"] == rz.RZ_EOVERFLOW
                assert st["hq_status"] & rz.RZ_STATUS_HQ_OVERFLOW
            else:
                assert st["state"] == rz.RZ_REQ_DONE and st["error"] == rz.RZ_OK
                assert rz.to_u32(img)[3] == 0xFFFFFF
            # the atomicMin method has no sums to overflow
            t = s.submit(cid, view, rz.RZ_MODE_ATOMICMIN, img=img)
            s.drain(60)
            assert s.poll(t)["state"] == rz.RZ_REQ_DONE
            del pts
    finally:
        s.close()


def test_requests_wait_for_the_callers_stream(rz, world, alone):
    """A request submitted right after its inputs were produced on another
    stream (a fresh copy of the cloud's planes and the fill of the output
    image, queued behind a long fill) waits for that stream's work: its image
    equals the one-view call's."""
    import torch
    clouds, pts, reqs = world
    side = torch.cuda.Stream()
    big = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    s = rz.Server(256 << 20, streams=4)
    try:
        outs = []
        for i in (1, 2, 5):
            c, v, m, bg = reqs[i]
            torch.cuda.synchronize()
            with torch.cuda.stream(side):
                big.fill_(i)                       # keeps the side stream busy first
                copy = rz.Points(*(t.clone() for t in (pts[c].x, pts[c].y, pts[c].z, pts[c].rgb)))
                img = torch.full((v.width * v.height,), -1, dtype=torch.int32, device="cuda")
            cid = s.add_cloud(copy)
            t = s.submit(cid, v, m, img=img, background=bg, after=side)
            outs.append((i, t, img, copy))
        s.drain(60)
        for i, t, img, _ in outs:
            assert s.poll(t)["state"] == rz.RZ_REQ_DONE
            assert np.array_equal(rz.to_u32(img), alone[i]), f"request {i}"
    finally:
        s.close()
        del big


def busy_stream(fills=100):
    """A side stream with about 20 ms of queued device work (fills of a
    1 GiB buffer), and the buffer, which must outlive that work."""
    import torch
    side = torch.cuda.Stream()
    buf = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(side):
        for k in range(fills):
            buf.fill_(k)
    return side, buf


def test_merged_requests_equal_alone(rz, world, alone):
    """With merge_views, queued requests of one cloud run as one multi-view
    launch; every image is still the one-view call's, bit for bit.  A
    splatting request of the largest cloud, whose work exceeds the work cap,
    runs first and alone, so that the others queue behind it and merge."""
    import torch
    clouds, pts, reqs = world
    s = rz.Server(256 << 20, streams=2, max_inflight=16, work_cap=pts[2].n, merge_views=8)
    ids = [s.add_cloud(p) for p in pts]
    v0 = reqs[0][1]
    blk_img = torch.empty(v0.width * v0.height, dtype=torch.int32, device="cuda")   # kept alive
    torch.cuda.synchronize()
    side, buf = busy_stream()
    # in flight until the side stream's work is done: the others queue
    blocker = s.submit(ids[2], v0, rz.RZ_MODE_HQ, img=blk_img, after=side)
    imgs, tickets = [], []
    for c, v, m, bg in reqs:
        img = torch.full((v.width * v.height,), -1, dtype=torch.int32, device="cuda")
        imgs.append(img)
        tickets.append(s.submit(ids[c], v, m, img=img, background=bg))
    s.drain(120)
    st = [s.poll(t) for t in tickets]
    assert s.poll(blocker)["state"] == rz.RZ_REQ_DONE
    stats = s.stats()
    s.close()
    torch.cuda.synchronize()
    del buf
    say(f"[serve] merged {stats['merged_requests']} requests in {stats['merged_launches']} "
        f"launches; groups {[x['group'] for x in st]}")
    assert all(x["state"] == rz.RZ_REQ_DONE and x["error"] == 0 for x in st)
    for i, (got, want) in enumerate(zip(imgs, alone)):
        assert np.array_equal(rz.to_u32(got), want), f"request {i} differs when merged"
    assert stats["merged_launches"] >= 1 and max(x["group"] for x in st) > 1
    assert stats["merged_requests"] == sum(1 for x in st if x["group"] > 1)


def test_merged_splat_overflow_fails_only_its_request(rz):
    """Two splatting requests of one cloud merged into one launch: the one
    whose pixel receives 16,843,010 fragments fails with RZ_EOVERFLOW, the
    other (its view culls every point) is served, with its own status."""
    import torch
    n = 16_843_010
    pts = rz.Points(torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"),
                    torch.full((n,), -10.0, device="cuda"),
                    torch.full((n,), 0xFFFFFF, dtype=torch.int32, device="cuda"))
    vp = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 0, 0], [0, 0, -1.0, 0]])
    hit = gen.View(vp, 1.0, 100.0, 2, 2)
    cull = gen.View(vp, 20.0, 100.0, 2, 2)      # every point nearer than near
    a = lambda v: (v + 255) // 256 * 256
    bw, bh = 1280, 720                          # the request that runs first
    blocker_bytes = a(8 * bw * bh) + a(16 * bw * bh) + 256
    small_bytes = a(8 * 4) + a(16 * 4) + 256
    # memory for the first request only: the two small ones queue behind it
    # and are admitted together once it is done
    budget = max(1 << 20, blocker_bytes + small_bytes // 2)
    assert blocker_bytes + small_bytes > budget >= 2 * small_bytes
    s = rz.Server(budget, streams=1, max_inflight=8, merge_views=4)
    try:
        cid = s.add_cloud(pts)
        other = s.add_cloud(rz.Points.from_cloud(gen.config1(n=100_000)[0]))
        v_big = gen.make_view((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, bw, bh, 0.01,
                              10.0)
        big_img = torch.empty(bw * bh, dtype=torch.int32, device="cuda")   # kept alive
        torch.cuda.synchronize()
        side, buf = busy_stream()
        # in flight until the side stream's work is done: the two queue
        first = s.submit(other, v_big, rz.RZ_MODE_HQ, img=big_img, after=side)
        img_hit = torch.zeros(4, dtype=torch.int32, device="cuda")
        img_cull = torch.zeros(4, dtype=torch.int32, device="cuda")
        t_hit = s.submit(cid, hit, rz.RZ_MODE_HQ, img=img_hit)
        t_cull = s.submit(cid, cull, rz.RZ_MODE_HQ, img=img_cull, background=0x123456)
        s.drain(60)
        assert s.poll(first)["state"] == rz.RZ_REQ_DONE
        st_hit, st_cull = s.poll(t_hit), s.poll(t_cull)
        assert st_hit["group"] == 2 and st_cull["group"] == 2
        assert st_hit["state"] == rz.RZ_REQ_FAILED and st_hit["error"] == rz.RZ_EOVERFLOW
        assert st_cull["state"] == rz.RZ_REQ_DONE and st_cull["error"] == rz.RZ_OK
        assert st_cull["hq_status"] == 0
        assert (rz.to_u32(img_cull) == 0x123456).all()
    finally:
        s.close()
        torch.cuda.synchronize()


def test_chained_requests_equal_alone(rz, world, alone):
    """With a work cap and exclusive requests, requests held back are
    admitted behind running ones on their streams (chained); every image is
    still the one-view call's, bit for bit."""
    import torch
    clouds, pts, reqs = world
    s = rz.Server(256 << 20, streams=4, max_inflight=16, work_cap=pts[2].n,
                  exclusive_work=pts[2].n)
    ids = [s.add_cloud(p) for p in pts]
    imgs, tickets = [], []
    for c, v, m, bg in reqs:
        img = torch.full((v.width * v.height,), -1, dtype=torch.int32, device="cuda")
        imgs.append(img)
        tickets.append(s.submit(ids[c], v, m, img=img, background=bg))
    s.drain(120)
    st = [s.poll(t) for t in tickets]
    stats = s.stats()
    s.close()
    say(f"[serve] chained {stats['chained_requests']} of {len(reqs)} requests")
    assert all(x["state"] == rz.RZ_REQ_DONE and x["error"] == 0 for x in st)
    for i, (got, want) in enumerate(zip(imgs, alone)):
        assert np.array_equal(rz.to_u32(got), want), f"request {i} differs when chained"
    assert stats["chained_requests"] > 0
