"""The serving workload at its full size: 8 resident clouds of 1M to 300M
points (826M in total, 13.2 GB of point planes), 96 requests submitted at
once over resolutions 256x256 to 2560x1440 and both methods, through a
4 GiB framebuffer budget on 4 streams.  Every served image equals its
one-view call, and the smallest request of every (cloud, method) pair
equals the oracle's whole image."""
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


def test_serving_workload_full_size(rz, oracle, stress_cloud):
    import torch
    t0 = time.time()
    clouds = []
    for i, n in enumerate(gen.SERVE_CLOUDS):
        say(f"[serve-full] cloud {i}: {n} points")
        clouds.append(stress_cloud[0] if n == 300_000_000 else gen.serve_cloud(i, n))
        assert clouds[-1].n == n
    pts = [rz.Points.from_cloud(c) for c in clouds]
    trace = gen.request_trace(96, 1e9, gen.CONFIG_SEEDS[5] + 2, len(clouds))
    assert max(v.width * v.height for _, _, v, _ in trace) == 2560 * 1440
    say(f"[serve-full] {sum(c.n for c in clouds) / 1e6:.0f}M points resident "
        f"({time.time() - t0:.0f} s)")
    imgs = [torch.full((v.width * v.height,), -1, dtype=torch.int32, device="cuda")
            for _, _, v, _ in trace]
    srv = rz.Server(4 << 30, streams=4)
    try:
        ids = [srv.add_cloud(p) for p in pts]
        tickets = [srv.submit(ids[c], v, m, img=img) for (_, c, v, m), img in zip(trace, imgs)]
        srv.drain(600)
        st = [srv.poll(t) for t in tickets]
        stats = srv.stats()
    finally:
        srv.close()
    assert all(x["state"] == rz.RZ_REQ_DONE and x["error"] == rz.RZ_OK for x in st)
    assert stats["peak_inflight"] > 1 and stats["peak_bytes"] <= 4 << 30
    say(f"[serve-full] served: peak in flight {stats['peak_inflight']}, "
        f"peak framebuffer memory {stats['peak_bytes'] / 1e6:.0f} MB")
    for k, ((_, c, v, m), img) in enumerate(zip(trace, imgs)):
        if m == 0:
            _, ref = rz.rasterize_atomicmin(pts[c], v)
        else:
            _, _, ref, status = rz.rasterize_hq_splat(pts[c], v)
            assert int(status.item()) == 0
        torch.cuda.synchronize()
        assert torch.equal(img, ref), f"request {k} (cloud {c}, {v.width}x{v.height}, mode {m})"
        del ref
    say("[serve-full] every served image equals its one-view call")
    smallest = {}
    for k, (_, c, v, m) in enumerate(trace):
        if (c, m) not in smallest or v.width * v.height < trace[smallest[(c, m)]][2].width * \
                trace[smallest[(c, m)]][2].height:
            smallest[(c, m)] = k
    assert len(smallest) == 2 * len(clouds)
    for (c, m), k in sorted(smallest.items()):
        _, _, v, _ = trace[k]
        cl = clouds[c]
        say(f"[serve-full] oracle: cloud {c} ({cl.n} points), mode {m}, {v.width}x{v.height}")
        if m == 0:
            _, want = oracle.render_atomicmin(cl.x, cl.y, cl.z, cl.rgb, v.vp, v.near, v.far,
                                              v.width, v.height)
        else:
            _, _, want = oracle.render_hq(cl.x, cl.y, cl.z, cl.rgb, v.vp, v.near, v.far,
                                          v.width, v.height)
        assert np.array_equal(rz.to_u32(imgs[k]), want), f"request {k} against the oracle"
    say(f"[serve-full] done in {time.time() - t0:.0f} s")
