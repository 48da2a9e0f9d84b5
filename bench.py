#!/usr/bin/env python3
"""Benchmark of the point rasterizer on one MI355X.

One step = one frame of both methods over the same resident cloud:
  atomicMin  : depth pass (k_raster_min) + resolve/clear (k_resolve_min)
  HQ splat   : depth pass + accumulate pass (k_hq_accum) + resolve (k_resolve_hq)
Value = points rasterized per second over the step (each method's frame
counts its N points once): Gpoints/s.  Inputs are resident in HBM before the
timed region.  Before the W warm-up steps the step runs untimed for
--settle-ms of wall time (reported as detail.settle), so that the timed steps
start at the GPU's sustained clock.  Per-kernel durations come from HIP events
recorded on the launch stream around each pass, averaged over the timed steps.

    python bench.py [--steps K] [--warmup W] [--workload terrain50m|spheres1m|...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpoints/s rasterized (atomicMin, HQ splat); served p50/p99 ms vs plain loop"
HBM_PEAK_GBS = 8000.0
# wave64 VALU issue without packed FP32: 256 CUs x 4 SIMDs, one instruction
# per SIMD every 4 cycles, 64 lanes, 2.4 GHz
VALU_ISSUE_PEAK = 256 * 64 * 2.4e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    from paper_1908_02681_amd import gen
    if name == "terrain50m":
        cloud, view = gen.config2()
        desc = "terrain 50M points, Morton order, 1920x1080 oblique camera"
    elif name == "terrain50m-shuffled":
        cloud, view = gen.config2()
        cloud = gen.shuffle(cloud, 1)
        desc = "terrain 50M points, shuffled, 1920x1080 oblique camera"
    elif name == "spheres1m":
        cloud, view = gen.config1()
        desc = "8 spheres 1M points, shuffled, 1024x768"
    elif name.startswith("stress300m"):
        # stress300m[-shuffled]-1440p|360p: 250M terrain points (5x density)
        # plus 20 dense spheres of 2.5M points
        parts = name.split("-")
        order = "shuffled" if "shuffled" in parts else "morton"
        res = parts[-1]
        if res not in ("1440p", "360p"):
            raise SystemExit(f"unknown workload {name}")
        log(f"[bench] generating the 300M-point stress cloud ({order})")
        cloud, views = gen.config3(order=order)
        view = views[0] if res == "1440p" else views[1]
        desc = (f"stress 300M points (250M terrain + 20 spheres of 2.5M), {order}, "
                f"{view.width}x{view.height}")
    else:
        raise SystemExit(f"unknown workload {name}")
    return cloud, view, desc


def cpu_baseline(cloud, view, eps, min_s=10.0, budget_s=20.0):
    """The oracle, single-threaded, on the same workload (whole frames):
    at least three frames and min_s seconds of work, at most budget_s."""
    from oracle import oracle
    oracle.build()
    n = cloud.n
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        oracle.render_atomicmin(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near,
                                view.far, view.width, view.height)
        t1 = time.perf_counter()
        oracle.render_hq(cloud.x, cloud.y, cloud.z, cloud.rgb, view.vp, view.near, view.far,
                         view.width, view.height, eps=eps)
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
        spent = time.perf_counter() - t_start
        if spent > budget_s or (len(times) >= 3 and spent >= min_s):
            break
    t_min = float(np.median([a for a, _ in times]))
    t_hq = float(np.median([b for _, b in times]))
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(line.split(":", 1)[1].strip() for line in f
                         if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {
        "value": round(2 * n / (t_min + t_hq) / 1e9, 6),
        "unit": "Gpoints/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{len(times)} full frames (atomicMin + HQ) of the same {n}-point workload; "
                  f"median atomicMin {t_min:.3f} s, HQ {t_hq:.3f} s; one thread on {model} "
                  f"({os.cpu_count()} host cores)",
    }


BATCH_SIZES = [(256, 256), (640, 480), (1280, 720), (1920, 1080)]


def calibration_copy(nbytes):
    """One device-to-device copy of nbytes: a plain copy kernel of known size
    whose HBM counters scale those of the kernels in the same counter run."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy of {src.numel() * 4} bytes done")


def settle(fn, ms):
    """Runs fn untimed for about ms of wall time (synchronising every few
    calls): a GPU left idle while the host generates inputs runs at a low
    clock, and a timed window of a few milliseconds started then measures the
    clock ramp, not the kernels (50M terrain: 195 Gpoints/s after 5 warm-up
    steps, 215 after 50).  Returns the steps run and the time taken."""
    import torch
    if ms <= 0:
        return {"steps": 0, "ms": 0.0}
    t0 = time.perf_counter()
    n = 0
    while True:
        fn()
        n += 1
        if n % 4 == 0:
            torch.cuda.synchronize()
            if (time.perf_counter() - t0) * 1e3 >= ms:
                break
    return {"steps": n, "ms": round((time.perf_counter() - t0) * 1e3, 1)}


def bench_batch(a):
    """64 views of one resident 100M-point terrain: one autotuned, graph-captured
    batch against the loop of 64 one-view calls (same views, same bits)."""
    import torch
    from paper_1908_02681_amd import gen, rz

    n = a.batch_points
    log(f"[batch] generating terrain {n}")
    cloud = gen.terrain(n, gen.CONFIG_SEEDS[4])
    views = gen.orbit_views(a.batch_views, gen.CONFIG_SEEDS[4], BATCH_SIZES)
    rng = np.random.default_rng([gen.CONFIG_SEEDS[4], 7])
    modes = rng.integers(0, 2, len(views)).tolist()
    pts = rz.Points.from_cloud(cloud)
    del cloud
    npix = sum(v.width * v.height for v in views)
    log(f"[batch] {len(views)} views, {npix / 1e6:.1f} Mpx, {sum(modes)} splatting")

    # plain loop: one call per view, buffers allocated once
    bufs = []
    for v, m in zip(views, modes):
        fb, acc = rz.new_framebuffer(v, 0, hq=(m == 1))
        img = torch.empty(v.width * v.height, dtype=torch.int32, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        bufs.append((fb, acc, img, st))

    def plain():
        for v, m, (fb, acc, img, st) in zip(views, modes, bufs):
            if m == 0:
                rz.rasterize_atomicmin(pts, v, fb=fb, img=img)
            else:
                rz.rasterize_hq_splat(pts, v, fb=fb, acc=acc, img=img, status=st)

    if a.batch_k:
        b = rz.Batch(pts, views, modes, views_per_group=a.batch_k, use_graph=False,
                     launch=tuple(a.batch_launch) if a.batch_launch else None)
        chosen = b.opts()
        log(f"[batch] fixed {chosen}")
    else:
        b = rz.Batch(pts, views, modes, use_graph=True)
        chosen, tuned_ms = b.autotune(reps=2)
        log(f"[batch] autotuned {chosen} ({tuned_ms:.3f} ms)")

    def timed(fn, steps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    ms_plain = timed(plain, a.steps, a.warmup)
    ms_batch = timed(b.run, a.steps, a.warmup)
    same = all(torch.equal(img, bimg) for (_, _, img, _), bimg in zip(bufs, b.imgs))
    log(f"[batch] plain {ms_plain:.3f} ms, batched {ms_batch:.3f} ms, identical={same}")
    if not same:
        raise SystemExit("batched images differ from the one-view calls")
    if a.calibrate_copy:
        calibration_copy(a.calibrate_copy)
    work = n * len(views)
    out = {
        "metric": METRIC, "value": round(work / (ms_batch * 1e-3) / 1e9, 3), "unit": "Gpoints/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_batch, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64->u64",
        "data": "synthetic",
        "config": {"workload": f"batched multi-view: terrain {n} points (Morton order), "
                               f"{len(views)} orbit cameras, resolutions {BATCH_SIZES}, "
                               f"{sum(modes)} splatting / {len(views) - sum(modes)} atomicMin",
                   "points": n, "views": len(views), "pixels": npix},
        "detail": {"plain_loop_ms": round(ms_plain, 4),
                   "plain_loop_gpts": round(work / (ms_plain * 1e-3) / 1e9, 3),
                   "speedup_vs_plain": round(ms_plain / ms_batch, 3),
                   ("fixed" if a.batch_k else "autotuned"): chosen,
                   "bit_identical_to_plain": same},
    }
    print(json.dumps(out), flush=True)


def serve_trace(n, rate, seed, nclouds):
    from paper_1908_02681_amd import gen
    return gen.request_trace(n, rate, seed, nclouds)


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else float("nan")


class ServingWorld:
    """Resident serving clouds, output image rings and the two ways of
    serving a request trace: the plain FIFO loop (one call, then a device
    synchronisation, per request) and the continuous-batching server."""

    def __init__(self, a, clouds=None, log_prefix="[serve]"):
        import torch
        from paper_1908_02681_amd import gen, rz
        self.torch, self.gen, self.rz, self.a = torch, gen, rz, a
        self.pts, self.npts = [], []
        for i, n in enumerate(gen.SERVE_CLOUDS[:a.serve_clouds]):
            c = clouds.get(i) if clouds else None
            if c is None:
                log(f"{log_prefix} generating cloud {i}: {n} points")
                c = gen.serve_cloud(i, n)
            self.pts.append(rz.Points.from_cloud(c))
            self.npts.append(c.n)
            del c
        torch.cuda.synchronize()
        log(f"{log_prefix} {sum(self.npts) / 1e6:.0f}M points resident")
        # one reusable output image ring per resolution (requests in flight never share)
        self.ring = a.serve_ring
        self.imgs = {sz: [torch.empty(sz[0] * sz[1], dtype=torch.int32, device="cuda")
                          for _ in range(self.ring)] for sz in gen.SERVE_SIZES}
        # plain loop buffers: one fb/acc per resolution
        self.fbs = {sz: rz.new_framebuffer(gen.View(np.eye(4), 1, 2, *sz), 0, hq=True)
                    for sz in gen.SERVE_SIZES}
        self.st_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()

    def plain_one(self, c, v, m, img):
        fb, acc = self.fbs[(v.width, v.height)]
        if m == 0:
            self.rz.rasterize_atomicmin(self.pts[c], v, fb=fb, img=img)
        else:
            self.rz.rasterize_hq_splat(self.pts[c], v, fb=fb, acc=acc, img=img,
                                       status=self.st_dev)

    def run_plain(self, trace):
        torch = self.torch
        lat, done_t = [], []
        t0 = time.perf_counter()
        for k, (t_arr, c, v, m) in enumerate(trace):
            while time.perf_counter() - t0 < t_arr:
                pass
            self.plain_one(c, v, m, self.imgs[(v.width, v.height)][k % self.ring])
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            lat.append((t - t_arr) * 1e3)
            done_t.append(t)
        return lat, trace[0][0], done_t[-1]

    def run_server(self, trace):
        rz, a = self.rz, self.a
        srv = rz.Server(a.serve_budget, streams=a.serve_streams, work_cap=self.work_cap(),
                        merge_views=a.serve_merge, exclusive_work=self.exclusive_work())
        ids = [srv.add_cloud(p) for p in self.pts]
        pending, status = {}, {}
        slot_owner = {sz: [None] * self.ring for sz in self.gen.SERVE_SIZES}

        def reap():
            for t in list(pending):
                st = srv.poll(t)
                if st["state"] >= rz.RZ_REQ_DONE:
                    status[t] = st
                    del pending[t]
        t0 = time.perf_counter()
        tick = []
        for k, (t_arr, c, v, m) in enumerate(trace):
            while time.perf_counter() - t0 < t_arr:
                if pending:
                    reap()
            sz = (v.width, v.height)
            j = k % self.ring
            prev = slot_owner[sz][j]
            while prev is not None and prev in pending:
                reap()
            late = time.perf_counter() - t0 - t_arr   # time spent before submission
            # the ring images were made and synchronised up front: no stream to wait for
            t = srv.submit(ids[c], v, m, img=self.imgs[sz][j], after=None)
            slot_owner[sz][j] = t
            pending[t] = k
            tick.append((t, late))
        srv.drain(600)
        reap()
        stats = srv.stats()
        srv.close()
        sts = [status[t] for t, _ in tick]
        if any(x["state"] != rz.RZ_REQ_DONE for x in sts):
            raise SystemExit("server request failed")
        # latency from arrival: the server's submit-to-done time plus any wait
        # of the request before it could be submitted
        lat = [(x["t_done_us"] - x["t_submit_us"]) / 1e3 + late * 1e3
               for x, (_, late) in zip(sts, tick)]
        first_arrival_us = sts[0]["t_submit_us"] - tick[0][1] * 1e6
        span = (max(x["t_done_us"] for x in sts) - first_arrival_us) / 1e6
        return lat, span, stats

    def work_cap(self):
        """The server's work cap: the option's value, or by default the work
        of the largest request (a splat frame of the largest cloud), so that
        such a request runs alone while smaller ones still overlap."""
        return self.a.serve_work_cap if self.a.serve_work_cap >= 0 else 2 * max(self.npts)

    def exclusive_work(self):
        """Requests at least this large run alone: the option's value, or by
        default none."""
        return self.a.serve_exclusive if self.a.serve_exclusive >= 0 else 0

    def capacity(self):
        """Requests per second of the plain loop on back-to-back requests."""
        probe = serve_trace(200, 1e9, self.gen.CONFIG_SEEDS[5], len(self.pts))
        for _ in range(2):
            self.run_plain(probe[:20])
        _, _, t_end = self.run_plain(probe)
        return len(probe) / t_end

    def load_row(self, rate, nreq):
        """Both ways of serving one Poisson trace at `rate` requests per second."""
        trace = serve_trace(nreq, rate, self.gen.CONFIG_SEEDS[5], len(self.pts))
        work = sum(self.npts[c] for _, c, _, _ in trace)
        lp, _, tp_end = self.run_plain(trace)
        ls, span, stats = self.run_server(trace)
        return {"offered_req_s": round(rate, 1), "requests": nreq,
                "server": {"req_s": round(len(trace) / span, 1),
                           "gpts": round(work / span / 1e9, 2),
                           "p50_ms": round(pct(ls, 50), 3), "p99_ms": round(pct(ls, 99), 3),
                           "peak_inflight": stats["peak_inflight"],
                           "merged_requests": stats["merged_requests"],
                           "chained_requests": stats["chained_requests"],
                           "peak_fb_MB": round(stats["peak_bytes"] / 1e6, 1)},
                "plain": {"req_s": round(len(trace) / (tp_end - trace[0][0]), 1),
                          "gpts": round(work / (tp_end - trace[0][0]) / 1e9, 2),
                          "p50_ms": round(pct(lp, 50), 3), "p99_ms": round(pct(lp, 99), 3)}}


def bench_serve(a):
    """Continuous-batching server vs the FIFO one-call-per-request loop on the
    same Poisson traces over 8 resident clouds."""
    import torch
    from paper_1908_02681_amd import gen, rz

    w = ServingWorld(a)
    pts, npts = w.pts, w.npts
    plain_one = w.plain_one
    cap = w.capacity()
    log(f"[serve] plain loop capacity ~{cap:.0f} req/s")
    rows = []
    for f in a.serve_loads:
        row = w.load_row(f * cap, a.serve_requests)
        log(f"[serve] load {f:.2f}: {row}")
        rows.append(row)
    # outside the timed runs: a burst of overlapping requests through the
    # server at full size, each image against its one-view call
    burst = serve_trace(64, 1e9, gen.CONFIG_SEEDS[5] + 1, len(pts))
    srv = rz.Server(a.serve_budget, streams=a.serve_streams, merge_views=a.serve_merge)
    ids = [srv.add_cloud(p) for p in pts]
    outs = []
    for _, c, v, m in burst:
        img = torch.empty(v.width * v.height, dtype=torch.int32, device="cuda")
        outs.append((srv.submit(ids[c], v, m, img=img), img))
    srv.drain(600)
    same = all(srv.poll(t)["state"] == rz.RZ_REQ_DONE for t, _ in outs)
    srv.close()
    for (_, c, v, m), (_, img) in zip(burst, outs):
        ref = torch.empty_like(img)
        plain_one(c, v, m, ref)
        torch.cuda.synchronize()
        same = same and torch.equal(img, ref)
    log(f"[serve] burst of {len(burst)} overlapping requests identical to one-view calls: {same}")
    if not same:
        raise SystemExit("served images differ from the one-view calls")
    del outs
    top = rows[-1]
    out = {
        "metric": METRIC, "value": top["server"]["gpts"], "unit": "Gpoints/s", "n_gpus": 1,
        "steps": a.serve_requests, "warmup": 0,
        "ms_per_step": round(1e3 / top["server"]["req_s"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64->u64", "data": "synthetic",
        "config": {"workload": f"serving: {len(pts)} resident clouds "
                               f"({', '.join(f'{n // 1_000_000}M' for n in npts)} points), Poisson "
                               f"arrivals, resolutions {gen.SERVE_SIZES}, methods 50/50, "
                               f"framebuffer budget {a.serve_budget >> 20} MiB, "
                               f"{a.serve_streams} streams",
                   "requests_per_rate": a.serve_requests, "plain_capacity_req_s": round(cap, 1),
                   "server_work_cap": w.work_cap()},
        "detail": {"rates": rows,
                   "p50_ms": top["server"]["p50_ms"], "p99_ms": top["server"]["p99_ms"],
                   "plain_p50_ms": top["plain"]["p50_ms"], "plain_p99_ms": top["plain"]["p99_ms"],
                   "throughput_vs_plain": round(top["server"]["req_s"] / top["plain"]["req_s"], 3),
                   "burst_identical_to_one_view_calls": len(burst)},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="terrain50m")
    ap.add_argument("--path", choices=("direct", "sorted"), default="direct",
                    help="direct: one atomic per fragment; sorted: screen-tile sort first")
    ap.add_argument("--point-size", type=int, default=1,
                    help="points of k x k pixels (direct path)")
    ap.add_argument("--flush-mall", action="store_true",
                    help="also time steps with a 1 GiB device fill before each (cold caches)")
    ap.add_argument("--shards", type=int, default=0,
                    help="also time one device's share of a sort-last split into G parts: "
                         "its depth pass (N/G points, full framebuffer) and the merge kernels")
    ap.add_argument("--depth", choices=("linear", "gl24", "f32rev"), default="linear",
                    help="depth encoding; gl24 and f32rev have no splat frame")
    ap.add_argument("--settle-ms", type=float, default=100.0,
                    help="before the warm-up steps, run the step untimed for this long (ms of "
                         "wall time), so that the GPU has left the idle clock it drops to "
                         "while the host generates the inputs; reported as detail.settle "
                         "(0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the stress, serving and viewpoint legs")
    ap.add_argument("--extras-budget", type=float, default=270.0,
                    help="seconds from the start of the run after which no further extra "
                         "leg starts (each leg is skipped, and named, when it would not fit)")
    ap.add_argument("--batch-points", type=int, default=100_000_000)
    ap.add_argument("--batch-views", type=int, default=64)
    ap.add_argument("--batch-k", type=int, default=0,
                    help="batch64: a fixed group size K, no graph and no autotuning "
                         "(for counter runs, which count every dispatch on its own)")
    ap.add_argument("--batch-launch", type=int, nargs=5, default=None,
                    metavar=("BLOCK", "PPT", "EARLY", "XCD", "BIN"),
                    help="with --batch-k: the launch shape of both passes of the batch")
    ap.add_argument("--serve-clouds", type=int, default=8)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-budget", type=int, default=4 << 30)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-ring", type=int, default=96)
    ap.add_argument("--serve-work-cap", type=int, default=-1,
                    help="server work cap in point passes (0: none; default: the work of the "
                         "largest request); see rz_server_opts")
    ap.add_argument("--serve-exclusive", type=int, default=-1,
                    help="server exclusive_work in point passes: requests at least this "
                         "large run alone (0 or default: none)")
    ap.add_argument("--serve-merge", type=int, default=0,
                    help="server merge_views: queued requests of one cloud run as one "
                         "multi-view launch (0: no merging)")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 0.8, 1.0, 1.3, 2.0])
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="after the timed region, copy BYTES between two device buffers "
                         "(a plain copy kernel of known size for scaling HBM counters)")
    a = ap.parse_args()
    a.t_start = time.perf_counter()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the sort-last "
              "composition across GPUs is designed, with its merge kernels timed on one GPU, "
              "but not run across GPUs", file=sys.stderr)
        raise SystemExit(2)

    import torch
    from paper_1908_02681_amd import rz

    assert torch.cuda.is_available(), "bench needs a HIP device"
    if a.workload == "batch64":
        return bench_batch(a)
    if a.workload == "serve":
        return bench_serve(a)
    eps = (1, 100)
    log(f"[bench] generating {a.workload}")
    cloud, view, desc = workload(a.workload)
    n, W, H = cloud.n, view.width, view.height
    npix = W * H
    pts = rz.Points.from_cloud(cloud)
    fb, acc = rz.new_framebuffer(view, 0, hq=True)
    img = torch.empty(npix, dtype=torch.int32, device="cuda")
    himg = torch.empty(npix, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] n={n} {W}x{H} launch={rz.get_launch()}")

    ws = rz.new_workspace(n, W, H) if a.path == "sorted" else None
    kinds = {"linear": rz.DEPTH_LINEAR, "gl24": rz.DEPTH_GL24, "f32rev": rz.DEPTH_F32REV}
    depth = (kinds[a.depth], 0.0)
    general = a.point_size > 1 or a.depth != "linear"
    with_hq = a.depth == "linear"
    if general and a.path != "direct":
        raise SystemExit("--point-size and --depth apply to the direct path")

    def step_general(ev):
        # the same two frames through rasterize_points (k x k points, any
        # depth encoding; the float encodings have no splat frame)
        if ev:
            ev[0].record()
        rz.rasterize_points(pts, view, depth, point_size=a.point_size, fb=fb, keep_keys=True)
        if ev:
            ev[1].record()
        rz.resolve_min(fb, npix, 0, img)
        if ev:
            ev[2].record()
        if with_hq:
            rz.rasterize_points(pts, view, depth, True, eps, a.point_size, fb=fb, acc=acc,
                                keep_keys=True)
        if ev:
            ev[3].record()
            ev[4].record()
        if with_hq:
            rz.resolve_hq(fb, acc, npix, 0, himg, status)
        if ev:
            ev[5].record()

    def step_sorted(ev):
        # the same two frames through the screen-sorted path (one call each)
        if ev:
            ev[0].record()
        rz.rasterize_sorted(pts, view, fb=fb, workspace=ws, keep_keys=True)
        if ev:
            ev[1].record()
        rz.resolve_min(fb, npix, 0, img)
        if ev:
            ev[2].record()
        rz.rasterize_sorted(pts, view, hq=True, eps=eps, fb=fb, acc=acc, workspace=ws,
                            keep_keys=True)
        if ev:
            ev[3].record()
            ev[4].record()
        rz.resolve_hq(fb, acc, npix, 0, himg, status)
        if ev:
            ev[5].record()

    def step(ev):
        if a.path == "sorted":
            return step_sorted(ev)
        if general:
            return step_general(ev)
        # atomicMin frame: depth pass, then resolve + clear
        if ev:
            ev[0].record()
        rz.rasterize_atomicmin(pts, view, fb=fb, keep_keys=True)
        if ev:
            ev[1].record()
        rz.resolve_min(fb, npix, 0, img)
        if ev:
            ev[2].record()
        # HQ frame: depth pass, accumulate pass, resolve
        rz.rasterize_atomicmin(pts, view, fb=fb, keep_keys=True)
        if ev:
            ev[3].record()
        rz.hq_accumulate(pts, view, fb, acc, eps=eps)
        if ev:
            ev[4].record()
        rz.resolve_hq(fb, acc, npix, 0, himg, status)
        if ev:
            ev[5].record()

    settled = settle(lambda: step(None), a.settle_ms)
    for _ in range(a.warmup):
        step(None)
    torch.cuda.synchronize()

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for k in range(a.steps):
        step(events[k])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    sums = np.zeros(5)
    for ev in events:
        sums += [ev[i].elapsed_time(ev[i + 1]) for i in range(5)]
    ms_per_step = (t3 - t2) * 1e3 / a.steps
    avg = sums / a.steps   # ms: raster(min), resolve_min, raster(hq), accum, resolve_hq
    if int(status.item()) != 0:
        raise SystemExit("splat count overflow reported")

    if general:
        kern = {
            "rasterize_points(atomicMin)": {"ms": avg[0], "bytes": 16 * n, "launches_per_step": 1},
            "k_resolve_min": {"ms": avg[1], "bytes": 20 * npix, "launches_per_step": 1},
        }
        if with_hq:
            kern["rasterize_points(HQ)"] = {"ms": avg[2], "bytes": 32 * n, "launches_per_step": 1}
            kern["k_resolve_hq"] = {"ms": avg[4], "bytes": 44 * npix, "launches_per_step": 1}
    elif a.path == "sorted":
        # whole calls, against the algorithmic bytes of the method (16 B per
        # point for the depth pass, 32 for the splat frame's two passes);
        # the sort's own traffic (count pass 12 B/pt, scatter 16 + 10, tile
        # minimum 10, splat sums 10) is reported beside it
        kern = {
            "rasterize_sorted(atomicMin)": {"ms": avg[0], "bytes": 16 * n,
                                            "sort_traffic_bytes": 48 * n,
                                            "launches_per_step": 1},
            "rasterize_sorted(HQ)": {"ms": avg[2], "bytes": 32 * n,
                                     "sort_traffic_bytes": 58 * n, "launches_per_step": 1},
            "k_resolve_min": {"ms": avg[1], "bytes": 20 * npix, "launches_per_step": 1},
            "k_resolve_hq": {"ms": avg[4], "bytes": 44 * npix, "launches_per_step": 1},
        }
    else:
        kern = {
            "k_raster_min": {"ms": (avg[0] + avg[2]) / 2, "bytes": 16 * n,
                             "launches_per_step": 2},
            "k_hq_accum": {"ms": avg[3], "bytes": 16 * n, "launches_per_step": 1},
            "k_resolve_min": {"ms": avg[1], "bytes": 20 * npix, "launches_per_step": 1},
            "k_resolve_hq": {"ms": avg[4], "bytes": 44 * npix, "launches_per_step": 1},
        }
    for k in kern.values():
        k["GBps"] = k["bytes"] / (k["ms"] * 1e-3) / 1e9
        if "sort_traffic_bytes" in k:
            k["sort_traffic_GBps"] = k["sort_traffic_bytes"] / (k["ms"] * 1e-3) / 1e9
    dom = max(kern, key=lambda k: kern[k]["ms"] * kern[k]["launches_per_step"])
    dk = kern[dom]
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            tr = json.load(f)
        rec = tr.get(a.workload if a.path == "direct" else f"{a.workload}:{a.path}", {}).get(dom)
        if rec and rec.get("source_hash") == kernel_source_hash(a.path):
            traffic = rec["bytes_per_launch"]
    # VALU issue of the dominant kernel: lane instructions per point from the
    # recorded counter pass (profiles/valu_terrain50m.md), rate from this run
    valu = None
    vfile = os.path.join(ROOT, "profiles", "valu_issue.json")
    if os.path.exists(vfile) and a.path == "direct" and not general:
        with open(vfile) as f:
            vrec = json.load(f).get(a.workload, {}).get(dom)
        if vrec and vrec.get("source_hash") == kernel_source_hash("direct"):
            rate = vrec["lane_instr_per_point"] * n / (dk["ms"] * 1e-3)
            valu = {"lane_instr_per_point": vrec["lane_instr_per_point"],
                    "achieved_T_per_s": round(rate / 1e12, 2),
                    "peak_T_per_s": VALU_ISSUE_PEAK / 1e12,
                    "frac": round(rate / VALU_ISSUE_PEAK, 4)}
    out = {
        "metric": METRIC,
        "value": round((2 if with_hq else 1) * n / (ms_per_step * 1e-3) / 1e9, 4),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64->u64",
        "data": "synthetic",
        "config": {"workload": desc, "points": n, "width": W, "height": H,
                   "eps": f"{eps[0]}/{eps[1]}",
                   "depth_map": {"linear": "linear 40-bit", "gl24": "24-bit window depth",
                                 "f32rev": "reversed float32 depth"}[a.depth],
                   "point_size": a.point_size, "path": a.path},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": round(dk["GBps"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dk["GBps"] / HBM_PEAK_GBS, 4), "traffic": traffic},
        "detail": {
            "atomicmin_gpts": round(n / ((avg[0] + avg[1]) * 1e-3) / 1e9, 3),
            "hq_gpts": (round(n / ((avg[2] + avg[3] + avg[4]) * 1e-3) / 1e9, 3)
                        if with_hq else None),
            "kernels_ms": {k: round(v["ms"], 4) for k, v in kern.items()},
            "kernels_GBps": {k: round(v["GBps"], 1) for k, v in kern.items()},
            "sort_traffic_GBps": {k: round(v["sort_traffic_GBps"], 1) for k, v in kern.items()
                                  if "sort_traffic_GBps" in v} or None,
            "evented_ms_per_step": round(float(avg.sum()), 4),
            "valu_issue": valu,
            "launch": rz.get_launch(),
            # untimed steps run before the warm-up steps (see settle)
            "settle": settled,
        },
    }
    if a.shards > 1:
        out["detail"]["sort_last"] = time_sort_last(rz, pts, view, a.shards, a.steps)
    if a.flush_mall:
        # the same steps, each after a 1 GiB fill that evicts L2 and the
        # 256 MB infinity cache; only the evented kernel time counts
        junk = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        fl = np.zeros(5)
        for k in range(a.steps):
            junk.fill_(k)
            torch.cuda.synchronize()
            step(events[k])
            torch.cuda.synchronize()
            fl += [events[k][i].elapsed_time(events[k][i + 1]) for i in range(5)]
        fl /= a.steps
        del junk
        out["detail"]["mall_flushed"] = {
            "evented_ms_per_step": round(float(fl.sum()), 4),
            "atomicmin_frame_ms": round(fl[0] + fl[1], 4),
            "hq_frame_ms": round(fl[2] + fl[3] + fl[4], 4) if with_hq else None}
    if a.calibrate_copy:
        calibration_copy(a.calibrate_copy)
    extras = (a.workload == "terrain50m" and a.path == "direct" and a.point_size == 1
              and a.depth == "linear" and not a.no_extras)
    if extras:
        del pts, fb, acc, img, himg, status
        torch.cuda.empty_cache()
        out["detail"].update(extra_legs(a))
    if not a.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(cloud, view, eps)
    print(json.dumps(out), flush=True)


def frame_times(rz, pts, view, path, steps, warmup, ws=None, settle_ms=0.0):
    """Median event times (ms) of one atomicMin frame and one HQ frame
    (depth pass, accumulate, resolve) over `steps` runs, each kind after
    settle_ms of untimed frames (see settle)."""
    import torch
    npix = view.width * view.height
    fb, acc = rz.new_framebuffer(view, 0, hq=True)
    img = torch.empty(npix, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = {}
    for hq in (False, True):
        def one(ev=None):
            if ev:
                ev[0].record()
            if path == "sorted":
                rz.rasterize_sorted(pts, view, hq=hq, fb=fb, acc=acc, img=img, status=st,
                                    workspace=ws)
            elif hq:
                rz.rasterize_hq_splat(pts, view, fb=fb, acc=acc, img=img, status=st)
            else:
                rz.rasterize_atomicmin(pts, view, fb=fb, img=img)
            if ev:
                ev[1].record()
        settle(one, settle_ms)
        for _ in range(warmup):
            one()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
        for e in evs:
            one(e)
        torch.cuda.synchronize()
        t = sorted(e[0].elapsed_time(e[1]) for e in evs)
        out["hq" if hq else "atomicmin"] = t[len(t) // 2]
    if int(st.item()) != 0:
        raise SystemExit("splat count overflow reported")
    return out


def extra_legs(a):
    """The rest of the metric on the default run, each leg started only while
    the run's wall clock allows it: the 300M-point stress cloud (Morton order
    by the direct path; shuffled by the best path per frame) at 2560x1440,
    the serving workload at 0.5, 0.8 and 1.0 times the plain loop's
    capacity, and the one-view calls of both methods on each of the 64 orbit
    cameras of the batched workload (viewpoint sensitivity)."""
    import torch
    from paper_1908_02681_amd import gen, rz
    detail, skipped = {}, []

    def left():
        return a.extras_budget - (time.perf_counter() - a.t_start)

    stress = None
    if left() > 90:
        log("[extras] generating the 300M-point stress cloud")
        stress, views = gen.config3()
        view = views[0]
        n = stress.n
        pts = rz.Points.from_cloud(stress)
        mort = frame_times(rz, pts, view, "direct", 10, 3, settle_ms=a.settle_ms)
        del pts
        torch.cuda.empty_cache()
        sh = gen.shuffle(stress, 3)
        pts = rz.Points.from_cloud(sh)
        del sh
        ws = rz.new_workspace(n, view.width, view.height)
        direct = frame_times(rz, pts, view, "direct", 5, 2, settle_ms=a.settle_ms)
        srt = frame_times(rz, pts, view, "sorted", 10, 3, ws, settle_ms=a.settle_ms)
        del pts, ws
        torch.cuda.empty_cache()
        best = {k: min(direct[k], srt[k]) for k in direct}
        bpath = {k: "sorted" if srt[k] <= direct[k] else "direct" for k in direct}

        def leg(t):
            return {"atomicmin_ms": round(t["atomicmin"], 4), "hq_ms": round(t["hq"], 4),
                    "atomicmin_gpts": round(n / t["atomicmin"] / 1e6, 2),
                    "hq_gpts": round(n / t["hq"] / 1e6, 2),
                    "atomicmin_hbm_frac": round(16 * n / (t["atomicmin"] * 1e-3) / 8e12, 4),
                    "hq_hbm_frac": round(32 * n / (t["hq"] * 1e-3) / 8e12, 4)}
        detail["stress300m"] = {
            "workload": f"stress 300M points (250M terrain + 20 spheres of 2.5M), "
                        f"{view.width}x{view.height}",
            "morton_direct": leg(mort),
            "shuffled_best": {**leg(best), "path": bpath},
            "shuffled_direct": leg(direct), "shuffled_sorted": leg(srt)}
        log(f"[extras] stress300m: {detail['stress300m']}")
    else:
        skipped.append("stress300m")

    if left() > 90:
        w = ServingWorld(a, clouds={7: stress} if stress is not None else None,
                         log_prefix="[extras]")
        stress = None
        cap = w.capacity()
        rows = [w.load_row(f * cap, 500) for f in (0.5, 0.8, 1.0)]
        detail["served"] = {
            "workload": f"{len(w.pts)} resident clouds "
                        f"({', '.join(f'{n // 1_000_000}M' for n in w.npts)} points), Poisson "
                        f"arrivals, resolutions 256x256 to 2560x1440, methods 50/50, "
                        f"{a.serve_budget >> 20} MiB framebuffer budget, {a.serve_streams} streams",
            "server_work_cap": w.work_cap(),
            "plain_capacity_req_s": round(cap, 1),
            "loads": rows}
        log(f"[extras] served: {detail['served']}")
        del w
        torch.cuda.empty_cache()
    else:
        skipped.append("served")
    stress = None

    if left() > 30:
        log("[extras] viewpoints: generating the 100M-point terrain")
        cloud = gen.terrain(100_000_000, gen.CONFIG_SEEDS[4])
        views = gen.orbit_views(64, gen.CONFIG_SEEDS[4], BATCH_SIZES)
        pts = rz.Points.from_cloud(cloud)
        n = cloud.n
        del cloud
        rates = {"atomicmin": [], "hq": []}
        for i, v in enumerate(views):   # the views follow each other: one settle
            t = frame_times(rz, pts, v, "direct", 3, 1, settle_ms=a.settle_ms if i == 0 else 0)
            for k in rates:
                rates[k].append(n / t[k] / 1e6)
        del pts
        torch.cuda.empty_cache()
        detail["viewpoints"] = {
            "workload": "terrain 100M points (Morton order), 64 orbit cameras (radius 600-1200 m, "
                        "elevation 20-60 deg, 256x256 to 1920x1080), one-view calls",
            **{k: {"min_gpts": round(min(r), 2), "median_gpts": round(float(np.median(r)), 2),
                   "max_gpts": round(max(r), 2)} for k, r in rates.items()}}
        log(f"[extras] viewpoints: {detail['viewpoints']}")
    else:
        skipped.append("viewpoints")
    detail["extras_skipped"] = skipped
    detail["extras_wall_s"] = round(time.perf_counter() - a.t_start, 1)
    return detail


def time_sort_last(rz, pts, view, G, steps):
    """One device's share of a G-way sort-last split: the depth pass of its
    N/G points into a full framebuffer, and the per-pixel merges that a
    reduction of the framebuffers applies (timed locally; no transfer)."""
    import torch
    n, npix = pts.n, view.width * view.height
    share = (n // G) // 4 * 4                      # keep the planes 16-byte aligned
    part = rz.Points(pts.x[:share], pts.y[:share], pts.z[:share], pts.rgb[:share])
    fb, _ = rz.new_framebuffer(view, 0)
    other, _ = rz.new_framebuffer(view, 0)
    rz.rasterize_atomicmin(pts, view, fb=other, keep_keys=True)
    acc = torch.zeros(2 * npix, dtype=torch.int64, device="cuda")
    acc2 = torch.ones(2 * npix, dtype=torch.int64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t = np.zeros(3)
    for _ in range(steps):
        rz.clear(fb, None, npix)
        ev[0].record()
        rz.rasterize_atomicmin(part, view, fb=fb, keep_keys=True)
        ev[1].record()
        rz.merge_min(fb, other, npix)
        ev[2].record()
        rz.merge_sum(acc, acc2, npix)
        ev[3].record()
        torch.cuda.synchronize()
        t += [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    t /= steps
    return {"shards": G, "points_per_shard": share,
            "local_depth_pass_ms": round(t[0], 4),
            "local_depth_pass_GBps": round(16 * share / (t[0] * 1e-3) / 1e9, 1),
            "merge_min_ms": round(t[1], 4),
            "merge_min_GBps": round(24 * npix / (t[1] * 1e-3) / 1e9, 1),
            "merge_sum_ms": round(t[2], 4),
            "merge_sum_GBps": round(48 * npix / (t[2] * 1e-3) / 1e9, 1)}


KERNEL_SOURCES = {
    "direct": ("rz_kernels.hip", "rz_device.h", "rz_internal.h", "rz_api.cpp"),
    "sorted": ("rz_sorted.hip", "rz_device.h", "rz_internal.h", "rz_api.cpp"),
    "general": ("rz_general.hip", "rz_kernels.hip", "rz_device.h", "rz_internal.h",
                "rz_api.cpp"),
    "merge": ("rz_merge.hip", "rz_kernels.hip", "rz_device.h", "rz_internal.h", "rz_api.cpp"),
}


def code_tokens(text):
    """C++ source without comments and with whitespace runs collapsed: edits
    to comments or layout leave a recorded measurement valid."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(path="direct"):
    """Hash of the code the measured kernels are built from: recorded HBM
    traffic and instruction counts are reported only while it still matches."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1908_02681_amd", "csrc")
    for f in KERNEL_SOURCES[path]:
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            h.update(code_tokens(fh.read()).encode())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
