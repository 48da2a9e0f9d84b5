"""Render-server scheduling on the host (dry-run backend: no device work):
admission by memory budget and in-flight slots, arrival order, continuous
admission as memory frees up, error isolation of failed requests, the work
cap and the merging of queued requests of one cloud."""
import time

import numpy as np
import pytest


@pytest.fixture(scope="module")
def rz():
    import os
    from paper_1908_02681_amd import build, rz as binding
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    binding.load()
    return binding


class _View:
    def __init__(self, w, h):
        self.vp = np.eye(4)
        self.vp[3] = [0, 0, 0, 1]
        self.near, self.far, self.width, self.height = 0.5, 2.0, w, h


def _server(rz, budget, us, streams=2, inflight=0):
    s = rz.Server(budget, streams=streams, max_inflight=inflight, dry_run=True, dry_run_us=us)
    cid = s.add_cloud(rz.rz_points(1, 1, 1, 1, 1000))
    return s, cid


def _wait(s, tickets, timeout=20.0):
    s.drain(timeout)
    return [s.poll(t) for t in tickets]


def _fb_bytes(w, h, hq):
    a = lambda v: (v + 255) // 256 * 256
    return a(8 * w * h) + (a(16 * w * h) if hq else 0) + 256


def test_budget_admits_one_at_a_time(rz):
    need = _fb_bytes(640, 480, False)
    s, cid = _server(rz, need + need // 2, 3000)
    ts = [s.submit(cid, _View(640, 480), 0) for _ in range(5)]
    st = _wait(s, ts)
    assert all(x["state"] == rz.RZ_REQ_DONE and x["error"] == 0 for x in st)
    stats = s.stats()
    assert stats["peak_inflight"] == 1 and stats["completed"] == 5
    assert stats["peak_bytes"] == need
    # arrival order, and each admitted only once the previous one finished
    for a, b in zip(st, st[1:]):
        assert b["t_admit_us"] >= a["t_done_us"] - 1.0
        assert b["t_admit_us"] >= a["t_admit_us"]
    for x in st:
        assert x["t_done_us"] - x["t_admit_us"] >= 3000 * 0.95
    s.close()


def test_slots_bound_concurrency(rz):
    s, cid = _server(rz, 512 << 20, 5000, streams=2, inflight=3)
    ts = [s.submit(cid, _View(256, 256), i % 2) for i in range(9)]
    st = _wait(s, ts)
    assert all(x["state"] == rz.RZ_REQ_DONE for x in st)
    assert s.stats()["peak_inflight"] == 3
    assert {x["stream"] for x in st} == {0, 1}
    s.close()


def test_continuous_admission_while_others_run(rz):
    """A request that arrives while others run starts as soon as memory
    frees up, not when the whole earlier batch has finished."""
    big = _fb_bytes(1920, 1080, True)
    small = _fb_bytes(256, 256, False)
    s, cid = _server(rz, big + small, 20000, streams=4)
    t_big = s.submit(cid, _View(1920, 1080), 1)
    t_small = [s.submit(cid, _View(256, 256), 0) for _ in range(3)]
    st_small = _wait(s, t_small)
    st_big = s.poll(t_big)
    assert st_big["state"] == rz.RZ_REQ_DONE
    # the first small request ran beside the big one; the remaining memory
    # holds one small framebuffer only, so never more than two at once and
    # never more memory than the budget
    assert st_small[0]["t_admit_us"] < st_big["t_admit_us"] + 5000
    assert st_small[0]["t_admit_us"] < st_big["t_done_us"]
    assert st_small[1]["t_admit_us"] >= min(st_small[0]["t_done_us"], st_big["t_done_us"]) - 1.0
    stats = s.stats()
    assert stats["peak_inflight"] >= 2 and stats["peak_bytes"] == big + small
    s.close()


def test_request_larger_than_budget_is_refused(rz):
    s, cid = _server(rz, 4 << 20, 10)
    with pytest.raises(rz.RzError) as e:
        s.submit(cid, _View(2560, 1440), 1)
    assert e.value.code == rz.RZ_EBUDGET
    with pytest.raises(rz.RzError) as e:
        s.submit(cid + 5, _View(64, 64), 0)
    assert e.value.code == rz.RZ_EINVAL
    with pytest.raises(rz.RzError) as e:
        s.submit(cid, _View(64, 64), 3)
    assert e.value.code == rz.RZ_EINVAL
    s.close()


def test_injected_failure_fails_only_that_request(rz):
    s, cid = _server(rz, 64 << 20, 500)
    inject = [False, True, False, True, False, False]
    ts = [s.submit(cid, _View(320, 240), i % 2, inject_failure=f) for i, f in enumerate(inject)]
    st = _wait(s, ts)
    for x, f in zip(st, inject):
        if f:
            assert x["state"] == rz.RZ_REQ_FAILED and x["error"] == rz.RZ_EHIP
        else:
            assert x["state"] == rz.RZ_REQ_DONE and x["error"] == 0
    stats = s.stats()
    assert stats["failed"] == 2 and stats["completed"] == 4
    assert stats["inflight"] == 0 and stats["queued"] == 0
    # the memory of failed requests came back: a request needing all of it fits
    t = s.submit(cid, _View(1600, 1600), 1)   # 91% of the budget
    assert _wait(s, [t])[0]["state"] == rz.RZ_REQ_DONE
    s.close()


def test_poll_forgets_finished_tickets(rz):
    s, cid = _server(rz, 64 << 20, 100)
    t = s.submit(cid, _View(64, 64), 0)
    s.drain(10)
    assert s.poll(t)["state"] == rz.RZ_REQ_DONE
    with pytest.raises(rz.RzError):
        s.poll(t)
    s.close()


def test_many_requests_from_threads(rz):
    import threading
    s, cid = _server(rz, 64 << 20, 200, streams=4)
    out, lock = [], threading.Lock()

    def worker(k):
        for i in range(50):
            t = s.submit(cid, _View(128 + k, 96), (i + k) % 2)
            with lock:
                out.append(t)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    st = _wait(s, out, timeout=60)
    assert len(set(out)) == 200 and all(x["state"] == rz.RZ_REQ_DONE for x in st)
    s.close()


def test_destroy_times_out_while_requests_run(rz):
    """rz_server_destroy waits at most its timeout: with a request still
    running it returns RZ_ESTATE and leaves the server usable."""
    s, cid = _server(rz, 64 << 20, 400_000)
    t = s.submit(cid, _View(64, 48), 0)
    t0 = time.perf_counter()
    with pytest.raises(rz.RzError) as e:
        s.close(timeout_s=0.05)
    assert e.value.code == rz.RZ_ESTATE
    assert time.perf_counter() - t0 < 0.3
    st = _wait(s, [t])[0]
    assert st["state"] == rz.RZ_REQ_DONE
    s.close(timeout_s=5.0)


def test_scheduler_sleeps_while_waiting(rz):
    """The scheduler blocks between events instead of spinning: a second of
    running requests costs the process far less than a second of CPU time."""
    s, cid = _server(rz, 64 << 20, 250_000, streams=1, inflight=1)
    ts = [s.submit(cid, _View(64, 48), 0) for _ in range(4)]
    c0, w0 = time.process_time(), time.perf_counter()
    st = _wait(s, ts)
    cpu, wall = time.process_time() - c0, time.perf_counter() - w0
    assert all(x["state"] == rz.RZ_REQ_DONE for x in st)
    assert wall > 0.9
    assert cpu < 0.25 * wall, (cpu, wall)
    s.close()


def test_work_cap_keeps_large_requests_apart(rz):
    """With a work cap, two large requests never run together while small
    ones still run beside a large one; arrival order is kept."""
    s = rz.Server(64 << 20, streams=4, dry_run=True, dry_run_us=20_000, work_cap=1200)
    big = s.add_cloud(rz.rz_points(1, 1, 1, 1, 1000))
    small = s.add_cloud(rz.rz_points(1, 1, 1, 1, 10))
    plan = [big, small, small, big, small, big]
    ts = [s.submit(c, _View(32, 32), 0) for c in plan]
    st = _wait(s, ts)
    s.close()
    assert all(x["state"] == rz.RZ_REQ_DONE for x in st)
    # when each request ran: every dry-run request runs 20 ms and ends at
    # t_done (one admitted behind a running request starts when that ends)
    spans = [(x["t_done_us"] - 20_000, x["t_done_us"]) for x in st]
    bigs = [spans[i] for i, c in enumerate(plan) if c == big]
    for (a0, a1), (b0, b1) in zip(bigs, bigs[1:]):
        assert b0 >= a1 - 1.0            # the next large request starts after the last ends
    # the first small requests ran while the first large one did
    assert spans[1][0] < spans[0][1] and spans[2][0] < spans[0][1]
    for a, b in zip(st, st[1:]):
        assert b["t_admit_us"] >= a["t_admit_us"]
    # a splatting request counts its points twice: 2 x 1000 > 1200, yet it
    # runs (alone) rather than waiting forever
    s = rz.Server(64 << 20, streams=2, dry_run=True, dry_run_us=1000, work_cap=1200)
    big = s.add_cloud(rz.rz_points(1, 1, 1, 1, 1000))
    st = _wait(s, [s.submit(big, _View(32, 32), 1) for _ in range(3)])
    s.close()
    assert all(x["state"] == rz.RZ_REQ_DONE for x in st)


def test_merge_groups_requests_of_one_cloud(rz):
    """With merge_views, queued requests of the admitted request's cloud
    join its launch (up to merge_views, never another cloud's, never past
    the work cap); the rest keep arrival order."""
    s = rz.Server(64 << 20, streams=2, max_inflight=8, dry_run=True, dry_run_us=30_000,
                  work_cap=1000, merge_views=4)
    big = s.add_cloud(rz.rz_points(1, 1, 1, 1, 1000))
    small = s.add_cloud(rz.rz_points(1, 1, 1, 1, 10))
    first = s.submit(big, _View(32, 32), 0)      # runs alone: nothing fits beside it
    time.sleep(0.005)
    plan = [small, big, small, small, big, small, small]
    ts = [s.submit(c, _View(32, 32), i % 2) for i, c in enumerate(plan)]
    st = _wait(s, [first] + ts)
    stats = s.stats()
    s.close()
    assert all(x["state"] == rz.RZ_REQ_DONE for x in st)
    first_st, st = st[0], st[1:]
    assert first_st["group"] == 1
    # the first small request and the next three small ones ran as one launch
    grouped = [0, 2, 3, 5]
    assert all(st[i]["group"] == 4 for i in grouped)
    assert len({st[i]["t_admit_us"] for i in grouped}) == 1
    assert all(st[i]["stream"] == st[0]["stream"] for i in grouped)
    # the large requests ran alone, after the group, in arrival order
    assert st[1]["group"] == 1 and st[4]["group"] == 1
    assert st[1]["t_admit_us"] >= st[0]["t_done_us"] - 1.0
    assert st[4]["t_admit_us"] >= st[1]["t_done_us"] - 1.0
    assert st[6]["group"] == 1
    assert stats["merged_launches"] == 1 and stats["merged_requests"] == 4


def test_merge_leaves_failures_alone(rz):
    """A request with an injected failure is never merged; it fails alone
    and the requests around it complete."""
    s = rz.Server(64 << 20, streams=1, max_inflight=8, dry_run=True, dry_run_us=20_000,
                  work_cap=1000, merge_views=8)
    big = s.add_cloud(rz.rz_points(1, 1, 1, 1, 1000))
    small = s.add_cloud(rz.rz_points(1, 1, 1, 1, 10))
    first = s.submit(big, _View(16, 16), 0)
    time.sleep(0.005)
    ts = [s.submit(small, _View(16, 16), 0, inject_failure=(i == 2)) for i in range(6)]
    st = _wait(s, [first] + ts)[1:]
    s.close()
    assert st[2]["state"] == rz.RZ_REQ_FAILED and st[2]["group"] == 1
    assert all(x["state"] == rz.RZ_REQ_DONE for i, x in enumerate(st) if i != 2)
    assert max(x["group"] for x in st) > 1


@pytest.mark.parametrize("bad", [-1, 9])
def test_merge_views_validation(rz, bad):
    with pytest.raises(rz.RzError):
        rz.Server(64 << 20, dry_run=True, merge_views=bad)


def test_exclusive_requests_run_alone(rz):
    """With exclusive_work, a request at least that large waits for an empty
    device and runs alone; smaller ones still overlap each other; arrival
    order is kept."""
    s = rz.Server(64 << 20, streams=4, max_inflight=8, dry_run=True, dry_run_us=20_000,
                  exclusive_work=1000)
    big = s.add_cloud(rz.rz_points(1, 1, 1, 1, 1000))
    small = s.add_cloud(rz.rz_points(1, 1, 1, 1, 10))
    plan = [small, small, big, small, small, big, small]
    st = _wait(s, [s.submit(c, _View(32, 32), 0) for c in plan])
    stats = s.stats()
    s.close()
    assert all(x["state"] == rz.RZ_REQ_DONE for x in st)
    spans = [(x["t_done_us"] - 20_000, x["t_done_us"]) for x in st]   # when each ran
    for i, c in enumerate(plan):
        if c != big:
            continue
        a0, a1 = spans[i]
        for j, (b0, b1) in enumerate(spans):
            if j != i:   # nothing else ran while it did
                assert b1 <= a0 + 1.0 or b0 >= a1 - 1.0, (i, j)
    # the first two small requests overlapped, and so did the two after the
    # first large one
    assert spans[1][0] < spans[0][1] and spans[4][0] < spans[3][1]
    for a, b in zip(st, st[1:]):
        assert b["t_admit_us"] >= a["t_admit_us"]
    assert stats["peak_inflight"] >= 2


def test_blocked_request_starts_behind_a_running_one(rz):
    """A request held back by the work cap is admitted behind a running
    request at least as large, on its stream: it is admitted at once, runs
    right after it (never beside it) and is counted as chained."""
    s = rz.Server(64 << 20, streams=4, max_inflight=8, dry_run=True, dry_run_us=20_000,
                  work_cap=1000)
    big = s.add_cloud(rz.rz_points(1, 1, 1, 1, 1000))
    small = s.add_cloud(rz.rz_points(1, 1, 1, 1, 10))
    first = s.submit(big, _View(32, 32), 0)
    time.sleep(0.003)
    second = s.submit(big, _View(32, 32), 0)
    third = s.submit(small, _View(32, 32), 0)    # nothing left to go behind: waits
    a, b, c = _wait(s, [first, second, third])
    stats = s.stats()
    s.close()
    assert a["state"] == b["state"] == c["state"] == rz.RZ_REQ_DONE
    assert b["t_admit_us"] < a["t_done_us"]              # admitted while the first ran
    assert b["stream"] == a["stream"]
    assert b["t_done_us"] >= a["t_done_us"] + 20_000 * 0.95   # and ran after it
    assert c["t_done_us"] >= b["t_done_us"] - 20_000 + 20_000 * 0.95 - 1.0
    assert stats["chained_requests"] == 1
