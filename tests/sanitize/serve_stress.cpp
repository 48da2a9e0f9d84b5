// Host-only checks built with a thread or an address and undefined-behaviour
// sanitizer by tests/test_sanitizers.py.
//  1. Argument validation of the one-view entry points (every depth map,
//     the piecewise tables at their limits): each call must return its
//     documented code before touching a device.
//  2. The render server's scheduler in its dry-run mode (no device work):
//     several threads submit, poll and read statistics at once while the
//     scheduler admits (merging queued requests of one cloud) and completes
//     requests; then drain, a destroy that times out while work is queued,
//     and a final destroy.
//  3. The batch autotune cache's file handling (stores and lookups from
//     several threads, malformed lines, bad keys) and the point-order
//     classifier on ragged, NaN-laden and empty inputs.
// The kernel launchers are stubs: none of these calls reaches a launch.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <unistd.h>

#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include "rz.h"
#include "rz_internal.h"

namespace rz {
hipError_t launch_raster_min(const Pts &, const Proj &, uint64_t *, const Tune &, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_hq_accum(const Pts &, const Proj &, uint32_t, uint32_t, const uint64_t *,
                           uint64_t *, const Tune &, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_resolve_min(uint64_t *, int64_t, uint32_t, uint32_t *, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_resolve_hq(uint64_t *, uint64_t *, int64_t, uint32_t, uint32_t *, uint32_t *,
                             hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_clear(uint64_t *, uint64_t *, int64_t, uint32_t, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_raster_points(const Pts &, const Proj &, int32_t, uint64_t *, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_hq_points(const Pts &, const Proj &, int32_t, uint32_t, uint32_t,
                            const uint64_t *, uint64_t *, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_multiview(bool, bool, const Pts &, const MvView *, int32_t, const Tune &,
                            hipStream_t)
{
    return hipErrorInvalidValue;
}
}  // namespace rz

static rz_request make_request(int32_t cloud, int32_t mode, int32_t w, int32_t h, uint32_t flags)
{
    rz_request r = {};
    r.cloud = cloud;
    r.mode = mode;
    for (int i = 0; i < 16; ++i)
        r.view.vp[i] = (i % 5 == 0) ? 1.0 : 0.0;   // identity: w = 1
    r.view.near_ = 0.5;
    r.view.far_ = 2.0;
    r.view.width = w;
    r.view.height = h;
    r.depth.kind = RZ_DEPTH_LINEAR;
    r.flags = flags;
    return r;
}

// Every call here must fail validation with the given code.
static int api_checks()
{
    int bad = 0;
    rz_points pts = {(const float *)16, (const float *)16, (const float *)16,
                     (const uint32_t *)16, 10};
    rz_request base = make_request(0, 0, 64, 48, 0);
    rz_view v = base.view;
    rz_depth_map dm = base.depth;
    uint64_t *fb = (uint64_t *)16;
    uint32_t *img = (uint32_t *)16;
    auto expect = [&](int got, int want) { bad += got != want; };
    expect(rasterize_atomicmin(nullptr, &v, &dm, 0, fb, img, 0, nullptr), RZ_EINVAL);
    expect(rasterize_atomicmin(&pts, nullptr, &dm, 0, fb, img, 0, nullptr), RZ_EINVAL);
    expect(rasterize_atomicmin(&pts, &v, &dm, 0, nullptr, img, 0, nullptr), RZ_EINVAL);
    expect(rasterize_atomicmin(&pts, &v, &dm, 0, fb, nullptr, 0, nullptr), RZ_EINVAL);
    rz_view far_view = v;
    far_view.far_ = 2e9;
    rz_depth_map mm = dm;
    mm.kind = RZ_DEPTH_SCALE;
    mm.scale = 1000.0;
    expect(rasterize_atomicmin(&pts, &far_view, &mm, 0, fb, img, 0, nullptr), RZ_EDEPTHRANGE);
    // piecewise tables: all RZ_MAX_RANGES ranges, then one range too many
    rz_depth_map pw = dm;
    pw.kind = RZ_DEPTH_PIECEWISE;
    pw.nranges = RZ_MAX_RANGES;
    for (int k = 0; k < RZ_MAX_RANGES; ++k) {
        pw.range_start[k] = k == 0 ? 0.0 : 0.25 * k;
        pw.range_scale[k] = 1.0e6;
    }
    expect(rasterize_atomicmin(&pts, &v, &pw, 0, fb, nullptr, 0, nullptr), RZ_EINVAL);
    pw.nranges = RZ_MAX_RANGES + 1;
    expect(rasterize_atomicmin(&pts, &v, &pw, 0, fb, img, 0, nullptr), RZ_EINVAL);
    rz_hq_params hq = {1, 0};
    expect(rasterize_hq_splat(&pts, &v, &dm, &hq, 0, fb, fb, img, (uint32_t *)16, 0, nullptr),
           RZ_EINVAL);
    hq.eps_den = 100;
    expect(rasterize_hq_splat(&pts, &v, &dm, &hq, 0, fb, fb, img, nullptr, 0, nullptr),
           RZ_EINVAL);
    expect(rasterize_points(&pts, &v, &dm, &hq, 17, 0, fb, fb, img, (uint32_t *)16, 0, nullptr),
           RZ_EINVAL);
    rz_depth_map gl = dm;
    gl.kind = RZ_DEPTH_GL24;
    expect(rasterize_points(&pts, &v, &gl, &hq, 1, 0, fb, fb, img, (uint32_t *)16, 0, nullptr),
           RZ_EINVAL);
    expect(rz_clear(nullptr, nullptr, 5, 0, nullptr), RZ_EINVAL);
    expect(rz_resolve_hq(fb, fb, 4, 0, img, nullptr, nullptr), RZ_EINVAL);
    rz_launch l = {96, 8, 1, 0, 2};
    expect(rz_set_launch(&l), RZ_EINVAL);
    return bad;
}

// The autotune cache and the order classifier (host code of rz_tune.cpp).
static int tune_checks()
{
    int bad = 0;
    char path[64];
    snprintf(path, sizeof(path), "/tmp/rz_tune_sanitize_%d.txt", (int)getpid());
    unlink(path);
    rz_tune_entry e = {};
    e.views_per_group = 4;
    e.depth = {64, 16, 1, 0, 2};
    e.accum = {128, 8, 1, 0, 3};
    e.ms = 1.5f;
    std::vector<std::thread> th;
    std::atomic<int> errs{0};
    for (int t = 0; t < 4; ++t) {
        th.emplace_back([&, t] {
            for (int i = 0; i < 20; ++i) {
                char key[96];
                snprintf(key, sizeof(key), "gfx950 n%d px%d v8 hq2 ordered", t, i);
                rz_tune_entry x = e;
                x.ms = (float)(t * 100 + i);
                rz_tune_entry got = {};
                if (rz_tune_cache_store(path, key, &x) != RZ_OK ||
                    rz_tune_cache_lookup(path, key, &got) != 1 || got.ms != x.ms)
                    errs++;
            }
        });
    }
    for (auto &x : th)
        x.join();
    bad += errs.load();
    FILE *f = fopen(path, "a");
    if (f) {
        fputs("gfx950 n1 px1 v8 hq2 ordered k=4 block=64\n", f);
        fputs("gfx950 n1 px1 v8 hq2 ordered k=99 block=64 ppt=16 early_out=1 xcd=0 bin=2 "
              "hq_block=64 hq_ppt=16 hq_early_out=1 hq_xcd=0 hq_bin=2 ms=1\n", f);
        fputs(std::string(5000, 'x').c_str(), f);
        fputs("\n\n#\n= = = = = = =\n", f);
        fclose(f);
    }
    rz_tune_entry got = {};
    if (rz_tune_cache_lookup(path, "gfx950 n1 px1 v8 hq2 ordered", &got) != 1 ||
        got.ms != 101.0f)
        bad++;
    if (rz_tune_cache_store(path, "bad key", &e) != RZ_EINVAL ||
        rz_tune_cache_lookup(path, " a b c d e f", &got) != RZ_EINVAL ||
        rz_tune_cache_lookup(nullptr, "a b c d e f", &got) != RZ_EINVAL)
        bad++;
    unlink(path);
    // order classes: a line, a shuffled line, NaNs, tiny and empty inputs
    const int n = 20000;
    std::vector<float> x(n), y(n), z(n);
    for (int i = 0; i < n; ++i) {
        x[i] = (float)i;
        y[i] = 0.5f * (float)i;
        z[i] = 0.f;
    }
    if (rz_order_class_host(x.data(), y.data(), z.data(), n) != 0)
        bad++;
    srand(7);
    for (int i = n - 1; i > 0; --i) {
        const int j = rand() % (i + 1);
        std::swap(x[i], x[j]);
        std::swap(y[i], y[j]);
    }
    if (rz_order_class_host(x.data(), y.data(), z.data(), n) != 1)
        bad++;
    for (int i = 0; i < n; i += 3)
        x[i] = NAN;
    (void)rz_order_class_host(x.data(), y.data(), z.data(), n);
    (void)rz_order_class_host(x.data(), y.data(), z.data(), 17);
    if (rz_order_class_host(nullptr, nullptr, nullptr, 0) != 1 ||
        rz_order_class_host(nullptr, y.data(), z.data(), 5) != RZ_EINVAL)
        bad++;
    return bad;
}

// argv[1]: the server's merge_views (default 4); with 0, requests held back
// by the work cap or an exclusive request are chained behind running ones
int main(int argc, char **argv)
{
    if (api_checks())
        return 6;
    if (tune_checks())
        return 7;
    rz_server_opts o = {};
    o.budget_bytes = 8u << 20;
    o.streams = 4;
    o.max_inflight = 6;
    o.dry_run = 1;
    o.dry_run_us = 300;
    o.work_cap = 5000;
    o.merge_views = argc > 1 ? atoi(argv[1]) : 4;
    o.exclusive_work = 3000;
    rz_server *s = nullptr;
    if (rz_server_create(&o, &s) != RZ_OK)
        return 1;
    int32_t ids[2];
    rz_points big = {(const float *)16, (const float *)16, (const float *)16,
                     (const uint32_t *)16, 3000};
    rz_points small = big;
    small.n = 50;
    if (rz_server_add_cloud(s, &big, &ids[0]) || rz_server_add_cloud(s, &small, &ids[1]))
        return 2;
    constexpr int kThreads = 4, kPer = 150;
    std::atomic<int> bad{0}, done{0};
    std::vector<std::vector<uint64_t>> tickets(kThreads);
    std::vector<std::thread> th;
    for (int t = 0; t < kThreads; ++t) {
        th.emplace_back([&, t] {
            for (int i = 0; i < kPer; ++i) {
                const int32_t sz = 16 + ((i * 7 + t) % 5) * 64;
                const uint32_t fl = (i % 37 == 5) ? RZ_REQ_INJECT_FAILURE : 0u;
                rz_request r = make_request(ids[(i + t) % 2], (i + t) % 2, sz, sz, fl);
                uint64_t k = 0;
                if (rz_server_submit(s, &r, &k) != RZ_OK)
                    bad++;
                tickets[t].push_back(k);
            }
        });
    }
    std::thread stats([&] {
        while (done.load() < kThreads * kPer) {
            rz_server_stats st;
            if (rz_server_get_stats(s, &st) != RZ_OK)
                bad++;
            std::this_thread::yield();
        }
    });
    for (auto &x : th)
        x.join();
    // poll from two threads until every ticket has been reported finished
    std::vector<std::thread> pollers;
    for (int p = 0; p < 2; ++p) {
        pollers.emplace_back([&, p] {
            for (int t = p; t < kThreads; t += 2) {
                for (uint64_t k : tickets[t]) {
                    for (;;) {
                        rz_request_status st;
                        if (rz_server_poll(s, k, &st) != RZ_OK) {
                            bad++;
                            break;
                        }
                        if (st.state == RZ_REQ_DONE || st.state == RZ_REQ_FAILED) {
                            done++;
                            break;
                        }
                        std::this_thread::yield();
                    }
                }
            }
        });
    }
    for (auto &x : pollers)
        x.join();
    stats.join();
    if (rz_server_drain(s, 30.0) != RZ_OK)
        return 3;
    rz_server_stats fin;
    const bool got = rz_server_get_stats(s, &fin) == RZ_OK;
    const uint64_t merged = got ? fin.merged_requests : 0;
    const uint64_t chained = got ? fin.chained_requests : 0;
    // a destroy that cannot finish in time leaves the server usable
    rz_request r = make_request(ids[0], 1, 64, 64, 0);
    uint64_t k = 0;
    rz_server_opts slow = o;
    (void)slow;
    for (int i = 0; i < 8; ++i)
        if (rz_server_submit(s, &r, &k) != RZ_OK)
            bad++;
    const int early = rz_server_destroy(s, 0.0);
    if (early != RZ_OK && early != RZ_ESTATE)
        bad++;
    if (early == RZ_ESTATE && rz_server_destroy(s, 30.0) != RZ_OK)
        return 4;
    printf("served %d requests, %d errors\n", done.load(), bad.load());
    printf("merged %llu requests\n", (unsigned long long)merged);
    printf("chained %llu requests\n", (unsigned long long)chained);
    return bad.load() == 0 && done.load() == kThreads * kPer ? 0 : 5;
}
