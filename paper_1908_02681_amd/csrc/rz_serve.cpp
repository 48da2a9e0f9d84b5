// Render server (declared in include/rz.h, "serving: continuous batching of
// render requests").
//
// One scheduler thread owns the device work.  Requests wait in a FIFO queue;
// the head is admitted as soon as its framebuffer memory fits the budget
// pool and an in-flight slot is free, then its kernels (clear, depth pass,
// splat accumulate, resolve: the same launchers as the one-view calls) are
// enqueued on the least loaded of several HIP streams, followed by an
// asynchronous copy of its splat status into a pinned host slot and an
// event.  The scheduler polls the events, stamps completion, and returns the
// memory and the slot, which admits the next requests while others still
// run.  A dry-run mode replaces the device by a host timer so that
// admission, budgeting and failure isolation can be tested without a GPU.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rz.h"
#include "rz_internal.h"

namespace rz {

int check_points(const rz_points *p);
int make_proj(const rz_view *v, const rz_depth_map *dm, Proj *P);
int check_hq(const rz_hq_params *hq, const Proj &P, uint32_t *num, uint32_t *den);
int hip_fail(hipError_t e);
Tune current_tune();
Tune current_tune_hq();

namespace {

constexpr uint64_t kAlign = 256;
constexpr int kMaxStreams = 16;

uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator of offsets inside the budget, with coalescing.
struct Pool {
    uint64_t size = 0;
    uint64_t used = 0;
    uint64_t peak = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> length

    void init(uint64_t n)
    {
        size = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(uint64_t n, uint64_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n;
                const uint64_t at = it->first + n;
                free_.erase(it);
                if (rest)
                    free_[at] = rest;
                used += n;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Req {
    uint64_t ticket = 0;
    rz_request r;
    Proj P;
    uint32_t num = 1, den = 100;
    uint64_t npix = 0;
    uint64_t fb_bytes = 0, acc_bytes = 0, bytes = 0, off = 0;
    int32_t state = RZ_REQ_QUEUED;
    int32_t error = RZ_OK;
    int32_t stream = -1;
    int32_t slot = -1;         // pinned status slot
    uint32_t hq_status = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    hipEvent_t ev = nullptr;
};

}  // namespace
}  // namespace rz

using namespace rz;

struct rz_server {
    rz_server_opts o;
    int device = 0;
    std::vector<Pts> clouds;
    char *dmem = nullptr;
    uint32_t *host_status = nullptr;      // pinned, one word per slot
    std::vector<int32_t> free_slots;
    Pool pool;
    std::vector<hipStream_t> streams;
    std::vector<int32_t> load;
    std::vector<hipEvent_t> events;
    std::mutex mu;
    std::condition_variable cv;           // work for the scheduler
    std::condition_variable idle_cv;      // everything finished
    std::deque<Req *> queue;
    std::vector<Req *> inflight;
    std::unordered_map<uint64_t, Req *> tickets;
    uint64_t next_ticket = 1;
    uint64_t submitted = 0, completed = 0, failed = 0;
    int32_t peak_inflight = 0;
    bool stop = false;
    std::thread th;
    std::chrono::steady_clock::time_point t0;

    double now_us() const
    {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
            .count();
    }
};

namespace {

void finish(rz_server *s, Req *r, int32_t state, int32_t error)
{
    r->state = state;
    r->error = error;
    r->t_done = s->now_us();
    if (r->slot >= 0) {
        if (!s->o.dry_run)
            r->hq_status = s->host_status[r->slot];
        s->free_slots.push_back(r->slot);
        r->slot = -1;
    }
    if (r->ev) {
        s->events.push_back(r->ev);
        r->ev = nullptr;
    }
    if (r->stream >= 0)
        s->load[r->stream]--;
    s->pool.release(r->off, r->bytes);
    if (state == RZ_REQ_DONE)
        s->completed++;
    else
        s->failed++;
}

// Enqueues the request's kernels; returns an RZ_* code.
int launch(rz_server *s, Req *r)
{
    hipStream_t st = s->streams[r->stream];
    uint64_t *fb = (uint64_t *)(s->dmem + r->off);
    uint64_t *acc = r->acc_bytes ? (uint64_t *)(s->dmem + r->off + r->fb_bytes) : nullptr;
    uint32_t *status = (uint32_t *)(s->dmem + r->off + r->fb_bytes + r->acc_bytes);
    const Pts &p = s->clouds[r->r.cloud];
    const Tune t = current_tune();
    hipError_t e = launch_clear(fb, acc, (int64_t)r->npix, r->r.background, st);
    if (e == hipSuccess)
        e = hipMemsetAsync(status, 0, sizeof(uint32_t), st);
    if (e == hipSuccess)
        e = launch_raster_min(p, r->P, fb, t, st);
    if (r->r.mode == RZ_MODE_HQ) {
        if (e == hipSuccess)
            e = launch_hq_accum(p, r->P, r->num, r->den, fb, acc, current_tune_hq(), st);
        if (e == hipSuccess)
            e = launch_resolve_hq(fb, acc, (int64_t)r->npix, r->r.background, r->r.img, status,
                                  st);
    } else if (e == hipSuccess) {
        e = launch_resolve_min(fb, (int64_t)r->npix, r->r.background, r->r.img, st);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(&s->host_status[r->slot], status, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) {
        if (s->events.empty()) {
            hipEvent_t ev;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess)
                s->events.push_back(ev);
        }
        if (e == hipSuccess) {
            r->ev = s->events.back();
            s->events.pop_back();
            e = hipEventRecord(r->ev, st);
        }
    }
    return e == hipSuccess ? RZ_OK : RZ_EHIP;
}

void admit(rz_server *s, Req *r)
{
    r->t_admit = s->now_us();
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    int32_t best = 0;
    for (int32_t i = 1; i < (int32_t)s->load.size(); ++i)
        if (s->load[i] < s->load[best])
            best = i;
    r->stream = best;
    s->load[best]++;
    r->state = RZ_REQ_RUNNING;
    s->inflight.push_back(r);
    s->peak_inflight = std::max(s->peak_inflight, (int32_t)s->inflight.size());
    int rc = RZ_OK;
    if (r->r.flags & RZ_REQ_INJECT_FAILURE) {
        rc = RZ_EHIP;
    } else if (!s->o.dry_run) {
        rc = launch(s, r);
        if (rc != RZ_OK)   // part of it may be queued: let it end before reuse
            (void)hipStreamSynchronize(s->streams[r->stream]);
    }
    if (rc != RZ_OK) {
        s->inflight.pop_back();
        finish(s, r, RZ_REQ_FAILED, rc);
    }
}

void scheduler(rz_server *s)
{
    if (!s->o.dry_run)
        (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // completions
        for (size_t i = 0; i < s->inflight.size();) {
            Req *r = s->inflight[i];
            int32_t state = -1, err = RZ_OK;
            if (s->o.dry_run) {
                if (s->now_us() >= r->t_admit + s->o.dry_run_us)
                    state = RZ_REQ_DONE;
            } else {
                const hipError_t q = hipEventQuery(r->ev);
                if (q == hipSuccess) {
                    state = RZ_REQ_DONE;
                } else if (q != hipErrorNotReady) {
                    state = RZ_REQ_FAILED;
                    err = RZ_EHIP;
                }
            }
            if (state >= 0) {
                s->inflight[i] = s->inflight.back();
                s->inflight.pop_back();
                finish(s, r, state, err);
            } else {
                ++i;
            }
        }
        // admissions, in arrival order
        while (!s->queue.empty() && (int32_t)s->inflight.size() < s->o.max_inflight &&
               !s->free_slots.empty()) {
            Req *r = s->queue.front();
            if (!s->pool.alloc(r->bytes, &r->off))
                break;
            s->queue.pop_front();
            admit(s, r);
        }
        if (s->inflight.empty() && s->queue.empty()) {
            s->idle_cv.notify_all();
            if (s->stop)
                break;
            s->cv.wait(lk, [s] { return s->stop || !s->queue.empty(); });
        } else {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

int validate(rz_server *s, const rz_request *q, Req *r)
{
    if (q->cloud < 0 || q->cloud >= (int32_t)s->clouds.size())
        return RZ_EINVAL;
    if (q->mode != RZ_MODE_ATOMICMIN && q->mode != RZ_MODE_HQ)
        return RZ_EINVAL;
    if ((q->flags & ~RZ_REQ_INJECT_FAILURE) || (!q->img && !s->o.dry_run))
        return RZ_EINVAL;
    int rc = make_proj(&q->view, &q->depth, &r->P);
    if (rc)
        return rc;
    if (r->P.zkind != 0)   // float depth encodings: one-view calls only
        return RZ_EINVAL;
    if (q->mode == RZ_MODE_HQ) {
        rz_hq_params hp = q->hq;
        if (hp.eps_den == 0) {
            hp.eps_num = 1;
            hp.eps_den = 100;
        }
        if ((rc = check_hq(&hp, r->P, &r->num, &r->den)))
            return rc;
    }
    r->r = *q;
    r->npix = (uint64_t)q->view.width * (uint64_t)q->view.height;
    r->fb_bytes = align_up(8 * r->npix);
    r->acc_bytes = q->mode == RZ_MODE_HQ ? align_up(16 * r->npix) : 0;
    r->bytes = r->fb_bytes + r->acc_bytes + kAlign;
    if (r->bytes > s->pool.size)
        return RZ_EBUDGET;
    return RZ_OK;
}

void release_device(rz_server *s)
{
    for (hipEvent_t e : s->events)
        (void)hipEventDestroy(e);
    s->events.clear();
    for (hipStream_t st : s->streams)
        (void)hipStreamDestroy(st);
    s->streams.clear();
    if (s->host_status)
        (void)hipHostFree(s->host_status);
    if (s->dmem)
        (void)hipFree(s->dmem);
    s->host_status = nullptr;
    s->dmem = nullptr;
}

}  // namespace

extern "C" {

int rz_server_create(const rz_server_opts *opts, rz_server **out)
{
    if (!opts || !out)
        return RZ_EINVAL;
    *out = nullptr;
    rz_server_opts o = *opts;
    if (o.streams == 0)
        o.streams = 4;
    if (o.max_inflight == 0)
        o.max_inflight = 4 * o.streams;
    if (o.streams < 1 || o.streams > kMaxStreams || o.max_inflight < 1 ||
        o.max_inflight > 1024 || o.budget_bytes < (1u << 20) || (o.dry_run & ~1) ||
        o.dry_run_us < 0)
        return RZ_EINVAL;
    rz_server *s = new (std::nothrow) rz_server();
    if (!s)
        return RZ_EINVAL;
    s->o = o;
    s->t0 = std::chrono::steady_clock::now();
    s->pool.init(o.budget_bytes / kAlign * kAlign);
    s->load.assign(o.streams, 0);
    for (int32_t i = o.max_inflight - 1; i >= 0; --i)
        s->free_slots.push_back(i);
    if (!o.dry_run) {
        hipError_t e = hipGetDevice(&s->device);
        if (e == hipSuccess)
            e = hipMalloc(&s->dmem, s->pool.size);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&s->host_status, sizeof(uint32_t) * o.max_inflight,
                              hipHostMallocDefault);
        for (int32_t i = 0; i < o.streams && e == hipSuccess; ++i) {
            hipStream_t st;
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e == hipSuccess)
                s->streams.push_back(st);
        }
        if (e != hipSuccess) {
            release_device(s);
            delete s;
            return hip_fail(e);
        }
    }
    s->th = std::thread(scheduler, s);
    *out = s;
    return RZ_OK;
}

int rz_server_add_cloud(rz_server *s, const rz_points *pts, int32_t *id)
{
    if (!s || !id)
        return RZ_EINVAL;
    int rc = check_points(pts);
    if (rc)
        return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    s->clouds.push_back(Pts{pts->x, pts->y, pts->z, pts->rgb, pts->n});
    *id = (int32_t)s->clouds.size() - 1;
    return RZ_OK;
}

int rz_server_submit(rz_server *s, const rz_request *req, uint64_t *ticket)
{
    if (!s || !req || !ticket)
        return RZ_EINVAL;
    Req *r = new (std::nothrow) Req();
    if (!r)
        return RZ_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    int rc = validate(s, req, r);
    if (rc) {
        delete r;
        return rc;
    }
    r->ticket = s->next_ticket++;
    r->t_submit = s->now_us();
    s->tickets[r->ticket] = r;
    s->queue.push_back(r);
    s->submitted++;
    *ticket = r->ticket;
    lk.unlock();
    s->cv.notify_one();
    return RZ_OK;
}

int rz_server_poll(rz_server *s, uint64_t ticket, rz_request_status *st)
{
    if (!s || !st)
        return RZ_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end())
        return RZ_EINVAL;
    Req *r = it->second;
    memset(st, 0, sizeof(*st));
    st->state = r->state;
    st->error = r->error;
    st->hq_status = r->hq_status;
    st->stream = r->stream < 0 ? 0u : (uint32_t)r->stream;
    st->t_submit_us = r->t_submit;
    st->t_admit_us = r->t_admit;
    st->t_done_us = r->t_done;
    if (r->state == RZ_REQ_DONE || r->state == RZ_REQ_FAILED) {
        s->tickets.erase(it);
        delete r;
    }
    return RZ_OK;
}

int rz_server_drain(rz_server *s, double timeout_s)
{
    if (!s)
        return RZ_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->idle_cv.wait_for(
        lk, std::chrono::duration<double>(timeout_s),
        [s] { return s->queue.empty() && s->inflight.empty(); });
    return ok ? RZ_OK : RZ_ESTATE;
}

int rz_server_get_stats(rz_server *s, rz_server_stats *st)
{
    if (!s || !st)
        return RZ_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    memset(st, 0, sizeof(*st));
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->peak_bytes = s->pool.peak;
    st->peak_inflight = s->peak_inflight;
    st->queued = (int32_t)s->queue.size();
    st->inflight = (int32_t)s->inflight.size();
    return RZ_OK;
}

int rz_server_destroy(rz_server *s)
{
    if (!s)
        return RZ_EINVAL;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->idle_cv.wait(lk, [s] { return s->queue.empty() && s->inflight.empty(); });
        s->stop = true;
    }
    s->cv.notify_all();
    s->th.join();
    for (auto &kv : s->tickets)
        delete kv.second;
    release_device(s);
    delete s;
    return RZ_OK;
}

}  // extern "C"
