// Render server (declared in include/rz.h, "serving: continuous batching of
// render requests").
//
// One scheduler thread owns the device work.  Requests wait in a FIFO queue;
// the head is admitted as soon as its framebuffer memory fits the budget
// pool, an in-flight slot is free and (with a work cap) the point passes in
// flight leave room for it.  With merging, later queued requests of the same
// cloud that fit at that moment join it as one multi-view launch.  Its
// kernels (clear, depth pass, splat accumulate, resolve: the same launchers
// as the one-view calls, or the batch engine's multi-view passes for a
// group) are enqueued on the stream with the least work in flight, after a
// wait for the event recorded at submission on the caller's stream (if it
// named one), and followed by an asynchronous copy of its splat status into
// a pinned host slot and a host function that marks the request finished
// and wakes the scheduler.  The scheduler sleeps until a submission or a completion wakes
// it, stamps completion, and returns the memory and the slot, which admits
// the next requests while others still run.  A dry-run mode replaces the
// device by a host timer so that admission, budgeting and failure isolation
// can be tested without a GPU.
//
// Locks: `mu` guards the queue, the in-flight list, the pool and the
// tickets, and is held while the scheduler enqueues device work.  `wake_mu`
// guards only the wake-up counter; it is never held across a HIP call, so
// the host functions, which run on a HIP runtime thread and take only
// `wake_mu`, can never wait on a thread that waits on the runtime.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
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
#include "rz_trace.h"

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
constexpr int kMergeWindow = 32;   // queued requests scanned for a merge
// Rough device time per point pass (about 200 G point passes per second on
// the one-view kernels): only to guess which running request ends first.
constexpr double kUsPerPointPass = 5e-6;
// Launch shape of a merged group's multi-view passes: the batch engine's
// measured best for groups of views (256 threads x 4 points, the 2 KiB
// per-wave tile).
constexpr Tune kGroupTune = {256, 4, 1, 0, 3};

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
    rz_server *srv = nullptr;
    uint64_t ticket = 0;
    rz_request r;
    Proj P;
    uint32_t num = 1, den = 100;
    uint64_t npix = 0;
    uint64_t fb_bytes = 0, acc_bytes = 0, bytes = 0, off = 0;
    int64_t work = 0;          // point passes: the cloud's n, twice for splatting
    int32_t state = RZ_REQ_QUEUED;
    int32_t error = RZ_OK;
    int32_t stream = -1;
    int32_t slot = -1;         // pinned status slot
    uint32_t hq_status = 0;
    int32_t group = 1;         // requests in its launch
    bool chained = false;      // a request was admitted behind it on its stream
    bool queued_behind = false;   // admitted behind another request
    double t_end_guess = 0;    // when its device work should end (dry run: does)
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::atomic<double> t_device_done{-1.0};   // stamped by the host function
    hipEvent_t after = nullptr;            // recorded on the caller's stream at submit
    std::atomic<bool> gpu_done{false};     // set by the host function after the work
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
    // merged groups: a view table of 2 * kMaxGroupViews entries per slot (the
    // group's head's slot), filled on the host in pinned memory and copied
    // to the device on the group's stream
    MvView *mv_stage = nullptr;
    MvView *mv_table = nullptr;
    std::vector<int32_t> free_slots;
    Pool pool;
    std::vector<hipStream_t> streams;
    std::vector<int64_t> load;   // work (point passes) in flight per stream
    std::vector<hipEvent_t> events;       // pool of ordering events
    std::mutex mu;
    std::condition_variable idle_cv;      // everything finished (with mu)
    std::mutex wake_mu;                   // only the counter below
    std::condition_variable wake_cv;      // submission, completion or stop
    uint64_t wake_seq = 0;
    std::deque<Req *> queue;
    std::vector<Req *> inflight;
    std::unordered_map<uint64_t, Req *> tickets;
    uint64_t next_ticket = 1;
    uint64_t submitted = 0, completed = 0, failed = 0;
    uint64_t merged_launches = 0, merged_requests = 0, chained_requests = 0;
    int64_t inflight_work = 0;
    int32_t inflight_exclusive = 0;       // requests in flight that run alone
    int32_t peak_inflight = 0;
    bool stop = false;
    std::thread th;
    std::chrono::steady_clock::time_point t0;

    double now_us() const
    {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
            .count();
    }
    void wake()
    {
        std::lock_guard<std::mutex> lk(wake_mu);
        ++wake_seq;
        wake_cv.notify_one();   // under the lock: see on_device_done
    }
};

namespace {

bool exclusive(const rz_server *s, const Req *r)
{
    return s->o.exclusive_work > 0 && r->work >= s->o.exclusive_work;
}

void finish(rz_server *s, Req *r, int32_t state, int32_t error)
{
    s->inflight_work -= r->work;   // only admitted requests finish
    if (exclusive(s, r))
        s->inflight_exclusive--;
    r->state = state;
    r->error = error;
    // the host function's stamp when the device work finished (in a dry
    // run, when its simulated work ended), else now (failures)
    const double dev = r->t_device_done.load(std::memory_order_relaxed);
    r->t_done = dev >= 0 ? dev
                         : (s->o.dry_run && state == RZ_REQ_DONE ? r->t_end_guess : s->now_us());
    if (r->slot >= 0) {
        if (!s->o.dry_run)
            r->hq_status = s->host_status[r->slot];
        s->free_slots.push_back(r->slot);
        r->slot = -1;
    }
    if (r->after) {
        s->events.push_back(r->after);
        r->after = nullptr;
    }
    if (r->stream >= 0)
        s->load[r->stream] -= r->work;
    s->pool.release(r->off, r->bytes);
    // a splat count beyond the exact range of the packed sums leaves some
    // pixels' colours unspecified: the request fails visibly
    if (state == RZ_REQ_DONE && r->r.mode == RZ_MODE_HQ &&
        (r->hq_status & RZ_STATUS_HQ_OVERFLOW)) {
        r->state = state = RZ_REQ_FAILED;
        r->error = RZ_EOVERFLOW;
    }
    if (state == RZ_REQ_DONE)
        s->completed++;
    else
        s->failed++;
}

// Host function enqueued after a request's device work: runs on a HIP
// runtime thread once that work has completed.  It takes only wake_mu and
// notifies under it, so once rz_server_destroy holds wake_mu after the last
// request finished, no host function touches the server any more.
void on_device_done(void *p)
{
    Req *r = static_cast<Req *>(p);
    rz_server *s = r->srv;
    r->t_device_done.store(s->now_us(), std::memory_order_relaxed);
    std::lock_guard<std::mutex> lk(s->wake_mu);
    r->gpu_done.store(true, std::memory_order_release);
    ++s->wake_seq;
    s->wake_cv.notify_one();
}

// Enqueues the request's kernels; returns an RZ_* code.
int launch(rz_server *s, Req *r)
{
    Range range(r->r.mode == RZ_MODE_HQ ? "rz_server request (splatting)"
                                        : "rz_server request (atomicMin)");
    hipStream_t st = s->streams[r->stream];
    uint64_t *fb = (uint64_t *)(s->dmem + r->off);
    uint64_t *acc = r->acc_bytes ? (uint64_t *)(s->dmem + r->off + r->fb_bytes) : nullptr;
    uint32_t *status = (uint32_t *)(s->dmem + r->off + r->fb_bytes + r->acc_bytes);
    const Pts &p = s->clouds[r->r.cloud];
    const Tune t = current_tune();
    hipError_t e = hipSuccess;
    if (r->after)
        e = hipStreamWaitEvent(st, r->after, 0);
    if (e == hipSuccess)
        e = launch_clear(fb, acc, (int64_t)r->npix, r->r.background, st);
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
    if (e == hipSuccess)
        e = hipLaunchHostFunc(st, on_device_done, r);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

// Enqueues a merged group (two or more requests of one cloud, one stream):
// per request its wait, clear and status reset; one multi-view depth launch
// over every view and one accumulate launch over the splatting ones (the
// view table is copied from the head's pinned slot to its device slot
// first); then per request its resolve, status copy and host function.
// Returns an RZ_* code.
int launch_group(rz_server *s, const std::vector<Req *> &g)
{
    Range range("rz_server merged requests");
    const Req *head = g[0];
    hipStream_t st = s->streams[head->stream];
    const Pts &p = s->clouds[head->r.cloud];
    MvView *stage = s->mv_stage + (size_t)head->slot * 2 * kMaxGroupViews;
    MvView *table = s->mv_table + (size_t)head->slot * 2 * kMaxGroupViews;
    int32_t nv = 0, nhq = 0;
    bool pw = false, pw_hq = false;
    hipError_t e = hipSuccess;
    for (Req *r : g) {
        uint64_t *fb = (uint64_t *)(s->dmem + r->off);
        uint64_t *acc = r->acc_bytes ? (uint64_t *)(s->dmem + r->off + r->fb_bytes) : nullptr;
        uint32_t *status = (uint32_t *)(s->dmem + r->off + r->fb_bytes + r->acc_bytes);
        if (e == hipSuccess && r->after)
            e = hipStreamWaitEvent(st, r->after, 0);
        if (e == hipSuccess)
            e = launch_clear(fb, acc, (int64_t)r->npix, r->r.background, st);
        if (e == hipSuccess)
            e = hipMemsetAsync(status, 0, sizeof(uint32_t), st);
        MvView m;
        memset(&m, 0, sizeof(m));
        m.P = r->P;
        m.fb = fb;
        m.acc = acc;
        m.eps_num = r->num;
        m.eps_den = r->den;
        stage[nv++] = m;
        pw = pw || r->P.nr > 0;
        if (r->r.mode == RZ_MODE_HQ) {
            stage[kMaxGroupViews + nhq++] = m;
            pw_hq = pw_hq || r->P.nr > 0;
        }
    }
    // the pinned slot is not written again before the head's slot is freed,
    // which happens only after the group's work (and so this copy) is done
    if (e == hipSuccess)
        e = hipMemcpyAsync(table, stage, sizeof(MvView) * 2 * kMaxGroupViews,
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_multiview(false, pw, p, table, nv, kGroupTune, st);
    if (e == hipSuccess && nhq > 0)
        e = launch_multiview(true, pw_hq, p, table + kMaxGroupViews, nhq, kGroupTune, st);
    for (Req *r : g) {
        uint64_t *fb = (uint64_t *)(s->dmem + r->off);
        uint64_t *acc = r->acc_bytes ? (uint64_t *)(s->dmem + r->off + r->fb_bytes) : nullptr;
        uint32_t *status = (uint32_t *)(s->dmem + r->off + r->fb_bytes + r->acc_bytes);
        if (e == hipSuccess)
            e = r->r.mode == RZ_MODE_HQ
                    ? launch_resolve_hq(fb, acc, (int64_t)r->npix, r->r.background, r->r.img,
                                        status, st)
                    : launch_resolve_min(fb, (int64_t)r->npix, r->r.background, r->r.img, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&s->host_status[r->slot], status, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, st);
    }
    for (Req *r : g)
        if (e == hipSuccess)
            e = hipLaunchHostFunc(st, on_device_done, r);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

// Admits a group of requests (one, or several of one cloud) on one stream:
// the stream with the least work in flight, or, with `behind`, that
// request's stream, where the group starts as soon as it ends.
void admit(rz_server *s, const std::vector<Req *> &g, Req *behind = nullptr)
{
    // the stream with the least work in flight: a small request does not
    // queue behind a large one while another stream is idle or lighter
    int32_t best = 0;
    for (int32_t i = 1; i < (int32_t)s->load.size(); ++i)
        if (s->load[i] < s->load[best])
            best = i;
    const double now = s->now_us();
    double start = now;
    if (behind) {
        best = behind->stream;
        behind->chained = true;
        start = std::max(now, behind->t_end_guess);
        s->chained_requests += g.size();
    }
    int64_t gwork = 0;
    for (Req *r : g)
        gwork += r->work;
    const double end = start + (s->o.dry_run ? (double)s->o.dry_run_us
                                             : (double)gwork * kUsPerPointPass);
    for (Req *r : g) {
        r->t_admit = now;
        r->t_end_guess = end;
        r->queued_behind = behind != nullptr;
        r->slot = s->free_slots.back();
        s->free_slots.pop_back();
        r->stream = best;
        s->load[best] += r->work;
        r->state = RZ_REQ_RUNNING;
        r->group = (int32_t)g.size();
        s->inflight_work += r->work;
        if (exclusive(s, r))
            s->inflight_exclusive++;
        s->inflight.push_back(r);
    }
    s->peak_inflight = std::max(s->peak_inflight, (int32_t)s->inflight.size());
    if (g.size() > 1) {
        s->merged_launches++;
        s->merged_requests += g.size();
    }
    int rc = RZ_OK;
    if (g.size() == 1 && (g[0]->r.flags & RZ_REQ_INJECT_FAILURE)) {
        rc = RZ_EHIP;
    } else if (!s->o.dry_run) {
        rc = g.size() == 1 ? launch(s, g[0]) : launch_group(s, g);
        if (rc != RZ_OK)   // part of it may be queued: let it end before reuse
            (void)hipStreamSynchronize(s->streams[best]);
    }
    if (rc != RZ_OK) {
        // the group fails together (its members are the last in flight)
        s->inflight.resize(s->inflight.size() - g.size());
        for (Req *r : g)
            finish(s, r, RZ_REQ_FAILED, rc);
    }
}

// The running request behind which the blocked head request r may start:
// one alone on the device that is exclusive, or one at least as large as r
// (so that the work running at once never grows), with nothing chained
// behind it yet, not itself waiting behind another (so that blocked
// requests do not line up on one stream) and not part of a merged group; if
// r must run alone, only a request alone on the device.  Of those, the one
// expected to end first.  With merging on, requests are not chained: a
// request held back is admitted by the scheduler, with the others of its
// cloud.
Req *chain_target(rz_server *s, const Req *r)
{
    if ((r->r.flags & RZ_REQ_INJECT_FAILURE) || s->o.merge_views > 1)
        return nullptr;
    Req *best = nullptr;
    for (Req *p : s->inflight) {
        if (p->chained || p->queued_behind || p->group != 1 || p->state != RZ_REQ_RUNNING)
            continue;
        const bool alone = s->inflight.size() == 1;
        const bool ok = (exclusive(s, p) && alone) ||
                        (p->work >= r->work && (!exclusive(s, r) || alone));
        if (ok && (!best || p->t_end_guess < best->t_end_guess))
            best = p;
    }
    return best;
}

void scheduler(rz_server *s)
{
    if (!s->o.dry_run)
        (void)hipSetDevice(s->device);
    uint64_t seen = 0;
    for (;;) {
        double next_deadline = -1.0;   // dry run: when the next request ends
        bool stop = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // completions
            for (size_t i = 0; i < s->inflight.size();) {
                Req *r = s->inflight[i];
                bool done;
                if (s->o.dry_run) {
                    const double end = r->t_end_guess;
                    done = s->now_us() >= end;
                    if (!done && (next_deadline < 0 || end < next_deadline))
                        next_deadline = end;
                } else {
                    done = r->gpu_done.load(std::memory_order_acquire);
                }
                if (done) {
                    s->inflight[i] = s->inflight.back();
                    s->inflight.pop_back();
                    finish(s, r, RZ_REQ_DONE, RZ_OK);
                } else {
                    ++i;
                }
            }
            // admissions, in arrival order
            while (!s->queue.empty() && (int32_t)s->inflight.size() < s->o.max_inflight &&
                   !s->free_slots.empty()) {
                Req *r = s->queue.front();
                // a request that runs alone waits for an empty device, and
                // nothing joins it; the work cap bounds the work in flight
                const bool blocked =
                    (s->o.work_cap > 0 && !s->inflight.empty() &&
                     s->inflight_work + r->work > s->o.work_cap) ||
                    s->inflight_exclusive > 0 || (exclusive(s, r) && !s->inflight.empty());
                // blocked: it may still go behind a running request on that
                // request's stream, so that it starts the moment the device
                // would otherwise wait for the scheduler
                Req *behind = blocked ? chain_target(s, r) : nullptr;
                if (blocked && !behind)
                    break;
                if (!s->pool.alloc(r->bytes, &r->off))
                    break;
                s->queue.pop_front();
                if (behind) {
                    admit(s, std::vector<Req *>{r}, behind);
                    if (s->o.dry_run && r->state == RZ_REQ_RUNNING &&
                        (next_deadline < 0 || r->t_end_guess < next_deadline))
                        next_deadline = r->t_end_guess;
                    continue;
                }
                std::vector<Req *> g{r};
                if (s->o.merge_views > 1 && !(r->r.flags & RZ_REQ_INJECT_FAILURE) &&
                    !exclusive(s, r)) {
                    // later requests of the same cloud that fit now join it
                    int64_t gwork = r->work;
                    int scanned = 0;
                    for (auto it = s->queue.begin();
                         it != s->queue.end() && scanned < kMergeWindow &&
                         (int32_t)g.size() < s->o.merge_views;
                         ++scanned) {
                        Req *q = *it;
                        const bool fits =
                            q->r.cloud == r->r.cloud && !(q->r.flags & RZ_REQ_INJECT_FAILURE) &&
                            !exclusive(s, q) &&
                            (int32_t)(s->inflight.size() + g.size()) < s->o.max_inflight &&
                            s->free_slots.size() > g.size() &&
                            (s->o.work_cap <= 0 ||
                             s->inflight_work + gwork + q->work <= s->o.work_cap);
                        if (fits && s->pool.alloc(q->bytes, &q->off)) {
                            g.push_back(q);
                            gwork += q->work;
                            it = s->queue.erase(it);
                        } else {
                            ++it;
                        }
                    }
                }
                admit(s, g);
                if (s->o.dry_run && r->state == RZ_REQ_RUNNING &&
                    (next_deadline < 0 || r->t_end_guess < next_deadline))
                    next_deadline = r->t_end_guess;
            }
            if (s->inflight.empty() && s->queue.empty()) {
                s->idle_cv.notify_all();
                stop = s->stop;
            }
        }
        if (stop)
            break;
        // sleep until a submission, a completion or a dry-run deadline
        std::unique_lock<std::mutex> wl(s->wake_mu);
        if (next_deadline >= 0) {
            const auto until =
                s->t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                            std::chrono::duration<double, std::micro>(next_deadline));
            s->wake_cv.wait_until(wl, until, [&] { return s->wake_seq != seen; });
        } else {
            s->wake_cv.wait(wl, [&] { return s->wake_seq != seen; });
        }
        seen = s->wake_seq;
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
    r->work = s->clouds[q->cloud].n * (q->mode == RZ_MODE_HQ ? 2 : 1);
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
    if (s->mv_stage)
        (void)hipHostFree(s->mv_stage);
    if (s->mv_table)
        (void)hipFree(s->mv_table);
    if (s->dmem)
        (void)hipFree(s->dmem);
    s->host_status = nullptr;
    s->mv_stage = nullptr;
    s->mv_table = nullptr;
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
        o.dry_run_us < 0 || o.work_cap < 0 || o.exclusive_work < 0 || o.merge_views < 0 ||
        o.merge_views > kMaxGroupViews)
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
        const size_t tables = sizeof(MvView) * 2 * kMaxGroupViews * (size_t)o.max_inflight;
        if (e == hipSuccess && o.merge_views > 1)
            e = hipHostMalloc((void **)&s->mv_stage, tables, hipHostMallocDefault);
        if (e == hipSuccess && o.merge_views > 1)
            e = hipMalloc((void **)&s->mv_table, tables);
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
    r->srv = s;
    std::unique_lock<std::mutex> lk(s->mu);
    int rc = validate(s, req, r);
    if (rc) {
        delete r;
        return rc;
    }
    if (req->after && !s->o.dry_run) {
        // order the request after the caller's work queued so far on its
        // stream (e.g. the fill of its image, or the upload of its cloud)
        hipError_t e = hipSuccess;
        if (s->events.empty()) {
            hipEvent_t ev;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess)
                s->events.push_back(ev);
        }
        if (e == hipSuccess) {
            r->after = s->events.back();
            s->events.pop_back();
            e = hipEventRecord(r->after, (hipStream_t)req->after);
        }
        if (e != hipSuccess) {
            if (r->after)
                s->events.push_back(r->after);
            delete r;
            return hip_fail(e);
        }
    }
    r->ticket = s->next_ticket++;
    r->t_submit = s->now_us();
    s->tickets[r->ticket] = r;
    s->queue.push_back(r);
    s->submitted++;
    *ticket = r->ticket;
    lk.unlock();
    s->wake();
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
    st->group = r->group;
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
    st->merged_launches = s->merged_launches;
    st->merged_requests = s->merged_requests;
    st->chained_requests = s->chained_requests;
    return RZ_OK;
}

int rz_server_destroy(rz_server *s, double timeout_s)
{
    if (!s || !(timeout_s >= 0.0))
        return RZ_EINVAL;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        const bool idle = s->idle_cv.wait_for(
            lk, std::chrono::duration<double>(timeout_s),
            [s] { return s->queue.empty() && s->inflight.empty(); });
        if (!idle)
            return RZ_ESTATE;   // still working: the server stays usable
        s->stop = true;
    }
    s->wake();
    s->th.join();
    // every request has finished, so every host function has set its flag;
    // wait for the streams (and their host functions) to end, then take
    // wake_mu once: no host function is inside its critical section after
    for (hipStream_t st : s->streams)
        (void)hipStreamSynchronize(st);
    { std::lock_guard<std::mutex> lk(s->wake_mu); }
    for (auto &kv : s->tickets)
        delete kv.second;
    release_device(s);
    delete s;
    return RZ_OK;
}

}  // extern "C"
