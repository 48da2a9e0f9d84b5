// Batched multi-view rendering (declared in include/rz.h, "batched
// multi-view rendering"): many views of one resident point cloud per
// submission, optionally replayed from one captured hipGraph, with a
// project-written autotuner over launch shape and views per group.
//
// Per group of K views, k_mv_raster_min loads each chunk of points once and
// runs the depth pass of section 2.1 for every view of the group (the view
// constants come from a device table, read with scalar loads).  The
// splatting views of the batch then share k_mv_hq_accum (section 2.2) in the
// same way, and k_mv_resolve resolves and clears every view in one launch.
// The per-chunk arithmetic is the same code as the one-view kernels
// (rz_device.h), so each view is bit-identical to its one-view call.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "rz.h"
#include "rz_device.h"
#include "rz_internal.h"
#include "rz_trace.h"

namespace rz {

int check_points(const rz_points *p);
int make_proj(const rz_view *v, const rz_depth_map *dm, Proj *P);
int check_hq(const rz_hq_params *hq, const Proj &P, uint32_t *num, uint32_t *den);
int hip_fail(hipError_t e);
Tune current_tune();
int order_class_windows(const float *x, const float *y, const float *z, int64_t m, int nwin);
int64_t order_sample_window();

namespace {

using namespace dev;

constexpr int kMaxK = kMaxGroupViews;
constexpr int kMaxViews = 4096;
constexpr int64_t kResolvePix = 512;   // pixels per resolve workgroup (256 x 2)

// One view of the fused resolve.
struct MvResolve {
    uint64_t *fb;
    uint64_t *acc;
    uint32_t *img;
    int64_t npix;
    int64_t block0;   // first resolve workgroup of this view
    uint64_t clear;
    uint32_t bg;
    int32_t hq;
};

// Depth passes of views[0 .. nv) over one chunk: the points are loaded
// once and stay in registers while each view is rasterized in turn.
template <int PPT, bool VEC, bool XCD, int BIN, bool PW>
__global__ void __launch_bounds__(512) k_mv_raster_min(Pts p, const MvView *__restrict__ views,
                                                       int32_t nv, int64_t nchunks,
                                                       uint32_t words)
{
    __shared__ uint64_t s_tile[BIN == kBinBlock ? kTileMin : 1];
    __shared__ uint32_t s_box[kMaxWaves][4];
    extern __shared__ uint64_t s_waves[];
    const int64_t chunk = chunk_index<XCD>();
    if (chunk >= nchunks)
        return;
    float x[PPT], y[PPT], z[PPT];
    uint32_t c[PPT];
    bool in[PPT];
    // points past the end load as NaN and are culled: no bounds flags
    load_points_nan<PPT, VEC>(p, chunk * (int64_t)blockDim.x * PPT, x, y, z, c);
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        in[j] = true;
    for (int32_t k = 0; k < nv; ++k) {
        const Proj P = views[k].P;
        if (BIN == kBinWave) {
            raster_chunk_wave<PPT, PW>(P, views[k].fb, x, y, z, c, in,
                                       s_waves + (threadIdx.x >> 6) * words, words);
        } else {
            if (BIN == kBinBlock && k > 0)
                __syncthreads();   // previous view's tile fully flushed
            raster_chunk<PPT, true, BIN == kBinBlock, PW>(P, views[k].fb, x, y, z, c, in, s_tile,
                                                      s_box);
        }
    }
}

// Accumulate passes of the splatting views views[0 .. nv) over one chunk.
template <int PPT, bool VEC, bool XCD, int BIN, bool PW>
__global__ void __launch_bounds__(512) k_mv_hq_accum(Pts p, const MvView *__restrict__ views,
                                                     int32_t nv, int64_t nchunks,
                                                     uint32_t words)
{
    __shared__ uint64_t s_tile[BIN == kBinBlock ? 2 * kTileHq : 2];
    __shared__ uint32_t s_box[kMaxWaves][4];
    extern __shared__ uint64_t s_waves[];
    const int64_t chunk = chunk_index<XCD>();
    if (chunk >= nchunks)
        return;
    float x[PPT], y[PPT], z[PPT];
    uint32_t c[PPT];
    bool in[PPT];
    // points past the end load as NaN and are culled: no bounds flags
    load_points_nan<PPT, VEC>(p, chunk * (int64_t)blockDim.x * PPT, x, y, z, c);
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        in[j] = true;
    for (int32_t k = 0; k < nv; ++k) {
        const Proj P = views[k].P;
        if (BIN == kBinWave) {
            accum_chunk_wave<PPT, PW>(P, views[k].eps_num, views[k].eps_den, views[k].fb,
                                      views[k].acc, x, y, z, c, in,
                                      s_waves + (threadIdx.x >> 6) * words, words);
        } else {
            if (BIN == kBinBlock && k > 0)
                __syncthreads();
            accum_chunk<PPT, BIN == kBinBlock, PW>(P, views[k].eps_num, views[k].eps_den,
                                                   views[k].fb, views[k].acc, x, y, z, c, in,
                                                   s_tile, s_box);
        }
    }
}

// The view of a resolve workgroup (uniform binary search over block0).
__device__ __forceinline__ int32_t find_view(const MvResolve *__restrict__ rv, int32_t nv,
                                             int64_t b)
{
    int32_t lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (rv[mid].block0 <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Resolve of every view in one launch: section 2.1's resolve/clear for the
// atomicMin views, section 2.2's third pass for the splatting views.
__global__ void __launch_bounds__(256) k_mv_resolve(const MvResolve *__restrict__ rv, int32_t nv,
                                                    uint32_t *__restrict__ status)
{
    const int32_t v = find_view(rv, nv, blockIdx.x);
    const MvResolve R = rv[v];
    const int64_t i0 = ((int64_t)blockIdx.x - R.block0) * kResolvePix + 2 * threadIdx.x;
    bool overflow = false;
    for (int64_t i = i0; i < i0 + 2 && i < R.npix; ++i) {
        if (R.hq) {
            R.img[i] = hq_colour(R.acc[2 * i], R.acc[2 * i + 1], R.bg, overflow);
            R.acc[2 * i] = 0;
            R.acc[2 * i + 1] = 0;
        } else {
            R.img[i] = (uint32_t)(R.fb[i] & kRgbMask);
        }
        R.fb[i] = R.clear;
    }
    if (overflow && status)
        atomicOr(status, RZ_STATUS_HQ_OVERFLOW);
}

// Order-independent 64-bit checksum of every image (used by the autotuner
// to check that a candidate launch shape renders the same bits).
__global__ void __launch_bounds__(256) k_mv_checksum(const MvResolve *__restrict__ rv, int32_t nv,
                                                     unsigned long long *__restrict__ out)
{
    const int32_t v = find_view(rv, nv, blockIdx.x);
    const MvResolve R = rv[v];
    const int64_t i0 = ((int64_t)blockIdx.x - R.block0) * kResolvePix + 2 * threadIdx.x;
    unsigned long long h = 0;
    for (int64_t i = i0; i < i0 + 2 && i < R.npix; ++i) {
        unsigned long long w = ((unsigned long long)R.img[i] << 20) ^ (unsigned long long)i ^
                               ((unsigned long long)v << 52);
        w *= 0x9E3779B97F4A7C15ull;
        w ^= w >> 29;
        h += w;
    }
    if (h)
        atomicAdd(out, h);
}

template <int PPT, bool VEC, bool XCD, int BIN>
hipError_t mv_launch_ppt(bool hq, bool pw, const Pts &p, const MvView *views, int32_t nv,
                         const Tune &t, hipStream_t s)
{
    const int64_t nchunks = (p.n + (int64_t)t.block * PPT - 1) / ((int64_t)t.block * PPT);
    const int64_t grid = XCD ? (nchunks + kXcds - 1) / kXcds * kXcds : nchunks;
    const uint32_t words = wave_tile_words(t.bin);
    const size_t lds =
        BIN == kBinWave ? (size_t)(t.block / 64) * words * sizeof(uint64_t) : 0;
    if (hq && pw)
        hipLaunchKernelGGL((k_mv_hq_accum<PPT, VEC, XCD, BIN, true>), dim3((uint32_t)grid),
                           dim3(t.block), lds, s, p, views, nv, nchunks, words);
    else if (hq)
        hipLaunchKernelGGL((k_mv_hq_accum<PPT, VEC, XCD, BIN, false>), dim3((uint32_t)grid),
                           dim3(t.block), lds, s, p, views, nv, nchunks, words);
    else if (pw)
        hipLaunchKernelGGL((k_mv_raster_min<PPT, VEC, XCD, BIN, true>), dim3((uint32_t)grid),
                           dim3(t.block), lds, s, p, views, nv, nchunks, words);
    else
        hipLaunchKernelGGL((k_mv_raster_min<PPT, VEC, XCD, BIN, false>), dim3((uint32_t)grid),
                           dim3(t.block), lds, s, p, views, nv, nchunks, words);
    return hipGetLastError();
}

template <int PPT, bool VEC, bool XCD>
hipError_t mv_launch_bin(bool hq, bool pw, const Pts &p, const MvView *views, int32_t nv,
                         const Tune &t, hipStream_t s)
{
    switch (t.bin) {
    case kBinBlock: return mv_launch_ppt<PPT, VEC, XCD, kBinBlock>(hq, pw, p, views, nv, t, s);
    case kBinWave:
    case kBinWaveSmall:
        return mv_launch_ppt<PPT, VEC, XCD, kBinWave>(hq, pw, p, views, nv, t, s);
    default: return mv_launch_ppt<PPT, VEC, XCD, kBinNone>(hq, pw, p, views, nv, t, s);
    }
}

template <int PPT>
hipError_t mv_launch_sel(bool hq, bool pw, const Pts &p, const MvView *views, int32_t nv,
                         const Tune &t, bool vec, hipStream_t s)
{
    if (vec)
        return t.xcd_remap ? mv_launch_bin<PPT, true, true>(hq, pw, p, views, nv, t, s)
                           : mv_launch_bin<PPT, true, false>(hq, pw, p, views, nv, t, s);
    return mv_launch_bin<PPT, false, false>(hq, pw, p, views, nv, t, s);
}

hipError_t mv_launch(bool hq, bool pw, const Pts &p, const MvView *views, int32_t nv,
                     const Tune &t, hipStream_t s)
{
    if (p.n == 0 || nv == 0)
        return hipSuccess;
    const bool vec = (((uintptr_t)p.x | (uintptr_t)p.y | (uintptr_t)p.z | (uintptr_t)p.rgb) &
                      15u) == 0;
    switch (t.ppt) {
    case 4: return mv_launch_sel<4>(hq, pw, p, views, nv, t, vec, s);
    case 8: return mv_launch_sel<8>(hq, pw, p, views, nv, t, vec, s);
    case 16: return mv_launch_sel<16>(hq, pw, p, views, nv, t, vec, s);
    default: return hipErrorInvalidValue;
    }
}

int check_launch(const rz_launch &l)
{
    if (!(l.block == 64 || l.block == 128 || l.block == 256 || l.block == 512))
        return RZ_EINVAL;
    if (!(l.ppt == 4 || l.ppt == 8 || l.ppt == 16))
        return RZ_EINVAL;
    if ((l.early_out & ~1) || (l.xcd_remap & ~1) || l.bin < 0 || l.bin > kBinWaveSmall)
        return RZ_EINVAL;
    return RZ_OK;
}

Tune tune_of(const rz_launch &l)
{
    Tune t;
    t.block = l.block;
    t.ppt = l.ppt;
    t.early_out = l.early_out;
    t.xcd_remap = l.xcd_remap;
    t.bin = l.bin;
    return t;
}

rz_launch launch_of(const Tune &t)
{
    rz_launch l;
    l.block = t.block;
    l.ppt = t.ppt;
    l.early_out = t.early_out;
    l.xcd_remap = t.xcd_remap;
    l.bin = t.bin;
    return l;
}

}  // namespace

hipError_t launch_multiview(bool hq, bool pw, const Pts &p, const MvView *views, int32_t nv,
                            const Tune &t, hipStream_t s)
{
    if (nv < 0 || nv > kMaxGroupViews)
        return hipErrorInvalidValue;
    Range r(hq ? "rz multi-view splat accumulate pass" : "rz multi-view depth pass");
    return mv_launch(hq, pw, p, views, nv, t, s);
}

}  // namespace rz

using namespace rz;

struct rz_batch {
    Pts pts;
    int32_t nviews = 0;
    int32_t nhq = 0;
    bool hq_pw = false;                   // some splatting view uses a piecewise map
    bool any_pw = false;                  // some view uses a piecewise map
    int64_t resolve_blocks = 0;
    void *dmem = nullptr;                 // one allocation: tables + checksum word
    MvView *d_raster = nullptr;           // all views
    MvView *d_accum = nullptr;            // splatting views
    MvResolve *d_resolve = nullptr;       // all views
    unsigned long long *d_sum = nullptr;  // autotuner checksum
    rz_batch_opts opts;
    Tune tune;      // depth passes (opts.launch)
    Tune tune_hq;   // accumulate passes: opts.launch, or the autotuner's pick
    int64_t total_px = 0;                 // pixels of all views
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

hipError_t enqueue(rz_batch *b, hipStream_t s)
{
    const int32_t K = b->opts.views_per_group;
    hipError_t e = hipSuccess;
    {
        Range r("rz batch: depth passes");
        for (int32_t g = 0; g < b->nviews && e == hipSuccess; g += K)
            e = mv_launch(false, b->any_pw, b->pts, b->d_raster + g, std::min(K, b->nviews - g),
                          b->tune, s);
    }
    if (b->nhq > 0) {
        Range r("rz batch: splat accumulate passes");
        for (int32_t g = 0; g < b->nhq && e == hipSuccess; g += K)
            e = mv_launch(true, b->hq_pw, b->pts, b->d_accum + g, std::min(K, b->nhq - g),
                          b->tune_hq, s);
    }
    if (e == hipSuccess && b->resolve_blocks > 0) {
        Range r("rz batch: resolve");
        hipLaunchKernelGGL(k_mv_resolve, dim3((uint32_t)b->resolve_blocks), dim3(256), 0, s,
                           b->d_resolve, b->nviews, b->opts.status);
        e = hipGetLastError();
    }
    return e;
}

void drop_graph(rz_batch *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// One run of the batch, then the checksum of every image (synchronous).
hipError_t run_checksum(rz_batch *b, hipStream_t s, unsigned long long *sum)
{
    hipError_t e = enqueue(b, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(b->d_sum, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess && b->resolve_blocks > 0) {
        hipLaunchKernelGGL(k_mv_checksum, dim3((uint32_t)b->resolve_blocks), dim3(256), 0, s,
                           b->d_resolve, b->nviews, b->d_sum);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(sum, b->d_sum, sizeof(*sum), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    return e;
}

// Median of reps timed runs (ms).
hipError_t time_runs(rz_batch *b, hipStream_t s, int32_t reps, float *med)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    std::vector<float> t;
    for (int32_t r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess)
            e = enqueue(b, s);
        if (e == hipSuccess)
            e = hipEventRecord(e1, s);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        t.push_back(ms);
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (e == hipSuccess) {
        std::sort(t.begin(), t.end());
        *med = t[t.size() / 2];
    }
    return e;
}

int capture(rz_batch *b)
{
    drop_graph(b);
    hipError_t e = hipSuccess;
    if (!b->cap_stream)
        e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess)
        return hip_fail(e);
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess)
        return hip_fail(e);
    hipError_t le = enqueue(b, b->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap_stream, &g);
    if (le != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return hip_fail(le);
    }
    if (e != hipSuccess)
        return hip_fail(e);
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return hip_fail(e);
    }
    return RZ_OK;
}

// The autotune cache key of a batch (see rz_batch_autotune_cached).
int batch_key(rz_batch *b, char *key, size_t len)
{
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess)
        return hip_fail(e);
    char arch[64];
    size_t i = 0;
    for (; i + 1 < sizeof(arch) && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i)
        arch[i] = prop.gcnArchName[i] == ' ' ? '_' : prop.gcnArchName[i];
    arch[i] = 0;
    if (!i)
        strcpy(arch, "unknown");
    // three windows of consecutive points, gathered on the host
    const int64_t n = b->pts.n;
    const int64_t m = std::min<int64_t>(n, order_sample_window());
    const int64_t starts[3] = {0, (n - m) / 2, n - m};
    std::vector<float> hx(3 * m), hy(3 * m), hz(3 * m);
    for (int w = 0; w < 3 && m > 0 && e == hipSuccess; ++w) {
        e = hipMemcpy(hx.data() + w * m, b->pts.x + starts[w], m * sizeof(float),
                      hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(hy.data() + w * m, b->pts.y + starts[w], m * sizeof(float),
                          hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(hz.data() + w * m, b->pts.z + starts[w], m * sizeof(float),
                          hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess)
        return hip_fail(e);
    const int order = order_class_windows(hx.data(), hy.data(), hz.data(), m, 3);
    const int nlog = n > 0 ? (int)lround(log2((double)n)) : 0;
    const int plog = b->total_px > 0 ? (int)lround(log2((double)b->total_px)) : 0;
    const int hq8 = (int)((b->nhq * 8 + b->nviews / 2) / b->nviews);
    snprintf(key, len, "%s n%d px%d v%d hq%d %s", arch, nlog, plog, b->nviews, hq8,
             order == 0 ? "ordered" : "shuffled");
    return RZ_OK;
}

}  // namespace

extern "C" {

int rz_batch_plan(const rz_points *pts, const rz_batch_view *views, int32_t nviews,
                  const rz_batch_opts *opts, rz_batch **out)
{
    if (!out || !views || nviews < 1 || nviews > kMaxViews)
        return RZ_EINVAL;
    *out = nullptr;
    int rc = check_points(pts);
    if (rc)
        return rc;
    rz_batch_opts o;
    memset(&o, 0, sizeof(o));
    if (opts)
        o = *opts;
    if (o.views_per_group == 0)
        o.views_per_group = 4;
    if (o.views_per_group < 1 || o.views_per_group > kMaxK || (o.use_graph & ~1))
        return RZ_EINVAL;
    if (o.launch.block == 0)
        o.launch = launch_of(current_tune());
    if ((rc = check_launch(o.launch)))
        return rc;

    std::vector<MvView> raster, accum;
    std::vector<MvResolve> res;
    int64_t blocks = 0;
    for (int32_t i = 0; i < nviews; ++i) {
        const rz_batch_view &v = views[i];
        MvView m;
        memset(&m, 0, sizeof(m));
        if ((rc = make_proj(&v.view, &v.depth, &m.P)))
            return rc;
        if (m.P.zkind != 0)   // float depth encodings: one-view calls only
            return RZ_EINVAL;
        const bool hq = v.mode == RZ_MODE_HQ;
        if (!hq && v.mode != RZ_MODE_ATOMICMIN)
            return RZ_EINVAL;
        if (!v.fb || !v.img || (hq && !v.acc))
            return RZ_EINVAL;
        if (hq) {
            rz_hq_params hp = v.hq;
            if (hp.eps_den == 0) {
                hp.eps_num = 1;
                hp.eps_den = 100;
            }
            if ((rc = check_hq(&hp, m.P, &m.eps_num, &m.eps_den)))
                return rc;
        }
        for (int32_t j = 0; j < i; ++j)   // buffers of two views must not coincide
            if (views[j].fb == v.fb || views[j].img == v.img || (hq && views[j].acc == v.acc))
                return RZ_EINVAL;
        m.fb = v.fb;
        m.acc = hq ? v.acc : nullptr;
        raster.push_back(m);
        if (hq)
            accum.push_back(m);
        MvResolve r;
        memset(&r, 0, sizeof(r));
        r.fb = v.fb;
        r.acc = m.acc;
        r.img = v.img;
        r.npix = (int64_t)m.P.width * m.P.height;
        r.block0 = blocks;
        r.clear = kDepthOnes | ((uint64_t)v.background & kRgbMask);
        r.bg = v.background & (uint32_t)kRgbMask;
        r.hq = hq ? 1 : 0;
        res.push_back(r);
        blocks += (r.npix + kResolvePix - 1) / kResolvePix;
    }

    if (!accum.empty() && !o.status)   // splat sums are resolved: overflow must be seen
        return RZ_EINVAL;
    rz_batch *b = new (std::nothrow) rz_batch();
    if (!b)
        return RZ_EINVAL;
    b->pts = Pts{pts->x, pts->y, pts->z, pts->rgb, pts->n};
    b->nviews = nviews;
    b->nhq = (int32_t)accum.size();
    for (const MvView &m : accum)
        b->hq_pw = b->hq_pw || m.P.nr > 0;
    for (const MvView &m : raster)
        b->any_pw = b->any_pw || m.P.nr > 0;
    b->resolve_blocks = blocks;
    for (const MvResolve &r : res)
        b->total_px += r.npix;
    b->opts = o;
    b->tune = tune_of(o.launch);
    b->tune_hq = b->tune;
    const size_t s1 = raster.size() * sizeof(MvView);
    const size_t s2 = accum.size() * sizeof(MvView);
    const size_t s3 = res.size() * sizeof(MvResolve);
    const size_t total = s1 + s2 + s3 + 64;
    hipError_t e = hipMalloc(&b->dmem, total);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e);
    }
    char *base = (char *)b->dmem;
    b->d_raster = (MvView *)base;
    b->d_accum = (MvView *)(base + s1);
    b->d_resolve = (MvResolve *)(base + s1 + s2);
    b->d_sum = (unsigned long long *)(base + ((s1 + s2 + s3 + 15) & ~(size_t)15));
    std::vector<char> host(total, 0);
    memcpy(host.data(), raster.data(), s1);
    if (s2)
        memcpy(host.data() + s1, accum.data(), s2);
    memcpy(host.data() + s1 + s2, res.data(), s3);
    e = hipMemcpy(b->dmem, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(b->dmem);
        delete b;
        return hip_fail(e);
    }
    if (o.use_graph) {
        if ((rc = capture(b))) {
            rz_batch_destroy(b);
            return rc;
        }
    }
    *out = b;
    return RZ_OK;
}

int rz_batch_capture(rz_batch *b)
{
    if (!b)
        return RZ_EINVAL;
    int rc = capture(b);
    if (rc == RZ_OK)
        b->opts.use_graph = 1;
    return rc;
}

int rz_batch_run(rz_batch *b, void *stream)
{
    Range range("rz_batch_run");
    if (!b)
        return RZ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = b->exec ? hipGraphLaunch(b->exec, s) : enqueue(b, s);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

int rz_batch_get_opts(const rz_batch *b, rz_batch_opts *opts)
{
    if (!b || !opts)
        return RZ_EINVAL;
    *opts = b->opts;
    return RZ_OK;
}

int rz_batch_autotune(rz_batch *b, void *stream, int32_t reps, rz_batch_opts *chosen,
                      float *best_ms)
{
    if (!b || reps < 1 || reps > 100)
        return RZ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const bool had_graph = b->exec != nullptr;
    drop_graph(b);
    struct Cand {
        int32_t k, block, ppt, bin, xcd, hq_block, hq_ppt;   // hq_*: accumulate passes
    };
    std::vector<Cand> cands;
    const int32_t ks[] = {1, 2, 4, 8};
    // the one-view defaults (64 x 16 for the depth passes with 128 x 8 for
    // the accumulate passes) first, then one shape for both
    for (int32_t k : ks)
        for (int32_t xcd : {0, 1})
            cands.push_back({k, 64, 16, 2, xcd, 128, 8});
    const int32_t shapes[][2] = {{64, 16}, {128, 8}, {256, 4}, {256, 8}, {512, 8}, {256, 16}};
    for (int32_t k : ks)
        for (auto &sh : shapes)
            for (int32_t xcd : {0, 1})
                cands.push_back({k, sh[0], sh[1], 2, xcd, sh[0], sh[1]});
    for (int32_t k : ks)
        for (auto &sh : shapes)
            cands.push_back({k, sh[0], sh[1], 1, 1, sh[0], sh[1]});
    // the small per-wave tile: more waves per SIMD for the leaner shapes,
    // which also get narrower and wider workgroups here
    const int32_t lean[][2] = {{64, 4}, {128, 4}, {512, 4}, {64, 8}};
    for (int32_t k : ks) {
        cands.push_back({k, 64, 16, kBinWaveSmall, 0, 128, 8});
        for (auto &sh : shapes)
            cands.push_back({k, sh[0], sh[1], kBinWaveSmall, 0, sh[0], sh[1]});
        for (auto &sh : lean)
            cands.push_back({k, sh[0], sh[1], kBinWaveSmall, 0, sh[0], sh[1]});
    }
    cands.push_back({4, 256, 16, 0, 1, 256, 16});

    hipError_t e = hipSuccess;
    unsigned long long ref = 0, sum = 0;
    bool have_ref = false;
    float best = 1e30f;
    rz_batch_opts best_opts = b->opts;
    Tune best_tune = b->tune, best_tune_hq = b->tune_hq;
    const rz_batch_opts saved = b->opts;
    const Tune saved_tune = b->tune, saved_tune_hq = b->tune_hq;
    for (size_t ci = 0; ci < cands.size() && e == hipSuccess; ++ci) {
        const Cand &c = cands[ci];
        b->opts.views_per_group = c.k;
        b->tune.block = c.block;
        b->tune.ppt = c.ppt;
        b->tune.bin = c.bin;
        b->tune.early_out = 1;
        b->tune.xcd_remap = c.xcd;
        b->tune_hq = b->tune;
        b->tune_hq.block = c.hq_block;
        b->tune_hq.ppt = c.hq_ppt;
        // correctness: one run, then the checksum of every image
        if ((e = run_checksum(b, s, &sum)) != hipSuccess)
            break;
        if (!have_ref) {
            ref = sum;
            have_ref = true;
        } else if (sum != ref) {
            continue;   // a candidate that renders other bits is never chosen
        }
        float med = 0.f;
        if ((e = time_runs(b, s, reps, &med)) != hipSuccess)
            break;
        if (med < best) {
            best = med;
            best_opts = b->opts;
            best_opts.launch = launch_of(b->tune);
            best_tune = b->tune;
            best_tune_hq = b->tune_hq;
        }
    }
    if (e != hipSuccess) {
        b->opts = saved;
        b->tune = saved_tune;
        b->tune_hq = saved_tune_hq;
        return hip_fail(e);
    }
    b->opts = best_opts;
    b->opts.use_graph = had_graph ? 1 : 0;
    b->tune = best_tune;
    b->tune_hq = best_tune_hq;
    if (had_graph) {
        int rc = capture(b);
        if (rc)
            return rc;
    }
    if (chosen)
        *chosen = b->opts;
    if (best_ms)
        *best_ms = best;
    return RZ_OK;
}

int rz_batch_autotune_cached(rz_batch *b, void *stream, int32_t reps, const char *cache_path,
                             rz_batch_opts *chosen, float *best_ms, int32_t *hit,
                             char *key_out, int32_t key_len)
{
    if (!b || !cache_path || reps < 1 || reps > 100 || (key_out && key_len < 1))
        return RZ_EINVAL;
    if (hit)
        *hit = 0;
    hipStream_t s = (hipStream_t)stream;
    char key[160];
    int rc = batch_key(b, key, sizeof(key));
    if (rc)
        return rc;
    if (key_out) {
        strncpy(key_out, key, (size_t)key_len - 1);
        key_out[key_len - 1] = 0;
    }
    rz_tune_entry ent;
    memset(&ent, 0, sizeof(ent));
    const int found = rz_tune_cache_lookup(cache_path, key, &ent);
    if (found < 0)
        return found;
    if (found == 1) {
        const bool had_graph = b->exec != nullptr;
        drop_graph(b);
        const rz_batch_opts saved = b->opts;
        const Tune saved_tune = b->tune, saved_tune_hq = b->tune_hq;
        // the library defaults give the reference checksum; the cached
        // options must render the same bits
        b->opts.views_per_group = 1;
        b->tune = Tune();
        b->tune_hq = kHqTune;
        unsigned long long ref = 0, sum = 0;
        hipError_t e = run_checksum(b, s, &ref);
        b->opts.views_per_group = ent.views_per_group;
        b->tune = tune_of(ent.depth);
        b->tune_hq = tune_of(ent.accum);
        if (e == hipSuccess)
            e = run_checksum(b, s, &sum);
        float med = 0.f;
        if (e == hipSuccess && sum == ref)
            e = time_runs(b, s, reps, &med);
        if (e != hipSuccess || sum != ref) {
            b->opts = saved;
            b->tune = saved_tune;
            b->tune_hq = saved_tune_hq;
            if (e != hipSuccess) {
                if (had_graph)
                    (void)capture(b);
                return hip_fail(e);
            }
            if (had_graph && (rc = capture(b)))
                return rc;
            // other bits under the cached options: fall through to the search
        } else {
            b->opts.launch = ent.depth;
            b->opts.use_graph = had_graph ? 1 : 0;
            if (had_graph && (rc = capture(b)))
                return rc;
            if (chosen)
                *chosen = b->opts;
            if (best_ms)
                *best_ms = med;
            if (hit)
                *hit = 1;
            return RZ_OK;
        }
    }
    float ms = 0.f;
    if ((rc = rz_batch_autotune(b, stream, reps, chosen, &ms)))
        return rc;
    if (best_ms)
        *best_ms = ms;
    ent.views_per_group = b->opts.views_per_group;
    ent.depth = launch_of(b->tune);
    ent.accum = launch_of(b->tune_hq);
    ent.ms = ms;
    return rz_tune_cache_store(cache_path, key, &ent);
}

int rz_batch_destroy(rz_batch *b)
{
    if (!b)
        return RZ_EINVAL;
    drop_graph(b);
    if (b->cap_stream)
        (void)hipStreamDestroy(b->cap_stream);
    if (b->dmem)
        (void)hipFree(b->dmem);
    delete b;
    return RZ_OK;
}

}  // extern "C"
