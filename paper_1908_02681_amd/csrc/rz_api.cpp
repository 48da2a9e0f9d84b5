// Host side of the C ABI declared in include/rz.h: argument validation,
// per-view constants (computed once per call in double precision) and the
// kernel launches.  Nothing here allocates device memory or synchronises.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include <hip/hip_runtime.h>

#include "rz.h"
#include "rz_internal.h"
#include "rz_trace.h"

namespace rz {

static thread_local int g_last_hip = 0;

bool roctx_on()
{
    static const bool on = [] {
        const char *v = getenv("RZ_ROCTX");
        return !(v && v[0] == '0' && v[1] == 0);
    }();
    return on;
}

int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return RZ_EHIP;
}

// Launch shapes, process wide: every call takes a copy under the lock, so a
// concurrent rz_set_launch never tears the shape a call launches with.
static std::mutex g_tune_mu;
static Tune g_tune;              // launch shape of the depth pass
static Tune g_tune_hq = kHqTune;  // and of the splat accumulate pass

Tune current_tune()
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    return g_tune;
}

Tune current_tune_hq()
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    return g_tune_hq;
}

constexpr double kQRange = 1099511627775.0;   // 2^40 - 1
constexpr int64_t kMaxPoints = 4294966784ll;  // 2^32 - 2^9
constexpr int32_t kMaxSide = 32768;
constexpr int32_t kMaxPointSize = 16;

static bool finite_all(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i]))
            return false;
    return true;
}

int check_points(const rz_points *p)
{
    if (!p || p->n < 0 || p->n > kMaxPoints)
        return RZ_EINVAL;
    if (p->n > 0 && (!p->x || !p->y || !p->z || !p->rgb))
        return RZ_EINVAL;
    return RZ_OK;
}

// Builds the per-view constants; validates the view and the depth map.
int make_proj(const rz_view *v, const rz_depth_map *dm, Proj *P)
{
    if (!v || !dm)
        return RZ_EINVAL;
    if (v->width < 1 || v->height < 1 || v->width > kMaxSide || v->height > kMaxSide)
        return RZ_EINVAL;
    if (!finite_all(v->vp, 16) || !isfinite(v->near_) || !isfinite(v->far_) ||
        !(v->near_ > 0.0) || !(v->far_ > v->near_))
        return RZ_EINVAL;
    double o, s;
    if (dm->kind == RZ_DEPTH_LINEAR) {
        o = v->near_;
        s = kQRange / (v->far_ - v->near_);
    } else if (dm->kind == RZ_DEPTH_SCALE) {
        if (!isfinite(dm->scale) || !(dm->scale > 0.0))
            return RZ_EINVAL;
        o = 0.0;
        s = dm->scale;
        if (!(v->far_ * s <= kQRange))
            return RZ_EDEPTHRANGE;
    } else if (dm->kind == RZ_DEPTH_PIECEWISE) {
        const int32_t nr = dm->nranges;
        if (nr < 1 || nr > RZ_MAX_RANGES || !isfinite(dm->range_start[0]) ||
            !(dm->range_start[0] <= v->near_))
            return RZ_EINVAL;
        // bases from consecutive starts (independent of far); only the
        // range that contains far bounds the depths that can occur
        double base = 0.0;
        for (int32_t k = 0; k < nr; ++k) {
            const double b = dm->range_start[k], sc = dm->range_scale[k];
            if (!isfinite(b) || !isfinite(sc) || !(sc > 0.0) ||
                (k > 0 && !(b > dm->range_start[k - 1])))
                return RZ_EINVAL;
            P->rb[k] = b;
            P->rs[k] = sc;
            P->rinv[k] = 1.0 / sc;
            P->rbase[k] = (uint64_t)base;
            if (b < v->far_) {
                const double end = k + 1 < nr && dm->range_start[k + 1] < v->far_
                                       ? dm->range_start[k + 1]
                                       : v->far_;
                if (!(base + floor((end - b) * sc) <= kQRange - 1.0))
                    return RZ_EDEPTHRANGE;
            }
            if (k + 1 < nr) {
                base += floor((dm->range_start[k + 1] - b) * sc) + 1.0;
                if (!(base < 9.0e18))
                    return RZ_EDEPTHRANGE;
            }
        }
        for (int32_t k = nr; k < 8; ++k) {
            P->rb[k] = 0.0;
            P->rs[k] = 1.0;
            P->rinv[k] = 1.0;
            P->rbase[k] = (1ull << 40) - 1;
        }
        P->rbase[nr] = (1ull << 40) - 1;
        P->rbase[8] = (1ull << 40) - 1;
        P->nr = nr;
        o = 0.0;
        s = 1.0;
    } else if (dm->kind == RZ_DEPTH_GL24 || dm->kind == RZ_DEPTH_F32REV) {
        o = 0.0;   // no integer map: the kernels encode the float depth
        s = 1.0;
    } else {
        return RZ_EINVAL;
    }
    P->zkind = dm->kind == RZ_DEPTH_GL24 || dm->kind == RZ_DEPTH_F32REV ? dm->kind : 0;
    if (dm->kind != RZ_DEPTH_PIECEWISE)
        P->nr = 0;
    if (!isfinite(s) || !(s > 0.0))
        return RZ_EDEPTHRANGE;
    const double z0 = floor(o * s);
    if (!(z0 >= 0.0 && z0 < 9.2e18))
        return RZ_EDEPTHRANGE;
    static const int rows[3] = {0, 1, 3};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c)
            P->m[4 * r + c] = (float)v->vp[4 * rows[r] + c];
    for (int c = 0; c < 4; ++c)
        P->mz[c] = (float)v->vp[8 + c];
    P->nearf = (float)v->near_;
    P->fw = (float)v->width;
    P->fh = (float)v->height;
    P->hw = 0.5f * P->fw;
    P->hh = 0.5f * P->fh;
    for (int c = 0; c < 4; ++c)
        P->v[c] = v->vp[12 + c];
    P->near_ = v->near_;
    P->far_ = v->far_;
    P->o = o;
    P->s = s;
    P->z0 = (uint64_t)z0;
    P->z0d = z0;
    P->wfp = z0 < 4503599627370496.0 ? 1 : 0;   // 2^52
    P->width = v->width;
    P->height = v->height;
    return RZ_OK;
}

// eps window limits: the integer test must not overflow 64 bits.
int check_hq(const rz_hq_params *hq, const Proj &P, uint32_t *num, uint32_t *den)
{
    uint32_t n = 1, d = 100;
    if (hq) {
        n = hq->eps_num;
        d = hq->eps_den;
    }
    if (d < 1 || d > (1u << 20) || n > (1u << 20) || P.zkind != 0)
        return RZ_EINVAL;
    // num * (2^40 + z0) < 2^63, and den * 2^40 < 2^63 holds by den <= 2^20
    // (the piecewise window is tested in double precision instead)
    if (P.nr == 0 && n > 0 &&
        (double)P.z0 + 1099511627776.0 >= 9223372036854775808.0 / (double)n)
        return RZ_EDEPTHRANGE;
    *num = n;
    *den = d;
    return RZ_OK;
}

}  // namespace rz

using namespace rz;

extern "C" {

int rasterize_atomicmin(const rz_points *pts, const rz_view *view, const rz_depth_map *depth,
                        uint32_t background, uint64_t *fb, uint32_t *img, uint32_t flags,
                        void *stream)
{
    Range range("rasterize_atomicmin");
    int rc = check_points(pts);
    if (rc)
        return rc;
    Proj P;
    if ((rc = make_proj(view, depth, &P)))
        return rc;
    if (!fb || (flags & ~RZ_KEEP_KEYS) || (!(flags & RZ_KEEP_KEYS) && !img))
        return RZ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Pts p{pts->x, pts->y, pts->z, pts->rgb, pts->n};
    hipError_t e = launch_raster_min(p, P, fb, current_tune(), s);   // every encoding
    if (e != hipSuccess)
        return hip_fail(e);
    if (!(flags & RZ_KEEP_KEYS)) {
        e = launch_resolve_min(fb, (int64_t)P.width * P.height, background, img, s);
        if (e != hipSuccess)
            return hip_fail(e);
    }
    return RZ_OK;
}

int rasterize_hq_splat(const rz_points *pts, const rz_view *view, const rz_depth_map *depth,
                       const rz_hq_params *hq, uint32_t background, uint64_t *fb, uint64_t *acc,
                       uint32_t *img, uint32_t *status, uint32_t flags, void *stream)
{
    Range range("rasterize_hq_splat");
    int rc = check_points(pts);
    if (rc)
        return rc;
    Proj P;
    if ((rc = make_proj(view, depth, &P)))
        return rc;
    uint32_t num, den;
    if ((rc = check_hq(hq, P, &num, &den)))
        return rc;
    if (!fb || !acc || (flags & ~RZ_KEEP_KEYS) ||
        (!(flags & RZ_KEEP_KEYS) && (!img || !status)))
        return RZ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Pts p{pts->x, pts->y, pts->z, pts->rgb, pts->n};
    hipError_t e = launch_raster_min(p, P, fb, current_tune(), s);
    if (e == hipSuccess)
        e = launch_hq_accum(p, P, num, den, fb, acc, current_tune_hq(), s);
    if (e == hipSuccess && !(flags & RZ_KEEP_KEYS))
        e = launch_resolve_hq(fb, acc, (int64_t)P.width * P.height, background, img, status, s);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

int rz_hq_accumulate(const rz_points *pts, const rz_view *view, const rz_depth_map *depth,
                     const rz_hq_params *hq, const uint64_t *fb, uint64_t *acc, void *stream)
{
    Range range("rz_hq_accumulate");
    int rc = check_points(pts);
    if (rc)
        return rc;
    Proj P;
    if ((rc = make_proj(view, depth, &P)))
        return rc;
    uint32_t num, den;
    if ((rc = check_hq(hq, P, &num, &den)))
        return rc;
    if (!fb || !acc)
        return RZ_EINVAL;
    const Pts p{pts->x, pts->y, pts->z, pts->rgb, pts->n};
    hipError_t e = launch_hq_accum(p, P, num, den, fb, acc, current_tune_hq(), (hipStream_t)stream);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

int rasterize_points(const rz_points *pts, const rz_view *view, const rz_depth_map *depth,
                     const rz_hq_params *hq, int32_t point_size, uint32_t background,
                     uint64_t *fb, uint64_t *acc, uint32_t *img, uint32_t *status,
                     uint32_t flags, void *stream)
{
    Range range("rasterize_points");
    int rc = check_points(pts);
    if (rc)
        return rc;
    Proj P;
    if ((rc = make_proj(view, depth, &P)))
        return rc;
    uint32_t num = 1, den = 100;
    if (hq && (rc = check_hq(hq, P, &num, &den)))
        return rc;
    if (point_size < 1 || point_size > kMaxPointSize || !fb || (hq && !acc) ||
        (flags & ~RZ_KEEP_KEYS) || (!(flags & RZ_KEEP_KEYS) && (!img || (hq && !status))))
        return RZ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Pts p{pts->x, pts->y, pts->z, pts->rgb, pts->n};
    // one-pixel points of every encoding take the depth-pass kernels (float
    // encodings are depth-only: check_hq rejects them with splatting)
    const bool general = point_size > 1;
    hipError_t e = general ? launch_raster_points(p, P, point_size, fb, s)
                           : launch_raster_min(p, P, fb, current_tune(), s);
    if (e == hipSuccess && hq)
        e = general ? launch_hq_points(p, P, point_size, num, den, fb, acc, s)
                    : launch_hq_accum(p, P, num, den, fb, acc, current_tune_hq(), s);
    const int64_t npix = (int64_t)P.width * P.height;
    if (e == hipSuccess && !(flags & RZ_KEEP_KEYS))
        e = hq ? launch_resolve_hq(fb, acc, npix, background, img, status, s)
               : launch_resolve_min(fb, npix, background, img, s);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

int rz_clear(uint64_t *fb, uint64_t *acc, int64_t npix, uint32_t background, void *stream)
{
    if (npix < 0 || (npix > 0 && !fb))
        return RZ_EINVAL;
    hipError_t e = launch_clear(fb, acc, npix, background, (hipStream_t)stream);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

int rz_resolve_min(uint64_t *fb, int64_t npix, uint32_t background, uint32_t *img, void *stream)
{
    if (npix < 0 || (npix > 0 && (!fb || !img)))
        return RZ_EINVAL;
    hipError_t e = launch_resolve_min(fb, npix, background, img, (hipStream_t)stream);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

int rz_resolve_hq(uint64_t *fb, uint64_t *acc, int64_t npix, uint32_t background, uint32_t *img,
                  uint32_t *status, void *stream)
{
    if (npix < 0 || !status || (npix > 0 && (!fb || !acc || !img)))
        return RZ_EINVAL;
    hipError_t e = launch_resolve_hq(fb, acc, npix, background, img, status, (hipStream_t)stream);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

int rz_set_launch(const rz_launch *l)
{
    if (!l) {   // back to the library defaults
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune = Tune();
        g_tune_hq = kHqTune;
        return RZ_OK;
    }
    if (!(l->block == 64 || l->block == 128 || l->block == 256 || l->block == 512))
        return RZ_EINVAL;
    if (!(l->ppt == 4 || l->ppt == 8 || l->ppt == 16))
        return RZ_EINVAL;
    if ((l->early_out & ~1) || (l->xcd_remap & ~1) || l->bin < 0 || l->bin > 3)
        return RZ_EINVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.block = l->block;
    g_tune.ppt = l->ppt;
    g_tune.early_out = l->early_out;
    g_tune.xcd_remap = l->xcd_remap;
    g_tune.bin = l->bin;
    g_tune_hq = g_tune;
    return RZ_OK;
}

int rz_get_launch(rz_launch *l)
{
    if (!l)
        return RZ_EINVAL;
    const Tune t = current_tune();
    l->block = t.block;
    l->ppt = t.ppt;
    l->early_out = t.early_out;
    l->xcd_remap = t.xcd_remap;
    l->bin = t.bin;
    return RZ_OK;
}

const char *rz_error_string(int code)
{
    switch (code) {
    case RZ_OK: return "ok";
    case RZ_EINVAL: return "invalid argument";
    case RZ_EDEPTHRANGE: return "depth range does not fit the 40-bit depth map";
    case RZ_EHIP: return "HIP runtime error";
    case RZ_EOVERFLOW: return "splat count overflow";
    case RZ_EBUDGET: return "request exceeds the memory budget";
    case RZ_ESTATE: return "object in the wrong state";
    case RZ_EIO: return "file could not be written";
    default: return "unknown error";
    }
}

int rz_last_hip_error(void) { return g_last_hip; }

int rz_version(void) { return 100; }

}  // extern "C"
