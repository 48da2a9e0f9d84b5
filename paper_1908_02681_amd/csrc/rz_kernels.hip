// HIP kernels of the point rasterizer for gfx950 (MI355X).
//
// Method: Schuetz & Wimmer, "Rendering Point Clouds with Compute Shaders"
// (arXiv 1908.02681), section 2.1 (atomicMin rasterization, resolve/clear)
// and section 2.2 (high-quality splatting: depth pass, eps-window
// accumulation, normalisation).
//
// Floating point: this file must be compiled with -ffp-contract=off (and
// the pragma below repeats it), so that the projection is the exact IEEE
// sequence of operations stated in include/rz.h: no fused multiply-add,
// correctly rounded f32 division, no flush of denormals.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rz.h"
#include "rz_internal.h"

#pragma clang fp contract(off)

namespace rz {
namespace {

constexpr double kQMax = 1099511627774.0;   // 2^40 - 2
constexpr int kXcds = 8;                     // XCDs of an MI355X

// The fragment of one point: pixel index and 40-bit depth (section 2.1).
// Returns false when the point is discarded.
__device__ __forceinline__ bool fragment(const Proj &P, float x, float y, float z,
                                         uint32_t &pix, uint64_t &q)
{
    float cx = P.m[0] * x;
    cx = cx + P.m[1] * y;
    cx = cx + P.m[2] * z;
    cx = cx + P.m[3];
    float cy = P.m[4] * x;
    cy = cy + P.m[5] * y;
    cy = cy + P.m[6] * z;
    cy = cy + P.m[7];
    float cw = P.m[8] * x;
    cw = cw + P.m[9] * y;
    cw = cw + P.m[10] * z;
    cw = cw + P.m[11];
    if (!(cw > 0.0f))
        return false;
    const float nx = cx / cw;
    const float ny = cy / cw;
    const float fx = (nx + 1.0f) * P.hw;
    const float fy = (ny + 1.0f) * P.hh;
    if (!(fx >= 0.0f && fx < P.fw && fy >= 0.0f && fy < P.fh))
        return false;
    const uint32_t px = (uint32_t)(int32_t)fx;
    const uint32_t py = (uint32_t)(int32_t)fy;

    // depth in double precision (section 1, section 2.1)
    double d = P.v[0] * (double)x;
    d = d + P.v[1] * (double)y;
    d = d + P.v[2] * (double)z;
    d = d + P.v[3];
    if (!(d >= P.near_ && d < P.far_))
        return false;
    double tf = floor((d - P.o) * P.s);
    if (tf > kQMax)
        tf = kQMax;
    // 0 <= tf < 2^40: split into two exact 32-bit halves
    const uint32_t hi = (uint32_t)(tf * 0x1p-32);
    const uint32_t lo = (uint32_t)(tf - (double)hi * 0x1p32);
    q = ((uint64_t)hi << 32) | lo;
    pix = py * (uint32_t)P.width + px;
    return true;
}

// Workgroup -> chunk of points.  Workgroups are dealt round-robin to the 8
// XCDs; with the remap, XCD k works through the k-th eighth of the point
// array, so spatially coherent (e.g. Morton-ordered) ranges share one L2.
template <bool XCD>
__device__ __forceinline__ int64_t chunk_index()
{
    const int64_t b = blockIdx.x;
    if (!XCD)
        return b;
    const int64_t per = gridDim.x / kXcds;   // grid is a multiple of 8
    return (b % kXcds) * per + b / kXcds;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// Streaming (non-temporal) access: the data is touched once.
template <typename T>
__device__ __forceinline__ T ldnt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void stnt(T v, T *p) { __builtin_nontemporal_store(v, p); }

// Loads the PPT points of this thread.  Vector form: PPT/4 groups of four
// consecutive points, group g at chunk + g*4*blockDim + 4*tid, so every
// load instruction of a wave reads one contiguous 1 KiB span per plane.
// Scalar form (tail chunk or unaligned planes): same point indices, bounds
// checked one by one.
template <int PPT, bool VEC>
__device__ __forceinline__ void load_points(const Pts &p, int64_t base, float (&x)[PPT],
                                            float (&y)[PPT], float (&z)[PPT],
                                            uint32_t (&c)[PPT], bool (&in)[PPT])
{
    const int64_t stride = 4 * (int64_t)blockDim.x;
    const int64_t first = base + 4 * (int64_t)threadIdx.x;
    const bool full = VEC && base + stride * (PPT / 4) <= p.n;
    if (full) {
#pragma unroll
        for (int g = 0; g < PPT / 4; ++g) {
            const int64_t i = first + g * stride;
            const f32x4 vx = ldnt(reinterpret_cast<const f32x4 *>(p.x + i));
            const f32x4 vy = ldnt(reinterpret_cast<const f32x4 *>(p.y + i));
            const f32x4 vz = ldnt(reinterpret_cast<const f32x4 *>(p.z + i));
            const u32x4 vc = ldnt(reinterpret_cast<const u32x4 *>(p.rgb + i));
            x[4 * g + 0] = vx.x; x[4 * g + 1] = vx.y; x[4 * g + 2] = vx.z; x[4 * g + 3] = vx.w;
            y[4 * g + 0] = vy.x; y[4 * g + 1] = vy.y; y[4 * g + 2] = vy.z; y[4 * g + 3] = vy.w;
            z[4 * g + 0] = vz.x; z[4 * g + 1] = vz.y; z[4 * g + 2] = vz.z; z[4 * g + 3] = vz.w;
            c[4 * g + 0] = vc.x; c[4 * g + 1] = vc.y; c[4 * g + 2] = vc.z; c[4 * g + 3] = vc.w;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                in[4 * g + k] = true;
        }
    } else {
#pragma unroll
        for (int g = 0; g < PPT / 4; ++g) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t i = first + g * stride + k;
                const bool ok = i < p.n;
                in[4 * g + k] = ok;
                x[4 * g + k] = ok ? p.x[i] : 0.0f;
                y[4 * g + k] = ok ? p.y[i] : 0.0f;
                z[4 * g + k] = ok ? p.z[i] : 0.0f;
                c[4 * g + k] = ok ? p.rgb[i] : 0u;
            }
        }
    }
}

// Depth pass (section 2.1): one 64-bit atomic minimum per surviving
// fragment.  Two refinements that never change the result, because the
// framebuffer only ever decreases and min is order independent:
//  - consecutive fragments of one thread that hit the same pixel are merged
//    in registers first;
//  - with EARLY, the current framebuffer value is read first and the atomic
//    is skipped when it is already <= the key (a stale read can only be
//    larger than the true value, so the skip is always safe).
template <int PPT, bool VEC, bool EARLY, bool XCD>
__global__ void __launch_bounds__(512) k_raster_min(Pts p, Proj P, uint64_t *__restrict__ fb,
                                                    int64_t nchunks)
{
    const int64_t chunk = chunk_index<XCD>();
    if (chunk >= nchunks)
        return;
    const int64_t base = chunk * (int64_t)blockDim.x * PPT;
    float x[PPT], y[PPT], z[PPT];
    uint32_t c[PPT];
    bool in[PPT];
    load_points<PPT, VEC>(p, base, x, y, z, c, in);

    // Straight-line selects only: no array element is updated inside a
    // divergent branch (a form this compiler has been seen to mis-allocate).
    uint32_t pix[PPT];
    uint64_t key[PPT];
    bool live[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        uint64_t q = 0;
        uint32_t px = 0;
        live[j] = in[j] && fragment(P, x[j], y[j], z[j], px, q);
        pix[j] = px;
        key[j] = (q << 24) | ((uint64_t)c[j] & kRgbMask);
    }
#pragma unroll
    for (int j = 1; j < PPT; ++j) {
        const bool same = live[j] && live[j - 1] && pix[j] == pix[j - 1];
        const uint64_t lo = key[j] < key[j - 1] ? key[j] : key[j - 1];
        key[j] = same ? lo : key[j];
        live[j - 1] = live[j - 1] && !same;
    }
    if (EARLY) {
        uint64_t cur[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            cur[j] = __hip_atomic_load(fb + (live[j] ? pix[j] : 0u), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            if (live[j] && key[j] < cur[j])
                __hip_atomic_fetch_min(fb + pix[j], key[j], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    } else {
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            if (live[j])
                __hip_atomic_fetch_min(fb + pix[j], key[j], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Accumulation pass of high-quality splatting (section 2.2).  Reprojects
// every point, compares its depth with the finished depth pass and, inside
// the eps window, adds its colour and a count with two 64-bit atomic adds:
// acc[2p] += R + (G << 32), acc[2p+1] += B + (1 << 32).  Consecutive
// accepted fragments of one thread in the same pixel are summed first.
template <int PPT, bool VEC, bool XCD>
__global__ void __launch_bounds__(512) k_hq_accum(Pts p, Proj P, uint32_t eps_num,
                                                  uint32_t eps_den,
                                                  const uint64_t *__restrict__ fb,
                                                  uint64_t *__restrict__ acc, int64_t nchunks)
{
    const int64_t chunk = chunk_index<XCD>();
    if (chunk >= nchunks)
        return;
    const int64_t base = chunk * (int64_t)blockDim.x * PPT;
    float x[PPT], y[PPT], z[PPT];
    uint32_t c[PPT];
    bool in[PPT];
    load_points<PPT, VEC>(p, base, x, y, z, c, in);

    uint32_t pix[PPT];
    uint64_t q[PPT];
    bool ok[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        uint32_t px = 0;
        uint64_t qq = 0;
        ok[j] = in[j] && fragment(P, x[j], y[j], z[j], px, qq);
        pix[j] = px;
        q[j] = qq;
    }
    // eps window against the finished depth pass; flags only, no in-branch
    // updates of the arrays (see k_raster_min)
    // all loads first (discarded fragments read pixel 0, always in bounds),
    // so that they are in flight together
    uint64_t fbv[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        fbv[j] = fb[ok[j] ? pix[j] : 0u];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint64_t qmin = fbv[j] >> 24;
        ok[j] = ok[j] &&
                (uint64_t)eps_den * (q[j] - qmin) <= (uint64_t)eps_num * (qmin + P.z0);
    }
    uint64_t w0[PPT], w1[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        w0[j] = (uint64_t)(c[j] & 0xFFu) | ((uint64_t)((c[j] >> 8) & 0xFFu) << 32);
        w1[j] = (uint64_t)((c[j] >> 16) & 0xFFu) | (1ull << 32);
    }
#pragma unroll
    for (int j = 1; j < PPT; ++j) {
        const bool same = ok[j] && ok[j - 1] && pix[j] == pix[j - 1];
        w0[j] += same ? w0[j - 1] : 0ull;
        w1[j] += same ? w1[j - 1] : 0ull;
        ok[j - 1] = ok[j - 1] && !same;
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (ok[j]) {
            uint64_t *a = acc + 2 * (uint64_t)pix[j];
            __hip_atomic_fetch_add(a, w0[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(a + 1, w1[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Resolve of section 2.1: colour bits to the image, framebuffer cleared.
__global__ void __launch_bounds__(256) k_resolve_min(uint64_t *__restrict__ fb, int64_t npix,
                                                     uint64_t clear, uint32_t *__restrict__ img,
                                                     bool vec)
{
    const int64_t i = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (vec && i + 1 < npix) {
        const u64x2 k = ldnt(reinterpret_cast<const u64x2 *>(fb + i));
        u32x2 o;
        o.x = (uint32_t)(k.x & kRgbMask);
        o.y = (uint32_t)(k.y & kRgbMask);
        stnt(o, reinterpret_cast<u32x2 *>(img + i));
        u64x2 cl;
        cl.x = clear;
        cl.y = clear;
        *reinterpret_cast<u64x2 *>(fb + i) = cl;
    } else {
        for (int64_t k = i; k < i + 2 && k < npix; ++k) {
            img[k] = (uint32_t)(fb[k] & kRgbMask);
            fb[k] = clear;
        }
    }
}

__device__ __forceinline__ uint32_t hq_colour(uint64_t w0, uint64_t w1, uint32_t bg,
                                              bool &overflow)
{
    const uint64_t cnt = w1 >> 32;
    if (cnt == 0)
        return bg;
    overflow = cnt > kHqCountMax;
    const double den = 2.0 * (double)cnt;
    // numerators < 2^34: the double quotient floors exactly
    const uint32_t r = (uint32_t)floor((2.0 * (double)(w0 & 0xFFFFFFFFull) + (double)cnt) / den);
    const uint32_t g = (uint32_t)floor((2.0 * (double)(w0 >> 32) + (double)cnt) / den);
    const uint32_t b = (uint32_t)floor((2.0 * (double)(w1 & 0xFFFFFFFFull) + (double)cnt) / den);
    return (r & 0xFFu) | ((g & 0xFFu) << 8) | ((b & 0xFFu) << 16);
}

// Third pass of section 2.2: average colour (or background), then fb and
// acc cleared.  fb is only written: a pixel has accepted fragments exactly
// when the depth pass wrote it, so the count alone decides.
__global__ void __launch_bounds__(256) k_resolve_hq(uint64_t *__restrict__ fb,
                                                    uint64_t *__restrict__ acc, int64_t npix,
                                                    uint64_t clear, uint32_t bg,
                                                    uint32_t *__restrict__ img,
                                                    uint32_t *__restrict__ status, bool vec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix)
        return;
    bool overflow = false;
    if (vec) {
        const u64x2 a = ldnt(reinterpret_cast<const u64x2 *>(acc + 2 * i));
        img[i] = hq_colour(a.x, a.y, bg, overflow);
        u64x2 zero;
        zero.x = 0;
        zero.y = 0;
        *reinterpret_cast<u64x2 *>(acc + 2 * i) = zero;
    } else {
        img[i] = hq_colour(acc[2 * i], acc[2 * i + 1], bg, overflow);
        acc[2 * i] = 0;
        acc[2 * i + 1] = 0;
    }
    fb[i] = clear;
    if (overflow && status)
        atomicOr(status, RZ_STATUS_HQ_OVERFLOW);
}

__global__ void __launch_bounds__(256) k_clear(uint64_t *__restrict__ fb,
                                               uint64_t *__restrict__ acc, int64_t npix,
                                               uint64_t clear)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix)
        return;
    fb[i] = clear;
    if (acc) {
        acc[2 * i] = 0;
        acc[2 * i + 1] = 0;
    }
}

bool aligned16(const void *ptr) { return ((uintptr_t)ptr & 15u) == 0; }

int64_t blocks_for(int64_t n, int64_t per) { return (n + per - 1) / per; }

template <int PPT, bool VEC, bool EARLY>
hipError_t raster_min_ppt(const Pts &p, const Proj &P, uint64_t *fb, const Tune &t,
                          hipStream_t s)
{
    const int64_t nchunks = blocks_for(p.n, (int64_t)t.block * PPT);
    int64_t grid = nchunks;
    if (t.xcd_remap) {
        grid = (nchunks + kXcds - 1) / kXcds * kXcds;
        hipLaunchKernelGGL((k_raster_min<PPT, VEC, EARLY, true>), dim3((uint32_t)grid),
                           dim3(t.block), 0, s, p, P, fb, nchunks);
    } else {
        hipLaunchKernelGGL((k_raster_min<PPT, VEC, EARLY, false>), dim3((uint32_t)grid),
                           dim3(t.block), 0, s, p, P, fb, nchunks);
    }
    return hipGetLastError();
}

template <int PPT, bool VEC>
hipError_t hq_accum_ppt(const Pts &p, const Proj &P, uint32_t num, uint32_t den,
                        const uint64_t *fb, uint64_t *acc, const Tune &t, hipStream_t s)
{
    const int64_t nchunks = blocks_for(p.n, (int64_t)t.block * PPT);
    int64_t grid = nchunks;
    if (t.xcd_remap) {
        grid = (nchunks + kXcds - 1) / kXcds * kXcds;
        hipLaunchKernelGGL((k_hq_accum<PPT, VEC, true>), dim3((uint32_t)grid), dim3(t.block),
                           0, s, p, P, num, den, fb, acc, nchunks);
    } else {
        hipLaunchKernelGGL((k_hq_accum<PPT, VEC, false>), dim3((uint32_t)grid), dim3(t.block),
                           0, s, p, P, num, den, fb, acc, nchunks);
    }
    return hipGetLastError();
}

bool planes_aligned(const Pts &p)
{
    return aligned16(p.x) && aligned16(p.y) && aligned16(p.z) && aligned16(p.rgb);
}

}  // namespace

hipError_t launch_raster_min(const Pts &p, const Proj &P, uint64_t *fb, const Tune &t,
                             hipStream_t s)
{
    if (p.n == 0)
        return hipSuccess;
    const bool vec = planes_aligned(p);
#define RZ_RASTER_CASE(PPT)                                                       \
    case PPT:                                                                     \
        if (vec)                                                                  \
            return t.early_out ? raster_min_ppt<PPT, true, true>(p, P, fb, t, s)  \
                               : raster_min_ppt<PPT, true, false>(p, P, fb, t, s); \
        return t.early_out ? raster_min_ppt<PPT, false, true>(p, P, fb, t, s)     \
                           : raster_min_ppt<PPT, false, false>(p, P, fb, t, s);
    switch (t.ppt) {
        RZ_RASTER_CASE(4)
        RZ_RASTER_CASE(8)
        RZ_RASTER_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef RZ_RASTER_CASE
}

hipError_t launch_hq_accum(const Pts &p, const Proj &P, uint32_t num, uint32_t den,
                           const uint64_t *fb, uint64_t *acc, const Tune &t, hipStream_t s)
{
    if (p.n == 0)
        return hipSuccess;
    const bool vec = planes_aligned(p);
    switch (t.ppt) {
    case 4:
        return vec ? hq_accum_ppt<4, true>(p, P, num, den, fb, acc, t, s)
                   : hq_accum_ppt<4, false>(p, P, num, den, fb, acc, t, s);
    case 8:
        return vec ? hq_accum_ppt<8, true>(p, P, num, den, fb, acc, t, s)
                   : hq_accum_ppt<8, false>(p, P, num, den, fb, acc, t, s);
    case 16:
        return vec ? hq_accum_ppt<16, true>(p, P, num, den, fb, acc, t, s)
                   : hq_accum_ppt<16, false>(p, P, num, den, fb, acc, t, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_resolve_min(uint64_t *fb, int64_t npix, uint32_t bg, uint32_t *img,
                              hipStream_t s)
{
    if (npix == 0)
        return hipSuccess;
    const uint64_t clear = kDepthOnes | ((uint64_t)bg & kRgbMask);
    const int64_t grid = blocks_for((npix + 1) / 2, 256);
    const bool vec = aligned16(fb) && ((uintptr_t)img & 7u) == 0;
    hipLaunchKernelGGL(k_resolve_min, dim3((uint32_t)grid), dim3(256), 0, s, fb, npix, clear,
                       img, vec);
    return hipGetLastError();
}

hipError_t launch_resolve_hq(uint64_t *fb, uint64_t *acc, int64_t npix, uint32_t bg,
                             uint32_t *img, uint32_t *status, hipStream_t s)
{
    if (npix == 0)
        return hipSuccess;
    const uint64_t clear = kDepthOnes | ((uint64_t)bg & kRgbMask);
    hipLaunchKernelGGL(k_resolve_hq, dim3((uint32_t)blocks_for(npix, 256)), dim3(256), 0, s, fb,
                       acc, npix, clear, bg & (uint32_t)kRgbMask, img, status, aligned16(acc));
    return hipGetLastError();
}

hipError_t launch_clear(uint64_t *fb, uint64_t *acc, int64_t npix, uint32_t bg, hipStream_t s)
{
    if (npix == 0)
        return hipSuccess;
    const uint64_t clear = kDepthOnes | ((uint64_t)bg & kRgbMask);
    hipLaunchKernelGGL(k_clear, dim3((uint32_t)blocks_for(npix, 256)), dim3(256), 0, s, fb, acc,
                       npix, clear);
    return hipGetLastError();
}

}  // namespace rz
