// Points larger than one pixel and the float depth encodings (declared in
// include/rz.h, rasterize_points).  A point of size k covers the k x k pixels
// px - r .. px - r + k - 1 (r = (k - 1) / 2) around its own pixel, clipped to
// the screen: k^2 fragments with one key in the depth pass (section 2.1), and
// in the splat pass (section 2.2) every covered pixel tests the point
// against its own nearest depth.  As in the one-pixel kernels, each wave
// gathers its fragments in a private 8 KiB LDS tile when the rectangle they
// cover fits (it does for spatially ordered clouds), and flushes it with one
// coalesced global atomic per touched pixel; otherwise every fragment takes
// an early-out read and a global atomic.  The depth pass first keeps only
// the smallest key of a thread's consecutive points with one centre pixel;
// the splat pass reads the rectangle's nearest depths into LDS once and
// adds one packed sum word per accepted covered pixel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rz.h"
#include "rz_device.h"
#include "rz_internal.h"
#include "rz_trace.h"

namespace rz {
namespace {

using namespace dev;

constexpr int kGenBlock = 256;
constexpr int kGenPpt = 4;   // one 16-byte group of points per thread
constexpr size_t kLds = (kGenBlock / 64) * kWaveTileWords * sizeof(uint64_t);
// Splat pass: per wave, one packed sum word and the nearest depth of each
// pixel of its tile.  A wave holds 64 * kGenPpt = 256 points, and a point
// adds to a pixel at most once, so a pixel's count stays <= 256 and its
// channel sums <= 255 * 256 < 2^17: R | G << 17 | B << 34 | count << 51
// never carries between fields.
constexpr uint64_t kOneR = 1ull, kOneG = 1ull << 17, kOneB = 1ull << 34, kOneC = 1ull << 51;
static_assert(64 * kGenPpt * 255 < (1 << 17) && 64 * kGenPpt < (1 << 13), "packed sums");
constexpr size_t kLdsHq = kLds;   // kWaveTileHq sum words + kWaveTileHq depths per wave

// Covered pixels [lo, hi) along one axis for a point of size k at pixel c.
__device__ __forceinline__ void cover(uint32_t c, int32_t k, int32_t size, int32_t &lo,
                                      int32_t &hi)
{
    const int32_t a = (int32_t)c - (k - 1) / 2;
    lo = a < 0 ? 0 : a;
    hi = a + k > size ? size : a + k;
}

// Rectangle covered by the squares of a wave's points (centres in box),
// clipped to the screen; tiled when it fits `limit` pixels.
struct Cover {
    int32_t x0, y0;
    uint32_t bw, bh;
    bool tiled;
};

__device__ __forceinline__ Cover wave_cover(const Box &box, int32_t k, int32_t width,
                                            int32_t height, uint32_t limit)
{
    Cover c{0, 0, 0, 0, false};
    if (box.x0 > box.x1)
        return c;
    const int32_t r = (k - 1) / 2;
    const int32_t x0 = (int32_t)box.x0 - r, y0 = (int32_t)box.y0 - r;
    const int32_t x1 = (int32_t)box.x1 - r + k - 1, y1 = (int32_t)box.y1 - r + k - 1;
    c.x0 = x0 < 0 ? 0 : x0;
    c.y0 = y0 < 0 ? 0 : y0;
    const int32_t cx1 = x1 > width - 1 ? width - 1 : x1;
    const int32_t cy1 = y1 > height - 1 ? height - 1 : y1;
    c.bw = (uint32_t)(cx1 - c.x0 + 1);
    c.bh = (uint32_t)(cy1 - c.y0 + 1);
    c.tiled = (uint64_t)c.bw * c.bh <= limit;
    return c;
}

template <bool VEC>
__global__ void __launch_bounds__(kGenBlock) k_raster_points(Pts p, Proj P, int32_t k,
                                                             uint64_t *__restrict__ fb)
{
    extern __shared__ uint64_t s_waves[];
    uint64_t *w_tile = s_waves + (threadIdx.x >> 6) * kWaveTileWords;
    const int64_t base = (int64_t)blockIdx.x * kGenBlock * kGenPpt;
    float x[kGenPpt], y[kGenPpt], z[kGenPpt];
    uint32_t c[kGenPpt];
    bool in[kGenPpt];
    load_points<kGenPpt, VEC>(p, base, x, y, z, c, in);
    uint32_t px[kGenPpt], py[kGenPpt];
    uint64_t key[kGenPpt];
    bool live[kGenPpt];
#pragma unroll
    for (int j = 0; j < kGenPpt; ++j) {
        uint32_t a = 0, b = 0;
        uint64_t q = 0;
        live[j] = fragment_any(P, x[j], y[j], z[j], a, b, q) & in[j];
        px[j] = a;
        py[j] = b;
        key[j] = (q << 24) | ((uint64_t)c[j] & kRgbMask);
    }
    // consecutive points of a thread with one centre pixel cover the same
    // square: keep only their smaller key (k^2 atomics saved per merge)
#pragma unroll
    for (int j = 1; j < kGenPpt; ++j) {
        const bool same = live[j] && live[j - 1] && px[j] == px[j - 1] && py[j] == py[j - 1];
        const uint64_t lo = key[j] < key[j - 1] ? key[j] : key[j - 1];
        key[j] = same ? lo : key[j];
        live[j - 1] = live[j - 1] && !same;
    }
    const Cover cv = wave_cover(wave_box<kGenPpt>(px, py, live), k, P.width, P.height,
                                kWaveTileMin);
    const uint32_t lane = threadIdx.x & 63u;
    if (cv.tiled) {
        const uint32_t area = cv.bw * cv.bh;
        for (uint32_t i = lane; i < area; i += 64)
            w_tile[i] = ~0ull;
        wave_sync();
#pragma unroll
        for (int j = 0; j < kGenPpt; ++j) {
            if (!live[j])
                continue;
            int32_t x0, x1, y0, y1;
            cover(px[j], k, P.width, x0, x1);
            cover(py[j], k, P.height, y0, y1);
            for (int32_t yy = y0; yy < y1; ++yy)
                for (int32_t xx = x0; xx < x1; ++xx)
                    __hip_atomic_fetch_min(&w_tile[(uint32_t)(yy - cv.y0) * cv.bw +
                                                   (uint32_t)(xx - cv.x0)],
                                           key[j], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        wave_sync();
        const float inv_bw = 1.0f / (float)cv.bw;
        for (uint32_t i = lane; i < area; i += 64) {
            const uint64_t v = w_tile[i];
            if (v != ~0ull) {
                uint32_t r, col;
                tile_rc(i, cv.bw, inv_bw, r, col);
                uint64_t *dst = fb + (int64_t)(cv.y0 + (int32_t)r) * P.width + cv.x0 + col;
                const uint64_t cur = __hip_atomic_load(dst, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                if (v < cur)
                    __hip_atomic_fetch_min(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        wave_sync();
        return;
    }
#pragma unroll
    for (int j = 0; j < kGenPpt; ++j) {
        if (!live[j])
            continue;
        int32_t x0, x1, y0, y1;
        cover(px[j], k, P.width, x0, x1);
        cover(py[j], k, P.height, y0, y1);
        for (int32_t yy = y0; yy < y1; ++yy) {
            for (int32_t xx = x0; xx < x1; ++xx) {
                uint64_t *dst = fb + (int64_t)yy * P.width + xx;
                const uint64_t cur = __hip_atomic_load(dst, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                if (key[j] < cur)
                    __hip_atomic_fetch_min(dst, key[j], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

template <bool VEC, bool PW>
__global__ void __launch_bounds__(kGenBlock) k_hq_points(Pts p, Proj P, int32_t k,
                                                         uint32_t eps_num, uint32_t eps_den,
                                                         const uint64_t *__restrict__ fb,
                                                         uint64_t *__restrict__ acc)
{
    extern __shared__ uint64_t s_waves[];
    uint64_t *w_tile = s_waves + (threadIdx.x >> 6) * kWaveTileWords;   // packed sums
    uint64_t *w_qmin = w_tile + kWaveTileHq;                           // nearest depths
    const int64_t base = (int64_t)blockIdx.x * kGenBlock * kGenPpt;
    float x[kGenPpt], y[kGenPpt], z[kGenPpt];
    uint32_t c[kGenPpt];
    bool in[kGenPpt];
    load_points<kGenPpt, VEC>(p, base, x, y, z, c, in);
    uint32_t px[kGenPpt], py[kGenPpt];
    uint64_t q[kGenPpt];
    bool live[kGenPpt];
#pragma unroll
    for (int j = 0; j < kGenPpt; ++j) {
        uint32_t a = 0, b = 0;
        uint64_t qq = 0;
        live[j] = fragment<PW>(P, x[j], y[j], z[j], a, b, qq) & in[j];
        px[j] = a;
        py[j] = b;
        q[j] = qq;
    }
    const Cover cv = wave_cover(wave_box<kGenPpt>(px, py, live), k, P.width, P.height,
                                kWaveTileHq);
    const uint32_t lane = threadIdx.x & 63u;
    if (cv.tiled) {
        // the nearest depth of every pixel of the rectangle, read once with
        // coalesced row loads, then looked up in LDS per covered pixel
        const uint32_t area = cv.bw * cv.bh;
        const float inv_bw = 1.0f / (float)cv.bw;
        for (uint32_t i = lane; i < area; i += 64) {
            uint32_t r, col;
            tile_rc(i, cv.bw, inv_bw, r, col);
            w_qmin[i] = fb[__umul24((uint32_t)cv.y0 + r, (uint32_t)P.width) + cv.x0 + col] >> 24;
            w_tile[i] = 0ull;
        }
        wave_sync();
#pragma unroll
        for (int j = 0; j < kGenPpt; ++j) {
            if (!live[j])
                continue;
            const uint32_t col = c[j];
            const uint64_t w = (col & 0xFFu) * kOneR + ((col >> 8) & 0xFFu) * kOneG +
                               ((col >> 16) & 0xFFu) * kOneB + kOneC;
            int32_t x0, x1, y0, y1;
            cover(px[j], k, P.width, x0, x1);
            cover(py[j], k, P.height, y0, y1);
            for (int32_t yy = y0; yy < y1; ++yy) {
                const uint32_t row = __umul24((uint32_t)(yy - cv.y0), cv.bw) - (uint32_t)cv.x0;
                for (int32_t xx = x0; xx < x1; ++xx) {
                    const uint32_t t = row + (uint32_t)xx;
                    if (!in_window_live<PW>(P, eps_num, eps_den, q[j], w_qmin[t], true))
                        continue;
                    __hip_atomic_fetch_add(&w_tile[t], w, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
        wave_sync();
        for (uint32_t i = lane; i < area; i += 64) {
            const uint64_t sw = w_tile[i];
            if (sw != 0ull) {   // unpack into the accumulator's two words
                const uint64_t a0 = (sw & 0x1FFFFull) | (((sw >> 17) & 0x1FFFFull) << 32);
                const uint64_t a1 = ((sw >> 34) & 0x1FFFFull) | ((sw >> 51) << 32);
                uint32_t r, col;
                tile_rc(i, cv.bw, inv_bw, r, col);
                uint64_t *dst =
                    acc + 2 * (uint64_t)(__umul24((uint32_t)cv.y0 + r, (uint32_t)P.width) +
                                         cv.x0 + col);
                __hip_atomic_fetch_add(dst, a0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(dst + 1, a1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        wave_sync();
        return;
    }
    // the squares spread too far for the tile: global reads and atomics
#pragma unroll
    for (int j = 0; j < kGenPpt; ++j) {
        if (!live[j])
            continue;
        const uint32_t col = c[j];
        const uint64_t w0 = (uint64_t)(col & 0xFFu) | ((uint64_t)((col >> 8) & 0xFFu) << 32);
        const uint64_t w1 = (uint64_t)((col >> 16) & 0xFFu) | (1ull << 32);
        int32_t x0, x1, y0, y1;
        cover(px[j], k, P.width, x0, x1);
        cover(py[j], k, P.height, y0, y1);
        for (int32_t yy = y0; yy < y1; ++yy) {
            for (int32_t xx = x0; xx < x1; ++xx) {
                const uint64_t pp = __umul24((uint32_t)yy, (uint32_t)P.width) + (uint32_t)xx;
                if (!in_window<PW>(P, eps_num, eps_den, q[j], fb[pp] >> 24))
                    continue;
                __hip_atomic_fetch_add(acc + 2 * pp, w0, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(acc + 2 * pp + 1, w1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

bool aligned16(const Pts &p)
{
    return (((uintptr_t)p.x | (uintptr_t)p.y | (uintptr_t)p.z | (uintptr_t)p.rgb) & 15u) == 0;
}

}  // namespace

hipError_t launch_raster_points(const Pts &p, const Proj &P, int32_t k, uint64_t *fb,
                                hipStream_t s)
{
    Range r("rz depth pass (k x k points)");
    if (p.n == 0)
        return hipSuccess;
    const dim3 grid((uint32_t)((p.n + kGenBlock * kGenPpt - 1) / (kGenBlock * kGenPpt)));
    if (aligned16(p))
        hipLaunchKernelGGL((k_raster_points<true>), grid, dim3(kGenBlock), kLds, s, p, P, k, fb);
    else
        hipLaunchKernelGGL((k_raster_points<false>), grid, dim3(kGenBlock), kLds, s, p, P, k, fb);
    return hipGetLastError();
}

hipError_t launch_hq_points(const Pts &p, const Proj &P, int32_t k, uint32_t eps_num,
                            uint32_t eps_den, const uint64_t *fb, uint64_t *acc, hipStream_t s)
{
    Range r("rz splat accumulate pass (k x k points)");
    if (p.n == 0)
        return hipSuccess;
    const dim3 grid((uint32_t)((p.n + kGenBlock * kGenPpt - 1) / (kGenBlock * kGenPpt)));
    const bool v = aligned16(p), pw = P.nr != 0;
    if (v && pw)
        hipLaunchKernelGGL((k_hq_points<true, true>), grid, dim3(kGenBlock), kLdsHq, s, p, P, k,
                           eps_num, eps_den, fb, acc);
    else if (v)
        hipLaunchKernelGGL((k_hq_points<true, false>), grid, dim3(kGenBlock), kLdsHq, s, p, P, k,
                           eps_num, eps_den, fb, acc);
    else if (pw)
        hipLaunchKernelGGL((k_hq_points<false, true>), grid, dim3(kGenBlock), kLdsHq, s, p, P, k,
                           eps_num, eps_den, fb, acc);
    else
        hipLaunchKernelGGL((k_hq_points<false, false>), grid, dim3(kGenBlock), kLdsHq, s, p, P, k,
                           eps_num, eps_den, fb, acc);
    return hipGetLastError();
}

}  // namespace rz
