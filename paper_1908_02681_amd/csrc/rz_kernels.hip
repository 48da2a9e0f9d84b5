// Single-view HIP kernels of the point rasterizer for gfx950 (MI355X) and
// their launchers: the depth pass (k_raster_min), the accumulate pass of
// high-quality splatting (k_hq_accum), the two resolve passes and clear.
//
// Method: Schuetz & Wimmer, "Rendering Point Clouds with Compute Shaders"
// (arXiv 1908.02681), section 2.1 and section 2.2.  The per-chunk bodies
// live in rz_device.h, shared with the multi-view batch kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rz.h"
#include "rz_device.h"
#include "rz_internal.h"
#include "rz_trace.h"

namespace rz {
namespace {

using namespace dev;

// Depth pass of section 2.1 for one view: one workgroup per chunk of
// blockDim * PPT consecutive points.
template <int PPT, bool VEC, bool EARLY, bool XCD, int BIN, bool PW>
__global__ void __launch_bounds__(512) k_raster_min(Pts p, Proj P, uint64_t *__restrict__ fb,
                                                    int64_t nchunks, uint32_t words)
{
    __shared__ uint64_t s_tile[BIN == kBinBlock ? kTileMin : 1];
    __shared__ uint32_t s_box[kMaxWaves][4];
    extern __shared__ uint64_t s_waves[];   // kBinWave: `words` per wave
    const int64_t chunk = chunk_index<XCD>();
    if (chunk >= nchunks)
        return;
    float x[PPT], y[PPT], z[PPT];
    uint32_t c[PPT];
    bool in[PPT];
    const int64_t base = chunk * (int64_t)blockDim.x * PPT;
    uint64_t *w_tile = s_waves + (threadIdx.x >> 6) * words;
    // no per-point bounds flags: points past the end load as NaN and are culled
    load_points_nan<PPT, VEC>(p, base, x, y, z, c);
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        in[j] = true;
    if (BIN == kBinWave)
        raster_chunk_wave<PPT, PW>(P, fb, x, y, z, c, in, w_tile, words);
    else
        raster_chunk<PPT, EARLY, BIN == kBinBlock, PW>(P, fb, x, y, z, c, in, s_tile, s_box);
}

// Depth pass for the float depth encodings (RZ_DEPTH_GL24, RZ_DEPTH_F32REV)
// at one pixel per point: the per-wave tile kernel with the encoding's key.
template <bool VEC, int ZK>
__global__ void __launch_bounds__(512) k_raster_min_zk(Pts p, Proj P, uint64_t *__restrict__ fb,
                                                       int64_t nchunks, uint32_t words)
{
    constexpr int PPT = 16;
    extern __shared__ uint64_t s_waves[];
    const int64_t chunk = blockIdx.x;
    if (chunk >= nchunks)
        return;
    float x[PPT], y[PPT], z[PPT];
    uint32_t c[PPT];
    bool in[PPT];
    load_points_nan<PPT, VEC>(p, chunk * (int64_t)blockDim.x * PPT, x, y, z, c);
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        in[j] = true;
    raster_chunk_wave<PPT, false, ZK>(P, fb, x, y, z, c, in,
                                      s_waves + (threadIdx.x >> 6) * words, words);
}

// Accumulation pass of section 2.2 for one view.
template <int PPT, bool VEC, bool XCD, int BIN, bool PW>
__global__ void __launch_bounds__(512) k_hq_accum(Pts p, Proj P, uint32_t eps_num,
                                                  uint32_t eps_den,
                                                  const uint64_t *__restrict__ fb,
                                                  uint64_t *__restrict__ acc, int64_t nchunks,
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
    const int64_t base = chunk * (int64_t)blockDim.x * PPT;
    uint64_t *w_tile = s_waves + (threadIdx.x >> 6) * words;
    load_points_nan<PPT, VEC>(p, base, x, y, z, c);
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        in[j] = true;
    if (BIN == kBinWave)
        accum_chunk_wave<PPT, PW>(P, eps_num, eps_den, fb, acc, x, y, z, c, in, w_tile, words);
    else
        accum_chunk<PPT, BIN == kBinBlock, PW>(P, eps_num, eps_den, fb, acc, x, y, z, c, in,
                                               s_tile, s_box);
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

// Dynamic LDS of a launch: the per-wave tiles of kBinWave / kBinWaveSmall.
size_t wave_lds(int bin, int block)
{
    return bin == kBinWave || bin == kBinWaveSmall
               ? (size_t)(block / 64) * wave_tile_words(bin) * sizeof(uint64_t)
               : 0;
}

template <int PPT, bool VEC, bool EARLY, int BIN, bool PW>
hipError_t raster_min_ppt(const Pts &p, const Proj &P, uint64_t *fb, const Tune &t,
                          hipStream_t s)
{
    const int64_t nchunks = blocks_for(p.n, (int64_t)t.block * PPT);
    const size_t lds = wave_lds(t.bin, t.block);
    const uint32_t words = wave_tile_words(t.bin);
    if (t.xcd_remap) {
        const int64_t grid = (nchunks + kXcds - 1) / kXcds * kXcds;
        hipLaunchKernelGGL((k_raster_min<PPT, VEC, EARLY, true, BIN, PW>), dim3((uint32_t)grid),
                           dim3(t.block), lds, s, p, P, fb, nchunks, words);
    } else {
        hipLaunchKernelGGL((k_raster_min<PPT, VEC, EARLY, false, BIN, PW>),
                           dim3((uint32_t)nchunks),
                           dim3(t.block), lds, s, p, P, fb, nchunks, words);
    }
    return hipGetLastError();
}

template <int PPT, bool VEC, int BIN, bool PW>
hipError_t hq_accum_ppt(const Pts &p, const Proj &P, uint32_t num, uint32_t den,
                        const uint64_t *fb, uint64_t *acc, const Tune &t, hipStream_t s)
{
    const int64_t nchunks = blocks_for(p.n, (int64_t)t.block * PPT);
    const size_t lds = wave_lds(t.bin, t.block);
    const uint32_t words = wave_tile_words(t.bin);
    if (t.xcd_remap) {
        const int64_t grid = (nchunks + kXcds - 1) / kXcds * kXcds;
        hipLaunchKernelGGL((k_hq_accum<PPT, VEC, true, BIN, PW>), dim3((uint32_t)grid),
                           dim3(t.block), lds, s, p, P, num, den, fb, acc, nchunks, words);
    } else {
        hipLaunchKernelGGL((k_hq_accum<PPT, VEC, false, BIN, PW>), dim3((uint32_t)nchunks),
                           dim3(t.block), lds, s, p, P, num, den, fb, acc, nchunks, words);
    }
    return hipGetLastError();
}

bool planes_aligned(const Pts &p)
{
    return aligned16(p.x) && aligned16(p.y) && aligned16(p.z) && aligned16(p.rgb);
}

template <int PPT, bool VEC, bool PW>
hipError_t raster_min_bin(const Pts &p, const Proj &P, uint64_t *fb, const Tune &t,
                          hipStream_t s)
{
    switch (t.bin) {
    case kBinBlock: return raster_min_ppt<PPT, VEC, true, kBinBlock, PW>(p, P, fb, t, s);
    case kBinWave:
    case kBinWaveSmall: return raster_min_ppt<PPT, VEC, true, kBinWave, PW>(p, P, fb, t, s);
    default:
        return t.early_out ? raster_min_ppt<PPT, VEC, true, kBinNone, PW>(p, P, fb, t, s)
                           : raster_min_ppt<PPT, VEC, false, kBinNone, PW>(p, P, fb, t, s);
    }
}

template <int PPT, bool VEC>
hipError_t raster_min_vec(const Pts &p, const Proj &P, uint64_t *fb, const Tune &t,
                          hipStream_t s)
{
    return P.nr ? raster_min_bin<PPT, VEC, true>(p, P, fb, t, s)
                : raster_min_bin<PPT, VEC, false>(p, P, fb, t, s);
}

template <int PPT>
hipError_t raster_min_dispatch(const Pts &p, const Proj &P, uint64_t *fb, const Tune &t,
                               hipStream_t s)
{
    return planes_aligned(p) ? raster_min_vec<PPT, true>(p, P, fb, t, s)
                             : raster_min_vec<PPT, false>(p, P, fb, t, s);
}

template <int PPT, bool VEC, bool PW>
hipError_t hq_accum_bin(const Pts &p, const Proj &P, uint32_t num, uint32_t den,
                        const uint64_t *fb, uint64_t *acc, const Tune &t, hipStream_t s)
{
    switch (t.bin) {
    case kBinBlock: return hq_accum_ppt<PPT, VEC, kBinBlock, PW>(p, P, num, den, fb, acc, t, s);
    case kBinWave:
    case kBinWaveSmall:
        return hq_accum_ppt<PPT, VEC, kBinWave, PW>(p, P, num, den, fb, acc, t, s);
    default: return hq_accum_ppt<PPT, VEC, kBinNone, PW>(p, P, num, den, fb, acc, t, s);
    }
}

template <int PPT, bool VEC>
hipError_t hq_accum_vec(const Pts &p, const Proj &P, uint32_t num, uint32_t den,
                        const uint64_t *fb, uint64_t *acc, const Tune &t, hipStream_t s)
{
    return P.nr ? hq_accum_bin<PPT, VEC, true>(p, P, num, den, fb, acc, t, s)
                : hq_accum_bin<PPT, VEC, false>(p, P, num, den, fb, acc, t, s);
}

template <int PPT>
hipError_t hq_accum_dispatch(const Pts &p, const Proj &P, uint32_t num, uint32_t den,
                             const uint64_t *fb, uint64_t *acc, const Tune &t, hipStream_t s)
{
    return planes_aligned(p) ? hq_accum_vec<PPT, true>(p, P, num, den, fb, acc, t, s)
                             : hq_accum_vec<PPT, false>(p, P, num, den, fb, acc, t, s);
}

template <int ZK>
hipError_t raster_min_zk(const Pts &p, const Proj &P, uint64_t *fb, const Tune &t, hipStream_t s)
{
    const int64_t nchunks = blocks_for(p.n, (int64_t)t.block * 16);
    const size_t lds = wave_lds(t.bin, t.block);
    const uint32_t words = wave_tile_words(t.bin);
    if (planes_aligned(p))
        hipLaunchKernelGGL((k_raster_min_zk<true, ZK>), dim3((uint32_t)nchunks), dim3(t.block),
                           lds, s, p, P, fb, nchunks, words);
    else
        hipLaunchKernelGGL((k_raster_min_zk<false, ZK>), dim3((uint32_t)nchunks), dim3(t.block),
                           lds, s, p, P, fb, nchunks, words);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_min(const Pts &p, const Proj &P, uint64_t *fb, const Tune &t,
                             hipStream_t s)
{
    Range r("rz depth pass");
    if (p.n == 0)
        return hipSuccess;
    if (P.zkind != 0) {
        // float depth encodings: the per-wave tile kernel (either tile
        // size) at 16 points per thread, the general point kernel for every
        // other launch shape
        if ((t.bin != kBinWave && t.bin != kBinWaveSmall) || t.ppt != 16 || t.xcd_remap)
            return launch_raster_points(p, P, 1, fb, s);
        return P.zkind == RZ_DEPTH_GL24 ? raster_min_zk<RZ_DEPTH_GL24>(p, P, fb, t, s)
                                        : raster_min_zk<RZ_DEPTH_F32REV>(p, P, fb, t, s);
    }
    switch (t.ppt) {
    case 4: return raster_min_dispatch<4>(p, P, fb, t, s);
    case 8: return raster_min_dispatch<8>(p, P, fb, t, s);
    case 16: return raster_min_dispatch<16>(p, P, fb, t, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hq_accum(const Pts &p, const Proj &P, uint32_t num, uint32_t den,
                           const uint64_t *fb, uint64_t *acc, const Tune &t, hipStream_t s)
{
    Range r("rz splat accumulate pass");
    if (p.n == 0)
        return hipSuccess;
    switch (t.ppt) {
    case 4: return hq_accum_dispatch<4>(p, P, num, den, fb, acc, t, s);
    case 8: return hq_accum_dispatch<8>(p, P, num, den, fb, acc, t, s);
    case 16: return hq_accum_dispatch<16>(p, P, num, den, fb, acc, t, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_resolve_min(uint64_t *fb, int64_t npix, uint32_t bg, uint32_t *img,
                              hipStream_t s)
{
    Range r("rz resolve (atomicMin)");
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
    Range r("rz resolve (splatting)");
    if (npix == 0)
        return hipSuccess;
    const uint64_t clear = kDepthOnes | ((uint64_t)bg & kRgbMask);
    hipLaunchKernelGGL(k_resolve_hq, dim3((uint32_t)blocks_for(npix, 256)), dim3(256), 0, s, fb,
                       acc, npix, clear, bg & (uint32_t)kRgbMask, img, status, aligned16(acc));
    return hipGetLastError();
}

hipError_t launch_clear(uint64_t *fb, uint64_t *acc, int64_t npix, uint32_t bg, hipStream_t s)
{
    Range r("rz clear");
    if (npix == 0)
        return hipSuccess;
    const uint64_t clear = kDepthOnes | ((uint64_t)bg & kRgbMask);
    hipLaunchKernelGGL(k_clear, dim3((uint32_t)blocks_for(npix, 256)), dim3(256), 0, s, fb, acc,
                       npix, clear);
    return hipGetLastError();
}

}  // namespace rz
