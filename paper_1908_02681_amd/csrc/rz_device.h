// Device-side building blocks of the point rasterizer for gfx950 (MI355X),
// shared by the one-view kernels (rz_kernels.hip), the multi-view batch
// kernels (rz_batch.hip), the general point-size and float-depth kernels
// (rz_general.hip), the screen-sorted path (rz_sorted.hip) and the
// reciprocal self-check (rz_check.hip).
//
// Method: Schuetz & Wimmer, "Rendering Point Clouds with Compute Shaders"
// (arXiv 1908.02681), section 2.1 (atomicMin rasterization, resolve/clear)
// and section 2.2 (high-quality splatting).
//
// Every file that includes this header must be compiled with
// -ffp-contract=off; the pragma below repeats it, so that the projection is
// the exact IEEE operation sequence stated in include/rz.h (fused
// multiply-adds only where written as such, correctly rounded f32 division,
// no flush of denormals).
//
// Code style rule for the point kernels: decisions are kept in separate
// boolean flags computed with selects; no element of a register array is
// updated inside a divergent branch.  This hipcc build was seen to
// mis-allocate that form (the reject copy of a phi was hoisted above the
// branch and overwritten).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rz.h"
#include "rz_internal.h"

#pragma clang fp contract(off)

namespace rz {
namespace dev {

constexpr double kQMax = 1099511627774.0;   // 2^40 - 2
constexpr int kXcds = 8;                     // XCDs of an MI355X
constexpr int kMaxWaves = 512 / 64;
constexpr uint32_t kTileMin = 4096;          // workgroup tile of the depth pass: 32 KiB
constexpr uint32_t kTileHq = 2048;           // workgroup tile of the accumulate pass: 32 KiB
constexpr uint32_t kWaveTileWords = 1024;    // per-wave tile: 8 KiB of LDS
constexpr uint32_t kWaveTileMin = kWaveTileWords;        // pixels (one key each)
constexpr uint32_t kWaveTileHq = kWaveTileWords / 2;     // pixels (two sums each)
// The small per-wave tile (2 KiB): a quarter of the LDS per wave, so that
// LDS no longer caps the waves per SIMD of kernels with few registers
// (measured: the multi-view kernels at 4 points per thread).
constexpr uint32_t kWaveTileSmallWords = 256;

// Tiling modes of the point kernels.  kBinWaveSmall is kBinWave with the
// small tile: the kernels take the tile size as an argument, so both modes
// share the kBinWave code.
enum : int { kBinNone = 0, kBinBlock = 1, kBinWave = 2, kBinWaveSmall = 3 };

// Words of one wave's tile in a per-wave tiling mode.
__host__ __device__ constexpr uint32_t wave_tile_words(int bin)
{
    return bin == kBinWaveSmall ? kWaveTileSmallWords : kWaveTileWords;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// Streaming (non-temporal) access: the data is touched once per pass.
template <typename T>
__device__ __forceinline__ T ldnt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void stnt(T v, T *p) { __builtin_nontemporal_store(v, p); }

// 0 <= t < 2^52, integral: t + 2^52 is exact and its 52 mantissa bits are t.
__device__ __forceinline__ uint64_t to_u64(double t)
{
    return (uint64_t)__double_as_longlong(t + 0x1p52) & 0xFFFFFFFFFFFFFull;
}

// True when the predicate holds on any active lane of the wave: the ballot
// mask itself (HIP's __any goes through an int and costs two more vector
// instructions per call).
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

// Piecewise depth map (section 2.1, sub-ranges with their own precision):
// range k with start rb[k] <= d < rb[k+1]; q = rbase[k] + floor((d - rb[k]) *
// rs[k]), which stays below rbase[k+1] because IEEE rounding is monotone.
__device__ __forceinline__ uint64_t piecewise_q(const Proj &P, double d)
{
    int k = 0;
    for (int i = 1; i < 8; ++i)
        k = (i < P.nr && d >= P.rb[i]) ? i : k;
    const double tf = floor((d - P.rb[k]) * P.rs[k]);
    const uint64_t q = P.rbase[k] + to_u64(tf);
    return q > (1ull << 40) - 2 ? (1ull << 40) - 2 : q;
}

// Linear depth of integer depth q under the piecewise map.
__device__ __forceinline__ double piecewise_depth(const Proj &P, uint64_t q)
{
    int k = 0;
    for (int i = 1; i < 8; ++i)
        k = (i < P.nr && q >= P.rbase[i]) ? i : k;
    return P.rb[k] + (double)(q - P.rbase[k]) * P.rinv[k];
}

// Section 2.2's window: does a fragment of depth q join the pixel whose
// nearest depth is qmin?  Linear maps: exact integer test; piecewise maps:
// the linear depths the integers stand for, in double precision.
template <bool PW>
__device__ __forceinline__ bool in_window(const Proj &P, uint32_t eps_num, uint32_t eps_den,
                                          uint64_t q, uint64_t qmin)
{
    if (!PW || P.nr == 0)   // PW kernels also serve linear views of a batch
        return (uint64_t)eps_den * (q - qmin) <= (uint64_t)eps_num * (qmin + P.z0);
    const double dq = piecewise_depth(P, q);
    const double dm = piecewise_depth(P, qmin);
    const double lhs = (double)eps_den * (dq - dm);
    const double rhs = (double)eps_num * dm;
    return lhs <= rhs;
}

// Integer depth below 2^52 as a double (exact): its bits under the
// exponent of 2^52, minus 2^52.
__device__ __forceinline__ double int52_to_double(uint64_t v)
{
    return __longlong_as_double((long long)(v | 0x4330000000000000ull)) - 0x1p52;
}

// live && in_window, for the accumulate passes.  Linear maps with z0 < 2^52
// decide in double precision first: D = q - qmin and S = qmin + z0 are
// exact there, den * D and num * S are each rounded once, and rounding is
// monotone, so when the rounded products differ they order the exact ones
// the same way.  Only equal rounded products (a fragment on the window's
// edge) take the integer test, in a branch a wave enters only when one of
// its live lanes needs it.  Same result as in_window for every input; the
// 64-bit integer products it avoids are quarter-rate instructions.
template <bool PW>
__device__ __forceinline__ bool in_window_live(const Proj &P, uint32_t eps_num, uint32_t eps_den,
                                               uint64_t q, uint64_t qmin, bool live)
{
    if ((PW && P.nr != 0) || !P.wfp)
        return live && in_window<PW>(P, eps_num, eps_den, q, qmin);
    const double dm = int52_to_double(qmin);
    const double lhs = (double)eps_den * (int52_to_double(q) - dm);
    const double rhs = (double)eps_num * (dm + P.z0d);
    bool ok = live & (lhs < rhs);
    const bool edge = live & (lhs == rhs);
    if (wave_any(edge)) {
        const bool ex = (uint64_t)eps_den * (q - qmin) <= (uint64_t)eps_num * (qmin + P.z0);
        ok = edge ? ex : ok;
    }
    return ok;
}

// The IEEE quotient 1 / w for w > 0, without the full division sequence:
// one Newton-Raphson correction of the hardware estimate, r + r * (1 - w r)
// with both steps fused (Markstein's method).  Run over every positive
// float on gfx950, it equals the correctly rounded reciprocal for all w in
// [2^-126, 2^126) and misses only for denormal w, w >= 2^126 and +inf;
// those lanes take the division.  For w <= 0 or NaN the value is never
// used (every caller culls the point), so it is left as it comes.
__device__ __forceinline__ float recip_newton(float w)
{
    const float r = __builtin_amdgcn_rcpf(w);
    const float e = __builtin_fmaf(-w, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

__device__ __forceinline__ float recip_rn(float w)
{
    float f = recip_newton(w);
    const bool slow = (w > 0.0f) & ((w < 0x1p-126f) | (w >= 0x1p126f));
    if (wave_any(slow)) {   // wave-uniform; no lane needs it in practice
        const float q = 1.0f / w;
        f = slow ? q : f;
    }
    return f;
}

// Translation column of the float matrix (clip x, y, w) and of the depth
// row in double, the addend of the first fused step of each row.
// lane_trans() returns it as per-lane values (identity DPP moves), made once
// per chunk: a fused multiply-add can take only one scalar-register operand
// on gfx950, so with the scalar copies every row of every point would need
// a move first.
struct Trans {
    float tx, ty, tw;
    double td;   // the depth row's translation (double precision)
};

__device__ __forceinline__ float lane_copy(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xE4, 0xF, 0xF,
                                                      false));   // quad_perm [0,1,2,3]
}

__device__ __forceinline__ double lane_copy(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __float_as_uint(lane_copy(__uint_as_float((uint32_t)b)));
    const uint32_t hi = __float_as_uint(lane_copy(__uint_as_float((uint32_t)(b >> 32))));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ Trans lane_trans(const Proj &P)
{
    return Trans{lane_copy(P.m[3]), lane_copy(P.m[7]), lane_copy(P.m[11]), lane_copy(P.v[3])};
}

__device__ __forceinline__ Trans scalar_trans(const Proj &P)
{
    return Trans{P.m[3], P.m[7], P.m[11], P.v[3]};
}

// Pixel of one point (section 2.1's projection in single precision: each
// clip coordinate a chain of fused multiply-adds from the translation
// column through the x, y and z terms), its clip w and 1 / w (rounded once;
// x and y are scaled by it, as a perspective divide does, and the viewport
// maps them with one fused scale and offset).  Returns false when the point
// is culled (w <= 0 or off screen).
// Straight-line code: the pixel of a culled point is 0, never a conversion
// of an out-of-range float.
__device__ __forceinline__ bool project(const Proj &P, const Trans &T, float x, float y, float z,
                                        uint32_t &px, uint32_t &py, float &cw, float &iw)
{
    float cx = __builtin_fmaf(P.m[0], x, T.tx);
    cx = __builtin_fmaf(P.m[1], y, cx);
    cx = __builtin_fmaf(P.m[2], z, cx);
    float cy = __builtin_fmaf(P.m[4], x, T.ty);
    cy = __builtin_fmaf(P.m[5], y, cy);
    cy = __builtin_fmaf(P.m[6], z, cy);
    cw = __builtin_fmaf(P.m[8], x, T.tw);
    cw = __builtin_fmaf(P.m[9], y, cw);
    cw = __builtin_fmaf(P.m[10], z, cw);
    iw = recip_rn(cw);
    const float nx = cx * iw;
    const float ny = cy * iw;
    const float fx = __builtin_fmaf(nx, P.hw, P.hw);   // viewport: scale and offset
    const float fy = __builtin_fmaf(ny, P.hh, P.hh);
    const bool vis = (cw > 0.0f) & (fx >= 0.0f) & (fx < P.fw) & (fy >= 0.0f) & (fy < P.fh);
    px = (uint32_t)(int32_t)(vis ? fx : 0.0f);
    py = (uint32_t)(int32_t)(vis ? fy : 0.0f);
    return vis;
}

// Depth in double precision (section 1, section 2.1): row 3 of VP, fused
// in the same order as the clip coordinates.
__device__ __forceinline__ double depth_of(const Proj &P, const Trans &T, float x, float y,
                                           float z)
{
    double d = __builtin_fma(P.v[0], (double)x, T.td);
    d = __builtin_fma(P.v[1], (double)y, d);
    d = __builtin_fma(P.v[2], (double)z, d);
    return d;
}

__device__ __forceinline__ double depth_of(const Proj &P, float x, float y, float z)
{
    return depth_of(P, scalar_trans(P), x, y, z);
}

// The fragment of one point: pixel coordinates and 40-bit depth (section
// 2.1).  Returns false when the point is discarded; q is then meaningless.
// Integer depth maps only (P.zkind == 0).  PW = false: linear or scale map
// only (P.nr == 0), so the piecewise tables are never read; PW = true serves
// every integer map.  Straight-line code apart from one wave-uniform skip
// of the depth when no lane of the wave is on screen.
// tq: q as a double for the linear and scale maps (meaningless for the
// piecewise map).
// vis: the point is on screen (w > 0, inside the framebuffer), whatever its
// depth.
template <bool PW>
__device__ __forceinline__ bool fragment(const Proj &P, const Trans &T, float x, float y, float z,
                                         uint32_t &px, uint32_t &py, uint64_t &q, double &tq,
                                         bool &vis)
{
    float cw, iw;
    vis = project(P, T, x, y, z, px, py, cw, iw);
    q = 0;
    tq = 0.0;
    if (!wave_any(vis))
        return false;
    const double d = depth_of(P, T, x, y, z);
    const bool in_range = d >= P.near_ && d < P.far_;
    if (!PW || P.nr == 0) {
        tq = fmin(floor((d - P.o) * P.s), kQMax);   // d < near gives garbage, unused
        q = to_u64(tq);
    } else {
        q = piecewise_q(P, in_range ? d : P.near_);
    }
    return vis && in_range;
}

template <bool PW>
__device__ __forceinline__ bool fragment(const Proj &P, const Trans &T, float x, float y, float z,
                                         uint32_t &px, uint32_t &py, uint64_t &q, double &tq)
{
    bool vis;
    return fragment<PW>(P, T, x, y, z, px, py, q, tq, vis);
}

template <bool PW>
__device__ __forceinline__ bool fragment(const Proj &P, const Trans &T, float x, float y, float z,
                                         uint32_t &px, uint32_t &py, uint64_t &q)
{
    double tq;
    return fragment<PW>(P, T, x, y, z, px, py, q, tq);
}

template <bool PW>
__device__ __forceinline__ bool fragment(const Proj &P, float x, float y, float z,
                                         uint32_t &px, uint32_t &py, uint64_t &q)
{
    return fragment<PW>(P, scalar_trans(P), x, y, z, px, py, q);
}

// fragment() for every depth encoding: the integer maps, the 24-bit window
// depth of the perspective matrix (RZ_DEPTH_GL24) and the complemented
// reversed float depth (RZ_DEPTH_F32REV).
__device__ __forceinline__ bool fragment_any(const Proj &P, float x, float y, float z,
                                             uint32_t &px, uint32_t &py, uint64_t &q)
{
    if (P.zkind == 0)
        return fragment<true>(P, x, y, z, px, py, q);
    float cw, iw;
    if (!project(P, scalar_trans(P), x, y, z, px, py, cw, iw))
        return false;
    const double d = depth_of(P, x, y, z);
    if (!(d >= P.near_ && d < P.far_))
        return false;
    if (P.zkind == RZ_DEPTH_F32REV) {
        const float zr = P.nearf / cw;
        q = 0xFFFFFFFFull - (uint64_t)__float_as_uint(zr);
        return true;
    }
    float cz = __builtin_fmaf(P.mz[0], x, P.mz[3]);
    cz = __builtin_fmaf(P.mz[1], y, cz);
    cz = __builtin_fmaf(P.mz[2], z, cz);
    const float nz = cz * iw;
    if (!(nz >= -1.0f && nz <= 1.0f))
        return false;
    const float zw = (nz + 1.0f) * 0.5f;
    const float t = zw * 16777215.0f;
    q = (uint64_t)(uint32_t)floor((double)t + 0.5);
    return true;
}

// fragment_any() for one float encoding, straight-line like fragment(): the
// same arithmetic, with selects in place of the early returns, and the
// 24-bit code converted only from a value inside the window.
template <int ZK>
__device__ __forceinline__ bool fragment_zk(const Proj &P, const Trans &T, float x, float y,
                                            float z, uint32_t &px, uint32_t &py, uint64_t &q)
{
    static_assert(ZK == RZ_DEPTH_GL24 || ZK == RZ_DEPTH_F32REV, "float encodings only");
    float cw, iw;
    const bool vis = project(P, T, x, y, z, px, py, cw, iw);
    q = 0;
    if (!wave_any(vis))
        return false;
    const double d = depth_of(P, T, x, y, z);
    const bool in_range = (d >= P.near_) & (d < P.far_);
    if (ZK == RZ_DEPTH_F32REV) {
        const float zr = P.nearf / cw;
        q = 0xFFFFFFFFull - (uint64_t)__float_as_uint(zr);
        return vis & in_range;
    }
    float cz = __builtin_fmaf(P.mz[0], x, P.mz[3]);
    cz = __builtin_fmaf(P.mz[1], y, cz);
    cz = __builtin_fmaf(P.mz[2], z, cz);
    const float nz = cz * iw;
    const bool clip = (nz >= -1.0f) & (nz <= 1.0f);
    const float zw = (nz + 1.0f) * 0.5f;
    const float t = zw * 16777215.0f;
    q = (uint64_t)(uint32_t)floor((double)(clip ? t : 0.0f) + 0.5);
    return vis & in_range & clip;
}

// The fragment of the kernels templated on the depth encoding: ZK = 0 for
// the integer maps, else RZ_DEPTH_GL24 or RZ_DEPTH_F32REV.
template <bool PW, int ZK>
__device__ __forceinline__ bool fragment_enc(const Proj &P, const Trans &T, float x, float y,
                                             float z, uint32_t &px, uint32_t &py, uint64_t &q)
{
    if constexpr (ZK == 0)
        return fragment<PW>(P, T, x, y, z, px, py, q);
    else
        return fragment_zk<ZK>(P, T, x, y, z, px, py, q);
}

// Workgroup -> chunk of points.  Workgroups are dealt round-robin to the 8
// XCDs; with the remap, XCD k works through the k-th eighth of the chunks,
// so spatially coherent (e.g. Morton-ordered) ranges share one L2.
template <bool XCD>
__device__ __forceinline__ int64_t chunk_index()
{
    const int64_t b = blockIdx.x;
    if (!XCD)
        return b;
    const int64_t per = gridDim.x / kXcds;   // grid is a multiple of 8
    return (b % kXcds) * per + b / kXcds;
}

// Loads the PPT points of this thread.  Vector form: PPT/4 groups of four
// consecutive points, group g at chunk + g*4*blockDim + 4*tid, so every
// load instruction of a wave reads one contiguous 1 KiB span per plane.
// Scalar form (tail chunk or unaligned planes): same point indices, bounds
// checked one by one.
template <int PPT>
__device__ __forceinline__ bool chunk_full(const Pts &p, int64_t base)
{
    return base + 4 * (int64_t)blockDim.x * (PPT / 4) <= p.n;
}

template <int PPT>
__device__ __forceinline__ void load_full(const Pts &p, int64_t base, float (&x)[PPT],
                                          float (&y)[PPT], float (&z)[PPT], uint32_t (&c)[PPT])
{
    const int64_t stride = 4 * (int64_t)blockDim.x;
    const int64_t first = base + 4 * (int64_t)threadIdx.x;
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
    }
}

template <int PPT>
__device__ __forceinline__ void load_ragged(const Pts &p, int64_t base, float (&x)[PPT],
                                            float (&y)[PPT], float (&z)[PPT],
                                            uint32_t (&c)[PPT], bool (&in)[PPT])
{
    const int64_t stride = 4 * (int64_t)blockDim.x;
    const int64_t first = base + 4 * (int64_t)threadIdx.x;
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

// The same loads for kernels that carry no per-point bounds flags: points
// past the end read as NaN, which every projection culls (a NaN coordinate
// makes clip w NaN, and w > 0 fails), so the chunk code is the same for the
// last chunk as for all others.
template <int PPT, bool VEC>
__device__ __forceinline__ void load_points_nan(const Pts &p, int64_t base, float (&x)[PPT],
                                                float (&y)[PPT], float (&z)[PPT],
                                                uint32_t (&c)[PPT])
{
    if (VEC && chunk_full<PPT>(p, base)) {
        load_full<PPT>(p, base, x, y, z, c);
        return;
    }
    const int64_t stride = 4 * (int64_t)blockDim.x;
    const int64_t first = base + 4 * (int64_t)threadIdx.x;
    const float nan = __builtin_nanf("");
#pragma unroll
    for (int g = 0; g < PPT / 4; ++g) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = first + g * stride + k;
            const bool ok = i < p.n;
            x[4 * g + k] = ok ? p.x[i] : nan;
            y[4 * g + k] = ok ? p.y[i] : nan;
            z[4 * g + k] = ok ? p.z[i] : nan;
            c[4 * g + k] = ok ? p.rgb[i] : 0u;
        }
    }
}

template <int PPT, bool VEC>
__device__ __forceinline__ void load_points(const Pts &p, int64_t base, float (&x)[PPT],
                                            float (&y)[PPT], float (&z)[PPT],
                                            uint32_t (&c)[PPT], bool (&in)[PPT])
{
    if (VEC && chunk_full<PPT>(p, base)) {
        load_full<PPT>(p, base, x, y, z, c);
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            in[j] = true;
    } else {
        load_ragged<PPT>(p, base, x, y, z, c, in);
    }
}

// Minimum over the 64 lanes of a wave with DPP moves (all lanes active):
// quads, 8-lane halves, 16-lane rows, then row broadcasts into lane 63.
__device__ __forceinline__ uint32_t wave_min(uint32_t v)
{
    // Each step moves a neighbour's value in by DPP and keeps the smaller.
    // Lanes the step does not write get the identity ~0, so the move folds
    // into the minimum (one v_min_u32 with a DPP operand per step).
#define RZ_DPP_MIN(ctrl, rows)                                                             \
    {                                                                                      \
        const uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, ctrl, rows,   \
                                                                 0xF, false);              \
        v = v < t ? v : t;                                                                 \
    }
    RZ_DPP_MIN(0xB1, 0xF)    // quad_perm [1,0,3,2]
    RZ_DPP_MIN(0x4E, 0xF)    // quad_perm [2,3,0,1]
    RZ_DPP_MIN(0x141, 0xF)   // row_half_mirror
    RZ_DPP_MIN(0x140, 0xF)   // row_mirror
    RZ_DPP_MIN(0x142, 0xA)   // row_bcast:15 into rows 1 and 3
    RZ_DPP_MIN(0x143, 0xC)   // row_bcast:31 into rows 2 and 3
#undef RZ_DPP_MIN
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// The same for the maximum (identity 0).
__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
#define RZ_DPP_MAX(ctrl, rows)                                                             \
    {                                                                                      \
        const uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, rows,    \
                                                                 0xF, false);              \
        v = v > t ? v : t;                                                                 \
    }
    RZ_DPP_MAX(0xB1, 0xF)
    RZ_DPP_MAX(0x4E, 0xF)
    RZ_DPP_MAX(0x141, 0xF)
    RZ_DPP_MAX(0x140, 0xF)
    RZ_DPP_MAX(0x142, 0xA)
    RZ_DPP_MAX(0x143, 0xC)
#undef RZ_DPP_MAX
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Screen rectangle of the live fragments of the workgroup.  Every thread
// must call it (it synchronises the workgroup); every thread gets the same
// answer.  Empty when x0 > x1.
struct Box {
    uint32_t x0, y0, x1, y1;
};

template <int PPT>
__device__ __forceinline__ Box block_box(const uint32_t (&px)[PPT], const uint32_t (&py)[PPT],
                                         const bool (&live)[PPT], uint32_t (*s_box)[4])
{
    uint32_t m[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint32_t a = live[j] ? px[j] : 0xFFFFFFFFu;
        const uint32_t b = live[j] ? py[j] : 0xFFFFFFFFu;
        const uint32_t c = live[j] ? ~px[j] : 0xFFFFFFFFu;
        const uint32_t d = live[j] ? ~py[j] : 0xFFFFFFFFu;
        m[0] = a < m[0] ? a : m[0];
        m[1] = b < m[1] ? b : m[1];
        m[2] = c < m[2] ? c : m[2];
        m[3] = d < m[3] ? d : m[3];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        m[k] = wave_min(m[k]);
    const uint32_t wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            s_box[wave][k] = m[k];
    }
    __syncthreads();
    const uint32_t nw = blockDim.x >> 6;
    for (uint32_t w = 0; w < nw; ++w) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            m[k] = s_box[w][k] < m[k] ? s_box[w][k] : m[k];
    }
    return Box{m[0], m[1], ~m[2], ~m[3]};
}

// Depth pass over one chunk already in registers (section 2.1): every
// surviving fragment takes part in a 64-bit minimum per pixel of fb.  None
// of the refinements changes the result, because min is order independent
// and the framebuffer only decreases:
//  - consecutive fragments of a thread in one pixel are merged in registers;
//  - BIN: when the workgroup's fragments fall in a small screen rectangle,
//    they are merged with LDS atomics in a tile first, and the tile is
//    flushed row by row (coalesced global atomics, one per touched pixel);
//  - EARLY: the framebuffer is read first and the atomic skipped when it is
//    already <= the key (a stale read can only be larger than the true
//    value, so the skip is always safe).
// With BIN every thread of the workgroup must call it; it returns with the
// workgroup past its last barrier but threads possibly still flushing, so a
// caller that reuses s_tile or s_box must synchronise first.
template <int PPT, bool EARLY, bool BIN, bool PW>
__device__ __forceinline__ void raster_chunk(const Proj &P, uint64_t *__restrict__ fb,
                                             const float (&x)[PPT], const float (&y)[PPT],
                                             const float (&z)[PPT], const uint32_t (&c)[PPT],
                                             const bool (&in)[PPT], uint64_t *s_tile,
                                             uint32_t (*s_box)[4])
{
    uint32_t px[PPT], py[PPT], pix[PPT];
    uint64_t key[PPT];
    bool live[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        uint64_t q = 0;
        uint32_t a = 0, b = 0;
        live[j] = fragment<PW>(P, x[j], y[j], z[j], a, b, q) & in[j];
        px[j] = a;
        py[j] = b;
        pix[j] = __umul24(b, (uint32_t)P.width) + a;   // both below 2^15
        key[j] = (q << 24) | ((uint64_t)c[j] & kRgbMask);
    }
#pragma unroll
    for (int j = 1; j < PPT; ++j) {
        const bool same = live[j] && live[j - 1] && pix[j] == pix[j - 1];
        const uint64_t lo = key[j] < key[j - 1] ? key[j] : key[j - 1];
        key[j] = same ? lo : key[j];
        live[j - 1] = live[j - 1] && !same;
    }

    bool direct[PPT];
    Box box{1, 1, 0, 0};
    uint32_t bw = 0, bh = 0;
    bool tiled = false;
    if (BIN) {
        box = block_box<PPT>(px, py, live, s_box);
        if (box.x0 <= box.x1) {
            bw = box.x1 - box.x0 + 1;
            bh = box.y1 - box.y0 + 1;
            tiled = (uint64_t)bw * bh <= kTileMin;
        }
    }
    if (tiled) {
        const uint32_t area = bw * bh;
        for (uint32_t i = threadIdx.x; i < area; i += blockDim.x)
            s_tile[i] = ~0ull;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const uint32_t tx = px[j] - box.x0, ty = py[j] - box.y0;
            const bool inside = live[j] && tx < bw && ty < bh;
            direct[j] = live[j] && !inside;
            if (inside)
                __hip_atomic_fetch_min(&s_tile[ty * bw + tx], key[j], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < area; i += blockDim.x) {
            const uint64_t v = s_tile[i];
            if (v != ~0ull) {
                const uint32_t r = i / bw;
                const uint32_t col = i - r * bw;
                uint64_t *dst = fb + (__umul24(box.y0 + r, (uint32_t)P.width) + box.x0 + col);
                const uint64_t cur = __hip_atomic_load(dst, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                if (v < cur)
                    __hip_atomic_fetch_min(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            direct[j] = live[j];
    }

    // fragments not merged in a tile go straight to the framebuffer
    if (EARLY) {
        uint64_t cur[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            cur[j] = __hip_atomic_load(fb + (direct[j] ? pix[j] : 0u), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            if (direct[j] && key[j] < cur[j])
                __hip_atomic_fetch_min(fb + pix[j], key[j], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    } else {
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            if (direct[j])
                __hip_atomic_fetch_min(fb + pix[j], key[j], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Orders the LDS accesses of one wave: LDS executes a wave's instructions in
// issue order, so only the compiler has to be kept from moving them.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row and column of tile entry i in a tile bw wide: i / bw through a float
// reciprocal, corrected to the exact quotient (i < 2^24, bw <= 2^15).
__device__ __forceinline__ void tile_rc(uint32_t i, uint32_t bw, float inv_bw, uint32_t &r,
                                        uint32_t &col)
{
    uint32_t q = (uint32_t)((float)i * inv_bw);
    q = __umul24(q, bw) > i ? q - 1 : q;          // products below 2^25
    q = __umul24(q + 1, bw) <= i ? q + 1 : q;
    r = q;
    col = i - __umul24(q, bw);
}

// Screen rectangle of the live fragments of one wave (no workgroup barrier).
template <int PPT>
__device__ __forceinline__ Box wave_box(const uint32_t (&px)[PPT], const uint32_t (&py)[PPT],
                                        const bool (&live)[PPT])
{
    static_assert(PPT % 2 == 0, "points are taken in pairs");
    uint32_t lx = 0xFFFFFFFFu, ly = 0xFFFFFFFFu, hx = 0u, hy = 0u;
#pragma unroll
    for (int j = 0; j < PPT; j += 2) {   // pairs: three-operand min and max
        const uint32_t a0 = live[j] ? px[j] : 0xFFFFFFFFu,
                       a1 = live[j + 1] ? px[j + 1] : 0xFFFFFFFFu;
        const uint32_t b0 = live[j] ? py[j] : 0xFFFFFFFFu,
                       b1 = live[j + 1] ? py[j + 1] : 0xFFFFFFFFu;
        const uint32_t c0 = live[j] ? px[j] : 0u, c1 = live[j + 1] ? px[j + 1] : 0u;
        const uint32_t d0 = live[j] ? py[j] : 0u, d1 = live[j + 1] ? py[j + 1] : 0u;
        lx = min(lx, min(a0, a1));
        ly = min(ly, min(b0, b1));
        hx = max(hx, max(c0, c1));
        hy = max(hy, max(d0, d1));
    }
    // no live lane: lx = ~0 > hx = 0, an empty box
    return Box{wave_min(lx), wave_min(ly), wave_max(hx), wave_max(hy)};
}

// wave_box() for the wave kernels, one select fewer per coordinate: a point
// that is off screen has pixel 0 (project()), which cannot raise a maximum,
// so the maxima are taken over all points; the minima only over the live
// ones.  Points on screen but outside [near, far) may widen the rectangle,
// which then still bounds every live fragment.
template <int PPT>
__device__ __forceinline__ Box wave_box_live_min(const uint32_t (&px)[PPT],
                                                 const uint32_t (&py)[PPT],
                                                 const bool (&live)[PPT])
{
    static_assert(PPT % 2 == 0, "points are taken in pairs");
    uint32_t lx = 0xFFFFFFFFu, ly = 0xFFFFFFFFu, hx = 0u, hy = 0u;
#pragma unroll
    for (int j = 0; j < PPT; j += 2) {   // pairs: three-operand min and max
        const uint32_t a0 = live[j] ? px[j] : 0xFFFFFFFFu,
                       a1 = live[j + 1] ? px[j + 1] : 0xFFFFFFFFu;
        const uint32_t b0 = live[j] ? py[j] : 0xFFFFFFFFu,
                       b1 = live[j + 1] ? py[j + 1] : 0xFFFFFFFFu;
        lx = min(lx, min(a0, a1));
        ly = min(ly, min(b0, b1));
        hx = max(hx, max(px[j], px[j + 1]));
        hy = max(hy, max(py[j], py[j + 1]));
    }
    // no live lane: lx = ~0 > hx, an empty box
    return Box{wave_min(lx), wave_min(ly), wave_max(hx), wave_max(hy)};
}

// Depth pass over one chunk with a private LDS tile per wave: like
// raster_chunk with BIN, but every wave gathers its own 64 * PPT fragments
// in its own slice of `words` keys (w_tile) and flushes it, so no workgroup
// barrier is needed.  Same result bits as raster_chunk, for any tile size.
template <int PPT, bool PW, int ZK = 0>
__device__ __forceinline__ void raster_chunk_wave(const Proj &P, uint64_t *__restrict__ fb,
                                                  const float (&x)[PPT], const float (&y)[PPT],
                                                  const float (&z)[PPT], const uint32_t (&c)[PPT],
                                                  const bool (&in)[PPT], uint64_t *w_tile,
                                                  uint32_t words)
{
    uint32_t px[PPT], py[PPT], pix[PPT];
    uint64_t key[PPT];
    bool live[PPT];
    const Trans T = lane_trans(P);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        uint64_t q = 0;
        uint32_t a = 0, b = 0;
        live[j] = fragment_enc<PW, ZK>(P, T, x[j], y[j], z[j], a, b, q) & in[j];
        px[j] = a;
        py[j] = b;
        key[j] = (q << 24) | ((uint64_t)c[j] & kRgbMask);
    }
    const Box box = wave_box_live_min<PPT>(px, py, live);
    const uint32_t lane = threadIdx.x & 63u;
    bool tiled = false;
    uint32_t bw = 0, bh = 0;
    if (box.x0 <= box.x1) {
        bw = box.x1 - box.x0 + 1;
        bh = box.y1 - box.y0 + 1;
        tiled = (uint64_t)bw * bh <= words;
    }
    if (tiled) {
        // the box bounds every live fragment of the wave, so all of them
        // land in the tile: entry (py - y0) * bw + (px - x0), computed
        // modulo 2^32 as py * bw + px - org
        const uint32_t area = bw * bh;
        const uint32_t org = box.y0 * bw + box.x0;
        for (uint32_t i = lane; i < area; i += 64)
            w_tile[i] = ~0ull;
        wave_sync();
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            if (live[j])
                __hip_atomic_fetch_min(&w_tile[__umul24(py[j], bw) + px[j] - org], key[j],
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        wave_sync();
        const float inv_bw = 1.0f / (float)bw;
        for (uint32_t i = lane; i < area; i += 64) {
            const uint64_t v = w_tile[i];
            if (v != ~0ull) {
                uint32_t r, col;
                tile_rc(i, bw, inv_bw, r, col);
                uint64_t *dst = fb + (__umul24(box.y0 + r, (uint32_t)P.width) + box.x0 + col);
                const uint64_t cur = __hip_atomic_load(dst, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                if (v < cur)
                    __hip_atomic_fetch_min(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        wave_sync();   // the tile is free for the next use
        return;
    }
    // the wave's fragments spread too far for the tile (or there are none):
    // runs of one pixel are merged in registers (LDS atomics need no such
    // help), then each remaining fragment takes an early-out read and a
    // global atomic
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        pix[j] = __umul24(py[j], (uint32_t)P.width) + px[j];   // both below 2^15
#pragma unroll
    for (int j = 1; j < PPT; ++j) {
        const bool same = live[j] && live[j - 1] && pix[j] == pix[j - 1];
        const uint64_t lo = key[j] < key[j - 1] ? key[j] : key[j - 1];
        key[j] = same ? lo : key[j];
        live[j - 1] = live[j - 1] && !same;
    }
    bool any_live = false;
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        any_live = any_live || live[j];
    if (wave_any(any_live)) {
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
    }
}

// Accumulation pass of high-quality splatting over one chunk (section 2.2).
// Reprojects every point, compares its depth with the finished depth pass
// and, inside the eps window, adds its colour and a count:
//   acc[2p] += R + (G << 32),  acc[2p+1] += B + (1 << 32).
// As in the depth pass, consecutive accepted fragments of a thread in one
// pixel are summed in registers, and with BIN the workgroup's sums are
// gathered in an LDS tile (64-bit LDS adds) and flushed once per pixel.
// Integer sums are order independent, so every variant gives the same bits.
// PW: the piecewise depth map's window test (linear depths in double).
// Barrier rules as for raster_chunk.
template <int PPT, bool BIN, bool PW>
__device__ __forceinline__ void accum_chunk(const Proj &P, uint32_t eps_num, uint32_t eps_den,
                                            const uint64_t *__restrict__ fb,
                                            uint64_t *__restrict__ acc,
                                            const float (&x)[PPT], const float (&y)[PPT],
                                            const float (&z)[PPT], const uint32_t (&c)[PPT],
                                            const bool (&in)[PPT], uint64_t *s_tile,
                                            uint32_t (*s_box)[4])
{
    uint32_t px[PPT], py[PPT], pix[PPT];
    uint64_t q[PPT];
    bool ok[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        uint32_t a = 0, b = 0;
        uint64_t qq = 0;
        ok[j] = fragment<PW>(P, x[j], y[j], z[j], a, b, qq) & in[j];
        px[j] = a;
        py[j] = b;
        pix[j] = __umul24(b, (uint32_t)P.width) + a;   // both below 2^15
        q[j] = qq;
    }
    // eps window against the finished depth pass: all loads first
    // (discarded fragments read pixel 0, always in bounds), then the tests
    uint64_t fbv[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        fbv[j] = fb[ok[j] ? pix[j] : 0u];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint64_t qmin = fbv[j] >> 24;
        ok[j] = in_window_live<PW>(P, eps_num, eps_den, q[j], qmin, ok[j]);
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

    bool direct[PPT];
    Box box{1, 1, 0, 0};
    uint32_t bw = 0, bh = 0;
    bool tiled = false;
    if (BIN) {
        box = block_box<PPT>(px, py, ok, s_box);
        if (box.x0 <= box.x1) {
            bw = box.x1 - box.x0 + 1;
            bh = box.y1 - box.y0 + 1;
            tiled = (uint64_t)bw * bh <= kTileHq;
        }
    }
    if (tiled) {
        const uint32_t area = bw * bh;
        for (uint32_t i = threadIdx.x; i < 2 * area; i += blockDim.x)
            s_tile[i] = 0ull;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const uint32_t tx = px[j] - box.x0, ty = py[j] - box.y0;
            const bool inside = ok[j] && tx < bw && ty < bh;
            direct[j] = ok[j] && !inside;
            if (inside) {
                uint64_t *t = &s_tile[2 * (ty * bw + tx)];
                __hip_atomic_fetch_add(t, w0[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(t + 1, w1[j], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < area; i += blockDim.x) {
            const uint64_t a1 = s_tile[2 * i + 1];
            if (a1 != 0ull) {
                const uint64_t a0 = s_tile[2 * i];
                const uint32_t r = i / bw;
                const uint32_t col = i - r * bw;
                uint64_t *dst =
                    acc + 2 * (uint64_t)(__umul24(box.y0 + r, (uint32_t)P.width) + box.x0 + col);
                __hip_atomic_fetch_add(dst, a0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(dst + 1, a1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            direct[j] = ok[j];
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (direct[j]) {
            uint64_t *a = acc + 2 * (uint64_t)pix[j];
            __hip_atomic_fetch_add(a, w0[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(a + 1, w1[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Accumulate pass over one chunk with a private LDS tile per wave of
// `words` words, one or two per pixel (see raster_chunk_wave and the
// weights below).  Same result bits as accum_chunk.
template <int PPT, bool PW>
__device__ __forceinline__ void accum_chunk_wave(const Proj &P, uint32_t eps_num,
                                                 uint32_t eps_den,
                                                 const uint64_t *__restrict__ fb,
                                                 uint64_t *__restrict__ acc,
                                                 const float (&x)[PPT], const float (&y)[PPT],
                                                 const float (&z)[PPT], const uint32_t (&c)[PPT],
                                                 const bool (&in)[PPT], uint64_t *w_tile,
                                                 uint32_t words)
{
    uint32_t px[PPT], py[PPT], pix[PPT];
    uint64_t q[PPT];
    double tq[PPT];
    bool ok[PPT];
    const Trans T = lane_trans(P);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        uint32_t a = 0, b = 0;
        uint64_t qq = 0;
        double t = 0.0;
        ok[j] = fragment<PW>(P, T, x[j], y[j], z[j], a, b, qq, t) & in[j];
        px[j] = a;
        py[j] = b;
        pix[j] = __umul24(b, (uint32_t)P.width) + a;   // both below 2^15
        q[j] = qq;
        tq[j] = t;
    }
    uint64_t fbv[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j)
        fbv[j] = fb[ok[j] ? pix[j] : 0u];
    if (PW && P.nr != 0) {
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            ok[j] = ok[j] && in_window<PW>(P, eps_num, eps_den, q[j], fbv[j] >> 24);
    } else if (!P.wfp) {   // linear or scale map, z0 >= 2^52: integer test only
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            ok[j] = ok[j] && in_window<false>(P, eps_num, eps_den, to_u64(tq[j]), fbv[j] >> 24);
    } else {
        // the double-precision pre-test of in_window_live(), with q as the
        // double the fragment floored, and one integer fallback per chunk
        bool edge[PPT];
        bool any_edge = false;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const double dm = int52_to_double(fbv[j] >> 24);
            const double lhs = (double)eps_den * (tq[j] - dm);
            const double rhs = (double)eps_num * (dm + P.z0d);
            edge[j] = ok[j] & (lhs == rhs);
            ok[j] = ok[j] & (lhs < rhs);
            any_edge = any_edge | edge[j];
        }
        if (wave_any(any_edge)) {   // reads the pixels again: rare
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const uint64_t qmin = fb[edge[j] ? pix[j] : 0u] >> 24;
                const bool ex = (uint64_t)eps_den * (to_u64(tq[j]) - qmin) <=
                                (uint64_t)eps_num * (qmin + P.z0);
                ok[j] = edge[j] ? ex : ok[j];
            }
        }
    }
    // Weights.  A wave of at most 512 points (PPT <= 8) adds one packed word
    // per fragment, R | G << 17 | B << 34 | count << 51: no field of a sum
    // over the wave can carry into the next (512 * 255 < 2^17, 512 < 2^13),
    // so the tile holds one word per pixel and each fragment takes one LDS
    // add; larger waves keep the accumulator's own two words.
    constexpr bool kPacked = PPT <= 8;
    constexpr uint32_t kPerPix = kPacked ? 1u : 2u;
    uint64_t w0[PPT], w1[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint32_t r = c[j] & 0xFFu, g = (c[j] >> 8) & 0xFFu, b = (c[j] >> 16) & 0xFFu;
        if (kPacked) {
            w0[j] = ((uint64_t)((b << 2) | (1u << 19)) << 32) | (r | (g << 17));
            w1[j] = 0;
        } else {
            w0[j] = (uint64_t)r | ((uint64_t)g << 32);
            w1[j] = (uint64_t)b | (1ull << 32);
        }
    }
    // runs of one pixel summed in registers: unlike the depth pass's LDS
    // minimum, the tile's LDS adds are slower than this merge on runs of
    // Morton-ordered points.  Only within each group of four consecutive
    // points: the next group lies 4 * blockDim points further on.
#pragma unroll
    for (int j = 1; j < PPT; ++j) {
        if (j % 4 == 0)
            continue;
        const bool same = ok[j] && ok[j - 1] && pix[j] == pix[j - 1];
        w0[j] += same ? w0[j - 1] : 0ull;
        if (!kPacked)
            w1[j] += same ? w1[j - 1] : 0ull;
        ok[j - 1] = ok[j - 1] && !same;
    }
    // the accumulator's two words of a packed sum
    auto unpack = [](uint64_t w, uint64_t &a0, uint64_t &a1) {
        a0 = (w & 0x1FFFFull) | (((w >> 17) & 0x1FFFFull) << 32);
        a1 = ((w >> 34) & 0x1FFFFull) | ((w >> 51) << 32);
    };
    const Box box = wave_box_live_min<PPT>(px, py, ok);
    const uint32_t lane = threadIdx.x & 63u;
    bool tiled = false;
    uint32_t bw = 0, bh = 0;
    if (box.x0 <= box.x1) {
        bw = box.x1 - box.x0 + 1;
        bh = box.y1 - box.y0 + 1;
        tiled = (uint64_t)bw * bh <= words / kPerPix;
    }
    if (tiled) {
        // every accepted fragment of the wave lies in the box (see
        // raster_chunk_wave)
        const uint32_t area = bw * bh;
        const uint32_t org = box.y0 * bw + box.x0;
        for (uint32_t i = lane; i < kPerPix * area; i += 64)
            w_tile[i] = 0ull;
        wave_sync();
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (ok[j]) {
                uint64_t *t = &w_tile[kPerPix * (__umul24(py[j], bw) + px[j] - org)];
                __hip_atomic_fetch_add(t, w0[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (!kPacked)
                    __hip_atomic_fetch_add(t + 1, w1[j], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        wave_sync();
        const float inv_bw = 1.0f / (float)bw;
        for (uint32_t i = lane; i < area; i += 64) {
            uint64_t a0, a1;
            if (kPacked) {
                unpack(w_tile[i], a0, a1);
            } else {
                a0 = w_tile[2 * i];
                a1 = w_tile[2 * i + 1];
            }
            if (a1 != 0ull) {   // count > 0
                uint32_t r, col;
                tile_rc(i, bw, inv_bw, r, col);
                uint64_t *dst =
                    acc + 2 * (uint64_t)(__umul24(box.y0 + r, (uint32_t)P.width) + box.x0 + col);
                __hip_atomic_fetch_add(dst, a0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(dst + 1, a1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        wave_sync();
        return;
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (ok[j]) {
            uint64_t a0 = w0[j], a1 = w1[j];
            if (kPacked)
                unpack(w0[j], a0, a1);
            uint64_t *a = acc + 2 * (uint64_t)pix[j];
            __hip_atomic_fetch_add(a, a0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(a + 1, a1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Colour of one pixel from its packed splat sums (section 2.2, third pass):
// per channel (2 * sum + count) / (2 * count), or the background.
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

}  // namespace dev
}  // namespace rz
