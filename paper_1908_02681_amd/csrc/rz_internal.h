// Internal declarations shared by the host side of the library and the
// kernel launchers.  Not part of the public C ABI (that is include/rz.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rz {

// Per-view constants of one rasterization, derived on the host in double
// precision and passed to the kernels by value.
struct Proj {
    float m[12];          // rows 0, 1 and 3 of (float)VP, row-major
    float fw, fh;         // framebuffer size as float
    float hw, hh;         // half of it
    float mz[4];          // row 2 of (float)VP (window depth encodings)
    float nearf;          // near as float (reversed float depth)
    int32_t zkind;        // 0: integer map (linear, scale, piecewise);
                          // RZ_DEPTH_GL24 or RZ_DEPTH_F32REV otherwise
    double v[4];          // row 3 of VP in double: the depth row
    double near_, far_;
    double o, s;          // q = floor((d - o) * s)
    uint64_t z0;          // floor(o * s)
    int32_t width, height;
    // piecewise depth map: nr > 0 selects it
    int32_t nr;
    int32_t pad_;
    double rb[8];         // range starts
    double rs[8];         // values per unit
    double rinv[8];       // 1 / rs
    uint64_t rbase[9];    // first integer of each range; rbase[nr] = 2^40 - 1
    double z0d;           // z0 as a double (exact when wfp is set)
    int32_t wfp;          // z0 < 2^52: the eps window may be pre-tested in double
    int32_t pad2_;
};

// Launch shape of the point kernels.  The defaults are those of the depth
// pass; the splat accumulate pass defaults to kHqTune (measured on the
// 50M-point terrain: 64 threads, 8 points each, the small per-wave tile).
struct Tune {
    int block = 64;        // threads per workgroup: 64, 128, 256 or 512
    int ppt = 16;          // points per thread: 4, 8 or 16
    int early_out = 1;     // read the framebuffer before the atomic
    int xcd_remap = 0;     // give each XCD a contiguous range of chunks
    int bin = 2;           // 0 none, 1 workgroup LDS tile, 2 per-wave LDS tile,
                           // 3 the small per-wave tile
};

constexpr Tune kHqTune = {64, 8, 1, 0, 3};

constexpr uint64_t kDepthOnes = 0xFFFFFFFFFF000000ull;
constexpr uint64_t kRgbMask = 0xFFFFFFull;
constexpr uint64_t kHqCountMax = 16843009ull;   // floor((2^32 - 1) / 255)

// Point planes on the device.
struct Pts {
    const float *x, *y, *z;
    const uint32_t *rgb;
    int64_t n;
};

hipError_t launch_raster_min(const Pts &p, const Proj &P, uint64_t *fb, const Tune &t,
                             hipStream_t s);
hipError_t launch_hq_accum(const Pts &p, const Proj &P, uint32_t eps_num, uint32_t eps_den,
                           const uint64_t *fb, uint64_t *acc, const Tune &t, hipStream_t s);
hipError_t launch_resolve_min(uint64_t *fb, int64_t npix, uint32_t bg, uint32_t *img,
                              hipStream_t s);
hipError_t launch_resolve_hq(uint64_t *fb, uint64_t *acc, int64_t npix, uint32_t bg,
                             uint32_t *img, uint32_t *status, hipStream_t s);
hipError_t launch_clear(uint64_t *fb, uint64_t *acc, int64_t npix, uint32_t bg, hipStream_t s);
// Points of size k >= 1 and every depth encoding (one fragment per covered
// pixel, early-out plus global atomics).
hipError_t launch_raster_points(const Pts &p, const Proj &P, int32_t k, uint64_t *fb,
                                hipStream_t s);

// One view of a multi-view pass (an entry of a device table): the batch
// engine's groups and the server's merged requests.
struct MvView {
    Proj P;
    uint64_t *fb;
    uint64_t *acc;
    uint32_t eps_num, eps_den;
};
constexpr int kMaxGroupViews = 8;   // views per multi-view launch

// Depth passes (hq false) or accumulate passes (hq true) of views[0 .. nv)
// (a device table, nv <= kMaxGroupViews) over the points, each chunk of
// points loaded once for all of them.  pw: some view uses a piecewise map.
hipError_t launch_multiview(bool hq, bool pw, const Pts &p, const MvView *views, int32_t nv,
                            const Tune &t, hipStream_t s);
hipError_t launch_hq_points(const Pts &p, const Proj &P, int32_t k, uint32_t eps_num,
                            uint32_t eps_den, const uint64_t *fb, uint64_t *acc, hipStream_t s);

}  // namespace rz
