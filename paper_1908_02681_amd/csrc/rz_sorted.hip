// Screen-sorted rendering (declared in include/rz.h): the same depth pass
// (section 2.1) and splat accumulation (section 2.2) for clouds in no
// particular order, where one global atomic per fragment would hit random
// framebuffer lines.  A counting sort by 32x32 screen tile first:
//   A  k_sort_count    per workgroup range: LDS histogram of fragment tiles
//   B  k_sort_prefix   per tile: prefix over workgroups, tile totals
//      k_sort_scan     exclusive scan of the totals (bucket starts)
//   C  k_sort_scatter  same fragments again: key and in-tile pixel into the
//                      tile's bucket at an LDS cursor
//   D  k_sort_raster   per chunk of a tile's bucket: LDS min, one coalesced
//                      global atomic per touched pixel
//   E  k_sort_accum    per chunk of a tile's bucket: eps window against the finished
//                      depth pass, LDS sums, one flush per pixel
// Every step is a minimum or an integer sum, so the result is the oracle's
// bit for bit regardless of the order in which fragments land.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rz.h"
#include "rz_device.h"
#include "rz_internal.h"

namespace rz {

int check_points(const rz_points *p);
int make_proj(const rz_view *v, const rz_depth_map *dm, Proj *P);
int check_hq(const rz_hq_params *hq, const Proj &P, uint32_t *num, uint32_t *den);
int hip_fail(hipError_t e);

namespace {

using namespace dev;

constexpr int kTileShift = 5;                 // 32 x 32 pixel tiles
constexpr int kTilePix = 1 << (2 * kTileShift);
constexpr int kMaxTiles = 8192;               // LDS histogram: 32 KiB
constexpr int kGroups = 1024;                 // workgroups of passes A and C
constexpr int kSortBlock = 256;
constexpr int kSortPpt = 8;
constexpr uint32_t kChunk = 8192;             // fragments per workgroup in passes D, E
constexpr int kPrefixTiles = 32;              // pass B: tiles per workgroup
constexpr int kPrefixSegs = 32;               // pass B: workgroup segments per tile

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

struct Layout {
    int32_t ntx = 0, nty = 0, ntiles = 0, groups = 0;
    int64_t per_wg = 0;
    int64_t chunks_max = 0;   // bound on the chunks of passes D and E
    size_t counts = 0, total = 0, start = 0, cstart = 0, keys = 0, lps = 0, bytes = 0;
};

Layout layout(int64_t n, int32_t w, int32_t h)
{
    Layout L;
    L.ntx = (w + (1 << kTileShift) - 1) >> kTileShift;
    L.nty = (h + (1 << kTileShift) - 1) >> kTileShift;
    L.ntiles = L.ntx * L.nty;
    const int64_t chunk = (int64_t)kSortBlock * kSortPpt;
    if (n > 0) {
        const int64_t want = (n + kGroups - 1) / kGroups;
        L.per_wg = (want + chunk - 1) / chunk * chunk;
        L.groups = (int32_t)((n + L.per_wg - 1) / L.per_wg);
    }
    // sum over tiles of ceil(count / kChunk) <= n / kChunk + ntiles
    L.chunks_max = (n + kChunk - 1) / kChunk + L.ntiles;
    L.counts = 0;
    L.total = align256(L.counts + (size_t)L.groups * L.ntiles * 4);
    L.start = align256(L.total + (size_t)L.ntiles * 4);
    L.cstart = align256(L.start + ((size_t)L.ntiles + 1) * 4);
    L.keys = align256(L.cstart + ((size_t)L.ntiles + 1) * 4);
    L.lps = align256(L.keys + (size_t)n * 8);
    L.bytes = align256(L.lps + (size_t)n * 2);
    return L;
}

// Pass A: number of fragments per screen tile in this workgroup's range.
template <int PPT, bool VEC>
__global__ void __launch_bounds__(kSortBlock) k_sort_count(Pts p, Proj P, uint32_t *counts,
                                                           int32_t ntx, int32_t ntiles,
                                                           int64_t per_wg)
{
    extern __shared__ uint32_t hist[];
    for (int32_t i = threadIdx.x; i < ntiles; i += blockDim.x)
        hist[i] = 0;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * per_wg;
    Pts q = p;
    q.n = lo + per_wg < p.n ? lo + per_wg : p.n;
    for (int64_t base = lo; base < q.n; base += (int64_t)blockDim.x * PPT) {
        float x[PPT], y[PPT], z[PPT];
        uint32_t c[PPT];
        bool in[PPT];
        load_points<PPT, VEC>(q, base, x, y, z, c, in);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            uint32_t px = 0, py = 0;
            uint64_t qq = 0;
            const bool live = in[j] && fragment(P, x[j], y[j], z[j], px, py, qq);
            if (live)
                atomicAdd(&hist[(py >> kTileShift) * (uint32_t)ntx + (px >> kTileShift)], 1u);
        }
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < ntiles; i += blockDim.x)
        counts[(int64_t)blockIdx.x * ntiles + i] = hist[i];
}

// Pass B, first half: per tile, each workgroup's offset inside the tile's
// bucket (exclusive prefix over workgroups, in place) and the tile total.
// A workgroup takes kPrefixTiles tiles; each of its kPrefixSegs segments
// sums a run of up to kPrefixSegs workgroups, the segment sums are scanned
// in LDS, and the segments write their offsets.  groups <= 1024.
__global__ void __launch_bounds__(kPrefixTiles * kPrefixSegs)
    k_sort_prefix(uint32_t *counts, int32_t groups, int32_t ntiles, uint32_t *total)
{
    __shared__ uint32_t s_seg[kPrefixSegs][kPrefixTiles];
    const int tt = threadIdx.x % kPrefixTiles, seg = threadIdx.x / kPrefixTiles;
    const int32_t t = blockIdx.x * kPrefixTiles + tt;
    const bool on = t < ntiles;
    const int32_t g0 = seg * kPrefixSegs;
    uint32_t c[kPrefixSegs];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPrefixSegs; ++k) {
        const int32_t g = g0 + k;
        c[k] = on && g < groups ? counts[(int64_t)g * ntiles + t] : 0u;
        sum += c[k];
    }
    s_seg[seg][tt] = sum;
    __syncthreads();
    if (seg == 0) {   // exclusive scan over the segments of tile tt
        uint32_t run = 0;
        for (int k = 0; k < kPrefixSegs; ++k) {
            const uint32_t v = s_seg[k][tt];
            s_seg[k][tt] = run;
            run += v;
        }
        if (on)
            total[t] = run;
    }
    __syncthreads();
    uint32_t run = s_seg[seg][tt];
#pragma unroll
    for (int k = 0; k < kPrefixSegs; ++k) {
        const int32_t g = g0 + k;
        if (on && g < groups)
            counts[(int64_t)g * ntiles + t] = run;
        run += c[k];
    }
}

// Pass B, second half: bucket starts = exclusive scan of the tile totals,
// and chunk starts = exclusive scan of ceil(total / kChunk) (the work items
// of passes D and E); start[ntiles] and cstart[ntiles] are the sums.  One
// workgroup of 1024 threads, 8 tiles each.
__global__ void __launch_bounds__(1024) k_sort_scan(const uint32_t *total, uint32_t *start,
                                                    uint32_t *cstart, int32_t ntiles)
{
    __shared__ uint32_t s_sum[1024], s_ch[1024];
    const int32_t t0 = threadIdx.x * 8;
    uint32_t v[8];
    uint32_t local = 0, lch = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = t0 + k < ntiles ? total[t0 + k] : 0u;
        local += v[k];
        lch += (v[k] + kChunk - 1) / kChunk;
    }
    s_sum[threadIdx.x] = local;
    s_ch[threadIdx.x] = lch;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive scans (Hillis-Steele)
        const bool has = threadIdx.x >= (uint32_t)off;
        const uint32_t add = has ? s_sum[threadIdx.x - off] : 0u;
        const uint32_t addc = has ? s_ch[threadIdx.x - off] : 0u;
        __syncthreads();
        s_sum[threadIdx.x] += add;
        s_ch[threadIdx.x] += addc;
        __syncthreads();
    }
    uint32_t run = s_sum[threadIdx.x] - local, runc = s_ch[threadIdx.x] - lch;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (t0 + k < ntiles) {
            start[t0 + k] = run;
            cstart[t0 + k] = runc;
        }
        run += v[k];
        runc += (v[k] + kChunk - 1) / kChunk;
    }
    if (threadIdx.x == 1023) {
        start[ntiles] = s_sum[1023];
        cstart[ntiles] = s_ch[1023];
    }
}

// Pass C: the same fragments as pass A (same range, same arithmetic), each
// written to its tile's bucket: the key, and the pixel inside the tile.
template <int PPT, bool VEC>
__global__ void __launch_bounds__(kSortBlock) k_sort_scatter(Pts p, Proj P,
                                                             const uint32_t *counts,
                                                             const uint32_t *start,
                                                             uint64_t *keys, uint16_t *lps,
                                                             int32_t ntx, int32_t ntiles,
                                                             int64_t per_wg)
{
    extern __shared__ uint32_t cursor[];
    for (int32_t i = threadIdx.x; i < ntiles; i += blockDim.x)
        cursor[i] = start[i] + counts[(int64_t)blockIdx.x * ntiles + i];
    const uint32_t end = start[ntiles];
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * per_wg;
    Pts q = p;
    q.n = lo + per_wg < p.n ? lo + per_wg : p.n;
    for (int64_t base = lo; base < q.n; base += (int64_t)blockDim.x * PPT) {
        float x[PPT], y[PPT], z[PPT];
        uint32_t c[PPT];
        bool in[PPT];
        load_points<PPT, VEC>(q, base, x, y, z, c, in);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            uint32_t px = 0, py = 0;
            uint64_t qq = 0;
            const bool live = in[j] && fragment(P, x[j], y[j], z[j], px, py, qq);
            if (live) {
                const uint32_t tile = (py >> kTileShift) * (uint32_t)ntx + (px >> kTileShift);
                const uint32_t pos = atomicAdd(&cursor[tile], 1u);
                if (pos >= end)   // unreachable: passes A and C see the same fragments
                    continue;
                keys[pos] = (qq << 24) | ((uint64_t)c[j] & kRgbMask);
                lps[pos] = (uint16_t)(((py & 31u) << kTileShift) | (px & 31u));
            }
        }
    }
}

// The chunk of this workgroup: tile t (the last tile whose first chunk is
// at or before blockIdx.x) and the range [lo, hi) of its bucket, at most
// kChunk fragments.  Workgroups beyond the last chunk get lo >= hi.
__device__ __forceinline__ void chunk_of(const uint32_t *start, const uint32_t *cstart,
                                         int32_t ntiles, int32_t &t, uint32_t &lo, uint32_t &hi)
{
    const uint32_t b = blockIdx.x;
    t = 0;
    hi = lo = 0;
    if (b >= cstart[ntiles])
        return;
    int32_t a = 0, z = ntiles;   // cstart[a] <= b < cstart[z]
    while (z - a > 1) {
        const int32_t m = (a + z) >> 1;
        if (cstart[m] <= b)
            a = m;
        else
            z = m;
    }
    t = a;
    const uint32_t end = start[t + 1];
    lo = start[t] + (b - cstart[t]) * kChunk;
    hi = end - lo > kChunk ? lo + kChunk : end;
}

constexpr int kUnroll = 4;   // bucket entries in flight per thread (D, E)

// Pass D: depth pass of one chunk of a tile's bucket (section 2.1's minimum).
__global__ void __launch_bounds__(256) k_sort_raster(const uint64_t *__restrict__ keys,
                                                     const uint16_t *__restrict__ lps,
                                                     const uint32_t *__restrict__ start,
                                                     const uint32_t *__restrict__ cstart,
                                                     uint64_t *__restrict__ fb, int32_t ntx,
                                                     int32_t ntiles, int32_t width)
{
    __shared__ uint64_t tile[kTilePix];
    int32_t t;
    uint32_t lo, hi;
    chunk_of(start, cstart, ntiles, t, lo, hi);
    if (lo >= hi)
        return;
    for (int i = threadIdx.x; i < kTilePix; i += blockDim.x)
        tile[i] = ~0ull;
    __syncthreads();
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kUnroll * blockDim.x) {
        uint64_t k[kUnroll];
        uint32_t l[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t i = i0 + (uint64_t)u * blockDim.x;
            ok[u] = i < hi;
            k[u] = ok[u] ? ldnt(keys + i) : ~0ull;
            l[u] = ok[u] ? lps[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (ok[u])
                __hip_atomic_fetch_min(&tile[l[u]], k[u], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    const uint32_t x0 = (uint32_t)(t % ntx) << kTileShift, y0 = (uint32_t)(t / ntx) << kTileShift;
    for (int l = threadIdx.x; l < kTilePix; l += blockDim.x) {
        const uint64_t v = tile[l];
        if (v != ~0ull) {   // a fragment landed here, so the pixel is on screen
            uint64_t *dst = fb + (uint64_t)(y0 + (l >> kTileShift)) * (uint32_t)width + x0 +
                            (l & 31);
            const uint64_t cur = __hip_atomic_load(dst, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            if (v < cur)
                __hip_atomic_fetch_min(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Pass E: splat accumulation of one chunk of a tile's bucket (section 2.2),
// from the bucket's keys; fb holds the finished depth pass.
template <bool PW>
__global__ void __launch_bounds__(256) k_sort_accum(const uint64_t *__restrict__ keys,
                                                    const uint16_t *__restrict__ lps,
                                                    const uint32_t *__restrict__ start,
                                                    const uint32_t *__restrict__ cstart, Proj P,
                                                    uint32_t eps_num, uint32_t eps_den,
                                                    const uint64_t *__restrict__ fb,
                                                    uint64_t *__restrict__ acc, int32_t ntx,
                                                    int32_t ntiles, int32_t width, int32_t height)
{
    __shared__ uint64_t qmin[kTilePix];
    __shared__ uint64_t sums[2 * kTilePix];
    int32_t t;
    uint32_t lo, hi;
    chunk_of(start, cstart, ntiles, t, lo, hi);
    if (lo >= hi)
        return;
    const uint32_t x0 = (uint32_t)(t % ntx) << kTileShift, y0 = (uint32_t)(t / ntx) << kTileShift;
    for (int l = threadIdx.x; l < kTilePix; l += blockDim.x) {
        const uint32_t x = x0 + (l & 31), y = y0 + (l >> kTileShift);
        const bool on = x < (uint32_t)width && y < (uint32_t)height;
        qmin[l] = on ? fb[(uint64_t)y * (uint32_t)width + x] >> 24 : 0ull;
        sums[2 * l] = 0ull;
        sums[2 * l + 1] = 0ull;
    }
    __syncthreads();
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kUnroll * blockDim.x) {
        uint64_t k[kUnroll];
        uint32_t l[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t i = i0 + (uint64_t)u * blockDim.x;
            ok[u] = i < hi;
            k[u] = ok[u] ? ldnt(keys + i) : 0ull;
            l[u] = ok[u] ? lps[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            ok[u] = ok[u] && in_window<PW>(P, eps_num, eps_den, k[u] >> 24, qmin[l[u]]);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (ok[u]) {
                const uint32_t c = (uint32_t)(k[u] & kRgbMask);
                const uint64_t w0 = (uint64_t)(c & 0xFFu) | ((uint64_t)((c >> 8) & 0xFFu) << 32);
                const uint64_t w1 = (uint64_t)((c >> 16) & 0xFFu) | (1ull << 32);
                __hip_atomic_fetch_add(&sums[2 * l[u]], w0, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(&sums[2 * l[u] + 1], w1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    __syncthreads();
    for (int l = threadIdx.x; l < kTilePix; l += blockDim.x) {
        const uint64_t a1 = sums[2 * l + 1];
        if (a1 != 0ull) {   // count > 0 (at most kChunk), so the pixel is on screen
            uint64_t *dst = acc + 2 * ((uint64_t)(y0 + (l >> kTileShift)) * (uint32_t)width +
                                       x0 + (l & 31));
            __hip_atomic_fetch_add(dst, sums[2 * l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(dst + 1, a1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

hipError_t sort_passes(const Pts &p, const Proj &P, const Layout &L, char *ws, bool vec,
                       hipStream_t s)
{
    uint32_t *counts = (uint32_t *)(ws + L.counts);
    uint32_t *total = (uint32_t *)(ws + L.total);
    uint32_t *start = (uint32_t *)(ws + L.start);
    uint32_t *cstart = (uint32_t *)(ws + L.cstart);
    uint64_t *keys = (uint64_t *)(ws + L.keys);
    uint16_t *lps = (uint16_t *)(ws + L.lps);
    const size_t lds = (size_t)L.ntiles * sizeof(uint32_t);
    if (vec)
        hipLaunchKernelGGL((k_sort_count<kSortPpt, true>), dim3(L.groups), dim3(kSortBlock), lds,
                           s, p, P, counts, L.ntx, L.ntiles, L.per_wg);
    else
        hipLaunchKernelGGL((k_sort_count<kSortPpt, false>), dim3(L.groups), dim3(kSortBlock), lds,
                           s, p, P, counts, L.ntx, L.ntiles, L.per_wg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sort_prefix, dim3((L.ntiles + kPrefixTiles - 1) / kPrefixTiles),
                       dim3(kPrefixTiles * kPrefixSegs), 0, s, counts, L.groups, L.ntiles, total);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, total, start, cstart, L.ntiles);
    if (vec)
        hipLaunchKernelGGL((k_sort_scatter<kSortPpt, true>), dim3(L.groups), dim3(kSortBlock),
                           lds, s, p, P, counts, start, keys, lps, L.ntx, L.ntiles, L.per_wg);
    else
        hipLaunchKernelGGL((k_sort_scatter<kSortPpt, false>), dim3(L.groups), dim3(kSortBlock),
                           lds, s, p, P, counts, start, keys, lps, L.ntx, L.ntiles, L.per_wg);
    return hipGetLastError();
}

}  // namespace
}  // namespace rz

using namespace rz;

extern "C" {

int64_t rz_sorted_workspace_bytes(int64_t n, int32_t width, int32_t height)
{
    if (n < 0 || width < 1 || height < 1)
        return -1;
    const Layout L = layout(n, width, height);
    return (int64_t)L.bytes;
}

int rasterize_sorted(const rz_points *pts, const rz_view *view, const rz_depth_map *depth,
                     const rz_hq_params *hq, uint32_t background, uint64_t *fb, uint64_t *acc,
                     uint32_t *img, uint32_t *status, void *workspace, int64_t workspace_bytes,
                     uint32_t flags, void *stream)
{
    int rc = check_points(pts);
    if (rc)
        return rc;
    Proj P;
    if ((rc = make_proj(view, depth, &P)))
        return rc;
    uint32_t num = 1, den = 100;
    if (hq && (rc = check_hq(hq, P, &num, &den)))
        return rc;
    if (!fb || (hq && !acc) || (flags & ~RZ_KEEP_KEYS) || (!(flags & RZ_KEEP_KEYS) && !img))
        return RZ_EINVAL;
    const Layout L = layout(pts->n, P.width, P.height);
    if (L.ntiles > kMaxTiles)
        return RZ_EINVAL;
    if (pts->n > 0 && (!workspace || ((uintptr_t)workspace & 255u) ||
                       workspace_bytes < (int64_t)L.bytes))
        return RZ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t npix = (int64_t)P.width * P.height;
    hipError_t e = hipSuccess;
    if (pts->n > 0) {
        const Pts p{pts->x, pts->y, pts->z, pts->rgb, pts->n};
        const bool vec = (((uintptr_t)p.x | (uintptr_t)p.y | (uintptr_t)p.z | (uintptr_t)p.rgb) &
                          15u) == 0;
        char *ws = (char *)workspace;
        e = sort_passes(p, P, L, ws, vec, s);
        const uint64_t *keys = (const uint64_t *)(ws + L.keys);
        const uint16_t *lps = (const uint16_t *)(ws + L.lps);
        const uint32_t *start = (const uint32_t *)(ws + L.start);
        const uint32_t *cstart = (const uint32_t *)(ws + L.cstart);
        const dim3 grid((uint32_t)L.chunks_max);   // workgroups past the last chunk exit
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_sort_raster, grid, dim3(256), 0, s, keys, lps, start, cstart, fb,
                               L.ntx, L.ntiles, P.width);
            e = hipGetLastError();
        }
        if (e == hipSuccess && hq) {
            if (P.nr)
                hipLaunchKernelGGL((k_sort_accum<true>), grid, dim3(256), 0, s, keys, lps, start,
                                   cstart, P, num, den, fb, acc, L.ntx, L.ntiles, P.width,
                                   P.height);
            else
                hipLaunchKernelGGL((k_sort_accum<false>), grid, dim3(256), 0, s, keys, lps, start,
                                   cstart, P, num, den, fb, acc, L.ntx, L.ntiles, P.width,
                                   P.height);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess && !(flags & RZ_KEEP_KEYS))
        e = hq ? launch_resolve_hq(fb, acc, npix, background, img, status, s)
               : launch_resolve_min(fb, npix, background, img, s);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

}  // extern "C"
