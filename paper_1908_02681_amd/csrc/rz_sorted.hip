// Screen-sorted rendering (declared in include/rz.h): the same depth pass
// (section 2.1) and splat accumulation (section 2.2) for clouds in no
// particular order, where one global atomic per fragment would hit random
// framebuffer lines.  The fragments are first sorted by 32x32 screen tile in
// two scatter levels, every write of the sort part of a run:
//   A   k_sort_count   per workgroup range of points: fragments per tile
//                      (LDS histogram, added to the totals) and per coarse
//                      bucket (256x256 px)
//   B   k_sort_prefix  per coarse bucket: each workgroup's offset (prefix
//                      over workgroups)
//       k_sort_scan    bucket starts and the work lists of C2, D and E
//   C1  k_sort_coarse  the fragments again; each workgroup appends to its
//                      own run of every coarse bucket through LDS cursors:
//                      key + pixel in bucket
//   C2  k_sort_fine    per chunk of 8192 entries of a coarse bucket: ranked
//                      by tile in LDS, one global atomic per tile reserves
//                      the chunk's run in the tile bucket: key + pixel in
//                      tile
//   D   k_sort_raster  per chunk of a tile bucket: LDS minimum, then one
//                      coalesced global atomic per touched pixel
//   E   k_sort_accum   per chunk of a tile bucket: eps window against the
//                      finished depth pass, LDS sums, one flush per pixel
// Only C2 places entries with global atomics, one per (chunk, tile).  Tiles
// are numbered coarse bucket first ("slots"): slot = coarse * 64 + 8 * (tile
// row in bucket) + (tile column in bucket), so a coarse bucket is the
// contiguous union of its 64 tile buckets; inside a coarse bucket the runs
// of A's workgroups follow in workgroup order.  Every reduction is a minimum or an
// integer sum, so the result is the oracle's bit for bit whatever order the
// fragments land in.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

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
constexpr int kCoarseShift = 3;               // 8 x 8 tiles per coarse bucket
constexpr int kSlotsPerCoarse = 1 << (2 * kCoarseShift);
constexpr int kMaxCoarse = 256;
constexpr int kMaxSlots = kMaxCoarse * kSlotsPerCoarse;   // pass A histogram: 64 KiB
constexpr int kGroups = 512;                  // workgroups of passes A and C1 (<= 1024)
constexpr int kSortBlock = 1024;
constexpr int kSortPpt = 8;                   // 8192 points per workgroup step
constexpr int kStep = kSortBlock * kSortPpt;
constexpr uint32_t kChunk = 8192;             // bucket entries per work item (C2, D, E)
constexpr int kUnroll = 4;                    // bucket entries in flight per thread (D, E)
constexpr int kPrefixCols = 32;               // pass B: columns per workgroup
constexpr int kPrefixSegs = 32;               // pass B: workgroup segments per column

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

struct Layout {
    int32_t ntx = 0, nty = 0, ccols = 0, crows = 0, ncoarse = 0, nslots = 0, groups = 0;
    int64_t per_wg = 0;
    int64_t cchunks_max = 0, fchunks_max = 0;   // bounds on the work lists
    size_t ccounts = 0, total = 0, ctotal = 0, fstart = 0, fchunk = 0;
    size_t fcursor = 0, cchunk = 0;
    size_t xkeys = 0, xlpc = 0, ykeys = 0, ylps = 0, bytes = 0;
};

Layout layout(int64_t n, int32_t w, int32_t h)
{
    Layout L;
    L.ntx = (w + (1 << kTileShift) - 1) >> kTileShift;
    L.nty = (h + (1 << kTileShift) - 1) >> kTileShift;
    L.ccols = (L.ntx + (1 << kCoarseShift) - 1) >> kCoarseShift;
    L.crows = (L.nty + (1 << kCoarseShift) - 1) >> kCoarseShift;
    L.ncoarse = L.ccols * L.crows;
    L.nslots = L.ncoarse * kSlotsPerCoarse;
    if (n > 0) {
        const int64_t want = (n + kGroups - 1) / kGroups;
        L.per_wg = (want + kStep - 1) / kStep * kStep;
        L.groups = (int32_t)((n + L.per_wg - 1) / L.per_wg);
    }
    // sum over buckets of ceil(count / kChunk) <= n / kChunk + buckets
    L.cchunks_max = (n + kChunk - 1) / kChunk + L.ncoarse;
    L.fchunks_max = (n + kChunk - 1) / kChunk + L.nslots;
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.ccounts = take((size_t)L.groups * L.ncoarse * 4);
    L.total = take((size_t)L.nslots * 4);
    L.ctotal = take((size_t)L.ncoarse * 4);
    L.fstart = take(((size_t)L.nslots + 1) * 4);
    L.fchunk = take(((size_t)L.nslots + 1) * 4);
    L.fcursor = take((size_t)L.nslots * 4);
    L.cchunk = take(((size_t)L.ncoarse + 1) * 4);
    L.xkeys = take((size_t)n * 8);
    L.xlpc = take((size_t)n * 2);
    L.ykeys = take((size_t)n * 8);
    L.ylps = take((size_t)n * 2);
    L.bytes = o;
    return L;
}

// Slot of the tile holding pixel (px, py).
__device__ __forceinline__ uint32_t slot_of(uint32_t px, uint32_t py, int32_t ccols)
{
    const uint32_t tx = px >> kTileShift, ty = py >> kTileShift;
    const uint32_t c = (ty >> kCoarseShift) * (uint32_t)ccols + (tx >> kCoarseShift);
    return (c << (2 * kCoarseShift)) | ((ty & 7u) << kCoarseShift) | (tx & 7u);
}

// First pixel of the tile of a slot.
__device__ __forceinline__ void slot_origin(uint32_t slot, int32_t ccols, uint32_t &x0,
                                            uint32_t &y0)
{
    const uint32_t c = slot >> (2 * kCoarseShift), f = slot & (kSlotsPerCoarse - 1);
    const uint32_t tx = (c % (uint32_t)ccols) * 8u + (f & 7u);
    const uint32_t ty = (c / (uint32_t)ccols) * 8u + (f >> kCoarseShift);
    x0 = tx << kTileShift;
    y0 = ty << kTileShift;
}

// Adds this lane's entry to the LDS counter hist[bin] and returns the
// counter before it (the entry's rank among the workgroup's entries of that
// bin).  A wave whose live lanes share one bin makes a single atomic.  Every
// lane of the wave must call it.
__device__ __forceinline__ uint32_t lds_rank(uint32_t *hist, uint32_t bin, bool live)
{
    const uint64_t m = __ballot(live);
    if (m == 0)
        return 0u;
    const uint32_t below =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    const int leader = __builtin_ctzll(m);
    const uint32_t b0 = __shfl(bin, leader);
    if (__all(!live || bin == b0)) {
        uint32_t base = 0;
        if (live && below == 0)
            base = atomicAdd(&hist[b0], (uint32_t)__popcll(m));
        return __shfl(base, leader) + below;
    }
    return live ? atomicAdd(&hist[bin], 1u) : 0u;
}

// Pass A: fragments per tile (added to total[], zero on entry) and per
// coarse bucket in this workgroup's contiguous range of points
// (ccounts[g][coarse]).
template <bool VEC, bool PW>
__global__ void __launch_bounds__(kSortBlock) k_sort_count(Pts p, Proj P, uint32_t *total,
                                                           uint32_t *ccounts, int32_t ccols,
                                                           int32_t nslots, int32_t ncoarse,
                                                           int64_t per_wg)
{
    extern __shared__ uint32_t hist[];
    for (int32_t i = threadIdx.x; i < nslots; i += blockDim.x)
        hist[i] = 0u;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * per_wg;
    Pts q = p;
    q.n = lo + per_wg < p.n ? lo + per_wg : p.n;
    for (int64_t base = lo; base < q.n; base += kStep) {
        float x[kSortPpt], y[kSortPpt], z[kSortPpt];
        uint32_t c[kSortPpt];
        bool in[kSortPpt];
        load_points<kSortPpt, VEC>(q, base, x, y, z, c, in);
#pragma unroll
        for (int j = 0; j < kSortPpt; ++j) {
            uint32_t px = 0, py = 0;
            uint64_t qq = 0;
            const bool live = fragment<PW>(P, x[j], y[j], z[j], px, py, qq) & in[j];
            lds_rank(hist, live ? slot_of(px, py, ccols) : 0u, live);
        }
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < nslots; i += blockDim.x) {
        const uint32_t v = hist[i];
        if (v)
            atomicAdd(&total[i], v);
    }
    if ((int32_t)threadIdx.x < ncoarse) {
        uint32_t sum = 0;
        for (int k = 0; k < kSlotsPerCoarse; ++k)
            sum += hist[threadIdx.x * kSlotsPerCoarse + k];
        ccounts[(int64_t)blockIdx.x * ncoarse + threadIdx.x] = sum;
    }
}

__global__ void k_sort_zero(uint32_t *p, int32_t n)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0u;
}

// Pass B, first part: for every column of the [groups][coarse] count matrix,
// the exclusive prefix over groups (in place) and the column total.  A
// workgroup takes kPrefixCols columns; each of its kPrefixSegs segments sums
// a run of up to kPrefixSegs groups, the segment sums are scanned in LDS, and
// the segments write their offsets (groups <= 1024).
__global__ void __launch_bounds__(kPrefixCols * kPrefixSegs)
    k_sort_prefix(uint32_t *m, int32_t groups, int32_t cols, uint32_t *total)
{
    __shared__ uint32_t s_seg[kPrefixSegs][kPrefixCols];
    const int tt = threadIdx.x % kPrefixCols, seg = threadIdx.x / kPrefixCols;
    const int32_t t = blockIdx.x * kPrefixCols + tt;
    const bool on = t < cols;
    const int32_t g0 = seg * kPrefixSegs;
    uint32_t c[kPrefixSegs];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPrefixSegs; ++k) {
        const int32_t g = g0 + k;
        c[k] = on && g < groups ? m[(int64_t)g * cols + t] : 0u;
        sum += c[k];
    }
    s_seg[seg][tt] = sum;
    __syncthreads();
    if (seg == 0) {   // exclusive scan over the segments of column tt
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
            m[(int64_t)g * cols + t] = run;
        run += c[k];
    }
}

// Pass B, second part: one workgroup of 1024 threads, 16 slots each
// (nslots <= 16384).
//   fstart  exclusive scan of the tile totals (tile bucket starts), and
//           fstart[nslots] = all fragments; fcursor = fstart;
//   fchunk  exclusive scan of ceil(total / kChunk): work items of D and E;
//   cchunk  exclusive scan of ceil(coarse total / kChunk): work items of C2.
__global__ void __launch_bounds__(1024) k_sort_scan(const uint32_t *total, uint32_t *fstart,
                                                    uint32_t *fchunk, uint32_t *fcursor,
                                                    uint32_t *cchunk, int32_t nslots,
                                                    int32_t ncoarse)
{
    constexpr int K = kMaxSlots / 1024;
    static_assert(kSlotsPerCoarse % K == 0, "a coarse bucket spans whole threads");
    constexpr int kThreadsPerCoarse = kSlotsPerCoarse / K;
    __shared__ uint32_t s_sum[1024], s_ch[1024];
    const int32_t t0 = threadIdx.x * K;
    uint32_t v[K];
    uint32_t local = 0, lch = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = t0 + k < nslots ? total[t0 + k] : 0u;
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
    for (int k = 0; k < K; ++k) {
        if (t0 + k < nslots) {
            fstart[t0 + k] = run;
            fcursor[t0 + k] = run;
            fchunk[t0 + k] = runc;
        }
        run += v[k];
        runc += (v[k] + kChunk - 1) / kChunk;
    }
    if (threadIdx.x == 1023) {
        fstart[nslots] = s_sum[1023];
        fchunk[nslots] = s_ch[1023];
    }
    // coarse buckets: s_sum holds the inclusive sums per thread
    uint32_t cn = 0;
    if ((int32_t)threadIdx.x < ncoarse) {
        const int32_t last = kThreadsPerCoarse * threadIdx.x + kThreadsPerCoarse - 1;
        const uint32_t end = s_sum[last];
        const uint32_t beg = threadIdx.x ? s_sum[last - kThreadsPerCoarse] : 0u;
        cn = (end - beg + kChunk - 1) / kChunk;
    }
    __syncthreads();
    s_ch[threadIdx.x] = cn;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t addc = threadIdx.x >= (uint32_t)off ? s_ch[threadIdx.x - off] : 0u;
        __syncthreads();
        s_ch[threadIdx.x] += addc;
        __syncthreads();
    }
    if ((int32_t)threadIdx.x < ncoarse)
        cchunk[threadIdx.x] = s_ch[threadIdx.x] - cn;
    if (threadIdx.x == 1023)
        cchunk[ncoarse] = s_ch[1023];
}

// Pass C1: the fragments of pass A again (same ranges, same arithmetic).
// Workgroup g owns the run of every coarse bucket that starts at the
// bucket's start plus g's offset from pass B; LDS cursors hand out its
// places.
template <bool VEC, bool PW>
__global__ void __launch_bounds__(kSortBlock) k_sort_coarse(Pts p, Proj P,
                                                            const uint32_t *__restrict__ coff,
                                                            const uint32_t *__restrict__ fstart,
                                                            uint64_t *xkeys, uint16_t *xlpc,
                                                            int32_t ccols, int32_t ncoarse,
                                                            int64_t per_wg)
{
    __shared__ uint32_t s_cur[kMaxCoarse];
    const uint64_t end = (uint64_t)p.n;   // bucket arrays hold n entries
    if ((int32_t)threadIdx.x < ncoarse)
        s_cur[threadIdx.x] = fstart[threadIdx.x * kSlotsPerCoarse] +
                             coff[(int64_t)blockIdx.x * ncoarse + threadIdx.x];
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * per_wg;
    Pts q = p;
    q.n = lo + per_wg < p.n ? lo + per_wg : p.n;
    for (int64_t base = lo; base < q.n; base += kStep) {
        float x[kSortPpt], y[kSortPpt], z[kSortPpt];
        uint32_t c[kSortPpt];
        bool in[kSortPpt];
        load_points<kSortPpt, VEC>(q, base, x, y, z, c, in);
#pragma unroll
        for (int j = 0; j < kSortPpt; ++j) {
            uint32_t px = 0, py = 0;
            uint64_t qq = 0;
            const bool live = fragment<PW>(P, x[j], y[j], z[j], px, py, qq) & in[j];
            const uint32_t cb = live ? slot_of(px, py, ccols) >> (2 * kCoarseShift) : 0u;
            const uint64_t pos = lds_rank(s_cur, cb, live);
            if (live && pos < end) {   // pos < end always: A and C1 agree
                xkeys[pos] = (qq << 24) | ((uint64_t)c[j] & kRgbMask);
                xlpc[pos] = (uint16_t)(((py & 255u) << 8) | (px & 255u));
            }
        }
    }
}

// Last index a with list[a] <= b (list[0] = 0 <= b < list[count]).
__device__ __forceinline__ int32_t find_item(const uint32_t *list, int32_t count, uint32_t b)
{
    int32_t a = 0, z = count;
    while (z - a > 1) {
        const int32_t m = (a + z) >> 1;
        if (list[m] <= b)
            a = m;
        else
            z = m;
    }
    return a;
}

// Pass C2: one chunk of a coarse bucket into the bucket's 64 tile buckets,
// ranked in LDS as in C1.
__global__ void __launch_bounds__(kSortBlock) k_sort_fine(const uint64_t *__restrict__ xkeys,
                                                          const uint16_t *__restrict__ xlpc,
                                                          const uint32_t *__restrict__ fstart,
                                                          const uint32_t *__restrict__ cchunk,
                                                          uint32_t *fcursor,
                                                          uint64_t *__restrict__ ykeys,
                                                          uint16_t *__restrict__ ylps,
                                                          int32_t ncoarse, int64_t n)
{
    __shared__ uint32_t s_cnt[kSlotsPerCoarse], s_base[kSlotsPerCoarse];
    const uint32_t b = blockIdx.x;
    if (b >= cchunk[ncoarse])
        return;
    const int32_t cb = find_item(cchunk, ncoarse, b);
    const uint32_t bucket_end = fstart[(cb + 1) * kSlotsPerCoarse];
    const uint32_t lo = fstart[cb * kSlotsPerCoarse] + (b - cchunk[cb]) * kChunk;
    const uint32_t hi = bucket_end - lo > kChunk ? lo + kChunk : bucket_end;
    if (threadIdx.x < kSlotsPerCoarse)
        s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    constexpr int K = kChunk / kSortBlock;
    uint64_t key[K];
    uint32_t f[K], lp[K], rank[K];
    bool ok[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const uint64_t i = (uint64_t)lo + (uint64_t)u * kSortBlock + threadIdx.x;
        ok[u] = i < hi;
        key[u] = ok[u] ? ldnt(xkeys + i) : 0ull;
        const uint32_t v = ok[u] ? (uint32_t)xlpc[i] : 0u;
        f[u] = ((v >> 13) << kCoarseShift) | ((v & 255u) >> kTileShift);
        lp[u] = (((v >> 8) & 31u) << kTileShift) | (v & 31u);
    }
#pragma unroll
    for (int u = 0; u < K; ++u)
        rank[u] = lds_rank(s_cnt, f[u], ok[u]);
    __syncthreads();
    if (threadIdx.x < kSlotsPerCoarse) {
        const uint32_t k = s_cnt[threadIdx.x];
        s_base[threadIdx.x] =
            k ? atomicAdd(&fcursor[cb * kSlotsPerCoarse + threadIdx.x], k) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const uint64_t pos = (uint64_t)s_base[f[u]] + rank[u];
        if (ok[u] && pos < (uint64_t)n) {   // pos < n always: the totals of A
            ykeys[pos] = key[u];
            ylps[pos] = (uint16_t)lp[u];
        }
    }
}

// The work item of this workgroup in passes D and E: slot t and the range
// [lo, hi) of its tile bucket, at most kChunk entries.  Workgroups past the
// last item get lo >= hi.
__device__ __forceinline__ void chunk_of(const uint32_t *fstart, const uint32_t *fchunk,
                                         int32_t nslots, int32_t &t, uint32_t &lo, uint32_t &hi)
{
    const uint32_t b = blockIdx.x;
    t = 0;
    hi = lo = 0;
    if (b >= fchunk[nslots])
        return;
    t = find_item(fchunk, nslots, b);
    const uint32_t end = fstart[t + 1];
    lo = fstart[t] + (b - fchunk[t]) * kChunk;
    hi = end - lo > kChunk ? lo + kChunk : end;
}

// Pass D: depth pass of one chunk of a tile bucket (section 2.1's minimum).
__global__ void __launch_bounds__(256) k_sort_raster(const uint64_t *__restrict__ keys,
                                                     const uint16_t *__restrict__ lps,
                                                     const uint32_t *__restrict__ fstart,
                                                     const uint32_t *__restrict__ fchunk,
                                                     uint64_t *__restrict__ fb, int32_t ccols,
                                                     int32_t nslots, int32_t width)
{
    __shared__ uint64_t tile[kTilePix];
    int32_t t;
    uint32_t lo, hi;
    chunk_of(fstart, fchunk, nslots, t, lo, hi);
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
    uint32_t x0, y0;
    slot_origin((uint32_t)t, ccols, x0, y0);
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

// Pass E: splat accumulation of one chunk of a tile bucket (section 2.2),
// from the bucket's keys; fb holds the finished depth pass.
template <bool PW>
__global__ void __launch_bounds__(256) k_sort_accum(const uint64_t *__restrict__ keys,
                                                    const uint16_t *__restrict__ lps,
                                                    const uint32_t *__restrict__ fstart,
                                                    const uint32_t *__restrict__ fchunk, Proj P,
                                                    uint32_t eps_num, uint32_t eps_den,
                                                    const uint64_t *__restrict__ fb,
                                                    uint64_t *__restrict__ acc, int32_t ccols,
                                                    int32_t nslots, int32_t width, int32_t height)
{
    __shared__ uint64_t qmin[kTilePix];
    __shared__ uint64_t sums[2 * kTilePix];
    int32_t t;
    uint32_t lo, hi;
    chunk_of(fstart, fchunk, nslots, t, lo, hi);
    if (lo >= hi)
        return;
    uint32_t x0, y0;
    slot_origin((uint32_t)t, ccols, x0, y0);
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

// Passes A to C2: leaves the tile buckets (ykeys, ylps) and their starts.
hipError_t sort_passes(const Pts &p, const Proj &P, const Layout &L, char *ws, bool vec,
                       hipStream_t s)
{
    uint32_t *ccounts = (uint32_t *)(ws + L.ccounts);
    uint32_t *total = (uint32_t *)(ws + L.total);
    uint32_t *ctotal = (uint32_t *)(ws + L.ctotal);
    uint32_t *fstart = (uint32_t *)(ws + L.fstart);
    uint32_t *fchunk = (uint32_t *)(ws + L.fchunk);
    uint32_t *fcursor = (uint32_t *)(ws + L.fcursor);
    uint32_t *cchunk = (uint32_t *)(ws + L.cchunk);
    uint64_t *xkeys = (uint64_t *)(ws + L.xkeys);
    uint16_t *xlpc = (uint16_t *)(ws + L.xlpc);
    uint64_t *ykeys = (uint64_t *)(ws + L.ykeys);
    uint16_t *ylps = (uint16_t *)(ws + L.ylps);
    hipLaunchKernelGGL(k_sort_zero, dim3((L.nslots + 255) / 256), dim3(256), 0, s, total,
                       L.nslots);
    const size_t lds = (size_t)L.nslots * sizeof(uint32_t);
    const dim3 g(L.groups), b(kSortBlock);
    const bool pw = P.nr != 0;
    if (vec && pw)
        hipLaunchKernelGGL((k_sort_count<true, true>), g, b, lds, s, p, P, total, ccounts,
                           L.ccols, L.nslots, L.ncoarse, L.per_wg);
    else if (vec)
        hipLaunchKernelGGL((k_sort_count<true, false>), g, b, lds, s, p, P, total, ccounts,
                           L.ccols, L.nslots, L.ncoarse, L.per_wg);
    else if (pw)
        hipLaunchKernelGGL((k_sort_count<false, true>), g, b, lds, s, p, P, total, ccounts,
                           L.ccols, L.nslots, L.ncoarse, L.per_wg);
    else
        hipLaunchKernelGGL((k_sort_count<false, false>), g, b, lds, s, p, P, total, ccounts,
                           L.ccols, L.nslots, L.ncoarse, L.per_wg);
    hipLaunchKernelGGL(k_sort_prefix, dim3((L.ncoarse + kPrefixCols - 1) / kPrefixCols),
                       dim3(kPrefixCols * kPrefixSegs), 0, s, ccounts, L.groups, L.ncoarse,
                       ctotal);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, total, fstart, fchunk, fcursor,
                       cchunk, L.nslots, L.ncoarse);
    if (vec && pw)
        hipLaunchKernelGGL((k_sort_coarse<true, true>), g, b, 0, s, p, P, ccounts, fstart, xkeys,
                           xlpc, L.ccols, L.ncoarse, L.per_wg);
    else if (vec)
        hipLaunchKernelGGL((k_sort_coarse<true, false>), g, b, 0, s, p, P, ccounts, fstart, xkeys,
                           xlpc, L.ccols, L.ncoarse, L.per_wg);
    else if (pw)
        hipLaunchKernelGGL((k_sort_coarse<false, true>), g, b, 0, s, p, P, ccounts, fstart, xkeys,
                           xlpc, L.ccols, L.ncoarse, L.per_wg);
    else
        hipLaunchKernelGGL((k_sort_coarse<false, false>), g, b, 0, s, p, P, ccounts, fstart,
                           xkeys, xlpc, L.ccols, L.ncoarse, L.per_wg);
    hipLaunchKernelGGL(k_sort_fine, dim3((uint32_t)L.cchunks_max), dim3(kSortBlock), 0, s, xkeys,
                       xlpc, fstart, cchunk, fcursor, ykeys, ylps, L.ncoarse, p.n);
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
    if (L.ncoarse > kMaxCoarse)
        return -1;
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
    if (P.zkind != 0)   // float depth encodings: one-view calls only
        return RZ_EINVAL;
    uint32_t num = 1, den = 100;
    if (hq && (rc = check_hq(hq, P, &num, &den)))
        return rc;
    if (!fb || (hq && !acc) || (flags & ~RZ_KEEP_KEYS) ||
        (!(flags & RZ_KEEP_KEYS) && (!img || (hq && !status))))
        return RZ_EINVAL;
    const Layout L = layout(pts->n, P.width, P.height);
    if (L.ncoarse > kMaxCoarse)
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
        const uint64_t *keys = (const uint64_t *)(ws + L.ykeys);
        const uint16_t *lps = (const uint16_t *)(ws + L.ylps);
        const uint32_t *fstart = (const uint32_t *)(ws + L.fstart);
        const uint32_t *fchunk = (const uint32_t *)(ws + L.fchunk);
        const dim3 grid((uint32_t)L.fchunks_max);   // workgroups past the last item exit
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_sort_raster, grid, dim3(256), 0, s, keys, lps, fstart, fchunk,
                               fb, L.ccols, L.nslots, P.width);
            e = hipGetLastError();
        }
        if (e == hipSuccess && hq) {
            if (P.nr)
                hipLaunchKernelGGL((k_sort_accum<true>), grid, dim3(256), 0, s, keys, lps, fstart,
                                   fchunk, P, num, den, fb, acc, L.ccols, L.nslots, P.width,
                                   P.height);
            else
                hipLaunchKernelGGL((k_sort_accum<false>), grid, dim3(256), 0, s, keys, lps,
                                   fstart, fchunk, P, num, den, fb, acc, L.ccols, L.nslots,
                                   P.width, P.height);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess && !(flags & RZ_KEEP_KEYS))
        e = hq ? launch_resolve_hq(fb, acc, npix, background, img, status, s)
               : launch_resolve_min(fb, npix, background, img, s);
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}


}  // extern "C"

// ---- allocation-free variant -----------------------------------------
//
// The workspace of rasterize_sorted_noalloc is a file-scope device array.
// In host code its name is only a stand-in for the symbol, so its device
// address is looked up once per device (with that device current) and kept;
// kernels and every host-side use take that address, never the name.
namespace rz {
namespace {

static __device__ __align__(256) unsigned char scratch[RZ_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (first call per device: the symbol
// lookup, under a lock).  Returns hipSuccess and sets *out.
hipError_t scratch_for_current_device(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!ptr || ((uintptr_t)ptr & 255u))
            return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace rz

extern "C" int rasterize_sorted_noalloc(const rz_points *pts, const rz_view *view,
                                        const rz_depth_map *depth, const rz_hq_params *hq,
                                        uint32_t background, uint64_t *fb, uint64_t *acc,
                                        uint32_t *img, uint32_t *status, uint32_t flags,
                                        void *stream)
{
    // the size checks of rasterize_sorted first, so that a call too large
    // for the scratch is refused before the symbol lookup
    if (!view || !pts)
        return RZ_EINVAL;
    const int64_t need = rz_sorted_workspace_bytes(pts->n, view->width, view->height);
    if (need < 0 || pts->n < 0)
        return RZ_EINVAL;
    if (need > (int64_t)RZ_NOALLOC_SCRATCH_BYTES)
        return RZ_EBUDGET;
    void *ws = nullptr;
    if (pts->n > 0) {
        const hipError_t e = rz::scratch_for_current_device(&ws);
        if (e != hipSuccess)
            return rz::hip_fail(e);
    }
    return rasterize_sorted(pts, view, depth, hq, background, fb, acc, img, status, ws,
                            (int64_t)RZ_NOALLOC_SCRATCH_BYTES, flags, stream);
}
