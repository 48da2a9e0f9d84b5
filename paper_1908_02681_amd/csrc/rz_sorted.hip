// Screen-sorted rendering (declared in include/rz.h): the same depth pass
// (section 2.1) and splat accumulation (section 2.2) for clouds in no
// particular order, where one global atomic per fragment would hit random
// framebuffer lines.  The fragments are sorted once, by bucket (a 64x64
// screen tile), and each bucket is then reduced in LDS:
//   A  k_sort_count    per workgroup range of points: on-screen points per
//                      bucket, from the single-precision projection alone
//                      (LDS histogram); one row of counts per workgroup
//   B  k_sort_prefix   per bucket: each workgroup's offset (prefix over
//                      workgroups) and the bucket's total
//      k_sort_scan     bucket starts and the chunk work list of E
//   C  k_sort_scatter  the same ranges again, with the whole fragment (depth
//                      in double precision).  Per step of 4096 points the
//                      workgroup sorts its entries by bucket in LDS (a
//                      counting sort), then writes each bucket's run at its
//                      own cursor in that bucket: consecutive lanes write
//                      consecutive entries.  Entry = key (u64) + pixel in
//                      the tile (u16).  (8192 points per step)
//   D  k_sort_raster   an equal share of the entries per workgroup; per run
//                      of one bucket in it: LDS minimum over the tile, then
//                      one coalesced early-out atomic per touched pixel
//   E  k_sort_accum    per chunk: the tile's nearest depths staged in LDS,
//                      the eps window, LDS sums, one flush per pixel
// A point that is on screen but outside [near, far) still takes its place
// (A counts it without the double-precision depth), with the key ~0: it
// never lowers a minimum, D never flushes a tile entry that only it
// reached, and E skips it.  Every reduction is a minimum or an integer sum,
// so the result is the oracle's bit for bit whatever order the fragments
// land in.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "rz.h"
#include "rz_device.h"
#include "rz_internal.h"
#include "rz_trace.h"

namespace rz {

int check_points(const rz_points *p);
int make_proj(const rz_view *v, const rz_depth_map *dm, Proj *P);
int check_hq(const rz_hq_params *hq, const Proj &P, uint32_t *num, uint32_t *den);
int hip_fail(hipError_t e);

namespace {

using namespace dev;

constexpr int kTileShift = 6;                 // buckets are 64 x 64 pixel tiles
constexpr int kTileSide = 1 << kTileShift;
constexpr int kTilePix = kTileSide * kTileSide;
constexpr int kMaxBuckets = 4096;             // A's histogram and C's offsets: 16 KiB
constexpr int kGroups = 512;                  // workgroups of passes A and C (<= 1024)
constexpr int kCountBlock = 1024;             // pass A: 8192 points per step
constexpr int kCountPpt = 8;
constexpr int kCountStep = kCountBlock * kCountPpt;
constexpr int kScBlock = 1024;                // pass C: 8192 points per step
constexpr int kScPpt = 8;
constexpr int kScStep = kScBlock * kScPpt;
constexpr int kScBuckets = kMaxBuckets / kScBlock;   // buckets per thread in C's scan
constexpr int kRasterBlock = 256;
constexpr int kRasterGroups = 512;            // pass D: two workgroups per CU
constexpr int kAccumBlock = 1024;
constexpr int kUnroll = 8;                    // bucket entries in flight per thread (D, E)
constexpr int kPrefixCols = 32;               // pass B: columns per workgroup
constexpr int kPrefixSegs = 32;               // pass B: workgroup segments per column
constexpr int kScanThreads = 1024;
static_assert(kCountStep % kScStep == 0, "A's ranges are whole steps of C");
static_assert(kMaxBuckets % kScBlock == 0 && kMaxBuckets % kScanThreads == 0, "scan shapes");
static_assert(kMaxBuckets <= 4096 && kTilePix <= 4096, "bucket and pixel fit 12 bits each");

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

struct Layout {
    int32_t ntx = 0, nty = 0, nb = 0, groups = 0;
    int64_t per_wg = 0;
    uint32_t chunk = 0;          // bucket entries per work item of E
    int64_t chunks_max = 0;      // bound on the work items
    size_t ccounts = 0, btotal = 0, bstart = 0, bchunk = 0, keys = 0, lps = 0, bytes = 0;
};

Layout layout(int64_t n, int32_t w, int32_t h)
{
    Layout L;
    L.ntx = (w + kTileSide - 1) >> kTileShift;
    L.nty = (h + kTileSide - 1) >> kTileShift;
    L.nb = L.ntx * L.nty;
    if (n > 0) {
        const int64_t want = (n + kGroups - 1) / kGroups;
        L.per_wg = (want + kCountStep - 1) / kCountStep * kCountStep;
        L.groups = (int32_t)((n + L.per_wg - 1) / L.per_wg);
    }
    // about 512 work items, at least 131072 entries each: a chunk's flush of
    // up to 4096 pixels (two global atomics each in the splat pass) stays
    // small beside its entries
    const int64_t c = ((n + 511) / 512 + 1023) / 1024 * 1024;
    L.chunk = (uint32_t)(c > 131072 ? c : 131072);
    // sum over buckets of ceil(count / chunk) <= n / chunk + buckets
    L.chunks_max = (n + L.chunk - 1) / L.chunk + L.nb;
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.ccounts = take((size_t)L.groups * L.nb * 4);
    L.btotal = take((size_t)L.nb * 4);
    L.bstart = take(((size_t)L.nb + 1) * 4);
    L.bchunk = take(((size_t)L.nb + 1 + L.chunks_max) * 4);   // + the bucket of each item
    L.keys = take((size_t)n * 8);
    L.lps = take((size_t)n * 2);
    L.bytes = o;
    return L;
}

// Bucket and pixel-in-tile of an on-screen pixel, packed: bucket << 12 | pixel.
__device__ __forceinline__ uint32_t bucket_pixel(uint32_t px, uint32_t py, int32_t ntx)
{
    const uint32_t b = __umul24(py >> kTileShift, (uint32_t)ntx) + (px >> kTileShift);
    return (b << 12) | ((py & (kTileSide - 1)) << kTileShift) | (px & (kTileSide - 1));
}

// Adds one to hist[bin] for every live lane; a wave whose live lanes share
// one bin makes a single atomic.  Every lane of the wave must call it.
__device__ __forceinline__ void lds_count(uint32_t *hist, uint32_t bin, bool live)
{
    const uint64_t m = __ballot(live);
    if (m == 0)
        return;
    const int leader = __builtin_ctzll(m);
    const uint32_t b0 = __shfl(bin, leader);
    if (__all(!live || bin == b0)) {
        if ((int)(threadIdx.x & 63u) == leader)
            atomicAdd(&hist[b0], (uint32_t)__popcll(m));
        return;
    }
    if (live)
        atomicAdd(&hist[bin], 1u);
}

// Inclusive prefix sum over the 64 lanes of a wave (all lanes active).
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v)
{
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)v, d);
        v += lane >= (uint32_t)d ? t : 0u;
    }
    return v;
}

// Pass A: on-screen points per bucket in this workgroup's contiguous range
// of points, written as row blockIdx.x of ccounts ([groups][nb]).
template <bool VEC>
__global__ void __launch_bounds__(kCountBlock) k_sort_count(Pts p, Proj P, uint32_t *ccounts,
                                                            int32_t ntx, int32_t nb,
                                                            int64_t per_wg)
{
    __shared__ uint32_t hist[kMaxBuckets];
    for (int32_t i = threadIdx.x; i < nb; i += blockDim.x)
        hist[i] = 0u;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * per_wg;
    Pts q = p;
    q.n = lo + per_wg < p.n ? lo + per_wg : p.n;
    const Trans T = lane_trans(P);
    for (int64_t base = lo; base < q.n; base += kCountStep) {
        float x[kCountPpt], y[kCountPpt], z[kCountPpt];
        uint32_t c[kCountPpt];
        load_points_nan<kCountPpt, VEC>(q, base, x, y, z, c);   // past the end: NaN, culled
#pragma unroll
        for (int j = 0; j < kCountPpt; ++j) {
            uint32_t px, py;
            float cw, iw;
            const bool vis = project(P, T, x[j], y[j], z[j], px, py, cw, iw);
            lds_count(hist, bucket_pixel(px, py, ntx) >> 12, vis);
        }
    }
    __syncthreads();
    uint32_t *row = ccounts + (int64_t)blockIdx.x * nb;
    for (int32_t i = threadIdx.x; i < nb; i += blockDim.x)
        row[i] = hist[i];
}

// Pass B, first part: for every column of the [groups][nb] count matrix,
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

// Pass B, second part: one workgroup, 4 buckets per thread.
//   bstart  exclusive scan of the bucket totals; bstart[nb] = all entries;
//   bchunk  exclusive scan of ceil(total / chunk): the work items of E;
//           bchunk[nb] = all work items, then from bchunk[nb + 1] on the
//           bucket of each work item.
__global__ void __launch_bounds__(kScanThreads) k_sort_scan(const uint32_t *total,
                                                            uint32_t *bstart, uint32_t *bchunk,
                                                            int32_t nb, uint32_t chunk)
{
    constexpr int K = kMaxBuckets / kScanThreads;
    __shared__ uint32_t s_sum[kScanThreads], s_ch[kScanThreads];
    __shared__ uint32_t s_first[kMaxBuckets + 1];   // each bucket's first item
    const int32_t t0 = threadIdx.x * K;
    uint32_t v[K];
    uint32_t local = 0, lch = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = t0 + k < nb ? total[t0 + k] : 0u;
        local += v[k];
        lch += (v[k] + chunk - 1) / chunk;
    }
    s_sum[threadIdx.x] = local;
    s_ch[threadIdx.x] = lch;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {   // inclusive scans (Hillis-Steele)
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
        if (t0 + k < nb) {
            bstart[t0 + k] = run;
            bchunk[t0 + k] = runc;
            s_first[t0 + k] = runc;
        }
        run += v[k];
        runc += (v[k] + chunk - 1) / chunk;
    }
    const uint32_t items = s_ch[kScanThreads - 1];
    if (threadIdx.x == kScanThreads - 1) {
        bstart[nb] = s_sum[kScanThreads - 1];
        bchunk[nb] = items;
    }
    __syncthreads();
    // the item table after bchunk[nb]: the bucket of each work item of E
    // (the last bucket whose first item is <= the item; empty buckets share
    // their successor's first item and never own one)
    uint32_t *item_bucket = bchunk + nb + 1;
    for (uint32_t i = threadIdx.x; i < items; i += kScanThreads)
        item_bucket[i] = (uint32_t)find_item(s_first, nb, i);
}

// Pass C: the fragments of pass A's ranges, sorted into the buckets.
// cursors holds, per workgroup row, the prefix offsets of pass B.  Thread t
// owns buckets t * kScBuckets .. t * kScBuckets + kScBuckets - 1 in every
// per-bucket phase and keeps the workgroup's cursors of those buckets in
// registers.
template <bool VEC, bool PW>
__global__ void __launch_bounds__(kScBlock) k_sort_scatter(Pts p, Proj P,
                                                           const uint32_t *__restrict__ cursors,
                                                           const uint32_t *__restrict__ bstart,
                                                           uint64_t *__restrict__ keys,
                                                           uint16_t *__restrict__ lps,
                                                           int32_t ntx, int32_t nb,
                                                           int64_t per_wg)
{
    __shared__ uint32_t s_off[kMaxBuckets];   // counts, then offsets, then deltas
    __shared__ uint64_t s_key[kScStep];       // the step's entries sorted by bucket
    __shared__ uint32_t s_lb[kScStep];        // bucket << 12 | pixel in tile
    __shared__ uint32_t s_wsum[kScBlock / 64];
    __shared__ uint32_t s_total;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const int32_t b0 = (int32_t)tid * kScBuckets;
    const uint32_t *row = cursors + (int64_t)blockIdx.x * nb;
    uint32_t cur[kScBuckets];   // this workgroup's next place in each of the thread's buckets
#pragma unroll
    for (int r = 0; r < kScBuckets; ++r)
        cur[r] = b0 + r < nb ? row[b0 + r] + bstart[b0 + r] : 0u;
    const int64_t lo = (int64_t)blockIdx.x * per_wg;
    Pts q = p;
    q.n = lo + per_wg < p.n ? lo + per_wg : p.n;
    const Trans T = lane_trans(P);
    // the points of the first step; each later step's are loaded while the
    // step before it sorts and writes its entries
    float x[kScPpt], y[kScPpt], z[kScPpt];
    uint32_t c[kScPpt];
    if (lo < q.n)
        load_points_nan<kScPpt, VEC>(q, lo, x, y, z, c);   // past the end: NaN, culled
    for (int64_t base = lo; base < q.n; base += kScStep) {
#pragma unroll
        for (int r = 0; r < kScBuckets; ++r)
            if (b0 + r < nb)
                s_off[b0 + r] = 0u;
        uint32_t lb[kScPpt], rank[kScPpt];   // rank ~0: not on screen
        uint64_t key[kScPpt];
        __syncthreads();   // counters zero (and the previous step's write-out done)
#pragma unroll
        for (int j = 0; j < kScPpt; ++j) {
            uint32_t px = 0, py = 0;
            uint64_t qq = 0;
            double tq;
            bool v = false;
            const bool live = fragment<PW>(P, T, x[j], y[j], z[j], px, py, qq, tq, v);
            key[j] = live ? (qq << 24) | ((uint64_t)c[j] & kRgbMask) : ~0ull;
            lb[j] = bucket_pixel(px, py, ntx);
            rank[j] = v ? atomicAdd(&s_off[lb[j] >> 12], 1u) : ~0u;
        }
        if (base + kScStep < q.n)   // workgroup-uniform
            load_points_nan<kScPpt, VEC>(q, base + kScStep, x, y, z, c);
        __syncthreads();   // counts complete
        // exclusive scan of the counts over the buckets; staging index i of
        // bucket b goes to cursor(b) + (i - off(b)): each bucket's delta
        uint32_t cnt[kScBuckets], delta[kScBuckets];
        uint32_t sum = 0;
#pragma unroll
        for (int r = 0; r < kScBuckets; ++r) {
            cnt[r] = b0 + r < nb ? s_off[b0 + r] : 0u;
            sum += cnt[r];
        }
        const uint32_t incl = wave_inclusive_sum(sum);
        if (lane == 63u)
            s_wsum[wave] = incl;
        __syncthreads();
        uint32_t run = incl - sum;
        for (uint32_t w = 0; w < wave; ++w)
            run += s_wsum[w];
#pragma unroll
        for (int r = 0; r < kScBuckets; ++r) {
            delta[r] = cur[r] - run;
            cur[r] += cnt[r];
            if (b0 + r < nb)
                s_off[b0 + r] = run;
            run += cnt[r];
        }
        if (tid == kScBlock - 1)
            s_total = run;
        __syncthreads();   // offsets complete
#pragma unroll
        for (int j = 0; j < kScPpt; ++j) {
            if (rank[j] != ~0u) {
                const uint32_t i = s_off[lb[j] >> 12] + rank[j];
                s_key[i] = key[j];
                s_lb[i] = lb[j];
            }
        }
        __syncthreads();   // staging complete, offsets read
#pragma unroll
        for (int r = 0; r < kScBuckets; ++r)
            if (b0 + r < nb)
                s_off[b0 + r] = delta[r];
        __syncthreads();   // deltas complete
        const uint32_t total = s_total;
        for (uint32_t i = tid; i < total; i += kScBlock) {
            const uint32_t e = s_lb[i];
            const uint32_t pos = s_off[e >> 12] + i;
            keys[pos] = s_key[i];
            lps[pos] = (uint16_t)(e & 0xFFFu);
        }
        __syncthreads();   // staging and deltas free for the next step
    }
}

// The work item b of a workgroup of pass E: bucket t and the range
// [lo, hi) of its entries, at most `chunk` of them.  Workgroups past the
// last item get lo >= hi.
__device__ __forceinline__ void chunk_of(const uint32_t *bstart, const uint32_t *bchunk,
                                         int32_t nb, uint32_t chunk, uint32_t b, int32_t &t,
                                         uint32_t &lo, uint32_t &hi)
{
    const uint32_t items = bchunk[nb];
    const uint32_t tb = bchunk[nb + 1 + b];   // in the table (b < its length), read early
    t = 0;
    hi = lo = 0;
    if (b >= items)
        return;
    t = (int32_t)tb;
    const uint32_t end = bstart[t + 1];
    lo = bstart[t] + (b - bchunk[t]) * chunk;
    hi = end - lo > chunk ? lo + chunk : end;
}

// Pass D: depth pass (section 2.1's minimum) over an equal share of the
// sorted entries per workgroup, whatever buckets it spans: each run of the
// share that lies in one bucket is reduced in the LDS tile, then flushed
// with one coalesced early-out atomic per touched pixel.  Equal shares keep
// every CU's load the same (work items of whole buckets left the CUs with
// two full items a third above the mean).
__global__ void __launch_bounds__(kRasterBlock) k_sort_raster(const uint64_t *__restrict__ keys,
                                                              const uint16_t *__restrict__ lps,
                                                              const uint32_t *__restrict__ bstart,
                                                              uint64_t *__restrict__ fb,
                                                              int32_t ntx, int32_t nb,
                                                              int32_t width)
{
    __shared__ uint64_t tile[kTilePix];
    __shared__ uint32_t s_start[kMaxBuckets + 1];
    for (int i = threadIdx.x; i <= nb; i += kRasterBlock)
        s_start[i] = bstart[i];
    __syncthreads();
    const uint32_t total = s_start[nb];
    const uint32_t per = (total + gridDim.x - 1) / gridDim.x;
    const uint64_t lo64 = (uint64_t)blockIdx.x * per;
    uint32_t lo = lo64 < total ? (uint32_t)lo64 : total;
    const uint32_t hi = total - lo > per ? lo + per : total;
    if (lo >= hi)
        return;
    // the bucket of entry lo: the last one starting at or before it (an empty
    // bucket shares its successor's start and is passed over)
    int32_t t = find_item(s_start, nb, lo);
    while (lo < hi) {
        const uint32_t end = s_start[t + 1] < hi ? s_start[t + 1] : hi;
        for (int i = threadIdx.x; i < kTilePix; i += kRasterBlock)
            tile[i] = ~0ull;
        __syncthreads();
        for (uint64_t i0 = lo + threadIdx.x; i0 < end; i0 += kUnroll * kRasterBlock) {
            uint64_t k[kUnroll];
            uint32_t l[kUnroll];
            bool ok[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t i = i0 + (uint64_t)u * kRasterBlock;
                ok[u] = i < end;
                k[u] = ok[u] ? ldnt(keys + i) : ~0ull;
                l[u] = ok[u] ? ldnt(lps + i) : 0u;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (ok[u])
                    __hip_atomic_fetch_min(&tile[l[u]], k[u], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        const uint32_t x0 = ((uint32_t)t % (uint32_t)ntx) << kTileShift;
        const uint32_t y0 = ((uint32_t)t / (uint32_t)ntx) << kTileShift;
        // the flush: all of the thread's early-out reads first, then its
        // atomics (framebuffer words only decrease, so a value read early is
        // still an upper bound when the atomic runs)
        constexpr int kFlush = kTilePix / kRasterBlock;
        uint64_t v[kFlush], cur[kFlush];
#pragma unroll
        for (int f = 0; f < kFlush; ++f) {
            const uint32_t l = threadIdx.x + f * kRasterBlock;
            v[f] = tile[l];
            cur[f] = 0ull;
            if (v[f] != ~0ull)   // a fragment in range landed here: the pixel is on screen
                cur[f] = __hip_atomic_load(fb + (uint64_t)(y0 + (l >> kTileShift)) *
                                                    (uint32_t)width +
                                               x0 + (l & (kTileSide - 1)),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int f = 0; f < kFlush; ++f) {
            const uint32_t l = threadIdx.x + f * kRasterBlock;
            if (v[f] < cur[f])
                __hip_atomic_fetch_min(fb + (uint64_t)(y0 + (l >> kTileShift)) *
                                                (uint32_t)width +
                                           x0 + (l & (kTileSide - 1)),
                                       v[f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        lo = end;
        ++t;
        while (t < nb && s_start[t + 1] <= lo)   // empty buckets
            ++t;
        __syncthreads();   // the tile is read before the next run clears it
    }
}

// Pass E: splat accumulation of one chunk of a bucket (section 2.2), from
// the bucket's keys; fb holds the finished depth pass.
template <bool PW>
__global__ void __launch_bounds__(kAccumBlock) k_sort_accum(const uint64_t *__restrict__ keys,
                                                            const uint16_t *__restrict__ lps,
                                                            const uint32_t *__restrict__ bstart,
                                                            const uint32_t *__restrict__ bchunk,
                                                            Proj P, uint32_t eps_num,
                                                            uint32_t eps_den,
                                                            const uint64_t *__restrict__ fb,
                                                            uint64_t *__restrict__ acc,
                                                            int32_t ntx, int32_t nb,
                                                            uint32_t chunk, int32_t width,
                                                            int32_t height)
{
    __shared__ uint64_t qmin[kTilePix];
    __shared__ uint64_t sums[2 * kTilePix];
    int32_t t;
    uint32_t lo, hi;
    chunk_of(bstart, bchunk, nb, chunk, blockIdx.x, t, lo, hi);
    if (lo >= hi)
        return;
    const uint32_t x0 = ((uint32_t)t % (uint32_t)ntx) << kTileShift;
    const uint32_t y0 = ((uint32_t)t / (uint32_t)ntx) << kTileShift;
    for (int l = threadIdx.x; l < kTilePix; l += blockDim.x) {
        const uint32_t x = x0 + (l & (kTileSide - 1)), y = y0 + (l >> kTileShift);
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
            const bool in = i < hi;
            k[u] = in ? ldnt(keys + i) : ~0ull;
            l[u] = in ? ldnt(lps + i) : 0u;
            ok[u] = k[u] != ~0ull;   // in range (the key ~0 marks a depth-culled point)
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            ok[u] = in_window_live<PW>(P, eps_num, eps_den, k[u] >> 24, qmin[l[u]], ok[u]);
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
        if (a1 != 0ull) {   // count > 0, so the pixel is on screen
            uint64_t *dst = acc + 2 * ((uint64_t)(y0 + (l >> kTileShift)) * (uint32_t)width +
                                       x0 + (l & (kTileSide - 1)));
            __hip_atomic_fetch_add(dst, sums[2 * l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(dst + 1, a1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <bool VEC, bool PW>
void launch_count_scatter(const Pts &p, const Proj &P, const Layout &L, uint32_t *ccounts,
                          uint32_t *btotal, uint32_t *bstart, uint32_t *bchunk, uint64_t *keys,
                          uint16_t *lps, hipStream_t s)
{
    hipLaunchKernelGGL((k_sort_count<VEC>), dim3(L.groups), dim3(kCountBlock), 0, s, p, P,
                       ccounts, L.ntx, L.nb, L.per_wg);
    hipLaunchKernelGGL(k_sort_prefix, dim3((L.nb + kPrefixCols - 1) / kPrefixCols),
                       dim3(kPrefixCols * kPrefixSegs), 0, s, ccounts, L.groups, L.nb, btotal);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kScanThreads), 0, s, btotal, bstart, bchunk,
                       L.nb, L.chunk);
    hipLaunchKernelGGL((k_sort_scatter<VEC, PW>), dim3(L.groups), dim3(kScBlock), 0, s, p, P,
                       ccounts, bstart, keys, lps, L.ntx, L.nb, L.per_wg);
}

// Passes A to C: leaves the buckets (keys, lps), their starts and the work
// list of E.
hipError_t sort_passes(const Pts &p, const Proj &P, const Layout &L, char *ws, bool vec,
                       hipStream_t s)
{
    Range r("rz sort: count, offsets, scatter");
    uint32_t *ccounts = (uint32_t *)(ws + L.ccounts);
    uint32_t *btotal = (uint32_t *)(ws + L.btotal);
    uint32_t *bstart = (uint32_t *)(ws + L.bstart);
    uint32_t *bchunk = (uint32_t *)(ws + L.bchunk);
    uint64_t *keys = (uint64_t *)(ws + L.keys);
    uint16_t *lps = (uint16_t *)(ws + L.lps);
    const bool pw = P.nr != 0;
    if (vec && pw)
        launch_count_scatter<true, true>(p, P, L, ccounts, btotal, bstart, bchunk, keys, lps, s);
    else if (vec)
        launch_count_scatter<true, false>(p, P, L, ccounts, btotal, bstart, bchunk, keys, lps, s);
    else if (pw)
        launch_count_scatter<false, true>(p, P, L, ccounts, btotal, bstart, bchunk, keys, lps, s);
    else
        launch_count_scatter<false, false>(p, P, L, ccounts, btotal, bstart, bchunk, keys, lps,
                                           s);
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
    if (L.nb > kMaxBuckets)
        return -1;
    return (int64_t)L.bytes;
}

int rasterize_sorted(const rz_points *pts, const rz_view *view, const rz_depth_map *depth,
                     const rz_hq_params *hq, uint32_t background, uint64_t *fb, uint64_t *acc,
                     uint32_t *img, uint32_t *status, void *workspace, int64_t workspace_bytes,
                     uint32_t flags, void *stream)
{
    Range range("rasterize_sorted");
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
    if (L.nb > kMaxBuckets)
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
        const uint32_t *bstart = (const uint32_t *)(ws + L.bstart);
        const uint32_t *bchunk = (const uint32_t *)(ws + L.bchunk);
        const dim3 grid((uint32_t)L.chunks_max);   // workgroups past the last item exit
        if (e == hipSuccess) {
            Range r("rz sort: bucket minima");
            hipLaunchKernelGGL(k_sort_raster, dim3(kRasterGroups), dim3(kRasterBlock), 0, s, keys,
                               lps, bstart, fb, L.ntx, L.nb, P.width);
            e = hipGetLastError();
        }
        if (e == hipSuccess && hq) {
            Range r("rz sort: bucket sums");
            if (P.nr)
                hipLaunchKernelGGL((k_sort_accum<true>), grid, dim3(kAccumBlock), 0, s, keys,
                                   lps, bstart, bchunk, P, num, den, fb, acc, L.ntx, L.nb,
                                   L.chunk, P.width, P.height);
            else
                hipLaunchKernelGGL((k_sort_accum<false>), grid, dim3(kAccumBlock), 0, s, keys,
                                   lps, bstart, bchunk, P, num, den, fb, acc, L.ntx, L.nb,
                                   L.chunk, P.width, P.height);
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
