/*
 * rz.h -- C ABI of the MI355X (gfx950) point-cloud rasterizer.
 *
 * The method is that of Schuetz & Wimmer, "Rendering Point Clouds with
 * Compute Shaders" (arXiv 1908.02681):
 *   - section 2.1 (rasterization via atomicMin): every point becomes a 64-bit
 *     key, its depth as a 40-bit integer in the upper bits and its 24-bit RGB
 *     colour in the lower bits; a 64-bit atomic minimum keeps the closest
 *     fragment of every pixel; a per-pixel pass copies the colour bits to the
 *     image and clears the framebuffer to 0xffffffffff000000 | background;
 *   - section 1 and section 2.1: the depth is computed in double precision
 *     and mapped linearly to the 40-bit integer (uniform precision, or the
 *     millimetre scale of the paper's example);
 *   - section 2.2 (high-quality splatting): after the depth pass, a second
 *     pass sums R, G, B and a count over the fragments whose linear depth is
 *     at most eps (1%) larger than their pixel's nearest depth; a third pass
 *     divides.
 *
 * Conventions shared by every entry point:
 *   - Pointers named "device" must point to device memory of the current HIP
 *     device (e.g. from hipMalloc or a torch CUDA tensor).  The caller owns
 *     every buffer; the plain calls allocate nothing.
 *   - Points are four planes (struct of arrays) of n elements: x, y, z
 *     (float32) and rgb (uint32, R | G << 8 | B << 16, bits 24..31 ignored).
 *   - Framebuffers are row-major, width * height elements, row 0 at the
 *     bottom of the image (OpenGL window convention).
 *   - The view-projection matrix vp is row-major and maps column vectors:
 *     clip = vp * (x, y, z, 1), each row evaluated as fused multiply-adds
 *     (one rounding each) in the order fma(r2, z, fma(r1, y, fma(r0, x, r3))).
 *     Pixel positions are computed in float32
 *     from (float)vp: ndc = clip.xy * (1 / clip.w) with the reciprocal
 *     rounded once, window = fma(ndc, size / 2, size / 2),
 *     pixel = floor(window) in [0, size).  The depth d is row 3 of vp in
 *     double precision (the clip w: linear view depth for a perspective
 *     matrix).  A fragment is kept iff clip.w > 0, the pixel is inside the
 *     framebuffer and near <= d < far.
 *   - Integer depth q = min(floor((d - o) * s), 2^40 - 2) with o, s from
 *     rz_depth_map; key = q << 24 | (rgb & 0xffffff).
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream) and return after enqueueing; argument errors are reported
 *     before anything is enqueued.  Calls are reentrant.
 *   - Return value: RZ_OK (0) or a negative RZ_E* code; rz_error_string()
 *     names it.  No C++ exception crosses this interface.
 *   - Every call and every pass it enqueues opens a roctx range (for a
 *     profiler's marker trace); the environment variable RZ_ROCTX=0, read
 *     once per process, turns them off.
 */
#ifndef RZ_H
#define RZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define RZ_OK 0
#define RZ_EINVAL (-1)       /* null pointer, bad size or flag            */
#define RZ_EDEPTHRANGE (-2)  /* depth map cannot hold [near, far) in 40 bits,
                                or the eps test could overflow 64 bits    */
#define RZ_EHIP (-3)         /* a HIP runtime call failed; see
                                rz_last_hip_error()                       */
#define RZ_EOVERFLOW (-4)    /* a splat count exceeded its exact range (the
                                error of a served request; the asynchronous
                                calls report it through their status word) */
#define RZ_EBUDGET (-5)      /* request does not fit the memory budget    */
#define RZ_ESTATE (-6)       /* object used in the wrong state            */
#define RZ_EIO (-7)          /* a file could not be written (autotune cache) */

/* ---- flags -------------------------------------------------------------- */
/* Skip the resolve step: fb (and acc) keep the raw keys (sums) so that they
   can be read back; img is not written and may be NULL. */
#define RZ_KEEP_KEYS 1u

/* bit set in *status by the splat resolve when a pixel's count exceeded the
   exactly representable range (see rasterize_hq_splat).  Every call that
   resolves splat sums requires a status word, so that such a result can
   never pass unnoticed. */
#define RZ_STATUS_HQ_OVERFLOW 1u

/* ---- depth maps (section 2.1) ----------------------------------------- */
/* o = near, s = (2^40 - 1) / (far - near): [near, far) spread uniformly
   over the 40-bit range. */
#define RZ_DEPTH_LINEAR 0
/* o = 0, s = scale: the paper's example is scale = 1000 for millimetre
   precision in a scene given in metres.  Requires far * scale <= 2^40 - 1. */
#define RZ_DEPTH_SCALE 1
/* Sub-ranges with their own precision (section 2.1, e.g. nm up to 10 m, um
   up to 10 km, mm beyond).  Range k starts at range_start[k] (strictly
   increasing, range_start[0] <= near) with range_scale[k] > 0 values per
   unit of depth:
     base[0] = 0,  base[k+1] = base[k] + floor((start[k+1] - start[k]) * scale[k]) + 1,
     q = base[k] + floor((d - start[k]) * scale[k])  for start[k] <= d < start[k+1],
   which never decreases with d.  Requires the last range to reach far
   within 2^40 - 1 values (else RZ_EDEPTHRANGE).  The splatting window then
   compares linear depths: den * (d(q) - d(qmin)) <= num * d(qmin) in double,
   with d(q) = start[k] + (q - base[k]) * (1 / scale[k]). */
#define RZ_DEPTH_PIECEWISE 2
#define RZ_MAX_RANGES 8
/* Encodings of a graphics depth buffer, for comparing precision with the
   40-bit integers (sections 1 and 2.1); depth pass only (rasterize_atomicmin
   and rasterize_points without hq; any other call returns RZ_EINVAL):
   RZ_DEPTH_GL24: z_ndc = clip.z * (1 / clip.w) in single precision (row 2 of the
   float matrix, same operation order as the other rows), z_win =
   (z_ndc + 1) * 0.5, depth = round(z_win * (2^24 - 1)) (ties up) as a 24-bit
   integer; fragments with z_ndc outside [-1, 1] are discarded.
   RZ_DEPTH_F32REV: z_rev = (float)near / clip.w in single precision (1 at
   the near plane, towards 0 far away), depth = 2^32 - 1 - (bit pattern of
   z_rev), so that nearer stays smaller.
   Both keep the [near, far) cull on the double-precision depth. */
#define RZ_DEPTH_GL24 3
#define RZ_DEPTH_F32REV 4

typedef struct rz_points {
    const float *x;        /* device, n floats */
    const float *y;        /* device, n floats */
    const float *z;        /* device, n floats */
    const uint32_t *rgb;   /* device, n words  */
    int64_t n;             /* 0 <= n < 2^32 - 2^9 */
} rz_points;

typedef struct rz_view {
    double vp[16];         /* row-major view-projection, column vectors   */
    double near_;          /* 0 < near < far, finite                      */
    double far_;
    int32_t width;         /* 1 <= width, height <= 32768                 */
    int32_t height;
} rz_view;

typedef struct rz_depth_map {
    int32_t kind;          /* RZ_DEPTH_LINEAR, _SCALE or _PIECEWISE       */
    double scale;          /* used by RZ_DEPTH_SCALE only; > 0            */
    int32_t nranges;       /* RZ_DEPTH_PIECEWISE: 1 .. RZ_MAX_RANGES      */
    double range_start[RZ_MAX_RANGES];
    double range_scale[RZ_MAX_RANGES];
} rz_depth_map;

typedef struct rz_hq_params {
    /* eps = eps_num / eps_den (section 2.2 uses 1/100).  A fragment of depth
       q joins pixel p iff eps_den * (q - qmin) <= eps_num * (qmin + z0),
       qmin = nearest depth of p, z0 = floor(o * s) (so that q + z0 is
       proportional to d); for RZ_DEPTH_PIECEWISE see there.
       1 <= eps_den <= 2^20, eps_num <= 2^20, and eps_num * (2^40 + z0) <
       2^63 (else RZ_EDEPTHRANGE). */
    uint32_t eps_num;
    uint32_t eps_den;
} rz_hq_params;

/*
 * Rasterization via atomicMin (section 2.1), then resolve.
 *   pts      points (device planes).
 *   view     camera and framebuffer size (host struct, read during the call).
 *   depth    depth map (host struct); any kind, RZ_DEPTH_GL24 and
 *            RZ_DEPTH_F32REV included.
 *   background  24-bit colour of empty pixels (upper 8 bits ignored).
 *   fb       device, width*height uint64.  Precondition: in the cleared state
 *            0xffffffffff000000 | background (rz_clear, or a previous resolve).
 *            After the call (without RZ_KEEP_KEYS) it is in that state again.
 *   img      device, width*height uint32, receives R | G << 8 | B << 16.
 *   flags    0 or RZ_KEEP_KEYS.
 *   stream   hipStream_t.
 * Errors: RZ_EINVAL, RZ_EDEPTHRANGE, RZ_EHIP.
 */
int rasterize_atomicmin(const rz_points *pts, const rz_view *view,
                        const rz_depth_map *depth, uint32_t background,
                        uint64_t *fb, uint32_t *img, uint32_t flags,
                        void *stream);

/*
 * High-quality splatting (section 2.2): depth pass (as above), accumulate
 * pass, normalise pass.
 *   hq       eps (host struct); NULL means 1/100.
 *   fb       as for rasterize_atomicmin (cleared on entry and on exit).
 *   acc      device, 2*width*height uint64, all zero on entry; zero again on
 *            exit (without RZ_KEEP_KEYS).  Per pixel p:
 *              acc[2p]   = sum R + (sum G << 32)
 *              acc[2p+1] = sum B + (count << 32)
 *            exact while count <= 16843009 = floor((2^32 - 1) / 255).
 *   img      device, width*height uint32: per channel
 *            (2 * sum + count) / (2 * count) (rounded half up), or the
 *            background where count = 0.
 *   status   device uint32, required unless RZ_KEEP_KEYS (then unused and
 *            may be NULL).  The resolve ORs RZ_STATUS_HQ_OVERFLOW into it if
 *            any pixel's count left the exact range (that pixel's colour is
 *            then unspecified); the caller zeroes it and reads it after the
 *            stream has reached the call.  It cannot happen when
 *            n <= 16843009.
 * Errors: RZ_EINVAL (also status NULL without RZ_KEEP_KEYS),
 * RZ_EDEPTHRANGE, RZ_EHIP.
 */
int rasterize_hq_splat(const rz_points *pts, const rz_view *view,
                       const rz_depth_map *depth, const rz_hq_params *hq,
                       uint32_t background, uint64_t *fb, uint64_t *acc,
                       uint32_t *img, uint32_t *status, uint32_t flags,
                       void *stream);

/*
 * Screen-sorted rendering, for clouds in no particular order (the paper
 * notes that shuffled points make the atomicMin method slower, section 3).
 * Same results as rasterize_atomicmin (hq == NULL) or rasterize_hq_splat
 * (hq != NULL), bit for bit, computed differently: the fragments are first
 * sorted into buckets per 64x64 screen tile (counted, then scattered once,
 * each workgroup sorting its share by bucket in LDS so that its writes are
 * runs), then each tile is reduced in LDS and merged into fb (and acc) with
 * one coalesced atomic per pixel; the splat sums are taken straight from the
 * buckets, without a second projection.
 *   workspace    device memory of at least
 *                rz_sorted_workspace_bytes(pts->n, width, height) bytes
 *                (about 10 bytes per point), owned by the caller, 256-byte
 *                aligned; its contents on entry do not matter.  May be NULL
 *                when pts->n == 0.
 *   Limits: ceil(width / 64) * ceil(height / 64) <= 4096 (e.g. 4096x4096
 *   or 7680x2160), else RZ_EINVAL; rz_sorted_workspace_bytes returns -1 for
 *   such a screen or a negative size.  Other arguments and errors as for
 *   the one-view calls (status required with hq unless RZ_KEEP_KEYS).
 */
int64_t rz_sorted_workspace_bytes(int64_t n, int32_t width, int32_t height);
int rasterize_sorted(const rz_points *pts, const rz_view *view,
                     const rz_depth_map *depth, const rz_hq_params *hq,
                     uint32_t background, uint64_t *fb, uint64_t *acc,
                     uint32_t *img, uint32_t *status, void *workspace,
                     int64_t workspace_bytes, uint32_t flags, void *stream);

/*
 * rasterize_sorted without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * hosts that forbid allocation): the workspace is a static device array of
 * RZ_NOALLOC_SCRATCH_BYTES per device, held by the library until the process
 * ends; the call itself allocates nothing (the array's device address is
 * looked up once per device, on the first call there).  The caller still
 * passes fb, acc, img and status as for rasterize_sorted, and gets the same
 * results bit for bit.
 *   Limit: rz_sorted_workspace_bytes(pts->n, width, height) <=
 *   RZ_NOALLOC_SCRATCH_BYTES (at 1920x1080 about 6 million points), else
 *   RZ_EBUDGET before anything is enqueued.
 *   Every call on one device shares that device's array and leaves it
 *   holding its own intermediate data: calls that overlap on one device
 *   (on two streams, or from two threads without ordering) race and give
 *   undefined results.  Calls on one stream, or ordered by the caller, are
 *   safe.
 * Errors: those of rasterize_sorted, RZ_EBUDGET, RZ_EHIP (symbol lookup).
 */
#define RZ_NOALLOC_SCRATCH_BYTES (64u << 20)
int rasterize_sorted_noalloc(const rz_points *pts, const rz_view *view,
                             const rz_depth_map *depth, const rz_hq_params *hq,
                             uint32_t background, uint64_t *fb, uint64_t *acc, uint32_t *img,
                             uint32_t *status, uint32_t flags, void *stream);

/*
 * Points larger than one pixel (the paper relates cost to the number of
 * fragments, section 3), and the depth encodings RZ_DEPTH_GL24 / _F32REV.
 * A point of size k (1 <= k <= 16) is culled by its centre as usual and then
 * covers the pixels px - r .. px - r + k - 1 and py - r .. py - r + k - 1,
 * r = (k - 1) / 2, around its pixel (px, py), clipped to the screen; every
 * covered pixel takes the point's key in the depth pass, and with hq every
 * covered pixel tests the point against its own nearest depth.
 *   hq       NULL: depth pass + resolve as rasterize_atomicmin; else the three
 *            passes of rasterize_hq_splat (depth maps 0-2 only).
 *   Other arguments as for rasterize_atomicmin / rasterize_hq_splat (acc and
 *   status are used only with hq; with hq and without RZ_KEEP_KEYS, status
 *   is required).  point_size 1 with an integer depth map runs the same
 *   kernels as those calls.
 * Errors: RZ_EINVAL (also point_size out of range, hq with a float depth
 * encoding), RZ_EDEPTHRANGE, RZ_EHIP.
 */
int rasterize_points(const rz_points *pts, const rz_view *view,
                     const rz_depth_map *depth, const rz_hq_params *hq,
                     int32_t point_size, uint32_t background, uint64_t *fb,
                     uint64_t *acc, uint32_t *img, uint32_t *status,
                     uint32_t flags, void *stream);

/*
 * Building blocks (section 2.1 resolve, section 2.2 third pass).
 * rz_clear: fb[p] = 0xffffffffff000000 | (background & 0xffffff) for
 *   p < npix, and acc[0 .. 2*npix) = 0 when acc is not NULL.
 * rz_resolve_min: img[p] = fb[p] & 0xffffff, then fb[p] = cleared value.
 * rz_resolve_hq: img from acc as in rasterize_hq_splat, then fb and acc
 *   cleared; status as above (required).
 * All pointers device; npix >= 0.
 */
int rz_clear(uint64_t *fb, uint64_t *acc, int64_t npix, uint32_t background,
             void *stream);
/*
 * Second pass of high-quality splatting alone (section 2.2): fb must hold
 * the finished depth pass of the same points and view (rasterize_atomicmin
 * with RZ_KEEP_KEYS); acc (2*width*height uint64, device) receives the
 * packed sums described at rasterize_hq_splat.  Together with
 * rz_resolve_hq this is the same work as rasterize_hq_splat.
 * Errors: RZ_EINVAL, RZ_EDEPTHRANGE, RZ_EHIP.
 */
int rz_hq_accumulate(const rz_points *pts, const rz_view *view,
                     const rz_depth_map *depth, const rz_hq_params *hq,
                     const uint64_t *fb, uint64_t *acc, void *stream);
int rz_resolve_min(uint64_t *fb, int64_t npix, uint32_t background,
                   uint32_t *img, void *stream);
int rz_resolve_hq(uint64_t *fb, uint64_t *acc, int64_t npix,
                  uint32_t background, uint32_t *img, uint32_t *status,
                  void *stream);

/*
 * Launch shape of the point kernels used by the plain calls above (process
 * wide; set it before the calls that should use it).  It never changes a
 * result: every shape computes the same integer minimum and sums.
 *   block      threads per workgroup: 64, 128, 256 or 512.
 *   ppt        points per thread: 4, 8 or 16.
 *   early_out  1: read the framebuffer and skip atomics that cannot lower it.
 *   xcd_remap  1: give each of the 8 XCDs one contiguous eighth of the points.
 *   bin        how fragments are merged before the global atomics:
 *              0: none (direct atomics); 1: one LDS tile per workgroup (when
 *              its fragments fall in a small screen rectangle); 2: one LDS
 *              tile per wave (no workgroup barrier), 8 KiB; 3: the same with
 *              a 2 KiB tile (more waves per SIMD when registers allow them;
 *              a wave whose fragments span more than 256 pixels, 128 when
 *              splatting, takes the direct atomics instead).
 */
typedef struct rz_launch {
    int32_t block;
    int32_t ppt;
    int32_t early_out;
    int32_t xcd_remap;
    int32_t bin;
} rz_launch;
/* Sets the launch shape of both point passes of the one-view calls and the
   server (RZ_EINVAL if out of range); NULL restores the library defaults
   (depth pass 64 threads x 16 points with the 8 KiB per-wave tile, splat
   pass 64 x 8 with the 2 KiB per-wave tile, early-out, no XCD remap).  rz_get_launch reports the depth pass's shape.
   Thread-safe: a call running concurrently launches with either the old
   or the new shape, and both give the same result. */
int rz_set_launch(const rz_launch *launch);
int rz_get_launch(rz_launch *launch);

/* ---- sort-last composition ------------------------------------------ */
/*
 * Combining the passes of disjoint parts of a cloud, each rendered into a
 * full framebuffer (by a device each, or one after the other): the depth
 * pass of the whole is the per-pixel minimum of the parts' depth passes
 * (section 2.1's minimum is associative), and the splat sums of the whole
 * are the sums of the parts' accumulate passes taken against that combined
 * depth pass (section 2.2).  Across devices the same per-pixel operations
 * are a MIN and a SUM reduction of the framebuffers.
 *   rz_merge_min  dst[p] = min(dst[p], src[p]) for p < npix (u64 keys).
 *   rz_merge_sum  dst[2p + k] += src[2p + k] for k = 0, 1 (packed sums as in
 *                 acc; exact while the merged counts stay within the range
 *                 of rasterize_hq_splat).
 * Device pointers, 16-byte aligned; dst and src must not overlap.  Errors:
 * RZ_EINVAL, RZ_EHIP.
 */
int rz_merge_min(uint64_t *dst, const uint64_t *src, int64_t npix, void *stream);
int rz_merge_sum(uint64_t *dst, const uint64_t *src, int64_t npix, void *stream);

/* ---- arithmetic self-check ------------------------------------------- */
/*
 * The perspective divide of section 2.1 needs 1 / w rounded once (the IEEE
 * quotient).  The kernels take it from the hardware reciprocal estimate
 * with one fused Newton-Raphson correction, and fall back to the full IEEE
 * division for denormal w and w >= 2^126.  rz_check_reciprocal runs that
 * same device function over the float bit patterns first_bits ..
 * first_bits + count - 1 and adds to *mismatches (a device counter the
 * caller zeroes) the number of positive w (including +inf) whose result
 * differs in any bit from 1.0f / w.  Patterns of w <= 0 and NaN are not
 * counted (the kernels cull those points).  Zero over all 2^31 positive
 * patterns is what the kernels' bit-exactness relies on; a caller moving
 * the library to another device or compiler can re-run it.  With flags =
 * RZ_CHECK_ESTIMATE_ONLY the corrected estimate is checked without the
 * fallback (it must be exact on [2^-126, 2^126), the range where the
 * kernels use it alone).
 * Errors: RZ_EINVAL (unknown flags, count < 0, first_bits + count > 2^32,
 * mismatches NULL or not 8-byte aligned), RZ_EHIP.
 */
#define RZ_CHECK_ESTIMATE_ONLY 1u
int rz_check_reciprocal(uint32_t first_bits, int64_t count, uint64_t *mismatches, uint32_t flags,
                        void *stream);
/*
 * The same reciprocal as the kernels' perspective divide (section 2.1),
 * applied elementwise: out[i] = 1 / w[i] as the point kernels compute it,
 * for a host to compare with its own IEEE quotients (the self-check above
 * compares on the device, against the device's division).  For w <= 0 and
 * NaN the value is whatever the estimate gives (the kernels cull those
 * points).  w and out are device arrays of n floats; n >= 0.  Errors:
 * RZ_EINVAL (n < 0, NULL arrays with n > 0), RZ_EHIP.
 */
int rz_reciprocal(const float *w, float *out, int64_t n, void *stream);

/* ---- batched multi-view rendering ------------------------------------ */
/*
 * Many views of one resident cloud in one submission.  Views are taken in
 * groups of K: a group's depth passes (section 2.1) read every point once and
 * project it into all K views; the splatting views of the group then share
 * one accumulate pass (section 2.2); one kernel resolves every view.  Each
 * view's fb, acc and img are bit-identical to those of the one-view calls.
 */
#define RZ_MODE_ATOMICMIN 0
#define RZ_MODE_HQ 1

typedef struct rz_batch_view {
    rz_view view;          /* camera and size, as for the one-view calls       */
    rz_depth_map depth;
    int32_t mode;          /* RZ_MODE_ATOMICMIN or RZ_MODE_HQ                 */
    rz_hq_params hq;       /* RZ_MODE_HQ only; eps_den == 0 means 1/100        */
    uint32_t background;
    uint64_t *fb;          /* device, width*height, cleared on entry; cleared
                              again by every run                               */
    uint64_t *acc;         /* device, 2*width*height, zero; RZ_MODE_HQ only    */
    uint32_t *img;         /* device, width*height, written by every run       */
} rz_batch_view;

typedef struct rz_batch_opts {
    int32_t views_per_group;  /* K in 1..8; 0 = 4                              */
    rz_launch launch;         /* launch shape; block == 0 = library default   */
    int32_t use_graph;        /* 1: runs replay one captured hipGraph          */
    uint32_t *status;         /* device: RZ_STATUS_HQ_OVERFLOW, as for
                                 rasterize_hq_splat; required when a view is
                                 RZ_MODE_HQ (else RZ_EINVAL), may be NULL
                                 otherwise                                     */
} rz_batch_opts;

typedef struct rz_batch rz_batch;   /* opaque; owns a small device table and,
                                       once captured, a hipGraph */

/* Validates every view (RZ_EINVAL / RZ_EDEPTHRANGE as the one-view calls),
   uploads the view table (one hipMalloc, synchronous) and returns the
   batch.  The points and the caller's buffers must outlive the batch.
   1 <= nviews <= 4096.  opts may be NULL (defaults, no graph). */
int rz_batch_plan(const rz_points *pts, const rz_batch_view *views,
                  int32_t nviews, const rz_batch_opts *opts, rz_batch **out);
/* Records the batch's kernels into a hipGraph (on an internal stream) and
   instantiates it; later runs replay it on the caller's stream. */
int rz_batch_capture(rz_batch *b);
/* Renders every view, asynchronously on `stream`. */
int rz_batch_run(rz_batch *b, void *stream);
/* Times the batch under candidate launch shapes and group sizes (reps runs
   each, median), keeps the fastest whose images hash to the same value as
   the first candidate's, and re-captures if the batch had a graph.  Runs
   synchronously on `stream`.  chosen may be NULL.  Candidates include the
   one-view calls' pair of shapes, one for the depth passes and another for
   the accumulate passes; opts.launch then reports the depth passes' shape. */
int rz_batch_autotune(rz_batch *b, void *stream, int32_t reps, rz_batch_opts *chosen,
                      float *best_ms);
/* Current options of the batch. */
int rz_batch_get_opts(const rz_batch *b, rz_batch_opts *opts);
/* Frees the table and the graph (waits for nothing: the caller must not
   destroy a batch whose run is still in flight). */
int rz_batch_destroy(rz_batch *b);

/* ---- autotune cache ----------------------------------------------------- */
/* The batch autotuner's choices persist in a text file, one line per key,
   so that a later process with a batch of the same class skips the search.
   Host-only calls (no device work) except rz_batch_autotune_cached. */
typedef struct rz_tune_entry {
    int32_t views_per_group;  /* K, 1..8                                     */
    rz_launch depth;          /* launch shape of the depth passes            */
    rz_launch accum;          /* launch shape of the accumulate passes       */
    float ms;                 /* the batch's time when the entry was chosen   */
} rz_tune_entry;

/* Point order class of HOST arrays x, y, z (n points): windows of up to 4096
   consecutive points at the start, middle and end of the arrays; a window is
   ordered when the median distance between consecutive finite points is at
   most 1/16 of its bounding-box diagonal (Morton or scan order), and the
   majority of windows with at least 16 such pairs decides.  Returns 0
   (ordered), 1 (shuffled, also when no window has 16 pairs) or RZ_EINVAL.
   The batch engine samples its device points the same way (section 3 of the
   paper: point order changes the atomic method's speed). */
int rz_order_class_host(const float *x, const float *y, const float *z, int64_t n);

/* key: six space-separated words without spaces inside, as built by
   rz_batch_autotune_cached: "<arch> n<log2 points> px<log2 pixels>
   v<views> hq<splatting views in eighths> <ordered|shuffled>".  Lookup
   returns 1 and fills *out when the file holds a valid line for key (the
   last one wins), 0 when it holds none or does not exist, RZ_EINVAL for a
   NULL argument or a malformed key.  Lines that do not parse are ignored. */
int rz_tune_cache_lookup(const char *path, const char *key, rz_tune_entry *out);
/* Replaces key's line (or adds it) and rewrites the file through a private
   temporary file and a rename, so that a reader never sees a torn file;
   lines that do not parse are dropped.  Writers in one process are
   serialised; between processes the last rename wins.  RZ_EINVAL for a bad
   key or an entry out of range, RZ_EIO when the file cannot be written. */
int rz_tune_cache_store(const char *path, const char *key, const rz_tune_entry *entry);

/* rz_batch_autotune through the cache at cache_path.  The key is built from
   the current device's architecture, the batch's point count and total
   pixels (log2, rounded), its view count, its share of splatting views and
   the order class of its points (three 4096-point windows copied to the
   host).  On a hit the cached options are first checked against the
   library-default options: one run of each, and the image checksums must
   agree (else the full search runs); they are then timed (reps runs, median)
   and applied, and *hit = 1.  On a miss the full search runs and its choice
   is stored (*hit = 0); RZ_EIO then means the batch is tuned but the file
   could not be written.  key_out (may be NULL) receives the key, at most
   key_len bytes with the terminating zero.  Synchronous on `stream`. */
int rz_batch_autotune_cached(rz_batch *b, void *stream, int32_t reps, const char *cache_path,
                             rz_batch_opts *chosen, float *best_ms, int32_t *hit,
                             char *key_out, int32_t key_len);

/* ---- serving: continuous batching of render requests ----------------- */
/*
 * A render server keeps point clouds resident and runs requests (one view of
 * one cloud, either method) as they arrive.  A scheduler thread admits
 * queued requests in arrival order whenever the framebuffer memory they need
 * (fb, plus acc for splatting) fits the server's device budget and an
 * in-flight slot is free, and spreads admitted requests over several HIP
 * streams so that their kernels overlap on the device.  A request's image is
 * bit-identical to the one-view call's, whatever else runs beside it.
 */
#define RZ_REQ_QUEUED 0
#define RZ_REQ_RUNNING 1
#define RZ_REQ_DONE 2
#define RZ_REQ_FAILED 3

/* rz_request.flags: the scheduler fails this request on purpose, as if its
   launch had failed (host-side fault injection for tests of error
   isolation; the device never sees the request). */
#define RZ_REQ_INJECT_FAILURE 1u

typedef struct rz_server_opts {
    uint64_t budget_bytes;   /* device memory for framebuffers; allocated once
                                at creation (>= 1 MiB)                         */
    int32_t streams;         /* HIP streams, 1..16; 0 = 4                     */
    int32_t max_inflight;    /* admitted and unfinished requests; 0 = 4*streams */
    int32_t dry_run;         /* 1: no device work at all; a request "runs" for
                                dry_run_us on the host (tests of admission and
                                error handling without a GPU)                  */
    int32_t dry_run_us;
    int64_t work_cap;        /* > 0: the head of the queue is admitted only while
                                the work in flight plus its own stays within
                                work_cap, or when nothing is in flight; a
                                request's work is its cloud's point count, twice
                                for splatting (two passes over the points).
                                Large requests then run (nearly) alone while
                                small ones still overlap them.  0: no limit.   */
    int32_t merge_views;     /* > 1: when a request is admitted, up to
                                merge_views - 1 more queued requests of the same
                                cloud (among the next 32 in the queue) that can
                                be admitted at once join it, and the group runs
                                as one multi-view launch: each chunk of points
                                is read once for all of its views (as a batch
                                does).  Requests of other clouds are never
                                merged; the results are the same bits as one
                                request at a time.  0 or 1: no merging; at most
                                8.                                             */
    int32_t pad;
    int64_t exclusive_work;  /* > 0: a request whose work (as for work_cap) is
                                at least exclusive_work runs alone: it is
                                admitted only when nothing is in flight, and
                                nothing else is admitted until it finishes
                                (requests behind it wait, in order).  Large
                                requests then keep the whole device, as in a
                                one-at-a-time loop, while small ones overlap
                                each other.  0: no such rule.                  */
} rz_server_opts;

typedef struct rz_request {
    int32_t cloud;           /* id returned by rz_server_add_cloud             */
    int32_t mode;            /* RZ_MODE_ATOMICMIN or RZ_MODE_HQ                */
    rz_view view;
    rz_depth_map depth;
    rz_hq_params hq;         /* RZ_MODE_HQ; eps_den == 0 means 1/100           */
    uint32_t background;
    uint32_t flags;          /* 0 or RZ_REQ_INJECT_FAILURE                     */
    uint32_t *img;           /* device, width*height, caller-owned; written by
                                the time the request is RZ_REQ_DONE            */
    void *after;             /* hipStream_t or NULL.  Not NULL: the request's
                                device work starts only after the work the
                                caller had queued on this stream when it
                                submitted (an event recorded at submission),
                                e.g. the fill of img or the upload of the
                                cloud.  NULL: the caller must have finished
                                such work (e.g. synchronised) before
                                submitting.                                    */
} rz_request;

typedef struct rz_request_status {
    int32_t state;           /* RZ_REQ_*                                      */
    int32_t error;           /* RZ_OK, or the RZ_E* code of a failed request:
                                RZ_EHIP (launch failed) or RZ_EOVERFLOW (a
                                splat count left the exact range; the image
                                was written but some colours are unspecified) */
    uint32_t hq_status;      /* RZ_STATUS_HQ_OVERFLOW bits (RZ_MODE_HQ)        */
    uint32_t stream;         /* stream index the request ran on               */
    int32_t group;           /* requests in its launch: 1 alone, more when it
                                was merged (rz_server_opts.merge_views)        */
    int32_t pad;
    double t_submit_us;      /* host steady clock, microseconds since the
                                server was created                            */
    double t_admit_us;
    double t_done_us;        /* when its device work had finished (the host
                                function after it ran), or when it failed    */
} rz_request_status;

typedef struct rz_server_stats {
    uint64_t submitted, completed, failed;
    uint64_t peak_bytes;     /* largest framebuffer memory in use at once     */
    int32_t peak_inflight;
    int32_t queued;          /* waiting for admission now                     */
    int32_t inflight;        /* admitted and unfinished now                   */
    int32_t pad;
    uint64_t merged_launches;  /* multi-view launches of two or more requests  */
    uint64_t merged_requests;  /* requests that ran in such a launch           */
    uint64_t chained_requests; /* requests admitted behind a running request on
                                  its stream because the work cap or an
                                  exclusive request held them back: they start
                                  when it ends, without waiting for the
                                  scheduler                                    */
} rz_server_stats;

typedef struct rz_server rz_server;

/* Creates the server: one device allocation of budget_bytes (none with
   dry_run), the streams, and the scheduler thread. */
int rz_server_create(const rz_server_opts *opts, rz_server **out);
/* Registers a resident cloud (device planes, caller-owned, must outlive the
   server).  Ids are 0, 1, 2, ... */
int rz_server_add_cloud(rz_server *s, const rz_points *pts, int32_t *id);
/* Queues a request; returns at once with a ticket.  RZ_EBUDGET if the
   request could never fit the budget; RZ_EINVAL / RZ_EDEPTHRANGE as the
   one-view calls.  Thread-safe. */
int rz_server_submit(rz_server *s, const rz_request *req, uint64_t *ticket);
/* State of a ticket (non-blocking).  A finished ticket is forgotten after
   it has been reported once as RZ_REQ_DONE or RZ_REQ_FAILED. */
int rz_server_poll(rz_server *s, uint64_t ticket, rz_request_status *st);
/* Waits until every submitted request has finished (or timeout_s passed:
   RZ_ESTATE). */
int rz_server_drain(rz_server *s, double timeout_s);
int rz_server_get_stats(rz_server *s, rz_server_stats *st);
/* Waits up to timeout_s seconds for every submitted request to finish, then
   stops the scheduler and frees the streams and the budget.  If requests are
   still queued or running at the timeout it returns RZ_ESTATE and leaves the
   server running (call again later, or drain first). */
int rz_server_destroy(rz_server *s, double timeout_s);

/* Name of an RZ_* return code (static string). */
const char *rz_error_string(int code);
/* hipError_t of the most recent RZ_EHIP failure on the calling thread. */
int rz_last_hip_error(void);
/* Library version: major * 10000 + minor * 100 + patch. */
int rz_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RZ_H */
