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
 *     clip = vp * (x, y, z, 1).  Pixel positions are computed in float32
 *     from (float)vp: ndc = clip.xy / clip.w, window = (ndc + 1) * size / 2,
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
#define RZ_EOVERFLOW (-4)    /* a splat count exceeded its exact range    */
#define RZ_EBUDGET (-5)      /* request does not fit the memory budget    */
#define RZ_ESTATE (-6)       /* object used in the wrong state            */

/* ---- flags -------------------------------------------------------------- */
/* Skip the resolve step: fb (and acc) keep the raw keys (sums) so that they
   can be read back; img is not written and may be NULL. */
#define RZ_KEEP_KEYS 1u

/* bit set in *status by the splat resolve when a pixel's count exceeded the
   exactly representable range (see rasterize_hq_splat) */
#define RZ_STATUS_HQ_OVERFLOW 1u

/* ---- depth maps (section 2.1) ----------------------------------------- */
/* o = near, s = (2^40 - 1) / (far - near): [near, far) spread uniformly
   over the 40-bit range. */
#define RZ_DEPTH_LINEAR 0
/* o = 0, s = scale: the paper's example is scale = 1000 for millimetre
   precision in a scene given in metres.  Requires far * scale <= 2^40 - 1. */
#define RZ_DEPTH_SCALE 1

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
    int32_t kind;          /* RZ_DEPTH_LINEAR or RZ_DEPTH_SCALE           */
    double scale;          /* used by RZ_DEPTH_SCALE only; > 0            */
} rz_depth_map;

typedef struct rz_hq_params {
    /* eps = eps_num / eps_den (section 2.2 uses 1/100).  A fragment of depth
       q joins pixel p iff eps_den * (q - qmin) <= eps_num * (qmin + z0),
       qmin = nearest depth of p, z0 = floor(o * s) (so that q + z0 is
       proportional to d).  1 <= eps_den <= 2^20, eps_num <= 2^20, and
       eps_num * (2^40 + z0) < 2^63 (else RZ_EDEPTHRANGE). */
    uint32_t eps_num;
    uint32_t eps_den;
} rz_hq_params;

/*
 * Rasterization via atomicMin (section 2.1), then resolve.
 *   pts      points (device planes).
 *   view     camera and framebuffer size (host struct, read during the call).
 *   depth    depth map (host struct).
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
 *   status   device uint32 or NULL.  The resolve ORs RZ_STATUS_HQ_OVERFLOW
 *            into it if any pixel's count left the exact range (that pixel's
 *            colour is then unspecified).  It cannot happen when n <= 16843009.
 * Errors: RZ_EINVAL, RZ_EDEPTHRANGE, RZ_EHIP.
 */
int rasterize_hq_splat(const rz_points *pts, const rz_view *view,
                       const rz_depth_map *depth, const rz_hq_params *hq,
                       uint32_t background, uint64_t *fb, uint64_t *acc,
                       uint32_t *img, uint32_t *status, uint32_t flags,
                       void *stream);

/*
 * Building blocks (section 2.1 resolve, section 2.2 third pass).
 * rz_clear: fb[p] = 0xffffffffff000000 | (background & 0xffffff) for
 *   p < npix, and acc[0 .. 2*npix) = 0 when acc is not NULL.
 * rz_resolve_min: img[p] = fb[p] & 0xffffff, then fb[p] = cleared value.
 * rz_resolve_hq: img from acc as in rasterize_hq_splat, then fb and acc
 *   cleared; status as above (may be NULL).
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
 *   bin        1: merge fragments of a workgroup in an LDS tile first (when
 *              they fall in a small screen rectangle); 0: direct atomics.
 */
typedef struct rz_launch {
    int32_t block;
    int32_t ppt;
    int32_t early_out;
    int32_t xcd_remap;
    int32_t bin;
} rz_launch;
int rz_set_launch(const rz_launch *launch);   /* RZ_EINVAL if out of range */
int rz_get_launch(rz_launch *launch);

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
