/*
 * rz_oracle.c -- plain CPU reference of the compute point rasterizer of
 * Schuetz & Wimmer, "Rendering Point Clouds with Compute Shaders"
 * (arXiv 1908.02681).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  The product path
 * (the HIP library under paper_1908_02681_amd/) never links, loads or calls
 * it, and the two share no source, header, table or helper.
 *
 * Plain, single-threaded and literal: every point is visited in input order,
 * every pixel in row order, one step of the method after the other.  Build
 * with -ffp-contract=off and without fast-math, so that every float and
 * double operation below is one IEEE-754 operation rounded to nearest: the
 * only fused multiply-adds are the explicit fmaf / fma calls (one rounding
 * each, as C99 defines them).
 *
 * What the method computes (section 2.1): each point becomes one fragment,
 * a 64-bit key whose upper 40 bits are an integer depth and whose lower 24
 * bits are the point's RGB colour; the framebuffer keeps, per pixel, the
 * smallest key (atomicMin).  A second per-pixel pass copies the colour bits
 * to the image and resets the framebuffer to depth all-ones plus the
 * background colour.  The result is a plain definition: fb[p] is the minimum
 * over the keys of all fragments that fall into pixel p, whatever their
 * order.  High-quality splatting (section 2.2) adds a pass that sums the
 * colours and counts the fragments whose linear depth is within a factor
 * (1 + eps) of the pixel's nearest depth, and a pass that divides.
 *
 * Readings of points the paper leaves open (all listed with reasons in the
 * design notes of the repository):
 *  - depth d is the clip-space w of the view-projection (row 3), computed in
 *    double precision; for a perspective matrix it is the linear view depth;
 *  - the matrix-vector products (clip coordinates and the depth) are chains
 *    of fused multiply-adds that start from the translation column and add
 *    the x, y and z terms in that order, as a shader compiler evaluates a
 *    matrix times a point;
 *  - projection to pixels is done in single precision: clip = VPf * p with
 *    VPf = (float)VP, ndc = clip.xy * (1 / clip.w) (the reciprocal correctly
 *    rounded once, as a perspective divide does), window = ndc * (size / 2) +
 *    size / 2 in one fused step (the viewport transform's scale and offset),
 *    pixel = floor(window), half-open [0, size), row 0 at the bottom;
 *  - fragments with w <= 0, outside the window, or with d outside
 *    [near, far) are discarded;
 *  - integer depth q = floor((d - o) * s), clamped to 2^40 - 2 so that a
 *    fragment always beats the cleared value 2^40 - 1;  "linear" maps
 *    [near, far) onto [0, 2^40 - 1) (o = near), "scale" is the paper's
 *    millimetre example (o = 0, s = 1000 for metres);
 *  - colour word = R | G << 8 | B << 16; on equal depth the smaller word wins;
 *  - the eps window is tested exactly in integers:
 *    den * (q - qmin) <= num * (qmin + z0) with z0 = floor(o * s), so that
 *    q + z0 is proportional to d;
 *  - the splat average rounds half up: (2 * sum + count) / (2 * count);
 *  - piecewise map (section 2.1's sub-ranges): range k starts at b[k] with
 *    sb[k] values per unit; q = base[k] + floor((d - b[k]) sb[k]),
 *    base[k+1] = base[k] + floor((b[k+1] - b[k]) sb[k]) + 1;
 *    its eps window compares the linear depths of q and qmin in double:
 *    den * (d(q) - d(qmin)) <= num * d(qmin), d(q) = b[k] + (q - base[k]) / sb[k]
 *    (the reciprocal of sb[k] computed once).
 *
 * Two more depth encodings stand for what a graphics pipeline keeps in its
 * depth buffer, the precision the paper's 40-bit integers are set against
 * (sections 1 and 2.1); they are for the depth pass only:
 *  - "gl24": window depth of the perspective matrix in single precision,
 *    z_ndc = clip.z * (1 / clip.w) (row 2 of the float matrix, same fused
 *    operation order as the other rows), z_win = (z_ndc + 1) / 2, kept as a 24-bit
 *    unsigned normalised integer round(z_win * (2^24 - 1)) (rounding to
 *    nearest, ties up), fragments with z_ndc outside [-1, 1] discarded;
 *  - "f32rev": reversed depth in single precision, z_rev = (float)near /
 *    clip.w (1 at the near plane, falling towards 0 far away), kept as its
 *    32-bit pattern complemented, 2^32 - 1 - bits(z_rev), so that nearer is
 *    smaller like every other key.
 * Both leave the near/far cull on d as for every map.
 *
 * Point size (section 3 on cost per fragment): a point of size k covers the
 * k x k pixels px - r .. px - r + k - 1, py - r .. py - r + k - 1 with
 * r = (k - 1) / 2 around its pixel (px, py), clipped to the screen; the point
 * itself is still culled by its centre.  Every covered pixel gets the same
 * key, and in the splat pass every covered pixel tests its own window.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define RZO_DEPTH_ONES 0xFFFFFFFFFF000000ull /* cleared depth, section 2.1 */
#define RZO_RGB_MASK 0xFFFFFFull
#define RZO_Q_MAX ((double)((1ull << 40) - 2)) /* largest fragment depth   */
#define RZO_Q_RANGE ((double)((1ull << 40) - 1))

enum { RZO_LINEAR = 0, RZO_SCALE = 1, RZO_PIECEWISE = 2, RZO_GL24 = 3, RZO_F32REV = 4 };
#define RZO_MAX_RANGES 8

typedef struct {
    float m[16];       /* view-projection rounded to float, row-major */
    double vp[16];     /* the same in double                          */
    double near_, far_;
    float nearf;       /* near rounded to float (f32rev)              */
    double o, s;       /* q = floor((d - o) * s)                      */
    uint64_t z0;       /* floor(o * s): q + z0 is proportional to d   */
    float fw, fh;      /* framebuffer size as float                   */
    float hw, hh;      /* half of it                                  */
    int32_t w, h;
    /* piecewise map (section 2.1, sub-ranges with their own precision):
       range k starts at depth b[k] with sb[k] values per unit and first
       integer base[k]; it ends where range k + 1 starts */
    int32_t kind, nr;
    double b[RZO_MAX_RANGES], sb[RZO_MAX_RANGES], inv[RZO_MAX_RANGES];
    uint64_t base[RZO_MAX_RANGES + 1];
} rzo_cam;

static int rzo_cam_init(rzo_cam *c, const double *vp, double near_, double far_,
                        int32_t w, int32_t h, int32_t kind, double scale)
{
    int i;
    c->kind = kind;
    c->nr = 0;
    if (w < 1 || h < 1 || !(near_ > 0.0) || !(far_ > near_))
        return -1;
    for (i = 0; i < 16; i++) {
        c->vp[i] = vp[i];
        c->m[i] = (float)vp[i];
    }
    c->near_ = near_;
    c->far_ = far_;
    c->nearf = (float)near_;
    if (kind == RZO_LINEAR) {
        c->o = near_;
        c->s = RZO_Q_RANGE / (far_ - near_);
    } else if (kind == RZO_SCALE) {
        c->o = 0.0;
        c->s = scale;
        if (!(scale > 0.0))
            return -1;
    } else if (kind == RZO_PIECEWISE) {
        c->o = 0.0;        /* the ranges are set by rzo_cam_ranges */
        c->s = 1.0;
    } else if (kind == RZO_GL24 || kind == RZO_F32REV) {
        c->o = 0.0;        /* no linear map: see rzo_fragment */
        c->s = 1.0;
    } else {
        return -1;
    }
    c->z0 = (uint64_t)floor(c->o * c->s);
    c->w = w;
    c->h = h;
    c->fw = (float)w;
    c->fh = (float)h;
    c->hw = 0.5f * c->fw;
    c->hh = 0.5f * c->fh;
    return 0;
}

/*
 * Piecewise map: nr ranges starting at b[0] <= near < b[1] < ..., each with
 * its own number of integer values per unit of depth.  Range k+1 starts one
 * integer above the largest value range k can produce, so q never decreases
 * with d.
 */
static int rzo_cam_ranges(rzo_cam *c, int32_t nr, const double *b, const double *sb)
{
    int k;
    if (nr < 1 || nr > RZO_MAX_RANGES || !(b[0] <= c->near_))
        return -1;
    c->nr = nr;
    c->base[0] = 0;
    for (k = 0; k < nr; k++) {
        if (!(sb[k] > 0.0) || (k > 0 && !(b[k] > b[k - 1])))
            return -1;
        c->b[k] = b[k];
        c->sb[k] = sb[k];
        c->inv[k] = 1.0 / sb[k];
        if (k + 1 < nr)
            c->base[k + 1] = c->base[k] + (uint64_t)floor((b[k + 1] - b[k]) * sb[k]) + 1;
    }
    c->base[nr] = (1ull << 40) - 1;
    return 0;
}

/* Depth -> 40-bit integer depth with the camera's map. */
static uint64_t rzo_quantise(const rzo_cam *c, double d)
{
    double t, tf;
    if (c->kind == RZO_PIECEWISE) {
        int k = 0;
        uint64_t qk;
        while (k + 1 < c->nr && d >= c->b[k + 1])
            k++;
        /* d < b[k+1] and IEEE rounding is monotone, so this never exceeds
           floor((b[k+1] - b[k]) * sb[k]) = base[k+1] - base[k] - 1 */
        t = (d - c->b[k]) * c->sb[k];
        tf = floor(t);
        qk = c->base[k] + (uint64_t)tf;
        return qk > (1ull << 40) - 2 ? (1ull << 40) - 2 : qk;
    }
    t = (d - c->o) * c->s;
    tf = floor(t);
    if (tf > RZO_Q_MAX)
        tf = RZO_Q_MAX;
    return (uint64_t)tf;
}

/* Linear depth of the start of integer depth q under a piecewise map. */
static double rzo_depth_of(const rzo_cam *c, uint64_t q)
{
    int k = 0;
    while (k + 1 < c->nr && q >= c->base[k + 1])
        k++;
    return c->b[k] + (double)(q - c->base[k]) * c->inv[k];
}

/*
 * The fragment of one point (section 2.1): its pixel index and its 40-bit
 * integer depth.  Returns 0 when the point is discarded.
 */
static int rzo_fragment(const rzo_cam *c, float x, float y, float z,
                        int64_t *pix, uint64_t *q)
{
    const float *m = c->m;
    const double *v = c->vp;
    float cx, cy, cw, iw, nx, ny, fx, fy;
    double d;
    int32_t px, py;

    /* clip coordinates in single precision: start from the translation
       column, then add the x, y and z terms, each with one rounding */
    cx = fmaf(m[0], x, m[3]);
    cx = fmaf(m[1], y, cx);
    cx = fmaf(m[2], z, cx);
    cy = fmaf(m[4], x, m[7]);
    cy = fmaf(m[5], y, cy);
    cy = fmaf(m[6], z, cy);
    cw = fmaf(m[12], x, m[15]);
    cw = fmaf(m[13], y, cw);
    cw = fmaf(m[14], z, cw);
    if (!(cw > 0.0f))
        return 0;

    /* perspective divide and viewport */
    iw = 1.0f / cw;
    nx = cx * iw;
    ny = cy * iw;
    fx = fmaf(nx, c->hw, c->hw);
    fy = fmaf(ny, c->hh, c->hh);
    if (!(fx >= 0.0f && fx < c->fw && fy >= 0.0f && fy < c->fh))
        return 0;
    px = (int32_t)fx;
    py = (int32_t)fy;

    /* depth in double precision (section 1, section 2.1), same order */
    d = fma(v[12], (double)x, v[15]);
    d = fma(v[13], (double)y, d);
    d = fma(v[14], (double)z, d);
    if (!(d >= c->near_ && d < c->far_))
        return 0;

    *pix = (int64_t)py * c->w + px;
    if (c->kind == RZO_GL24) {
        /* window depth of the perspective matrix, 24-bit normalised */
        float cz, nz, zw, t;
        cz = fmaf(m[8], x, m[11]);
        cz = fmaf(m[9], y, cz);
        cz = fmaf(m[10], z, cz);
        nz = cz * iw;
        if (!(nz >= -1.0f && nz <= 1.0f))
            return 0;
        zw = (nz + 1.0f) * 0.5f;
        t = zw * 16777215.0f;
        *q = (uint64_t)floor((double)t + 0.5);
        return 1;
    }
    if (c->kind == RZO_F32REV) {
        /* reversed single-precision depth, complemented bit pattern */
        union { float f; uint32_t u; } zr;
        zr.f = c->nearf / cw;
        *q = (uint64_t)(0xFFFFFFFFu - zr.u);
        return 1;
    }
    /* integer part of the scaled depth, kept inside 40 bits */
    *q = rzo_quantise(c, d);
    return 1;
}

/* Pixel range [lo, hi) covered along one axis by a point of size k whose
   centre pixel is c, clipped to [0, size). */
static void rzo_span(int64_t c, int32_t k, int32_t size, int64_t *lo, int64_t *hi)
{
    const int64_t r = (k - 1) / 2;
    *lo = c - r < 0 ? 0 : c - r;
    *hi = c - r + k > size ? size : c - r + k;
}

/* ---------------------------------------------------------------------- */
/* exported entry points (called through ctypes by the tests)             */
/* ---------------------------------------------------------------------- */

/* Depth-map constants (o, s, z0) as the oracle derives them. */
int rzo_depth_constants(const double *vp, double near_, double far_, int32_t w,
                        int32_t h, int32_t kind, double scale, int32_t nr,
                        const double *rb, const double *rs, double *o, double *s,
                        uint64_t *z0)
{
    rzo_cam c;
    if (rzo_cam_init(&c, vp, near_, far_, w, h, kind, scale))
        return -1;
    if (kind == RZO_PIECEWISE && rzo_cam_ranges(&c, nr, rb, rs))
        return -1;
    *o = c.o;
    *s = c.s;
    *z0 = c.z0;
    return 0;
}

/* Per-point fragments: pix[i] = pixel index or -1, q[i] = integer depth. */
int rzo_fragments(const float *x, const float *y, const float *z, int64_t n,
                  const double *vp, double near_, double far_, int32_t w,
                  int32_t h, int32_t kind, double scale, int32_t nr,
                  const double *rb, const double *rs, int64_t *pix, uint64_t *q)
{
    rzo_cam c;
    int64_t i;
    if (rzo_cam_init(&c, vp, near_, far_, w, h, kind, scale))
        return -1;
    if (kind == RZO_PIECEWISE && rzo_cam_ranges(&c, nr, rb, rs))
        return -1;
    for (i = 0; i < n; i++) {
        int64_t p;
        uint64_t qq;
        if (rzo_fragment(&c, x[i], y[i], z[i], &p, &qq)) {
            pix[i] = p;
            q[i] = qq;
        } else {
            pix[i] = -1;
            q[i] = 0;
        }
    }
    return 0;
}

/* Reset a framebuffer: depth all ones, colour = background (section 2.1). */
void rzo_clear(uint64_t *fb, int64_t npix, uint32_t bg)
{
    int64_t p;
    for (p = 0; p < npix; p++)
        fb[p] = RZO_DEPTH_ONES | ((uint64_t)bg & RZO_RGB_MASK);
}

/*
 * Rasterization via atomicMin (section 2.1): depth shifted 24 bits left,
 * colour in the low 24 bits, the smaller key kept.
 */
int rzo_raster_min(const float *x, const float *y, const float *z,
                   const uint32_t *rgb, int64_t n, const double *vp,
                   double near_, double far_, int32_t w, int32_t h,
                   int32_t kind, double scale, int32_t nr, const double *rb,
                   const double *rs, int32_t psize, uint64_t *fb)
{
    rzo_cam c;
    int64_t i;
    if (psize < 1 || rzo_cam_init(&c, vp, near_, far_, w, h, kind, scale))
        return -1;
    if (kind == RZO_PIECEWISE && rzo_cam_ranges(&c, nr, rb, rs))
        return -1;
    for (i = 0; i < n; i++) {
        int64_t p, x0, x1, y0, y1, xx, yy;
        uint64_t q, key;
        if (!rzo_fragment(&c, x[i], y[i], z[i], &p, &q))
            continue;
        key = (q << 24) | ((uint64_t)rgb[i] & RZO_RGB_MASK);
        rzo_span(p % w, psize, w, &x0, &x1);
        rzo_span(p / w, psize, h, &y0, &y1);
        for (yy = y0; yy < y1; yy++)
            for (xx = x0; xx < x1; xx++)
                if (key < fb[yy * w + xx])
                    fb[yy * w + xx] = key;
    }
    return 0;
}

/*
 * Second step of section 2.1: copy the colour bits of every pixel into the
 * image, then clear the framebuffer for the next frame.
 */
void rzo_resolve_min(uint64_t *fb, int64_t npix, uint32_t bg, uint32_t *img)
{
    int64_t p;
    for (p = 0; p < npix; p++) {
        img[p] = (uint32_t)(fb[p] & RZO_RGB_MASK);
        fb[p] = RZO_DEPTH_ONES | ((uint64_t)bg & RZO_RGB_MASK);
    }
}

/*
 * Second pass of high-quality splatting (section 2.2): every fragment whose
 * depth is at most eps larger than the nearest depth of its pixel adds its
 * red, green and blue values and increments the pixel's counter.  sums holds
 * four exact 64-bit totals per pixel: R, G, B, count.
 */
int rzo_hq_accumulate(const float *x, const float *y, const float *z,
                      const uint32_t *rgb, int64_t n, const double *vp,
                      double near_, double far_, int32_t w, int32_t h,
                      int32_t kind, double scale, int32_t nr, const double *rb,
                      const double *rs, int32_t psize, uint32_t eps_num,
                      uint32_t eps_den, const uint64_t *fb, uint64_t *sums)
{
    rzo_cam c;
    int64_t i;
    if (eps_den == 0 || psize < 1 || kind == RZO_GL24 || kind == RZO_F32REV)
        return -1;
    if (rzo_cam_init(&c, vp, near_, far_, w, h, kind, scale))
        return -1;
    if (kind == RZO_PIECEWISE && rzo_cam_ranges(&c, nr, rb, rs))
        return -1;
    for (i = 0; i < n; i++) {
        int64_t p, x0, x1, y0, y1, xx, yy;
        uint64_t q;
        uint32_t col;
        if (!rzo_fragment(&c, x[i], y[i], z[i], &p, &q))
            continue;
        col = rgb[i];
        rzo_span(p % w, psize, w, &x0, &x1);
        rzo_span(p / w, psize, h, &y0, &y1);
        for (yy = y0; yy < y1; yy++) {
            for (xx = x0; xx < x1; xx++) {
                const int64_t pp = yy * w + xx;
                const uint64_t qmin = fb[pp] >> 24;
                if (q < qmin)
                    return -2; /* fb does not hold this cloud's depth pass */
                if (c.kind == RZO_PIECEWISE) {
                    /* q + z0 is not proportional to d here: compare the
                       linear depths the two integers stand for, in double */
                    const double dq = rzo_depth_of(&c, q);
                    const double dm = rzo_depth_of(&c, qmin);
                    const double lhs = (double)eps_den * (dq - dm);
                    const double rhs = (double)eps_num * dm;
                    if (!(lhs <= rhs))
                        continue;
                } else if ((unsigned __int128)eps_den * (q - qmin) >
                           (unsigned __int128)eps_num * ((unsigned __int128)qmin + c.z0)) {
                    continue;   /* exact: 128-bit products cannot overflow */
                }
                sums[4 * pp + 0] += col & 0xFFu;
                sums[4 * pp + 1] += (col >> 8) & 0xFFu;
                sums[4 * pp + 2] += (col >> 16) & 0xFFu;
                sums[4 * pp + 3] += 1;
            }
        }
    }
    return 0;
}

/*
 * Third pass of high-quality splatting (section 2.2): the average colour of
 * the accepted fragments, or the background where none was accepted; then
 * the framebuffer and the sums are cleared.
 */
void rzo_hq_resolve(uint64_t *sums, uint64_t *fb, int64_t npix, uint32_t bg,
                    uint32_t *img)
{
    int64_t p;
    for (p = 0; p < npix; p++) {
        uint64_t cnt = sums[4 * p + 3];
        if (cnt == 0) {
            img[p] = bg & 0xFFFFFFu;
        } else {
            uint64_t r = (2 * sums[4 * p + 0] + cnt) / (2 * cnt);
            uint64_t g = (2 * sums[4 * p + 1] + cnt) / (2 * cnt);
            uint64_t b = (2 * sums[4 * p + 2] + cnt) / (2 * cnt);
            img[p] = (uint32_t)(r | (g << 8) | (b << 16));
        }
        sums[4 * p + 0] = 0;
        sums[4 * p + 1] = 0;
        sums[4 * p + 2] = 0;
        sums[4 * p + 3] = 0;
        fb[p] = RZO_DEPTH_ONES | ((uint64_t)bg & RZO_RGB_MASK);
    }
}

/*
 * Sort-last composition (the sharded form of both passes): the depth passes
 * of disjoint parts of a cloud, each into a full framebuffer, combine into
 * the depth pass of the whole cloud by a per-pixel minimum; the splat sums
 * of the parts, each accumulated against the combined depth pass, add up to
 * the sums of the whole cloud.
 */
void rzo_merge_min(uint64_t *dst, const uint64_t *src, int64_t npix)
{
    int64_t p;
    for (p = 0; p < npix; p++)
        if (src[p] < dst[p])
            dst[p] = src[p];
}

/* sums: four exact words per pixel (R, G, B, count) */
void rzo_merge_sum(uint64_t *dst, const uint64_t *src, int64_t npix)
{
    int64_t i;
    for (i = 0; i < 4 * npix; i++)
        dst[i] += src[i];
}
