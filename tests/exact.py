"""Exact (rational) statement of where a point lands and at which depth.

An independent check of the oracle's floating-point projection: the same
mathematics (projective transform with the float-rounded matrix, viewport,
floor; depth row in double, floor((d - o) s)), evaluated with Python
Fractions, so that no operation order or rounding is involved.  A point whose
floor decisions lie closer to an integer (or a cull boundary) than the
rounding error of the float pipeline could move them is reported as
ambiguous; tests drop such points, so the comparison on the rest is exact.
"""
from __future__ import annotations

from fractions import Fraction as F

import numpy as np

U32 = F(1, 1 << 24)   # unit roundoff of binary32
U64 = F(1, 1 << 53)   # unit roundoff of binary64
SAFETY = 8


def _floor(v: F) -> int:
    return v.numerator // v.denominator


def _dist_int(v: F) -> F:
    f = v - _floor(v)
    return min(f, 1 - f)


class ExactCamera:
    def __init__(self, vp, near, far, width, height, o, s):
        vp = np.asarray(vp, np.float64).reshape(16)
        self.m = [F(float(np.float32(a))) for a in vp]   # (float)VP, exactly
        self.v = [F(float(a)) for a in vp]                # VP, exactly
        self.near, self.far = F(float(near)), F(float(far))
        self.W, self.H = int(width), int(height)
        self.o, self.s = F(float(o)), F(float(s))

    def fragment(self, x, y, z):
        """('cull', None, None), ('frag', pixel, q) or ('ambiguous', None, None)."""
        X, Y, Z = (F(float(np.float32(a))) for a in (x, y, z))
        if any(not np.isfinite(a) for a in (x, y, z)):
            return ("ambiguous", None, None)
        m, v = self.m, self.v

        def row(r, mat):
            terms = [mat[4 * r] * X, mat[4 * r + 1] * Y, mat[4 * r + 2] * Z, mat[4 * r + 3]]
            return sum(terms), sum(abs(t) for t in terms)

        cx, sx = row(0, m)
        cy, sy = row(1, m)
        cw, sw = row(3, m)
        ecw = SAFETY * 4 * U32 * sw
        if cw <= ecw:
            return ("cull", None, None) if cw < -ecw else ("ambiguous", None, None)
        ex, ey = SAFETY * 4 * U32 * sx, SAFETY * 4 * U32 * sy
        nx, ny = cx / cw, cy / cw
        # error of the float ndc, then of the window coordinate
        enx = (ex + abs(nx) * ecw) / (cw - ecw) + SAFETY * U32 * abs(nx)
        eny = (ey + abs(ny) * ecw) / (cw - ecw) + SAFETY * U32 * abs(ny)
        hw, hh = F(self.W, 2), F(self.H, 2)
        fx, fy = (nx + 1) * hw, (ny + 1) * hh
        efx = (enx + SAFETY * U32 * abs(nx + 1)) * hw + SAFETY * U32 * abs(fx)
        efy = (eny + SAFETY * U32 * abs(ny + 1)) * hh + SAFETY * U32 * abs(fy)
        for val, err, lim in ((fx, efx, self.W), (fy, efy, self.H)):
            if abs(val) <= err or abs(val - lim) <= err:
                return ("ambiguous", None, None)
        inside = 0 <= fx < self.W and 0 <= fy < self.H
        if not inside:
            return ("cull", None, None)
        if _dist_int(fx) <= efx or _dist_int(fy) <= efy:
            return ("ambiguous", None, None)
        px, py = _floor(fx), _floor(fy)

        d, sd = row(3, v)
        ed = SAFETY * 4 * U64 * sd
        if abs(d - self.near) <= ed or abs(d - self.far) <= ed:
            return ("ambiguous", None, None)
        if not (self.near <= d < self.far):
            return ("cull", None, None)
        t = (d - self.o) * self.s
        et = (ed + SAFETY * U64 * abs(d - self.o)) * self.s + SAFETY * U64 * abs(t)
        if _dist_int(t) <= et:
            return ("ambiguous", None, None)
        q = min(_floor(t), (1 << 40) - 2)
        return ("frag", py * self.W + px, q)

    def depth(self, x, y, z) -> F:
        X, Y, Z = (F(float(np.float32(a))) for a in (x, y, z))
        v = self.v
        return v[12] * X + v[13] * Y + v[14] * Z + v[15]


def fragments(cam: ExactCamera, x, y, z):
    """Lists status, pixel, q for every point."""
    out = [cam.fragment(a, b, c) for a, b, c in zip(x, y, z)]
    status = np.array([o[0] for o in out])
    pix = np.array([o[1] if o[0] == "frag" else -1 for o in out], np.int64)
    q = np.array([o[2] if o[0] == "frag" else 0 for o in out], dtype=object)
    return status, pix, q


def brute_force_min(pix, q, rgb, npix, clear):
    """Per pixel, the smallest (q << 24 | rgb) over the points in it."""
    fb = [clear] * npix
    for p, qq, c in zip(pix, q, rgb):
        if p < 0:
            continue
        key = (int(qq) << 24) | (int(c) & 0xFFFFFF)
        if key < fb[p]:
            fb[p] = key
    return np.array(fb, dtype=np.uint64)


def round_ieee(v: F, p: int, emin: int) -> F:
    """v rounded to the nearest binary floating-point number with p significand
    bits and least normal exponent emin, ties to even (IEEE 754, section 4.3.1);
    no overflow in these inputs."""
    if v == 0:
        return F(0)
    sign, a = (-1, -v) if v < 0 else (1, v)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if F(2) ** e > a:
        e -= 1
    ulp = F(2) ** (max(e, emin) - p + 1)
    m = a / ulp
    k = m.numerator // m.denominator
    r = m - k
    if r > F(1, 2) or (r == F(1, 2) and k % 2 == 1):
        k += 1
    return sign * k * ulp


def r32(v):
    return round_ieee(v, 24, -126)


def r64(v):
    return round_ieee(v, 53, -1022)
