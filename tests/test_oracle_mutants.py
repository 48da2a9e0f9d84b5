"""The oracle's pins must catch plausible mistakes.  Each mutant below plants
one mistake in a private copy of the oracle source (on the CPU), and at least
one pin of tests/test_oracle.py has to fail on it."""
import ctypes
import os
import subprocess

import pytest

from oracle import oracle as O
from tests import test_oracle as T

MUTANTS = {
    "transposed matrix": ("cx = fmaf(m[1], y, cx);", "cx = fmaf(m[4], y, cx);"),
    "dropped translation": ("cx = fmaf(m[0], x, m[3]);", "cx = m[0] * x;"),
    "wrong w row": ("cw = fmaf(m[12], x, m[15]);", "cw = fmaf(m[8], x, m[15]);"),
    "viewport sign": ("fx = fmaf(nx, c->hw, c->hw);", "fx = fmaf(nx, c->hw, -c->hw);"),
    "half sizes swapped": ("fy = fmaf(ny, c->hh, c->hh);", "fy = fmaf(ny, c->hw, c->hw);"),
    "ndc scales by the wrong reciprocal": ("ny = cy * iw;", "ny = cy / cx;"),
    "reciprocal of the wrong row": ("iw = 1.0f / cw;", "iw = 1.0f / cx;"),
    "window edge inclusive": ("fx < c->fw", "fx <= c->fw"),
    "clip row unfused": ("cx = fmaf(m[0], x, m[3]);\n    cx = fmaf(m[1], y, cx);\n    cx = fmaf(m[2], z, cx);",
                         "cx = ((m[0] * x + m[1] * y) + m[2] * z) + m[3];"),
    "depth row unfused": ("d = fma(v[13], (double)y, d);\n    d = fma(v[14], (double)z, d);",
                          "d = (d + v[13] * (double)y) + v[14] * (double)z;"),
    "division instead of the reciprocal": ("nx = cx * iw;", "nx = cx / cw;"),
    "viewport unfused": ("fx = fmaf(nx, c->hw, c->hw);", "fx = (nx + 1.0f) * c->hw;"),
    "depth from row 2": ("d = fma(v[12], (double)x, v[15]);", "d = fma(v[8], (double)x, v[15]);"),
    "depth offset dropped": ("d = fma(v[12], (double)x, v[15]);", "d = v[12] * (double)x;"),
    "depth in single precision": ("d = fma(v[14], (double)z, d);",
                                  "d = fma(v[14], (double)z, d);\n    d = (double)cw;"),
    "far inclusive": ("d < c->far_", "d <= c->far_"),
    "near exclusive": ("d >= c->near_", "d > c->near_"),
    "round instead of floor": ("    t = (d - c->o) * c->s;\n    tf = floor(t);",
                               "    t = (d - c->o) * c->s;\n    tf = round(t);"),
    "no clamp below clear depth": ("#define RZO_Q_MAX ((double)((1ull << 40) - 2))",
                                   "#define RZO_Q_MAX ((double)((1ull << 40) - 1))"),
    "linear range off by one": ("#define RZO_Q_RANGE ((double)((1ull << 40) - 1))",
                                "#define RZO_Q_RANGE ((double)((1ull << 40)))"),
    "pixel index transposed": ("*pix = (int64_t)py * c->w + px;", "*pix = (int64_t)px * c->h + py;"),
    "colour shift 23": ("key = (q << 24)", "key = (q << 23)"),
    "max instead of min": ("if (key < fb[yy * w + xx])", "if (key > fb[yy * w + xx])"),
    "colour mask 16 bits": ("key = (q << 24) | ((uint64_t)rgb[i] & RZO_RGB_MASK);",
                            "key = (q << 24) | ((uint64_t)rgb[i] & 0xFFFFu);"),
    "eps window exclusive": ("(unsigned __int128)eps_den * (q - qmin) >\n",
                             "(unsigned __int128)eps_den * (q - qmin) >=\n"),
    "eps offset z0 dropped": ("((unsigned __int128)qmin + c.z0)", "((unsigned __int128)qmin)"),
    "eps num and den swapped": ("if ((unsigned __int128)eps_den * (q - qmin) >\n                           (unsigned __int128)eps_num",
                                "if ((unsigned __int128)eps_num * (q - qmin) >\n                           (unsigned __int128)eps_den"),
    "piecewise base off by one": ("+ (uint64_t)floor((b[k + 1] - b[k]) * sb[k]) + 1;",
                                  "+ (uint64_t)floor((b[k + 1] - b[k]) * sb[k]);"),
    "piecewise range boundary exclusive": ("while (k + 1 < c->nr && d >= c->b[k + 1])",
                                           "while (k + 1 < c->nr && d > c->b[k + 1])"),
    "piecewise range start not subtracted": ("t = (d - c->b[k]) * c->sb[k];", "t = d * c->sb[k];"),
    "piecewise window from the wrong depth": ("const double rhs = (double)eps_num * dm;",
                                              "const double rhs = (double)eps_num * dq;"),
    "truncating average": ("uint64_t r = (2 * sums[4 * p + 0] + cnt) / (2 * cnt);",
                           "uint64_t r = sums[4 * p + 0] / cnt;"),
    "green reads blue": ("sums[4 * pp + 1] += (col >> 8) & 0xFFu;",
                         "sums[4 * pp + 1] += (col >> 16) & 0xFFu;"),
    "count steps by two": ("sums[4 * pp + 3] += 1;", "sums[4 * pp + 3] += 2;"),
    "resolve clear drops background": (
        "img[p] = (uint32_t)(fb[p] & RZO_RGB_MASK);\n        fb[p] = RZO_DEPTH_ONES | ((uint64_t)bg & RZO_RGB_MASK);",
        "img[p] = (uint32_t)(fb[p] & RZO_RGB_MASK);\n        fb[p] = RZO_DEPTH_ONES;"),
    "splat background lost": ("img[p] = bg & 0xFFFFFFu;", "img[p] = 0;"),
    "splat sums not cleared": ("        sums[4 * p + 3] = 0;\n", ""),
    "gl24 z from the w row": ("cz = fmaf(m[10], z, cz);", "cz = fmaf(m[14], z, cz);"),
    "gl24 window offset dropped": ("zw = (nz + 1.0f) * 0.5f;", "zw = nz * 0.5f;"),
    "gl24 truncates": ("*q = (uint64_t)floor((double)t + 0.5);", "*q = (uint64_t)floor((double)t);"),
    "gl24 not clipped": ("        if (!(nz >= -1.0f && nz <= 1.0f))\n            return 0;\n", ""),
    "gl24 23 bits": ("t = zw * 16777215.0f;", "t = zw * 8388607.0f;"),
    "f32rev not complemented": ("*q = (uint64_t)(0xFFFFFFFFu - zr.u);", "*q = (uint64_t)zr.u;"),
    "f32rev from far": ("zr.f = c->nearf / cw;", "zr.f = (float)c->far_ / cw;"),
    "point square one short": ("*hi = c - r + k > size ? size : c - r + k;",
                               "*hi = c - r + k - 1 > size ? size : c - r + k - 1;"),
    "point square not centred": ("const int64_t r = (k - 1) / 2;", "const int64_t r = 0;"),
    "point square radius rounded up": ("const int64_t r = (k - 1) / 2;", "const int64_t r = k / 2;"),
    "splat footprint only the centre": (
        "rzo_span(p % w, psize, w, &x0, &x1);\n        rzo_span(p / w, psize, h, &y0, &y1);\n        for (yy = y0; yy < y1; yy++) {",
        "rzo_span(p % w, 1, w, &x0, &x1);\n        rzo_span(p / w, 1, h, &y0, &y1);\n        for (yy = y0; yy < y1; yy++) {"),
    "splat window of the centre pixel": ("const uint64_t qmin = fb[pp] >> 24;",
                                         "const uint64_t qmin = fb[p] >> 24;"),
    "merge keeps the larger key": ("if (src[p] < dst[p])\n            dst[p] = src[p];",
                                   "if (src[p] > dst[p])\n            dst[p] = src[p];"),
    "merge sum drops the count": ("for (i = 0; i < 4 * npix; i++)", "for (i = 0; i < 4 * npix; i += 4)"),
}

PINS = [
    (T.test_clear_value_matches_paper, {}),
    (T.test_empty_cloud_gives_background, {}),
    *[(T.test_hand_cases, {"case": i}) for i in range(len(T._gold("hand_cases.json")["cases"]))],
    (T.test_depth_edges, {}),
    (T.test_depth_clamps_below_clear_depth, {}),
    (T.test_moon_in_millimetres, {}),
    (T.test_linear_map_is_uniform, {}),
    (T.test_window_edges_and_culling, {}),
    (T.test_behind_camera_and_outside_range_culled, {}),
    (T.test_optical_axis_hits_centre_pixel, {}),
    (T.test_resolve_clears_framebuffer, {}),
    (T.test_fragments_match_exact_projection, {"seed": 1, "kind": 0, "scale": 0.0}),
    *[(T.test_projection_rounding_follows_the_fused_reading, {"offset": f}) for f in (0.0, 3.0e5)],
    (T.test_framebuffer_matches_brute_force, {"seed": 5}),
    (T.test_eps_window_relative_to_linear_depth, {}),
    (T.test_piecewise_paper_example, {}),
    (T.test_piecewise_window_uses_linear_depth, {}),
    (T.test_piecewise_range_boundary, {}),
    (T.test_hq_depth_pass_equals_basic, {}),
    (T.test_hq_huge_eps_averages_whole_pixel, {}),
    (T.test_hq_integer_window_matches_linear_depth, {}),
    (T.test_gl24_window_depth_codes, {}),
    (T.test_f32rev_codes, {}),
    (T.test_gl24_codes_follow_the_perspective_depth, {}),
    (T.test_depth_buffer_precision_at_one_kilometre, {}),
    (T.test_point_size_corner_hand_case, {}),
    *[(T.test_point_size_is_a_min_filter, {"k": k}) for k in (2, 3, 4, 5)],
    *[(T.test_point_size_splat_sums_are_box_sums, {"k": k}) for k in (2, 3)],
    (T.test_point_size_splat_window_per_covered_pixel, {}),
    (T.test_sort_last_depth_merge, {}),
    (T.test_sort_last_splat_merge, {}),
]


def _first_failing_pin(lib):
    saved = O._lib
    O._lib = lib
    try:
        for fn, kw in PINS:
            try:
                fn(O, **kw)
            except (AssertionError, ValueError):
                return f"{fn.__name__}{kw or ''}"
        return None
    finally:
        O._lib = saved


def test_unmutated_oracle_passes_every_pin():
    O.build()
    assert _first_failing_pin(O.configure(ctypes.CDLL(O.LIB))) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(O.SRC).read()
    assert src.count(old) == 1, f"mutation site of {name!r} is not unique"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    flags = [f for f in O.CFLAGS if f != "-Werror"]
    subprocess.run(["gcc", *flags, str(path), "-o", str(so), "-lm"], check=True)
    lib = O.configure(ctypes.CDLL(str(so)))
    assert _first_failing_pin(lib) is not None, f"no pin catches: {name}"
