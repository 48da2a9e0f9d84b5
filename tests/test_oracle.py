"""Pins of the CPU oracle against facts that do not come from the oracle:
values the paper prints, hand-computed cases, an exact rational statement of
the projection, closed forms and invariants (sections 2.1 and 2.2)."""
import json
import math
import os
from fractions import Fraction as F

import numpy as np
import pytest

from paper_1908_02681_amd import gen
from tests.exact import ExactCamera, brute_force_min, fragments as exact_fragments

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LINEAR, SCALE = 0, 1


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _axis_camera():
    """Camera at the origin looking down -z: clip = (x, y, 0, -z)."""
    vp = np.zeros((4, 4))
    vp[0, 0] = vp[1, 1] = 1.0
    vp[3, 2] = -1.0
    return vp


def _pts(rows):
    a = np.array([[r[0], r[1], r[2]] for r in rows], np.float32)
    c = np.array([int(r[3], 16) for r in rows], np.uint32)
    return a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy(), c


# --------------------------------------------------------------------------
# values printed in the paper
# --------------------------------------------------------------------------

def test_clear_value_matches_paper(oracle):
    g = _gold("paper_constants.json")
    assert oracle.clear_value(0) == int(g["clear_value"]["value"], 16)
    assert oracle.clear_value(0x123456) == int(g["clear_value"]["value"], 16) | 0x123456
    # the background bits never reach the depth bytes
    assert oracle.clear_value(0xFF123456) == int(g["clear_value"]["value"], 16) | 0x123456


def test_bit_budget_matches_paper():
    g = _gold("paper_constants.json")
    assert g["color_shift"]["value"] + g["depth_bits"]["value"] == 64
    assert 2 ** g["depth_bits"]["value"] >= g["values_in_40_bits_at_least"]["value"]
    # 1 trillion mm = 1 billion m: the mm map covers 1e9 m inside 40 bits
    assert g["mm_range_metres"]["value"] * g["mm_scale"]["value"] < 2 ** 40
    pw = g["piecewise_example"]
    counts = [(b - a) * s for (a, b), s in zip(pw["ranges_m"], pw["values_per_m"])]
    assert max(counts) <= pw["max_values_per_range"]
    assert sum(counts) <= pw["total_values"]


def test_empty_cloud_gives_background(oracle):
    vp = _axis_camera()
    e = np.zeros(0, np.float32)
    keys, img = oracle.render_atomicmin(e, e, e, np.zeros(0, np.uint32), vp, 1, 100, 7, 5,
                                        bg=0x0A0B0C)
    assert (keys == oracle.clear_value(0x0A0B0C)).all()
    assert (img == 0x0A0B0C).all()
    keys, sums, img = oracle.render_hq(e, e, e, np.zeros(0, np.uint32), vp, 1, 100, 7, 5,
                                       bg=0x0A0B0C)
    assert (sums == 0).all() and (img == 0x0A0B0C).all()


@pytest.mark.parametrize("case", range(len(_gold("hand_cases.json")["cases"])))
def test_hand_cases(oracle, case):
    g = _gold("hand_cases.json")
    c = g["cases"][case]
    x, y, z, rgb = _pts(c["points"])
    vp = np.array(g["vp"], np.float64)
    args = (vp, g["near"], g["far"], g["width"], g["height"], SCALE, g["scale"])
    for perm in (np.arange(x.size), np.arange(x.size)[::-1]):
        xs, ys, zs, cs = x[perm], y[perm], z[perm], rgb[perm]
        if "key" in c:
            keys, img = oracle.render_atomicmin(xs, ys, zs, cs, *args)
            assert int(keys[c["pixel"]]) == int(c["key"], 16)
            assert int(img[c["pixel"]]) == int(c["image"], 16)
        if "sums" in c:
            keys, sums, img = oracle.render_hq(xs, ys, zs, cs, *args, eps=tuple(c["eps"]))
            assert sums[c["pixel"]].tolist() == c["sums"]
            assert int(img[c["pixel"]]) == int(c["hq_image"], 16)
        # all other pixels stay background
        others = np.ones(g["width"] * g["height"], bool)
        others[c["pixel"]] = False
        assert (img[others] == 0).all()


# --------------------------------------------------------------------------
# closed forms of the depth map and the viewport
# --------------------------------------------------------------------------

def test_optical_axis_hits_centre_pixel(oracle):
    W, H = 640, 480
    v = gen.make_view((1.0, 2.0, 3.0), (4.0, -1.0, 0.5), (0, 0, 1), 50.0, W, H, 0.1, 100.0)
    eye, tgt = np.array([1.0, 2.0, 3.0]), np.array([4.0, -1.0, 0.5])
    dirv = (tgt - eye) / np.linalg.norm(tgt - eye)
    ts = np.linspace(0.5, 50, 100)
    p = (eye[None, :] + ts[:, None] * dirv[None, :]).astype(np.float32)
    pix, q = oracle.fragments(p[:, 0], p[:, 1], p[:, 2], v.vp, v.near, v.far, W, H)
    # rounding of the float positions moves a point by << 1 pixel around the
    # centre corner (W/2, H/2): it lands in one of the 4 pixels meeting there
    centre = {(H // 2 - a) * W + (W // 2 - b) for a in (0, 1) for b in (0, 1)}
    assert set(pix.tolist()) <= centre
    # depth along the axis grows with the distance
    assert (np.diff(q.astype(np.int64)) > 0).all()


def test_depth_edges(oracle):
    vp = _axis_camera()
    near, far = 0.5, 8.0
    # d = near exactly -> q = 0; far itself is excluded; just below far is
    # the top of the range
    z = np.array([-near, -far, -np.nextafter(np.float32(far), np.float32(0)), -0.49999997],
                 np.float32)
    e = np.zeros_like(z)
    pix, q = oracle.fragments(e, e, z, vp, near, far, 2, 2, LINEAR)
    assert pix[0] == 3 and q[0] == 0
    assert pix[1] == -1 and pix[3] == -1
    o, s, z0 = oracle.depth_constants(vp, near, far, 2, 2, LINEAR)
    assert o == near and s == (2 ** 40 - 1) / (far - near)
    exact = (F(float(-z[2])) - F(near)) * F(s)
    assert q[2] == math.floor(exact) and q[2] < 2 ** 40 - 1


def test_depth_clamps_below_clear_depth(oracle):
    """The rounding edge next to far is kept strictly below the cleared depth."""
    vp = np.zeros((4, 4))
    vp[3, 0] = 1.0
    vp[3, 3] = float(2 ** 40 - 3)
    x = np.array([1.5, 1.75, 2.25, 2.5], np.float32)
    e = np.zeros_like(x)
    pix, q = oracle.fragments(x, e, e, vp, 1.0, 2.0 ** 40 - 0.25, 2, 2, SCALE, 1.0)
    assert (pix == 3).all()
    assert q.tolist() == [2 ** 40 - 2] * 4


def test_moon_in_millimetres(oracle):
    """Section 2.1: with the 1000x (mm) map, the Moon's distance still fits."""
    vp = _axis_camera()
    z = np.array([-384_400_000.0, -1.0, -0.5], np.float32)
    e = np.zeros_like(z)
    g = _gold("paper_constants.json")
    pix, q = oracle.fragments(e, e, z, vp, 0.25, 1e9, 2, 2, SCALE, g["mm_scale"]["value"])
    assert q.tolist() == [384_400_000_000, 1000, 500]


def test_linear_map_is_uniform(oracle):
    """A uniform map: equal depth steps give equal integer steps (section 2.1)."""
    vp = _axis_camera()
    near, far = 1.0, 1025.0    # s = (2^40 - 1) / 1024
    z = -np.arange(1, 1025, 16, dtype=np.float32)
    e = np.zeros_like(z)
    pix, q = oracle.fragments(e, e, z, vp, near, far, 2, 2, LINEAR)
    exact = [math.floor((F(int(-zz)) - 1) * F((2 ** 40 - 1) / 1024)) for zz in z]
    assert q.tolist() == exact
    steps = np.diff(q.astype(np.int64))
    assert steps.max() - steps.min() <= 1


def test_window_edges_and_culling(oracle):
    """Orthographic-like camera with exact arithmetic: window x = (x + 1) W/2."""
    W, H = 8, 4
    vp = np.eye(4)
    vp[2, :] = 0
    vp[3, :] = [0, 0, 0, 1]            # w = 1, d = 1
    xs = np.array([-1.0, -0.75, 0.999, 1.0, -1.0000001, 0.0, 0.0, np.nan, np.inf, 0.0],
                  np.float32)
    ys = np.array([-1.0, 0.0, 0.999, 0.0, 0.0, -1.0, 1.0, 0.0, 0.0, -np.inf], np.float32)
    zs = np.zeros_like(xs)
    pix, q = oracle.fragments(xs, ys, zs, vp, 0.5, 2.0, W, H, LINEAR)
    exp = [0 * W + 0, 2 * W + 1, 3 * W + 7, -1, -1, 0 * W + 4, -1, -1, -1, -1]
    assert pix.tolist() == exp


def test_behind_camera_and_outside_range_culled(oracle):
    vp = _axis_camera()
    z = np.array([5.0, 0.0, -0.1, -2000.0, -10.0], np.float32)
    e = np.zeros_like(z)
    pix, q = oracle.fragments(e, e, z, vp, 1.0, 1000.0, 2, 2, LINEAR)
    assert pix.tolist() == [-1, -1, -1, -1, 3]


# --------------------------------------------------------------------------
# exact rational statement of the projection, and per-pixel brute force
# --------------------------------------------------------------------------

def _random_scene(seed, n, W, H, kind=LINEAR, scale=0.0):
    rng = np.random.default_rng(seed)
    v = gen.make_view(rng.uniform(-3, 3, 3) + np.array([0, 0, 6.0]), rng.uniform(-0.5, 0.5, 3),
                      (0.2, 1.0, 0.1), 55.0, W, H, 0.3, 12.0)
    pts = rng.uniform(-4, 4, size=(n, 3)).astype(np.float32)
    # a dense cluster so that pixels receive many candidates
    pts[: n // 2] = (rng.normal(0, 0.4, size=(n // 2, 3))).astype(np.float32)
    rgb = rng.integers(0, 1 << 24, size=n, dtype=np.uint32)
    # a few exact depth ties with different colours
    pts[n // 2: n // 2 + 20] = pts[n // 2 + 20: n // 2 + 40]
    return v, pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(), rgb


@pytest.mark.parametrize("seed,kind,scale", [(1, LINEAR, 0.0), (2, LINEAR, 0.0), (3, SCALE, 1000.0),
                                             (4, SCALE, 2.0 ** 30)])
def test_fragments_match_exact_projection(oracle, seed, kind, scale):
    W, H = 48, 32
    v, x, y, z, rgb = _random_scene(seed, 1500, W, H, kind, scale)
    o, s, z0 = oracle.depth_constants(v.vp, v.near, v.far, W, H, kind, scale)
    cam = ExactCamera(v.vp, v.near, v.far, W, H, o, s)
    status, epix, eq = exact_fragments(cam, x, y, z)
    assert (status == "ambiguous").mean() < 0.05
    assert (status == "frag").sum() > 300 and (status == "cull").sum() > 100
    pix, q = oracle.fragments(x, y, z, v.vp, v.near, v.far, W, H, kind, scale)
    ok = status != "ambiguous"
    assert (pix[ok] == epix[ok]).all()
    fr = status == "frag"
    assert [int(a) for a in q[fr]] == [int(a) for a in eq[fr]]


@pytest.mark.parametrize("seed", [5, 6])
def test_framebuffer_matches_brute_force(oracle, seed):
    W, H = 40, 24
    v, x, y, z, rgb = _random_scene(seed, 2000, W, H)
    o, s, z0 = oracle.depth_constants(v.vp, v.near, v.far, W, H)
    cam = ExactCamera(v.vp, v.near, v.far, W, H, o, s)
    status, epix, eq = exact_fragments(cam, x, y, z)
    keep = status != "ambiguous"
    x, y, z, rgb, epix, eq = x[keep], y[keep], z[keep], rgb[keep], epix[keep], eq[keep]
    clear = oracle.clear_value(0x203040)
    want = brute_force_min(epix, eq, rgb, W * H, clear)
    keys, img = oracle.render_atomicmin(x, y, z, rgb, v.vp, v.near, v.far, W, H, bg=0x203040)
    assert (keys == want).all()
    assert (img == (want & np.uint64(0xFFFFFF)).astype(np.uint32)).all()
    assert (keys != clear).sum() > 100


def test_key_fields_round_trip(oracle):
    W, H = 64, 48
    v, x, y, z, rgb = _random_scene(7, 3000, W, H)
    pix, q = oracle.fragments(x, y, z, v.vp, v.near, v.far, W, H)
    keys, img = oracle.render_atomicmin(x, y, z, rgb, v.vp, v.near, v.far, W, H)
    hit = keys != oracle.clear_value(0)
    # every written key is the key of a point of that pixel: depth field = q,
    # colour field = rgb of that point
    for p in np.flatnonzero(hit)[:200]:
        cand = {(int(qq) << 24) | (int(c) & 0xFFFFFF) for qq, c in
                zip(q[pix == p], rgb[pix == p])}
        assert int(keys[p]) in cand
        assert int(keys[p]) == min(cand)
    assert ((keys[hit] >> np.uint64(24)) < 2 ** 40 - 1).all()


# --------------------------------------------------------------------------
# order invariance and the high-quality splatting invariants
# --------------------------------------------------------------------------

def _small_terrain():
    c = gen.terrain(40_000, 11, extent=100.0, amplitude=10.0, wavelength=40.0)
    v = gen.terrain_view(96, 64, extent=100.0, distance=120.0, near=0.5, far=400.0)
    return c, v


def test_order_invariance(oracle):
    c, v = _small_terrain()
    a = oracle.render_hq(c.x, c.y, c.z, c.rgb, v.vp, v.near, v.far, v.width, v.height)
    for seed in (1, 2):
        s = gen.shuffle(c, seed)
        b = oracle.render_hq(s.x, s.y, s.z, s.rgb, v.vp, v.near, v.far, v.width, v.height)
        for u, w in zip(a, b):
            assert (u == w).all()


def test_hq_depth_pass_equals_basic(oracle):
    c, v = _small_terrain()
    keys, img = oracle.render_atomicmin(c.x, c.y, c.z, c.rgb, v.vp, v.near, v.far, v.width,
                                        v.height)
    k2, sums, img2 = oracle.render_hq(c.x, c.y, c.z, c.rgb, v.vp, v.near, v.far, v.width,
                                      v.height)
    assert (keys == k2).all()
    # a pixel has accepted fragments exactly when it was written
    assert ((sums[:, 3] > 0) == (keys != oracle.clear_value(0))).all()
    # with several fragments per pixel the window is actually used
    assert sums[:, 3].max() > 3


def test_hq_eps_zero_keeps_only_nearest(oracle):
    c, v = _small_terrain()
    keys, img = oracle.render_atomicmin(c.x, c.y, c.z, c.rgb, v.vp, v.near, v.far, v.width,
                                        v.height)
    _, sums, img0 = oracle.render_hq(c.x, c.y, c.z, c.rgb, v.vp, v.near, v.far, v.width,
                                     v.height, eps=(0, 1))
    one = sums[:, 3] == 1
    assert one.sum() > 100
    assert (img0[one] == img[one]).all()


def test_hq_huge_eps_averages_whole_pixel(oracle):
    """eps >> 1 accepts every fragment of a pixel: plain per-pixel averages."""
    W, H = 40, 24
    v, x, y, z, rgb = _random_scene(8, 2000, W, H)
    o, s, z0 = oracle.depth_constants(v.vp, v.near, v.far, W, H)
    cam = ExactCamera(v.vp, v.near, v.far, W, H, o, s)
    status, epix, eq = exact_fragments(cam, x, y, z)
    keep = status != "ambiguous"
    x, y, z, rgb, epix = x[keep], y[keep], z[keep], rgb[keep], epix[keep]
    assert z0 > 2 ** 20
    _, sums, img = oracle.render_hq(x, y, z, rgb, v.vp, v.near, v.far, W, H,
                                    eps=(2 ** 20, 1), bg=0x010203)
    inside = epix >= 0
    for ch in range(3):
        want = np.bincount(epix[inside], weights=((rgb[inside] >> (8 * ch)) & 255),
                           minlength=W * H)
        assert (sums[:, ch] == want.astype(np.uint64)).all()
    cnt = np.bincount(epix[inside], minlength=W * H)
    assert (sums[:, 3] == cnt).all()
    for p in range(W * H):
        if cnt[p] == 0:
            assert img[p] == 0x010203
            continue
        exp = 0
        for ch in range(3):
            avg = F(int(sums[p, ch]), int(cnt[p]))
            exp |= math.floor(avg + F(1, 2)) << (8 * ch)
        assert int(img[p]) == exp


def test_hq_integer_window_matches_linear_depth(oracle):
    """The integer eps test agrees with 'linear depth at most 1% larger than
    the nearest' wherever the real-number margin exceeds two depth quanta."""
    c, v = _small_terrain()
    W, H = v.width, v.height
    keys, _ = oracle.render_atomicmin(c.x, c.y, c.z, c.rgb, v.vp, v.near, v.far, W, H)
    o, s, z0 = oracle.depth_constants(v.vp, v.near, v.far, W, H)
    pix, q = oracle.fragments(c.x, c.y, c.z, v.vp, v.near, v.far, W, H)
    cam = ExactCamera(v.vp, v.near, v.far, W, H, o, s)
    sel = np.flatnonzero(pix >= 0)[::7][:3000]
    qmin = keys[pix[sel]] >> np.uint64(24)
    agree = checked = 0
    for i, qm in zip(sel, qmin):
        d = cam.depth(c.x[i], c.y[i], c.z[i])
        dmin = F(int(qm)) / F(s) + F(o)           # depth of the nearest fragment
        margin = F(101, 100) * dmin - d
        if abs(margin) * F(s) <= 2:
            continue
        checked += 1
        integer_ok = 100 * (int(q[i]) - int(qm)) <= int(qm) + z0
        agree += integer_ok == (margin >= 0)
    assert checked > 2000 and agree == checked


def test_eps_window_relative_to_linear_depth(oracle):
    """Section 2.2 states the window in linear depth (1% of the distance), not
    in stored integer depth: with the linear map of [50, 150) the offset of
    the near plane matters.  Nearest at d = 100, d = 100.9 is within 1%
    (accepted), d = 101.2 is not; worked out by hand."""
    vp = _axis_camera()
    z = np.array([-100.0, -100.9, -101.2], np.float32)
    e = np.zeros_like(z)
    rgb = np.array([10, 20, 200], np.uint32)
    _, sums, img = oracle.render_hq(e, e, z, rgb, vp, 50.0, 150.0, 2, 2, LINEAR, eps=(1, 100))
    assert sums[3].tolist() == [30, 0, 0, 2]
    assert img[3] == 15


def test_z_fighting_free_at_one_millimetre(oracle):
    """Two interleaved surfaces 1 mm apart at ~1 km: the 40-bit buffer always
    shows the nearer one (teaser (a) vs (b), section 1)."""
    rng = np.random.default_rng(3)
    n = 20000
    W, H = 64, 64
    v = gen.make_view((0, 0, 1000.0), (0, 0, 0), (0, 1, 0), 1.0, W, H, 0.5, 4000.0)
    x = rng.uniform(-8, 8, n).astype(np.float32)
    y = rng.uniform(-8, 8, n).astype(np.float32)
    z = np.where(np.arange(n) % 2 == 0, np.float32(0.0), np.float32(-0.001)).astype(np.float32)
    rgb = np.where(np.arange(n) % 2 == 0, 0x0000FF, 0x00FF00).astype(np.uint32)
    keys, img = oracle.render_atomicmin(x, y, z, rgb, v.vp, v.near, v.far, W, H)
    near_px = set(oracle.fragments(x[::2], y[::2], z[::2], v.vp, v.near, v.far, W, H)[0].tolist())
    near_px.discard(-1)
    assert len(near_px) > 3000
    assert all(img[p] == 0x0000FF for p in near_px)


def test_resolve_clears_framebuffer(oracle):
    """The resolve step leaves the framebuffer cleared for the next frame
    (section 2.1), in both the basic and the splatting variant."""
    c, v = _small_terrain()
    bg = 0x405060
    fb = oracle.raster_min(c.x, c.y, c.z, c.rgb, v.vp, v.near, v.far, v.width, v.height, bg=bg)
    assert (fb != oracle.clear_value(bg)).sum() > 1000
    oracle.resolve_min(fb, bg)
    assert (fb == oracle.clear_value(bg)).all()
    fb = oracle.raster_min(c.x, c.y, c.z, c.rgb, v.vp, v.near, v.far, v.width, v.height, bg=bg)
    sums = oracle.hq_accumulate(c.x, c.y, c.z, c.rgb, v.vp, v.near, v.far, v.width, v.height, fb)
    oracle.hq_resolve(sums, fb, bg)
    assert (fb == oracle.clear_value(bg)).all() and (sums == 0).all()


# --------------------------------------------------------------------------
# piecewise depth map (section 2.1: sub-ranges with their own precision)
# --------------------------------------------------------------------------

def _paper_ranges():
    pw = _gold("paper_constants.json")["piecewise_example"]
    return tuple((a, sc) for (a, _), sc in zip(pw["ranges_m"], pw["values_per_m"]))


def _piecewise_q_exact(d, ranges):
    """Integer depth by the definition, in exact rationals."""
    starts = [F(a) for a, _ in ranges]
    scales = [F(sc) for _, sc in ranges]
    base = [0]
    for k in range(len(ranges) - 1):
        base.append(base[k] + math.floor((starts[k + 1] - starts[k]) * scales[k]) + 1)
    k = max(i for i, a in enumerate(starts) if F(d) >= a)
    return base[k] + math.floor((F(d) - starts[k]) * scales[k]), base


def test_piecewise_paper_example(oracle):
    """nm up to 10 m, um up to 10 km, mm beyond: every range uses at most
    10 billion values, 30 billion in all (section 2.1)."""
    ranges = _paper_ranges()
    g = _gold("paper_constants.json")["piecewise_example"]
    vp = _axis_camera()
    ds = np.array([0.5, 5.0, 9.5, np.nextafter(np.float32(10), np.float32(0)), 10.0, 10.5, 9999.5,
                   10000.0, 12345.5, 1.0e6, 9.0e6], np.float32)
    e = np.zeros_like(ds)
    pix, q = oracle.fragments(e, e, -ds, vp, 0.25, 1.0e7, 2, 2, oracle.PIECEWISE, ranges)
    assert (pix == 3).all()
    for d, qq in zip(ds, q):
        want, base = _piecewise_q_exact(float(d), ranges)
        assert int(qq) == want, (float(d), int(qq), want)
    # bases: 1e10 + 1 and 1e10 + 1 + 9.99e9 + 1; the last value is below 3e10
    _, base = _piecewise_q_exact(1.0, ranges)
    assert base == [0, 10_000_000_001, 19_990_000_002]
    top = base[2] + math.floor((F(10_000_000) - F(10_000)) * F(1000))
    assert top <= g["total_values"] and max(base[1], base[2] - base[1]) <= g["max_values_per_range"] + 1
    # dense sweep: never decreasing, and distinct float32 depths stay
    # distinct (nm near the camera, mm far away)
    for lo, hi in ((0.3, 12.0), (9990.0, 10020.0), (9.0e5, 9.1e5)):
        d = np.unique(np.linspace(lo, hi, 20001).astype(np.float32))
        e = np.zeros_like(d)
        _, qq = oracle.fragments(e, e, -d, vp, 0.25, 1.0e7, 2, 2, oracle.PIECEWISE, ranges)
        qq = qq.astype(np.int64)
        assert (np.diff(qq) > 0).all()


def test_piecewise_window_uses_linear_depth(oracle):
    """With sub-ranges the 1% window is taken in linear depth, relative to the
    nearest depth, also across a range boundary: nearest 5.00 m, 5.04 m in,
    5.0505 m out (1.01 x 5.00 = 5.05), 5.06 m out; nearest 9.95 m, 10.04 m in
    (next range), 10.06 m out.  Worked out by hand."""
    ranges = _paper_ranges()
    vp = _axis_camera()
    for zs in ([5.0, 5.04, 5.0505, 5.06], [9.95, 10.04, 10.0496, 10.06]):
        z = -np.array(zs, np.float32)
        e = np.zeros_like(z)
        rgb = np.array([10, 20, 100, 200], np.uint32)
        _, sums, _ = oracle.render_hq(e, e, z, rgb, vp, 0.25, 1.0e7, 2, 2, oracle.PIECEWISE,
                                      ranges)
        assert sums[3].tolist() == [30, 0, 0, 2]


def test_piecewise_range_boundary(oracle):
    """Range 1 starts one integer above the largest value of range 0, also
    when the next start is not on range 0's grid."""
    vp = _axis_camera()
    ranges = ((0.0, 3.0), (1.0, 1000.0))        # base[1] = floor(1 * 3) + 1 = 4
    d = np.array([0.5, 0.99999994, 1.0, 1.001], np.float32)
    e = np.zeros_like(d)
    _, q = oracle.fragments(e, e, -d, vp, 0.25, 10.0, 2, 2, oracle.PIECEWISE, ranges)
    assert q.tolist() == [1, 2, 4, 5]
    ranges = ((0.0, 2.5), (1.0, 1000.0))        # base[1] = floor(2.5) + 1 = 3
    d = np.array([0.9999999, 1.0], np.float32)
    e = np.zeros_like(d)
    _, q = oracle.fragments(e, e, -d, vp, 0.25, 10.0, 2, 2, oracle.PIECEWISE, ranges)
    assert q.tolist() == [2, 3]
