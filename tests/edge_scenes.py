"""Point sets where the rounding of the single-precision projection and of
the double-precision depth row decides the result (section 1 fixes the
precisions, not the operation order).  Shared by the oracle's pin against
the IEEE definition of each rounded step and by the GPU parity tests, so
that the kernels see exactly the points on which the fused and unfused
readings differ.  Inputs only: no rasterizer arithmetic here."""
from fractions import Fraction as F

import numpy as np

from paper_1908_02681_amd import gen

EDGE_W, EDGE_H = 15000, 12000    # half sizes that are not powers of two


def random_scene(seed, n, W, H):
    """A random camera looking at n points in a cube, half of them in a
    dense cluster, with 20 exact depth ties of different colours."""
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


def rounding_edge_scene(offset):
    """1500 random points plus 500 points unprojected from within 10^-4
    pixel of a pixel corner of a 15000 x 12000 screen, where the rounding of
    the divide and the viewport decides the floor.  With offset != 0 the
    whole scene (camera and points) sits that far from the origin
    (georeferenced coordinates), where the terms of the depth row cancel
    and its rounding decides the 40-bit depth.  Returns (view, x, y, z, rgb)."""
    W, H = EDGE_W, EDGE_H
    v, x, y, z, rgb = random_scene(11, 1500, W, H)
    rng = np.random.default_rng(13)
    corner = rng.integers(1, [W, H], size=(500, 2)) + rng.uniform(-1e-4, 1e-4, (500, 2))
    ndc = np.column_stack([2 * corner / [W, H] - 1, rng.uniform(-0.9, 0.9, 500), np.ones(500)])
    world = np.linalg.solve(np.asarray(v.vp, np.float64).reshape(4, 4), ndc.T).T
    world = (world[:, :3] / world[:, 3:]).astype(np.float32)
    x, y, z = (np.concatenate([a, world[:, k]]) for k, a in enumerate((x, y, z)))
    rgb = np.concatenate([rgb, np.random.default_rng(14).integers(0, 1 << 24, 500,
                                                                  dtype=np.uint32)])
    if offset:
        off = np.array([offset, 0.5 * offset, -0.25 * offset])
        rng = np.random.default_rng(12)
        v = gen.make_view(rng.uniform(-3, 3, 3) + np.array([0, 0, 6.0]) + off,
                          rng.uniform(-0.5, 0.5, 3) + off, (0.2, 1.0, 0.1), 55.0, W, H, 0.3, 12.0)
        x, y, z = ((a + np.float32(b)).astype(np.float32) for a, b in zip((x, y, z), off))
    return v, x, y, z, rgb


# probe depths around an edge, in steps of 2^-23 of the edge's depth, from
# below the float resolution of the coordinates to well beyond it
OFFSETS = (-512, -128, -32, -12, -6, -3, -1, 0, 1, 3, 6, 12, 32, 128, 512)
PROBE_RGB = 0x010203


def _ray_points(view, pixels, depths, rng):
    """Points on the rays through random spots of the given pixels, at the
    given depths (the depth is row 3 of VP, affine along a ray), rounded to
    float32."""
    vp = np.asarray(view.vp, np.float64).reshape(4, 4)
    inv = np.linalg.inv(vp)
    out = []
    for p, ds in zip(pixels, depths):
        px, py = p % view.width + rng.uniform(0.3, 0.7), p // view.width + rng.uniform(0.3, 0.7)
        nx, ny = 2 * px / view.width - 1, 2 * py / view.height - 1
        a = inv @ np.array([nx, ny, -1.0, 1.0])
        b = inv @ np.array([nx, ny, 1.0, 1.0])
        a, b = a[:3] / a[3], b[:3] / b[3]
        da, db = vp[3, :3] @ a + vp[3, 3], vp[3, :3] @ b + vp[3, 3]
        for d in ds:
            t = (d - da) / (db - da)
            out.append(a + t * (b - a))
    return np.asarray(out, np.float32)


def window_edge_scene(oracle, seed, kind, scale, eps, offset):
    """A random cloud on a 64 x 48 screen, and probe points on the rays
    through 120 of its pixels at depths around each pixel's splat window
    edge (section 2.2: where q reaches qmax + 1, from the oracle's depth
    pass), and through 30 other pixels around the near and far planes, at
    relative offsets OFFSETS * 2^-23.  The scene sits `offset` from the
    origin.  Returns a dict: view, fb (the oracle's depth pass of cloud and
    probes together), depth (o, s, z0), base (the cloud, float32 (n, 3)),
    rgb (its colours), probes (float32 (m, 3), colour 0x010203)."""
    W, H = 64, 48
    rng = np.random.default_rng(seed)
    off = np.array([offset, 0.5 * offset, -0.25 * offset])
    eye = rng.uniform(-2, 2, 3) + np.array([0, 0, 6.0]) + off
    view = gen.make_view(eye, rng.uniform(-0.3, 0.3, 3) + off, (0.2, 1.0, 0.1), 50.0, W, H,
                         0.5, 40.0)
    base = (rng.normal(0, 0.8, size=(6000, 3)) + off).astype(np.float32)
    rgb = rng.integers(0, 1 << 24, size=6000, dtype=np.uint32)
    args = (view.vp, view.near, view.far, W, H, kind, scale)
    fb, _ = oracle.render_atomicmin(base[:, 0], base[:, 1], base[:, 2], rgb, *args[:5],
                                    kind, scale)
    o, s, z0 = oracle.depth_constants(*args)
    clear = np.uint64(oracle.clear_value(0))
    hit = np.flatnonzero(fb != clear)
    pick = rng.choice(hit, size=min(120, hit.size), replace=False)
    num, den = eps
    depths = []
    for p in pick:
        qmin = int(fb[p]) >> 24
        qmax = qmin + (num * (qmin + int(z0))) // den
        edge = F(o) + F(qmax + 1) / F(s)          # where q reaches qmax + 1
        depths.append([float(edge * (1 + F(k, 1 << 23))) for k in OFFSETS])
    near_far = [[view.near * (1 + k * 2.0 ** -23) for k in OFFSETS] +
                [view.far * (1 + k * 2.0 ** -23) for k in OFFSETS]
                for _ in range(30)]
    rest = np.setdiff1d(np.arange(W * H), pick)
    pts = np.concatenate([_ray_points(view, pick, depths, rng),
                          _ray_points(view, rng.choice(rest, 30, replace=False), near_far, rng)])
    # the depth pass of the whole cloud, probes included (the accumulate
    # pass always runs against the depth pass of its own points)
    allp = np.concatenate([base, pts])
    allc = np.concatenate([rgb, np.full(len(pts), PROBE_RGB, np.uint32)])
    fb, _ = oracle.render_atomicmin(allp[:, 0], allp[:, 1], allp[:, 2], allc, *args[:5],
                                    kind, scale)
    return {"view": view, "fb": fb, "depth": (o, s, z0), "base": base, "rgb": rgb,
            "probes": pts}
