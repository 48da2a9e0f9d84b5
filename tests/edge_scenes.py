"""Point sets where the rounding of the single-precision projection and of
the double-precision depth row decides the result (section 1 fixes the
precisions, not the operation order).  Shared by the oracle's pin against
the IEEE definition of each rounded step and by the GPU parity tests, so
that the kernels see exactly the points on which the fused and unfused
readings differ.  Inputs only: no rasterizer arithmetic here."""
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
