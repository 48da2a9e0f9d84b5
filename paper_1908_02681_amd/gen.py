"""Seeded synthetic point clouds and cameras.

This module produces inputs only.  It holds none of the rasterizer's
arithmetic (no projection, depth quantisation, key packing or blending):
it builds point arrays and view-projection matrices, which both the CPU
oracle and the HIP path take as given.

The paper measures real scans (Heidentor, Retz, Morro Bay; Table 1) that are
not available here.  The generators below stand in for them with the same
kind of structure: a dense LIDAR-like terrain delivered in a locality
preserving (Morton) order, closed object surfaces (spheres), and the same
clouds randomly shuffled, which the paper reports as the harder order
(section 3).

Point layout (struct of arrays): x, y, z float32 planes and one uint32 colour
plane holding R | G << 8 | B << 16 (top byte zero).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Cloud", "View", "look_at", "perspective", "make_view", "spheres",
    "terrain", "terrain_height", "buildings", "concat", "shuffle",
    "orbit_views", "config1", "config2", "config3", "CONFIG_SEEDS",
    "SERVE_SIZES", "SERVE_CLOUDS", "serve_cloud", "request_trace",
]

# Seeds of the five benchmark workloads (1M spheres, 50M terrain, 300M
# stress cloud, 100M batched cloud, serving clouds).
CONFIG_SEEDS = {1: 0, 2: 1, 3: 2, 4: 3, 5: 4}


@dataclass
class Cloud:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    rgb: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def take(self, idx) -> "Cloud":
        return Cloud(self.x[idx], self.y[idx], self.z[idx], self.rgb[idx], self.name)


@dataclass
class View:
    """A camera: row-major view-projection matrix (clip = VP @ [x, y, z, 1]),
    near/far of the depth range and the framebuffer size."""
    vp: np.ndarray
    near: float
    far: float
    width: int
    height: int
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# cameras (OpenGL conventions: camera looks down -z in view space)
# --------------------------------------------------------------------------

def look_at(eye, target, up) -> np.ndarray:
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    up = np.asarray(up, np.float64)
    f = target - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, up)
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    m = np.eye(4)
    m[0, :3] = s
    m[1, :3] = u
    m[2, :3] = -f
    m[0, 3] = -s @ eye
    m[1, 3] = -u @ eye
    m[2, 3] = f @ eye
    return m


def perspective(fovy_deg: float, aspect: float, near: float, far: float) -> np.ndarray:
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    m = np.zeros((4, 4))
    m[0, 0] = f / aspect
    m[1, 1] = f
    m[2, 2] = (far + near) / (near - far)
    m[2, 3] = 2.0 * far * near / (near - far)
    m[3, 2] = -1.0
    return m


def make_view(eye, target, up, fovy, width, height, near, far, **meta) -> View:
    vp = perspective(fovy, width / height, near, far) @ look_at(eye, target, up)
    return View(np.ascontiguousarray(vp, np.float64), float(near), float(far),
                int(width), int(height), dict(meta, eye=list(map(float, eye)),
                                              target=list(map(float, target))))


# --------------------------------------------------------------------------
# element-wise work in chunks on a thread pool (numpy releases the GIL in
# its array loops); every chunk computes exactly what one whole-array
# expression would, so the result does not depend on the thread count
# --------------------------------------------------------------------------

_CHUNK = 1 << 22


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n: int, fn):
    """fn(a, b) for consecutive ranges covering [0, n), on a thread pool."""
    ranges = [(a, min(n, a + _CHUNK)) for a in range(0, n, _CHUNK)]
    if len(ranges) <= 1:
        for a, b in ranges:
            fn(a, b)
        return
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda r: fn(*r), ranges))


# --------------------------------------------------------------------------
# integer hash used for lattice noise (Wellons' "lowbias32" mixer)
# --------------------------------------------------------------------------

def _mix32(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint32, copy=True)
    v ^= v >> np.uint32(16)
    v *= np.uint32(0x7FEB352D)
    v ^= v >> np.uint32(15)
    v *= np.uint32(0x846CA68B)
    v ^= v >> np.uint32(16)
    return v


def _lattice(nx: int, ny: int, octave: int, seed: int) -> np.ndarray:
    """Uniform values in [-1, 1) on an (ny, nx) integer lattice."""
    iy, ix = np.meshgrid(np.arange(ny, dtype=np.uint32),
                         np.arange(nx, dtype=np.uint32), indexing="ij")
    h = _mix32(ix * np.uint32(0x9E3779B1) ^ _mix32(iy + np.uint32(0x632BE5AB * (octave + 1) & 0xFFFFFFFF))
               ^ np.uint32((seed * 0x85EBCA77) & 0xFFFFFFFF))
    return (h >> np.uint32(8)).astype(np.float64) * (2.0 / (1 << 24)) - 1.0


def _smooth(t):
    return t * t * (3.0 - 2.0 * t)


def terrain_height(px, py, seed: int, extent=1000.0, amplitude=50.0,
                   wavelength=200.0, octaves=6, persistence=0.5) -> np.ndarray:
    """Fractal value noise evaluated at arbitrary (px, py), float64.  Used for a
    few query points (building footprints); the bulk grid uses the separable
    form in ``_height_grid``, which evaluates the same function."""
    px = np.asarray(px, np.float64)
    py = np.asarray(py, np.float64)
    z = np.zeros(np.broadcast(px, py).shape)
    amp, total = 1.0, 0.0
    for k in range(octaves):
        lam = wavelength / (2 ** k)
        nodes = int(math.ceil(extent / lam)) + 2
        lat = _lattice(nodes, nodes, k, seed)
        u, v = px / lam, py / lam
        iu = np.clip(np.floor(u).astype(np.int64), 0, nodes - 2)
        iv = np.clip(np.floor(v).astype(np.int64), 0, nodes - 2)
        tu, tv = _smooth(u - iu), _smooth(v - iv)
        a = lat[iv, iu] * (1 - tu) + lat[iv, iu + 1] * tu
        b = lat[iv + 1, iu] * (1 - tu) + lat[iv + 1, iu + 1] * tu
        z += amp * (a * (1 - tv) + b * tv)
        total += amp
        amp *= persistence
    return z * (amplitude / total)


def _chunked_rows(g: int, fn):
    """fn(a, b) over row ranges of a g x g grid, about _CHUNK cells each."""
    per = max(1, _CHUNK // max(1, g))
    ranges = [(a, min(g, a + per)) for a in range(0, g, per)]
    if len(ranges) <= 1:
        for a, b in ranges:
            fn(a, b)
        return
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda r: fn(*r), ranges))


def _height_grid(g: int, h: float, seed: int, extent, amplitude, wavelength,
                 octaves, persistence) -> np.ndarray:
    """Value noise at the g x g cell centres ((i + 0.5) h, (j + 0.5) h), as a
    float32 (row j, column i) array.  Bilinear lattice interpolation is
    separable, so each octave is one interpolation along x on the lattice
    rows followed by a row gather along y."""
    c = (np.arange(g, dtype=np.float64) + 0.5) * h
    z = np.zeros((g, g), np.float32)
    amp, total = 1.0, 0.0
    for k in range(octaves):
        lam = wavelength / (2 ** k)
        nodes = int(math.ceil(extent / lam)) + 2
        lat = _lattice(nodes, nodes, k, seed)
        u = c / lam
        iu = np.clip(np.floor(u).astype(np.int64), 0, nodes - 2)
        t = _smooth(u - iu)
        rows = (lat[:, iu] * (1 - t)[None, :] + lat[:, iu + 1] * t[None, :]).astype(np.float32)
        w1 = (amp * t).astype(np.float32)[:, None]
        w0 = (amp * (1 - t)).astype(np.float32)[:, None]

        def add_rows(a, b, rows=rows, iu=iu, w0=w0, w1=w1):
            z[a:b] += rows[iu[a:b]] * w0[a:b]
            z[a:b] += rows[iu[a:b] + 1] * w1[a:b]
        _chunked_rows(g, add_rows)
        total += amp
        amp *= persistence
    z *= np.float32(amplitude / total)
    return z


def _compact_table() -> np.ndarray:
    """Even bits of every 16-bit value, packed into 8 bits."""
    v = np.arange(1 << 16, dtype=np.uint32)
    out = np.zeros(1 << 16, np.uint32)
    for b in range(8):
        out |= ((v >> np.uint32(2 * b)) & np.uint32(1)) << np.uint32(b)
    return out


_COMPACT = _compact_table()


def _compact1by1(v: np.ndarray) -> np.ndarray:
    """Even bits of v (uint32, at most 32 bits), packed: the x part of a Z code."""
    t = _COMPACT
    return t[v & np.uint32(0xFFFF)] | (t[v >> np.uint32(16)] << np.uint32(8))


_BLOCK_BITS = 8   # Z order in blocks of 256 x 256 cells


def _block_pattern():
    """Z order inside one 256 x 256 block: the cell (i, j) of every code."""
    code = np.arange(1 << (2 * _BLOCK_BITS), dtype=np.uint32)
    return (_compact1by1(code).astype(np.int32),
            _compact1by1(code >> np.uint32(1)).astype(np.int32))


def _morton_cells(g: int, n: int):
    """The first n cells of a g x g grid in Z (Morton) order, as (i, j).

    A Z code splits into the code of a 256 x 256 block (high bits) and the
    code inside the block (low bits), so the order is: blocks in Z order of
    their block coordinates, each block's cells in the fixed in-block Z
    order, cells outside the grid dropped."""
    k = max(1, int(math.ceil(math.log2(g))))
    if k > 16:
        raise ValueError("grid side above 65536")
    side = 1 << _BLOCK_BITS
    nb = (g + side - 1) // side                      # blocks per axis
    bcode = np.arange(1 << (2 * max(0, k - _BLOCK_BITS)), dtype=np.uint32)
    bi, bj = _compact1by1(bcode), _compact1by1(bcode >> np.uint32(1))
    keep = (bi < nb) & (bj < nb)
    bi, bj = bi[keep].astype(np.int64), bj[keep].astype(np.int64)
    pi, pj = _block_pattern()
    out_i, out_j, have = [], [], 0
    step = max(1, (1 << 26) // pi.size)              # blocks per piece
    for b0 in range(0, bi.size, step):
        i = (bi[b0:b0 + step, None] * side + pi[None, :]).ravel()
        j = (bj[b0:b0 + step, None] * side + pj[None, :]).ravel()
        inside = (i < g) & (j < g)
        if not inside.all():
            i, j = i[inside], j[inside]
        out_i.append(i)
        out_j.append(j)
        have += i.size
        if have >= n:
            break
    return np.concatenate(out_i)[:n], np.concatenate(out_j)[:n]


_RAMP_T = np.array([0.0, 0.35, 0.7, 1.0])
_RAMP_C = np.array([[40, 90, 30], [110, 160, 60], [140, 110, 70], [225, 222, 212]], np.float64)


def _pack_rgb(r, g, b) -> np.ndarray:
    return (r.astype(np.uint32) | (g.astype(np.uint32) << np.uint32(8))
            | (b.astype(np.uint32) << np.uint32(16)))


def terrain(n: int, seed: int, extent=1000.0, amplitude=50.0, wavelength=200.0,
            octaves=6, persistence=0.5, jitter=0.02, order="morton") -> Cloud:
    """LIDAR-like terrain: a jittered g x g grid over extent x extent metres
    (g = ceil(sqrt(n)), spacing h = extent / g), height = fractal value noise,
    Gaussian jitter of jitter*h on x, y and z, colour = height ramp plus
    uniform noise in [-12, 12] per channel.  ``order="morton"`` delivers the
    first n grid cells in Z order; ``"shuffled"`` then permutes them."""
    n = int(n)
    rng = np.random.default_rng([seed, 0x7E77A1])
    g = max(1, int(math.ceil(math.sqrt(n))))
    h = extent / g

    def draws():
        # the random draws, in their fixed order (one stream), made on a
        # thread of their own while the grid and the cell order are computed
        j = [rng.standard_normal(n, dtype=np.float32) for _ in range(3)]
        return j, [rng.integers(-12, 13, size=n, dtype=np.int16) for _ in range(3)]
    with ThreadPoolExecutor(1) as ex:
        pending = ex.submit(draws)
        zg = _height_grid(g, h, seed, extent, amplitude, wavelength, octaves, persistence)
        ci, cj = _morton_cells(g, n)
        (jx, jy, jz), noise = pending.result()
    sig = np.float32(jitter * h)
    x = np.empty(n, np.float32)
    y = np.empty(n, np.float32)
    z = np.empty(n, np.float32)
    rgb = np.empty(n, np.uint32)
    lo, hi = -amplitude, amplitude
    hf = np.float32(h)

    def fill(a, b):
        x[a:b] = (ci[a:b].astype(np.float32) + np.float32(0.5)) * hf + jx[a:b] * sig
        y[a:b] = (cj[a:b].astype(np.float32) + np.float32(0.5)) * hf + jy[a:b] * sig
        zc = zg[cj[a:b], ci[a:b]]
        z[a:b] = zc + jz[a:b] * sig
        tn = np.clip((zc.astype(np.float64) - lo) / (hi - lo), 0.0, 1.0)
        chans = []
        for ch in range(3):
            base = np.interp(tn, _RAMP_T, _RAMP_C[:, ch])
            chans.append(np.clip(np.rint(base) + noise[ch][a:b], 0, 255).astype(np.uint8))
        rgb[a:b] = _pack_rgb(*chans)
    _chunked(n, fill)
    del zg, jx, jy, jz, noise, ci, cj
    c = Cloud(x, y, z, rgb, f"terrain{n}")
    if order == "shuffled":
        c = shuffle(c, seed)
    return c


def spheres(n: int, seed: int, count=8, rmin=0.1, rmax=0.5, box=1.0) -> Cloud:
    """n points uniformly distributed over the surfaces of ``count`` spheres
    (radius U[rmin, rmax], centre U[0, box]^3).  The sphere of each point is
    drawn with probability proportional to r^2 (uniform area density), its
    direction is a normalised N(0, I3) sample, its colour uniform RGB8.
    Points are i.i.d., so the cloud is in random order."""
    n = int(n)
    rng = np.random.default_rng([seed, 0x5B4E7E])
    centres = rng.uniform(0.0, box, size=(count, 3))
    radii = rng.uniform(rmin, rmax, size=count)
    p = radii ** 2
    which = rng.choice(count, size=n, p=p / p.sum())
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pos = centres[which] + radii[which, None] * d
    col = rng.integers(0, 256, size=(n, 3), dtype=np.uint16)
    return Cloud(np.ascontiguousarray(pos[:, 0], np.float32),
                 np.ascontiguousarray(pos[:, 1], np.float32),
                 np.ascontiguousarray(pos[:, 2], np.float32),
                 _pack_rgb(col[:, 0], col[:, 1], col[:, 2]), f"spheres{n}")


def _morton3_order(x, y, z) -> np.ndarray:
    """Permutation sorting points by a 3D Morton code (21 bits per axis)."""
    def spread(v):
        v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v
    q = []
    for a in (x, y, z):
        a = a.astype(np.float64)
        lo, hi = a.min(), a.max()
        q.append(np.floor((a - lo) / max(hi - lo, 1e-30) * ((1 << 21) - 1)))
    code = spread(q[0]) | (spread(q[1]) << np.uint64(1)) | (spread(q[2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


def buildings(count: int, per: int, seed: int, extent=1000.0, rmin=10.0, rmax=40.0,
              terrain_seed=None, **terrain_kw) -> Cloud:
    """``count`` dense spheres ("buildings") of ``per`` points each, radius
    U[rmin, rmax], standing on the terrain surface; each sphere's points are
    in 3D Morton order, spheres one after another."""
    rng = np.random.default_rng([seed, 0xB01D])
    cx = rng.uniform(0.1 * extent, 0.9 * extent, count)
    cy = rng.uniform(0.1 * extent, 0.9 * extent, count)
    r = rng.uniform(rmin, rmax, count)
    ground = terrain_height(cx, cy, seed if terrain_seed is None else terrain_seed,
                            extent=extent, **terrain_kw)

    def one(b):   # each sphere from its own seed: built on a thread pool
        s = spheres(per, seed * 1000 + b, count=1, rmin=1.0, rmax=1.0, box=0.0)
        x = (s.x.astype(np.float64) * r[b] + cx[b]).astype(np.float32)
        y = (s.y.astype(np.float64) * r[b] + cy[b]).astype(np.float32)
        z = (s.z.astype(np.float64) * r[b] + ground[b] + 0.5 * r[b]).astype(np.float32)
        o = _morton3_order(x, y, z)
        return Cloud(x[o], y[o], z[o], s.rgb[o])
    with ThreadPoolExecutor(_threads()) as ex:
        parts = list(ex.map(one, range(count)))
    return concat(parts, f"buildings{count}x{per}")


def concat(parts, name="") -> Cloud:
    return Cloud(np.concatenate([p.x for p in parts]), np.concatenate([p.y for p in parts]),
                 np.concatenate([p.z for p in parts]), np.concatenate([p.rgb for p in parts]), name)


def shuffle(c: Cloud, seed: int) -> Cloud:
    perm = np.random.default_rng([seed, 0x5F0FF1E]).permutation(c.n)
    out = c.take(perm)
    out.name = c.name + "-shuffled"
    return out


def orbit_views(count: int, seed: int, sizes, extent=1000.0, rmin=600.0, rmax=1200.0,
                elev=(20.0, 60.0), fovy=60.0, near=0.5, far=4000.0):
    """Cameras on a random orbit around the terrain centre: radius
    U[rmin, rmax], azimuth U[0, 2 pi), elevation U[elev], resolution drawn
    uniformly from ``sizes``."""
    rng = np.random.default_rng([seed, 0x0B17])
    views = []
    c = np.array([extent / 2, extent / 2, 0.0])
    for _ in range(count):
        rad = rng.uniform(rmin, rmax)
        az = rng.uniform(0.0, 2 * math.pi)
        el = math.radians(rng.uniform(*elev))
        w, h = sizes[int(rng.integers(0, len(sizes)))]
        eye = c + rad * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az),
                                  math.sin(el)])
        views.append(make_view(eye, c, (0, 0, 1), fovy, w, h, near, far))
    return views


def terrain_view(width=1920, height=1080, extent=1000.0, distance=1000.0,
                 elevation_deg=45.0, fovy=60.0, near=0.5, far=4000.0) -> View:
    """Oblique camera looking at the terrain centre from the south."""
    c = np.array([extent / 2, extent / 2, 0.0])
    el = math.radians(elevation_deg)
    eye = c + distance * np.array([0.0, -math.cos(el), math.sin(el)])
    return make_view(eye, c, (0, 0, 1), fovy, width, height, near, far)


def config1(seed: int = CONFIG_SEEDS[1], n: int = 1_000_000):
    """1M points on 8 random spheres; 1024x768 camera (fov 60, near 0.01,
    far 10) at (0.5, 0.5, 2.5) looking at the unit-cube centre."""
    cloud = spheres(n, seed)
    view = make_view((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, 1024, 768, 0.01, 10.0)
    return cloud, view


def config2(seed: int = CONFIG_SEEDS[2], n: int = 50_000_000):
    """50M-point Morton-ordered terrain, 1920x1080 oblique camera."""
    return terrain(n, seed), terrain_view()


def config3(seed: int = CONFIG_SEEDS[3], n_terrain: int = 250_000_000,
            n_buildings: int = 20, per_building: int = 2_500_000, order="morton"):
    """Contention stress cloud: dense terrain plus dense spheres."""
    t = terrain(n_terrain, seed)
    b = buildings(n_buildings, per_building, seed, terrain_seed=seed)
    c = concat([t, b], f"stress{t.n + b.n}")
    del t, b
    if order == "shuffled":
        c = shuffle(c, seed)
    return c, [terrain_view(2560, 1440), terrain_view(640, 360)]


# --------------------------------------------------------------------------
# serving workload: resident clouds and request traces
# --------------------------------------------------------------------------

SERVE_SIZES = [(256, 256), (640, 480), (1280, 720), (1920, 1080), (2560, 1440)]
SERVE_CLOUDS = [1_000_000, 5_000_000, 20_000_000, 50_000_000, 100_000_000, 150_000_000,
                200_000_000, 300_000_000]


def serve_cloud(i: int, n: int) -> Cloud:
    """Cloud i of the serving workload: the sphere generator for the first
    (1M points), the stress generator (terrain plus dense spheres) for a
    300M-point cloud, terrain otherwise."""
    if i == 0:
        return config1(n=n)[0]
    if n == 300_000_000:
        return config3()[0]
    return terrain(n, CONFIG_SEEDS[5] * 10 + i)


def request_trace(count: int, rate: float, seed: int, nclouds: int, sizes=SERVE_SIZES):
    """Poisson arrivals at `rate` per second: a list of (arrival time in s,
    cloud index, view, mode).  Each request picks a cloud, a resolution, a
    method (0 atomicMin, 1 splatting) and a random orbit camera uniformly;
    cloud 0 (the spheres in the unit cube) gets a close orbit of its own."""
    rng = np.random.default_rng([seed, int(rate)])
    arrivals = np.cumsum(rng.exponential(1.0 / rate, count))
    out = []
    for i in range(count):
        c = int(rng.integers(0, nclouds))
        w, h = sizes[int(rng.integers(0, len(sizes)))]
        if c == 0:
            v = orbit_views(1, int(rng.integers(1 << 30)), [(w, h)], extent=1.0, rmin=1.5,
                            rmax=3.0, elev=(-60.0, 60.0), near=0.01, far=10.0)[0]
        else:
            v = orbit_views(1, int(rng.integers(1 << 30)), [(w, h)])[0]
        out.append((float(arrivals[i]), c, v, int(rng.integers(0, 2))))
    return out
