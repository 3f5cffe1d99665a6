"""Seeded synthetic point clouds standing in for the paper's benchmark scans.

The paper measures on S3DIS / ScanNet rooms and SemanticKITTI Velodyne scans
(Sec. 5.1, Sec. 5.6), none of which are available here.  These generators
produce clouds with the same shape: indoor rooms of tens of thousands of
points sampled on planar and curved surfaces, and spinning-LiDAR sweeps of
~100k (64 beams) up to ~1M (128 beams) points in azimuth-major order.

This module holds only input generation.  It contains none of the sampling
method's arithmetic and is shared by the oracle side and the device side.
Everything is drawn with numpy PCG64 ``default_rng`` in float64 and cast to
float32 at the end, so the same seed gives the same bytes on every machine.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

__all__ = [
    "cube", "room", "lidar", "dense_lidar", "lidar_stage_sizes", "batch",
    "fingerprint", "ROOM_N", "LIDAR_N", "DENSE_N",
]

ROOM_N = 80_000
LIDAR_N = 114_624          # 64 beams x 1800 azimuth steps minus 576 dropped returns
DENSE_N = 1_048_576        # 128 beams x 8192 azimuth steps, nothing dropped


def fingerprint(xyz: np.ndarray) -> str:
    """SHA-256 of the little-endian float32 bytes of a cloud."""
    a = np.ascontiguousarray(xyz, dtype="<f4")
    return hashlib.sha256(a.tobytes()).hexdigest()


def cube(seed: int = 0, n: int = 4096) -> np.ndarray:
    """``n`` points uniform in the unit cube [0,1)^3, float32 [n,3]."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.random((n, 3), dtype=np.float32))


# ----------------------------------------------------------------------------
# Indoor room: floor, ceiling, four walls, boxes resting on the floor, spheres.
# ----------------------------------------------------------------------------

def _rect(rng, n, origin, u, v):
    """n points uniform on the parallelogram origin + a*u + b*v, a,b in [0,1)."""
    ab = rng.random((n, 2))
    return origin[None, :] + ab[:, :1] * u[None, :] + ab[:, 1:] * v[None, :]


def room(seed: int = 0, n: int = ROOM_N, size=(10.0, 8.0, 3.0), n_boxes: int = 20,
         n_spheres: int = 10, noise: float = 0.005) -> np.ndarray:
    """Room-like cloud of exactly ``n`` float32 points.

    A ``size`` box room (floor, ceiling and four walls), ``n_boxes``
    axis-aligned boxes with sides U[0.3, 2] m resting on the floor (five
    faces each, the bottom is hidden), ``n_spheres`` spheres with radius
    U[0.2, 0.8] m fully inside the room.  Point counts per surface are
    multinomial in the surface areas; points are uniform on each surface with
    iid N(0, noise^2) jitter per coordinate; the result is shuffled.
    """
    rng = np.random.default_rng(seed)
    W, D, H = size
    surfaces = []  # (area, sampler(k) -> [k,3])

    def add_rect(origin, u, v):
        o, uu, vv = (np.asarray(t, dtype=np.float64) for t in (origin, u, v))
        area = float(np.linalg.norm(np.cross(uu, vv)))
        surfaces.append((area, lambda k, o=o, uu=uu, vv=vv: _rect(rng, k, o, uu, vv)))

    add_rect((0, 0, 0), (W, 0, 0), (0, D, 0))        # floor
    add_rect((0, 0, H), (W, 0, 0), (0, D, 0))        # ceiling
    add_rect((0, 0, 0), (0, D, 0), (0, 0, H))        # wall x = 0
    add_rect((W, 0, 0), (0, D, 0), (0, 0, H))        # wall x = W
    add_rect((0, 0, 0), (W, 0, 0), (0, 0, H))        # wall y = 0
    add_rect((0, D, 0), (W, 0, 0), (0, 0, H))        # wall y = D

    for _ in range(n_boxes):
        sx, sy, sz = rng.uniform(0.3, 2.0, size=3)
        x0 = rng.uniform(0.0, W - sx)
        y0 = rng.uniform(0.0, D - sy)
        add_rect((x0, y0, sz), (sx, 0, 0), (0, sy, 0))        # top
        add_rect((x0, y0, 0), (0, sy, 0), (0, 0, sz))         # -x side
        add_rect((x0 + sx, y0, 0), (0, sy, 0), (0, 0, sz))    # +x side
        add_rect((x0, y0, 0), (sx, 0, 0), (0, 0, sz))         # -y side
        add_rect((x0, y0 + sy, 0), (sx, 0, 0), (0, 0, sz))    # +y side

    for _ in range(n_spheres):
        r = rng.uniform(0.2, 0.8)
        c = np.array([rng.uniform(r, W - r), rng.uniform(r, D - r), rng.uniform(r, H - r)])

        def sph(k, c=c, r=r):
            v = rng.normal(size=(k, 3))
            v /= np.linalg.norm(v, axis=1, keepdims=True)
            return c[None, :] + r * v

        surfaces.append((4.0 * math.pi * r * r, sph))

    areas = np.array([a for a, _ in surfaces])
    counts = rng.multinomial(n, areas / areas.sum())
    parts = [f(int(k)) for (_, f), k in zip(surfaces, counts) if k > 0]
    pts = np.concatenate(parts, axis=0)
    pts += rng.normal(0.0, noise, size=pts.shape)
    pts = pts[rng.permutation(n)]
    return np.ascontiguousarray(pts.astype(np.float32))


# ----------------------------------------------------------------------------
# Spinning LiDAR: ray cast from the origin against ground, boxes and a far wall.
# ----------------------------------------------------------------------------

def lidar(seed: int = 0, beams: int = 64, azimuth_steps: int = 1800, drop: int = 576,
          n_boxes: int = 40, ground_z: float = -1.7, wall_range: float = 80.0,
          elev_deg=(-25.0, 3.0), range_noise: float = 0.02,
          n_out: int | None = None) -> np.ndarray:
    """LiDAR-like sweep as float32 [N,3] in azimuth-major order.

    Sensor at the origin; ``beams`` elevations evenly spaced over
    ``elev_deg``; ``azimuth_steps`` evenly spaced azimuths.  Every ray hits
    the nearest of: the ground plane z = ``ground_z``, ``n_boxes``
    axis-aligned boxes (sides U[1,5] m, standing on the ground, centres at
    horizontal range U[5,80] m and uniform azimuth), or a vertical cylinder
    of radius ``wall_range`` around the sensor (so every ray returns).  The
    range gets N(0, range_noise^2) noise along the ray.  Then ``drop``
    returns chosen at random are removed (or, with ``n_out``, exactly enough
    to leave ``n_out`` points); the azimuth-major order is kept.
    """
    rng = np.random.default_rng(seed)
    # scene
    boxes = []
    for _ in range(n_boxes):
        sx, sy, sz = rng.uniform(1.0, 5.0, size=3)
        rr = rng.uniform(5.0, 80.0)
        th = rng.uniform(0.0, 2.0 * math.pi)
        cx, cy = rr * math.cos(th), rr * math.sin(th)
        lo = np.array([cx - sx / 2, cy - sy / 2, ground_z])
        hi = np.array([cx + sx / 2, cy + sy / 2, ground_z + sz])
        boxes.append((lo, hi))
    # rays, azimuth-major: index = a * beams + b
    el = np.deg2rad(np.linspace(elev_deg[0], elev_deg[1], beams))
    az = np.arange(azimuth_steps, dtype=np.float64) * (2.0 * math.pi / azimuth_steps)
    cel, sel = np.cos(el), np.sin(el)
    dx = (np.cos(az)[:, None] * cel[None, :]).ravel()
    dy = (np.sin(az)[:, None] * cel[None, :]).ravel()
    dz = np.broadcast_to(sel[None, :], (azimuth_steps, beams)).ravel().copy()
    nr = dx.size
    # far wall (cylinder) always hit since |elevation| < 90 deg
    t = wall_range / np.sqrt(dx * dx + dy * dy)
    # ground
    down = dz < 0
    tg = np.full(nr, np.inf)
    tg[down] = ground_z / dz[down]
    t = np.minimum(t, tg)
    # boxes (slab method); the sensor is outside every box
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = [1.0 / dx, 1.0 / dy, 1.0 / dz]
        for lo, hi in boxes:
            tn = np.full(nr, -np.inf)
            tf = np.full(nr, np.inf)
            for a, d in enumerate((dx, dy, dz)):
                t1 = lo[a] * inv[a]
                t2 = hi[a] * inv[a]
                par = d == 0.0
                t1 = np.where(par, np.where((lo[a] <= 0) & (0 <= hi[a]), -np.inf, np.inf), t1)
                t2 = np.where(par, np.where((lo[a] <= 0) & (0 <= hi[a]), np.inf, -np.inf), t2)
                tn = np.maximum(tn, np.minimum(t1, t2))
                tf = np.minimum(tf, np.maximum(t1, t2))
            hit = (tn <= tf) & (tn > 0)
            t = np.where(hit & (tn < t), tn, t)
    t = t + rng.normal(0.0, range_noise, size=nr)
    pts = np.stack([t * dx, t * dy, t * dz], axis=1)
    keep_n = nr - drop if n_out is None else n_out
    if keep_n < nr:
        keep = np.sort(rng.choice(nr, size=keep_n, replace=False))
        pts = pts[keep]
    return np.ascontiguousarray(pts.astype(np.float32))


def dense_lidar(seed: int = 0) -> np.ndarray:
    """128 beams x 8192 azimuth steps of the LiDAR scene, nothing dropped (N = 1,048,576)."""
    return lidar(seed, beams=128, azimuth_steps=8192, drop=0)


def lidar_stage_sizes(n: int = LIDAR_N, stages: int = 4):
    """Multi-stage sample counts N -> N/4 -> N/16 -> N/64 as a point backbone runs them."""
    return [n // (4 ** k) for k in range(stages)]


def batch(seed: int = 0, b: int = 32, n_lo: int = 8000, n_hi: int = 120_000):
    """Uneven batch: ``b`` clouds with N_i log-uniform in [n_lo, n_hi].

    Even i: room generator with N_i points; odd i: LiDAR generator with 64
    beams and ceil(N_i / (64 * 0.995)) azimuth steps, randomly thinned to
    exactly N_i.  M_i = N_i // 4.  Returns (xyz float32 [sum N_i, 3],
    offsets int32 [b+1], m int32 [b]).
    """
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=b))).astype(np.int64)
    clouds = []
    for i, ni in enumerate(sizes):
        ni = int(ni)
        sub = [seed, i]
        if i % 2 == 0:
            clouds.append(room(np.random.SeedSequence(sub), n=ni))
        else:
            steps = int(math.ceil(ni / (64 * 0.995)))
            clouds.append(lidar(np.random.SeedSequence(sub), beams=64, azimuth_steps=steps, n_out=ni))
    offsets = np.zeros(b + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(sizes)
    m = (sizes // 4).astype(np.int32)
    xyz = np.ascontiguousarray(np.concatenate(clouds, axis=0).astype(np.float32))
    return xyz, offsets, m
