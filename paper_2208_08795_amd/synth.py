"""Seeded synthetic point clouds (NumPy only; no sampling arithmetic here).

These stand in for the paper's inputs, which are not available here: the
ShapeNet / ModelNet40 / S3DIS objects of its PointNet++ tasks (Table I:
1024-4096 points per normalised object) and real LiDAR scans (Sec. III-A: a
rotating LiDAR's firing order leaves a cloud approximately sorted).  No item of
those datasets is reproduced; every cloud is drawn from a seeded generator.

Generators:
  * ``uniform_cube``      -- points uniform in [0,1)^3, sorted by x;
  * ``object_cloud``      -- the surfaces of 1-4 random primitives (box,
    sphere, cylinder), normalised to the unit sphere, sorted by x and then
    approximately sorted (shuffled inside consecutive bins of ``window``);
  * ``lidar_scan``        -- a synthetic 64-beam rotating sensor over a ground
    plane, 20 random boxes and an enclosing wall, stored in firing order
    (column-major, so the cloud is approximately sorted by azimuth);
  * ``batch_of_objects``  -- many object clouds of log-uniform size;
  * ``frame_stream``      -- LiDAR frames of uniform random size with Poisson
    arrival times, for the serving loop.

All coordinates are float32, C-contiguous, shape (N, 3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _rng(seed) -> np.random.Generator:
    return seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)


def approx_sort(points: np.ndarray, key: np.ndarray, window: int, rng) -> np.ndarray:
    """Stable sort by ``key``, then shuffle inside consecutive bins of ``window``.

    Every point of a later bin has a key >= every point of an earlier bin, and
    points inside a bin are in random order: the paper's definition of an
    approximately sorted cloud (Sec. IV-B, footnote; it uses bins of 128).
    ``window`` <= 1 gives the exact sort.
    """
    rng = _rng(rng)
    order = np.argsort(key, kind="stable")
    if window > 1:
        n = order.shape[0]
        for lo in range(0, n, window):
            seg = order[lo:lo + window]
            order[lo:lo + window] = seg[rng.permutation(seg.shape[0])]
    return np.ascontiguousarray(points[order], dtype=np.float32)


def uniform_cube(n: int = 2048, seed=0) -> np.ndarray:
    """n points uniform in the unit cube, sorted ascending by x."""
    rng = _rng(seed)
    p = rng.random((n, 3), dtype=np.float32)
    return np.ascontiguousarray(p[np.argsort(p[:, 0], kind="stable")])


def _random_rotation(rng) -> np.ndarray:
    """Uniform random rotation from a uniform unit quaternion (Shoemake)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _box_surface(rng, count, ext):
    a, b, c = ext
    faces = np.array([b * c, b * c, a * c, a * c, a * b, a * b])
    f = rng.choice(6, size=count, p=faces / faces.sum())
    u = rng.random((count, 3)) - 0.5
    p = u * np.array([a, b, c])
    axis, sign = f // 2, np.where(f % 2 == 0, -0.5, 0.5)
    p[np.arange(count), axis] = sign * np.array([a, b, c])[axis]
    return p


def _sphere_surface(rng, count, r):
    v = rng.standard_normal((count, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return r * v


def _cylinder_surface(rng, count, r, h):
    side, cap = 2 * math.pi * r * h, math.pi * r * r
    part = rng.choice(3, size=count, p=np.array([side, cap, cap]) / (side + 2 * cap))
    theta = rng.random(count) * 2 * math.pi
    rad = np.where(part == 0, r, r * np.sqrt(rng.random(count)))
    z = np.where(part == 0, (rng.random(count) - 0.5) * h, np.where(part == 1, -h / 2, h / 2))
    return np.stack([rad * np.cos(theta), rad * np.sin(theta), z], axis=1)


def object_cloud(n: int = 8192, seed=0, window: int = 16) -> np.ndarray:
    """Surface samples of 1-4 random primitives, unit-sphere normalised.

    Primitive type is uniform over {box, sphere, cylinder}; extents uniform in
    [0.2, 1.0]; orientation uniform; translation uniform in [-1, 1]^3.  Points
    are distributed over primitives and faces in proportion to surface area,
    then the cloud is centred, scaled to the unit sphere, sorted by x and
    shuffled inside bins of ``window`` positions.
    """
    rng = _rng(seed)
    kinds = rng.integers(0, 3, size=int(rng.integers(1, 5)))
    ext = rng.uniform(0.2, 1.0, size=(kinds.shape[0], 3))
    areas = []
    for t, e in zip(kinds, ext):
        if t == 0:
            areas.append(2 * (e[0] * e[1] + e[1] * e[2] + e[0] * e[2]))
        elif t == 1:
            areas.append(4 * math.pi * (e[0] / 2) ** 2)
        else:
            r = e[0] / 2
            areas.append(2 * math.pi * r * e[2] + 2 * math.pi * r * r)
    areas = np.array(areas)
    counts = rng.multinomial(n, areas / areas.sum())
    parts = []
    for t, e, cnt in zip(kinds, ext, counts):
        rot, shift = _random_rotation(rng), rng.uniform(-1.0, 1.0, size=3)
        if cnt == 0:
            continue
        if t == 0:
            p = _box_surface(rng, cnt, e)
        elif t == 1:
            p = _sphere_surface(rng, cnt, e[0] / 2)
        else:
            p = _cylinder_surface(rng, cnt, e[0] / 2, e[2])
        parts.append(p @ rot.T + shift)
    pts = np.concatenate(parts, axis=0)
    pts -= pts.mean(axis=0)
    pts /= np.linalg.norm(pts, axis=1).max()
    pts = pts.astype(np.float32)
    return approx_sort(pts, pts[:, 0], window, rng)


@dataclass
class LidarScene:
    """Ground plane z=0, axis-aligned boxes resting on it, a cylindrical wall."""
    box_lo: np.ndarray       # (B, 3)
    box_hi: np.ndarray       # (B, 3)
    wall_radius: float = 60.0
    sensor_height: float = 1.8


def lidar_scene(rng, n_boxes: int = 20) -> LidarScene:
    rng = _rng(rng)
    radius = rng.uniform(4.0, 40.0, n_boxes)
    angle = rng.uniform(0.0, 2 * math.pi, n_boxes)
    size = rng.uniform(0.5, 4.0, (n_boxes, 3))
    centre = np.stack([radius * np.cos(angle), radius * np.sin(angle)], axis=1)
    lo = np.concatenate([centre - size[:, :2] / 2, np.zeros((n_boxes, 1))], axis=1)
    hi = np.concatenate([centre + size[:, :2] / 2, size[:, 2:3]], axis=1)
    return LidarScene(lo, hi)


def lidar_scan(columns: int = 512, seed=0, beams: int = 64, n: int | None = None,
               noise: float = 0.02, n_boxes: int = 20,
               scene: LidarScene | None = None) -> np.ndarray:
    """A synthetic rotating-LiDAR frame in firing order.

    ``beams`` elevations evenly spaced over [-25, 3] degrees, ``columns``
    azimuths evenly spaced over 360 degrees, sensor at (0, 0, 1.8 m).  Each ray
    takes its first hit among the ground, the boxes and the wall (every ray
    hits the wall, so the point count is exact), plus Gaussian range noise.
    Point index = column * beams + beam, so the cloud is approximately sorted
    by azimuth.  ``n`` truncates the frame.
    """
    rng = _rng(seed)
    if scene is None:
        scene = lidar_scene(rng, n_boxes)
    el = np.deg2rad(np.linspace(-25.0, 3.0, beams))
    az = 2 * math.pi * np.arange(columns) / columns
    az_g, el_g = np.meshgrid(az, el, indexing="ij")          # (columns, beams)
    d = np.stack([np.cos(el_g) * np.cos(az_g), np.cos(el_g) * np.sin(az_g),
                  np.sin(el_g)], axis=-1).reshape(-1, 3)
    if n is not None:
        d = d[:n]
    origin = np.array([0.0, 0.0, scene.sensor_height])
    horiz = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
    t = scene.wall_radius / horiz
    down = d[:, 2] < 0
    t[down] = np.minimum(t[down], scene.sensor_height / -d[down, 2])
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        for lo, hi in zip(scene.box_lo, scene.box_hi):
            t0 = (lo - origin) * inv
            t1 = (hi - origin) * inv
            tmin = np.nanmax(np.minimum(t0, t1), axis=1)
            tmax = np.nanmin(np.maximum(t0, t1), axis=1)
            hit = (tmax >= np.maximum(tmin, 0.0)) & (tmin > 0.0)
            t[hit] = np.minimum(t[hit], tmin[hit])
    r = t + rng.normal(0.0, noise, t.shape[0])
    pts = origin + r[:, None] * d
    return np.ascontiguousarray(pts, dtype=np.float32)


def batch_of_objects(count: int = 256, seed=0, n_min: int = 1024, n_max: int = 32768,
                     window: int = 16):
    """``count`` object clouds with N log-uniform in [n_min, n_max]."""
    rng = _rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), count))).astype(int)
    sizes = np.clip(sizes, n_min, n_max)
    seeds = rng.integers(0, 2**63 - 1, count)
    return [object_cloud(int(nn), int(s), window) for nn, s in zip(sizes, seeds)]


@dataclass
class Frame:
    points: np.ndarray
    c: int
    m: int
    k: int
    start: int
    arrival: float            # seconds from the start of the stream


def frame_stream(rate: float, count: int, seed=0, n_min: int = 16384, n_max: int = 131072,
                 ms=(8, 16, 32), k: int = 64, c_div: int = 8, beams: int = 64):
    """LiDAR frames of N uniform in [n_min, n_max] with Poisson arrivals."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    frames = []
    for i in range(count):
        n = int(rng.integers(n_min, n_max + 1))
        cols = -(-n // beams)
        pts = lidar_scan(cols, int(rng.integers(0, 2**63 - 1)), beams=beams, n=n)
        m = int(rng.choice(np.asarray(ms)))
        frames.append(Frame(pts, n // c_div, m, k, 0, float(arrivals[i])))
    return frames
