"""Seeded synthetic point clouds shared by the oracle tests, the GPU tests and the bench.

This module only draws coordinates. It holds none of the sampler's arithmetic, so both
the CPU oracle and the HIP path can be fed identical bytes from it.

The shapes follow the workloads the paper evaluates on (KITTI-like 16,384-point scenes,
64-beam LiDAR sweeps, and large indoor/outdoor scenes, Sec. 4.1 and Fig. 5/7); the
datasets themselves are not used. Every generator returns a C-contiguous float32 array
of shape [N, 3].
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "uniform_box_with_ground",
    "lidar_scan",
    "scene_planes_blobs",
    "batch_lidar_clouds",
    "serving_trace",
    "lattice",
    "random_cloud",
]


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1, 3))


def uniform_box_with_ground(n: int = 16384, seed: int = 1) -> np.ndarray:
    """Half the points uniform in a 70 x 80 x 4 m box (x in [0,70), y in [-40,40),
    z in [-3,1)), half uniform on the ground plane z = -1.7 over the same x-y
    rectangle, shuffled. KITTI-scale scene (16,384 points)."""
    rng = np.random.default_rng(seed)
    h = n // 2
    box = np.empty((h, 3))
    box[:, 0] = rng.uniform(0.0, 70.0, h)
    box[:, 1] = rng.uniform(-40.0, 40.0, h)
    box[:, 2] = rng.uniform(-3.0, 1.0, h)
    g = n - h
    ground = np.empty((g, 3))
    ground[:, 0] = rng.uniform(0.0, 70.0, g)
    ground[:, 1] = rng.uniform(-40.0, 40.0, g)
    ground[:, 2] = -1.7
    pts = np.concatenate([box, ground])
    pts = pts[rng.permutation(n)]
    return _f32(pts)


def _lidar_boxes(rng, n_boxes: int):
    """Axis-aligned boxes resting on z = 0: centres uniform in [-40,40]^2 outside a
    3 m radius around the sensor, footprint sides U[1,8] m, heights U[1,4] m."""
    lo = np.empty((n_boxes, 3))
    hi = np.empty((n_boxes, 3))
    k = 0
    while k < n_boxes:
        c = rng.uniform(-40.0, 40.0, 2)
        if math.hypot(c[0], c[1]) < 3.0:
            continue
        sx, sy = rng.uniform(1.0, 8.0, 2)
        h = rng.uniform(1.0, 4.0)
        lo[k] = (c[0] - sx / 2, c[1] - sy / 2, 0.0)
        hi[k] = (c[0] + sx / 2, c[1] + sy / 2, h)
        k += 1
    return lo, hi


def _cast_rays(rng, n_azimuth: int, n_beams: int, boxes, sensor_h: float,
               max_range: float, noise_sigma: float) -> np.ndarray:
    """Nearest hit of each ray against the ground plane z = 0 and the boxes; misses
    are dropped; Gaussian range noise along the ray. Azimuth-major order."""
    elev = np.deg2rad(np.linspace(-24.8, 2.0, n_beams))
    az = 2.0 * np.pi * np.arange(n_azimuth) / n_azimuth
    # azimuth-major: all beams of azimuth step 0, then step 1, ...
    A, E = np.meshgrid(az, elev, indexing="ij")
    d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1).reshape(-1, 3)
    o = np.array([0.0, 0.0, sensor_h])
    t = np.full(d.shape[0], np.inf)
    # ground plane
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = -o[2] / d[:, 2]
    tg[~(d[:, 2] < 0)] = np.inf
    t = np.minimum(t, tg)
    lo, hi = boxes
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
    for b in range(lo.shape[0]):
        t1 = (lo[b] - o) * inv
        t2 = (hi[b] - o) * inv
        tmin = np.nanmax(np.minimum(t1, t2), axis=1)
        tmax = np.nanmin(np.maximum(t1, t2), axis=1)
        hit = (tmax >= np.maximum(tmin, 0.0))
        tb = np.where(hit, np.maximum(tmin, 0.0), np.inf)
        t = np.minimum(t, tb)
    keep = np.isfinite(t) & (t <= max_range) & (t > 0)
    r = t[keep] + rng.normal(0.0, noise_sigma, int(keep.sum()))
    return o + d[keep] * r[:, None]


def lidar_scan(seed: int = 2, n_azimuth: int = 2048, n_beams: int = 64,
               n_boxes: int = 30) -> np.ndarray:
    """Synthetic 64-beam LiDAR sweep: sensor at (0, 0, 1.8 m), elevations
    linspace(-24.8 deg, +2 deg, 64), n_azimuth steps of 2*pi/n_azimuth, a z = 0 ground
    plane plus 30 seeded boxes, range noise sigma = 2 cm, max range 120 m."""
    rng = np.random.default_rng(seed)
    boxes = _lidar_boxes(rng, n_boxes)
    return _f32(_cast_rays(rng, n_azimuth, n_beams, boxes, 1.8, 120.0, 0.02))


def scene_planes_blobs(n: int = 1 << 20, seed: int = 3, n_planes: int = 6,
                       n_blobs: int = 200, size=(50.0, 50.0, 10.0),
                       plane_frac: float = 0.4) -> np.ndarray:
    """Scene-scale cloud in a 50 x 50 x 10 m volume: 40 % of the points on 6 random
    planes (random unit normal through a uniform point; uniform volume samples
    projected onto the plane, rejected when outside the volume), 60 % in 200
    Gaussian blobs with per-axis sigma ~ U[0.05, 1] m, equal shares. Globally
    shuffled, so the index order carries no locality."""
    rng = np.random.default_rng(seed)
    size = np.asarray(size, dtype=np.float64)
    n_plane = int(round(n * plane_frac))
    n_blob = n - n_plane
    parts = []
    per_plane = [n_plane // n_planes + (1 if i < n_plane % n_planes else 0) for i in range(n_planes)]
    for cnt in per_plane:
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        p0 = rng.uniform(0.0, 1.0, 3) * size
        got = []
        have = 0
        while have < cnt:
            q = rng.uniform(0.0, 1.0, (max(2 * (cnt - have), 1024), 3)) * size
            q = q - ((q - p0) @ nrm)[:, None] * nrm[None, :]
            ok = np.all((q >= 0.0) & (q < size), axis=1)
            q = q[ok][: cnt - have]
            got.append(q)
            have += q.shape[0]
        parts.append(np.concatenate(got) if got else np.zeros((0, 3)))
    per_blob = [n_blob // n_blobs + (1 if i < n_blob % n_blobs else 0) for i in range(n_blobs)]
    centres = rng.uniform(0.0, 1.0, (n_blobs, 3)) * size
    sig = rng.uniform(0.05, 1.0, (n_blobs, 3))
    for b, cnt in enumerate(per_blob):
        parts.append(centres[b] + rng.normal(size=(cnt, 3)) * sig[b])
    pts = np.concatenate(parts)
    pts = pts[rng.permutation(n)]
    return _f32(pts)


def batch_lidar_clouds(n_clouds: int = 64, seed0: int = 1000, n_min: int = 20000,
                       n_max: int = 200000, ratio: int = 4):
    """Uneven LiDAR-shaped clouds: cloud i uses seed seed0 + i, N_i ~ U{n_min..n_max},
    generated as lidar_scan with ceil(N_i / (64 * 0.85)) azimuth steps (more if the
    sweep has fewer hits), keeping the first N_i hits; M_i = N_i // ratio."""
    clouds, ms = [], []
    for i in range(n_clouds):
        rng = np.random.default_rng(seed0 + i)
        n_i = int(rng.integers(n_min, n_max + 1))
        az = int(math.ceil(n_i / (64 * 0.85)))
        boxes = _lidar_boxes(rng, 30)
        while True:
            pts = _cast_rays(rng, az, 64, boxes, 1.8, 120.0, 0.02)
            if pts.shape[0] >= n_i:
                break
            if pts.shape[0] < az * 64 // 4:
                boxes = _lidar_boxes(rng, 30)  # a box encloses the sensor
            else:
                az = int(math.ceil(az * 1.25))
        clouds.append(_f32(pts[:n_i]))
        ms.append(n_i // ratio)
    return clouds, ms


def lidar_points(n: int, seed: int = 0, beams: int = 64):
    """A LiDAR-shaped sweep (as lidar_scan: ground, 30 boxes, 64 beams) with exactly n
    points: ceil(n / (beams * 0.85)) azimuth steps (more if the sweep has fewer hits),
    the first n hits kept (azimuth-major order). Boxes are drawn again if one encloses
    the sensor (then no ray leaves it)."""
    rng = np.random.default_rng(seed)
    az = int(math.ceil(n / (beams * 0.85)))
    boxes = _lidar_boxes(rng, 30)
    while True:
        pts = _cast_rays(rng, az, beams, boxes, 1.8, 120.0, 0.02)
        if pts.shape[0] >= n:
            return _f32(pts[:n])
        if pts.shape[0] < az * beams // 4:
            boxes = _lidar_boxes(rng, 30)  # a box encloses the sensor: every ray is lost
        else:
            az = int(math.ceil(az * 1.25))


def serving_trace(n_requests: int = 10000, rate_hz: float = 2000.0, seed: int = 7,
                  median_n: float = 1e5, sigma_ln: float = 1.0, n_lo: int = 1024,
                  n_hi: int = 2097152):
    """Poisson arrival trace: exponential inter-arrival times at rate_hz; N lognormal
    around median_n (clamped to [n_lo, n_hi]); kind 0 = LiDAR-like, 1 = scene-like with
    probability 1/2; M = N/4 or N/16 with probability 1/2. Returns a dict of arrays."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps)
    n = np.clip(np.round(np.exp(rng.normal(math.log(median_n), sigma_ln, n_requests))),
                n_lo, n_hi).astype(np.int64)
    kind = rng.integers(0, 2, n_requests)
    div = np.where(rng.integers(0, 2, n_requests) == 0, 4, 16)
    m = np.maximum(n // div, 1)
    return {"t_arrival": t, "n": n, "m": m, "kind": kind}


def serving_bases(n_max: int = 1 << 21):
    """The two base clouds the serving requests are windows of: a LiDAR sweep (seed 32,
    azimuth-major, so a window of consecutive points is a sector) and a scene cloud
    (seed 31, shuffled), each of n_max points."""
    scene = scene_planes_blobs(n_max, seed=31)
    lidar = lidar_scan(seed=32, n_azimuth=int(math.ceil(n_max / (64 * 0.85))) + 2048)[:n_max]
    return [np.ascontiguousarray(lidar), np.ascontiguousarray(scene)]


def serving_windows(trace, n_base: int, seed: int = 8):
    """Start offset of each request's window in its base cloud (uniform over the
    windows that fit)."""
    rng = np.random.default_rng(seed)
    return np.array([int(rng.integers(0, n_base - int(n) + 1)) for n in trace["n"]], dtype=np.int64)


def lattice(side: int = 8) -> np.ndarray:
    """Integer lattice {0..side-1}^3; point (x, y, z) has index x + side*y + side^2*z."""
    z, y, x = np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij")
    return _f32(np.stack([x.ravel(), y.ravel(), z.ravel()], -1))


def random_cloud(n: int, seed: int, scale: float = 10.0, kind: str = "uniform") -> np.ndarray:
    """Small generic clouds for tests: 'uniform' in a cube, 'clustered' around a few
    centres, 'quantised' on a 0.25 m grid (many exact duplicates and boundary hits)."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        p = rng.uniform(0.0, scale, (n, 3))
    elif kind == "clustered":
        c = rng.uniform(0.0, scale, (max(1, n // 50), 3))
        p = c[rng.integers(0, c.shape[0], n)] + rng.normal(0.0, scale * 0.02, (n, 3))
    elif kind == "quantised":
        p = np.floor(rng.uniform(0.0, scale, (n, 3)) * 4.0) / 4.0
    else:
        raise ValueError(kind)
    return _f32(p)
