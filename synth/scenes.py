"""Seeded synthetic scenes: planes-and-spheres, indoor rooms, ray-cast LiDAR.

These stand in for the paper's KITTI / MulRan scans and Kimera-Multi maps
(Section IV-A), which are not available here.  Nothing in this module
computes any part of the registration method; it only draws geometry.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_ROOT = 2409


def rng_for(config: int, item: int = 0, *extra: int) -> np.random.Generator:
    """PCG64 generator seeded from SeedSequence([2409, config, item, ...])."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, config, item, *extra])))


@dataclasses.dataclass(frozen=True)
class Params:
    """Faster-PFH parameters (Section IV-B states them in units of the voxel size v)."""

    voxel: float
    r_normal: float
    r_fpfh: float
    tau_num: int = 3
    tau_lin: float = 0.99
    n_bins: int = 11

    @staticmethod
    def from_voxel(v: float, normal_mult: float = 3.5, fpfh_mult: float = 5.0) -> "Params":
        return Params(voxel=v, r_normal=normal_mult * v, r_fpfh=fpfh_mult * v)


def params_c0() -> Params:
    return Params(voxel=0.05, r_normal=0.10, r_fpfh=0.25)


def params_c1(v: float = 0.3) -> Params:
    return Params(voxel=v, r_normal=3.0 * v, r_fpfh=5.0 * v)


def params_indoor(v: float = 0.025) -> Params:
    return Params.from_voxel(v)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation on SO(3) from a normalised 4-D Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ]
    )


def _soa(points_n3: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(points_n3, dtype=np.float64).T.astype(np.float32))


def _unit_sphere(rng, n):
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# Planes + spheres scene (small single pair)
# ---------------------------------------------------------------------------

def _sphere_centres(rng, k, lo, hi, min_sep):
    centres = []
    while len(centres) < k:
        c = rng.uniform(lo, hi, 3)
        if all(np.linalg.norm(c - o) >= min_sep for o in centres):
            centres.append(c)
    return np.array(centres)


def planes_spheres_scene(rng, n=5000, side=2.0, radius=0.3):
    """Planes x=0, y=0, z=0 over [0, side]^2 plus two spheres, uniform by area."""
    centres = _sphere_centres(rng, 2, 0.45, 1.55, 0.7)
    areas = np.array([side * side] * 3 + [4 * math.pi * radius * radius] * 2)
    which = rng.choice(5, size=n, p=areas / areas.sum())
    pts = np.empty((n, 3))
    for s in range(3):
        idx = np.nonzero(which == s)[0]
        uv = rng.uniform(0.0, side, (idx.size, 2))
        cols = [c for c in range(3) if c != s]
        pts[idx, s] = 0.0
        pts[idx, cols[0]] = uv[:, 0]
        pts[idx, cols[1]] = uv[:, 1]
    for s in range(2):
        idx = np.nonzero(which == 3 + s)[0]
        pts[idx] = centres[s] + radius * _unit_sphere(rng, idx.size)
    return pts


def _make_target(rng, src, outlier_frac, noise_sigma, R, t):
    tgt = src @ R.T + t
    if noise_sigma > 0:
        tgt = tgt + rng.normal(0.0, noise_sigma, tgt.shape)
    n = tgt.shape[0]
    n_out = int(round(outlier_frac * n))
    inlier = np.ones(n, dtype=bool)
    if n_out > 0:
        lo, hi = tgt.min(axis=0), tgt.max(axis=0)
        sel = rng.choice(n, size=n_out, replace=False)
        tgt[sel] = rng.uniform(lo, hi, (n_out, 3))
        inlier[sel] = False
    return tgt, inlier


def c0_pair(item: int = 0) -> dict:
    """Planes+spheres source (5,000 points) and a transformed, noisy, outlier-laden target."""
    rng = rng_for(0, item)
    src = planes_spheres_scene(rng)
    R = random_rotation(rng)
    t = rng.uniform(-1.0, 1.0, 3)
    tgt, inlier = _make_target(rng, src, 0.30, 0.01, R, t)
    vp_src = np.array([3.0, 3.0, 3.0])
    return dict(
        src=_soa(src),
        tgt=_soa(tgt),
        vp_src=vp_src,
        vp_tgt=R @ vp_src + t,
        R=R,
        t=t,
        inlier=inlier,
        params=params_c0(),
        name="planes+spheres 5k",
    )


# ---------------------------------------------------------------------------
# Ray-cast spinning LiDAR
# ---------------------------------------------------------------------------

# HDL-64E-like beam table: 32 beams from +2 deg down in 1/3 deg steps, 32 beams
# from -8.83 deg down in 1/2 deg steps (spans -24.33 .. +2 deg).
HDL64_ELEVATIONS = np.concatenate([2.0 - np.arange(32) / 3.0, -8.83 - 0.5 * np.arange(32)])


def _boxes(rng, n_boxes, sensors_xy, height, r_min=20.0, r_max=70.0):
    """Axis-aligned boxes (sides U[1, 10] m) resting on the ground, centres uniform by
    area in the annulus r_min..r_max around the first sensor."""
    boxes = []
    while len(boxes) < n_boxes:
        size = rng.uniform(1.0, 10.0, 3)
        rad = math.sqrt(rng.uniform(r_min * r_min, r_max * r_max))
        ang = rng.uniform(0.0, 2 * math.pi)
        c = np.array([rad * math.cos(ang), rad * math.sin(ang)])
        lo = np.array([c[0] - size[0] / 2, c[1] - size[1] / 2, 0.0])
        hi = np.array([c[0] + size[0] / 2, c[1] + size[1] / 2, size[2]])
        inside = False
        for s in sensors_xy:
            p = np.array([s[0], s[1], height])
            if np.all(p >= lo - 0.5) and np.all(p <= hi + 0.5):
                inside = True
        if not inside:
            boxes.append((lo, hi))
    return boxes


def lidar_scan(rng, origin, yaw, boxes, n_beams=64, n_az=1875, max_range=100.0, range_sigma=0.02):
    """Ray-cast one spinning-LiDAR sweep; returns points in the sensor frame (n, 3).
    n_beams=64 uses the HDL-64E-like table; other counts interpolate its span."""
    if n_beams == 64:
        el_deg = np.sort(HDL64_ELEVATIONS)
    else:
        el_deg = np.interp(np.linspace(0, 63, n_beams), np.arange(64), np.sort(HDL64_ELEVATIONS))
    el = np.deg2rad(el_deg)
    az = 2 * math.pi * np.arange(n_az) / n_az
    E, A = np.meshgrid(el, az, indexing="ij")
    d_local = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1).reshape(-1, 3)
    cy, sy = math.cos(yaw), math.sin(yaw)
    Rz = np.array([[cy, -sy, 0.0], [sy, cy, 0.0], [0.0, 0.0, 1.0]])
    d = d_local @ Rz.T
    o = np.asarray(origin, dtype=np.float64)
    tbest = np.full(d.shape[0], np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(d[:, 2] < 0, -o[2] / d[:, 2], np.inf)
        tbest = np.minimum(tbest, tg)
        inv = 1.0 / d
        for lo, hi in boxes:
            t1 = (lo - o) * inv
            t2 = (hi - o) * inv
            tn = np.nanmax(np.minimum(t1, t2), axis=1)
            tf = np.nanmin(np.maximum(t1, t2), axis=1)
            hit = (tn <= tf) & (tn > 0)
            tbest = np.where(hit & (tn < tbest), tn, tbest)
    ok = tbest <= max_range
    r = tbest[ok] + rng.normal(0.0, range_sigma, int(ok.sum()))
    pts_world = o + d[ok] * r[:, None]
    # sensor frame: translate to the sensor and undo its yaw
    return (pts_world - o) @ Rz


def lidar_pair(config: int, item: int, v: float, n_beams=64, n_az=1875, outlier_frac=0.20,
               n_boxes=40, normal_mult=3.0, fpfh_mult=5.0) -> dict:
    rng = rng_for(config, item)
    height = 1.73
    yaw = rng.uniform(0.0, 2 * math.pi)
    dist = rng.uniform(2.0, 10.0)
    ang = rng.uniform(0.0, 2 * math.pi)
    s0 = np.array([0.0, 0.0, height])
    s1 = np.array([dist * math.cos(ang), dist * math.sin(ang), height])
    boxes = _boxes(rng, n_boxes, [s0[:2], s1[:2]], height)
    src = lidar_scan(rng, s0, 0.0, boxes, n_beams, n_az)
    tgt = lidar_scan(rng, s1, yaw, boxes, n_beams, n_az)
    n = tgt.shape[0]
    n_out = int(round(outlier_frac * n))
    lo, hi = tgt.min(axis=0), tgt.max(axis=0)
    sel = rng.choice(n, size=n_out, replace=False)
    tgt[sel] = rng.uniform(lo, hi, (n_out, 3))
    cy, sy = math.cos(yaw), math.sin(yaw)
    Rz = np.array([[cy, -sy, 0.0], [sy, cy, 0.0], [0.0, 0.0, 1.0]])
    R = Rz.T
    t = Rz.T @ (s0 - s1)
    return dict(
        src=_soa(src),
        tgt=_soa(tgt),
        vp_src=np.zeros(3),
        vp_tgt=np.zeros(3),
        R=R,
        t=t,
        params=Params(voxel=v, r_normal=normal_mult * v, r_fpfh=fpfh_mult * v),
        name=f"lidar {n_beams}x{n_az} v={v:g}",
    )


def c1_pair(item: int = 0) -> dict:
    """64 x 1,875 ray-cast scan pair, voxel 0.3 m, r_normal 0.9 m, r_FPFH 1.5 m."""
    d = lidar_pair(1, item, 0.3)
    d["name"] = "lidar 64x1875 v=0.3"
    return d


# ---------------------------------------------------------------------------
# Indoor rooms (planes + spheres + cylinders)
# ---------------------------------------------------------------------------

def indoor_scene(rng, n_points):
    W, L = rng.uniform(3.0, 10.0, 2)
    H = rng.uniform(2.4, 3.2)
    n_sph = int(rng.integers(2, 7))
    n_cyl = int(rng.integers(2, 7))
    sph = []
    for _ in range(n_sph):
        r = rng.uniform(0.1, 0.5)
        c = np.array([rng.uniform(r, W - r), rng.uniform(r, L - r), rng.uniform(r, H - r)])
        sph.append((c, r))
    cyl = []
    for _ in range(n_cyl):
        r = rng.uniform(0.05, 0.3)
        h = rng.uniform(0.5, 2.5)
        c = np.array([rng.uniform(r, W - r), rng.uniform(r, L - r)])
        cyl.append((c, r, min(h, H)))
    surfaces = [("z", 0.0, W, L), ("z", H, W, L), ("x", 0.0, L, H), ("x", W, L, H), ("y", 0.0, W, H), ("y", L, W, H)]
    areas = [a * b for _, _, a, b in surfaces]
    areas += [4 * math.pi * r * r for _, r in sph]
    areas += [2 * math.pi * r * h for _, r, h in cyl]
    areas = np.array(areas)
    which = rng.choice(areas.size, size=n_points, p=areas / areas.sum())
    pts = np.empty((n_points, 3))
    for s, (axis, off, a, b) in enumerate(surfaces):
        idx = np.nonzero(which == s)[0]
        u = rng.uniform(0.0, a, idx.size)
        w = rng.uniform(0.0, b, idx.size)
        if axis == "z":
            pts[idx] = np.stack([u, w, np.full(idx.size, off)], 1)
        elif axis == "x":
            pts[idx] = np.stack([np.full(idx.size, off), u, w], 1)
        else:
            pts[idx] = np.stack([u, np.full(idx.size, off), w], 1)
    base = len(surfaces)
    for k, (c, r) in enumerate(sph):
        idx = np.nonzero(which == base + k)[0]
        pts[idx] = c + r * _unit_sphere(rng, idx.size)
    base += len(sph)
    for k, (c, r, h) in enumerate(cyl):
        idx = np.nonzero(which == base + k)[0]
        th = rng.uniform(0.0, 2 * math.pi, idx.size)
        pts[idx] = np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th), rng.uniform(0.0, h, idx.size)], 1)
    total_area = float(areas.sum())
    vp = np.array([W / 2, L / 2, 1.5])
    return pts, vp, total_area


def _raw_for_kept(m_target, area, v):
    """Raw sample count whose expected occupied-voxel count is about m_target (uniform surface sampling)."""
    cells = area / (v * v)
    if m_target >= 0.9 * cells:
        return int(3 * cells)
    return int(math.ceil(-cells * math.log1p(-m_target / cells)))


def indoor_pair(config: int, item: int, m_target: int, v: float = 0.025, n_raw: int = 0) -> dict:
    """Indoor room pair; the raw count follows m_target unless n_raw is given."""
    rng = rng_for(config, item)
    _, _, area = indoor_scene(rng_for(config, item, 1), 16)  # size-probe draw of the same room
    rng_room = rng_for(config, item, 1)
    if n_raw <= 0:
        n_raw = _raw_for_kept(m_target, area, v)
    src, vp, _ = indoor_scene(rng_room, n_raw)
    R = random_rotation(rng)
    t = rng.uniform(-1.0, 1.0, 3)
    tgt, inlier = _make_target(rng, src, 0.30, 0.01, R, t)
    return dict(
        src=_soa(src),
        tgt=_soa(tgt),
        vp_src=vp,
        vp_tgt=R @ vp + t,
        R=R,
        t=t,
        inlier=inlier,
        params=params_indoor(v),
        m_target=m_target,
        name=f"indoor m~{m_target} v={v:g}",
    )


def c2_sizes(n_pairs: int = 64, config: int = 2) -> np.ndarray:
    """Kept-size targets of the uneven batch, log-uniform in [2k, 60k]."""
    rng = rng_for(config, 0)
    return np.round(np.exp(rng.uniform(math.log(2000), math.log(60000), n_pairs))).astype(int)


def c2_batch(n_pairs: int = 64, config: int = 2, items=None) -> list:
    """Uneven batch: kept sizes log-uniform in [2k, 60k]; first half indoor, second half LiDAR-like.
    items: the pair indices to generate (default all); each pair has its own seed, so a
    selection gives the same pairs as the whole batch."""
    sizes = c2_sizes(n_pairs, config)
    pairs = []
    half = n_pairs // 2
    for i in (range(n_pairs) if items is None else items):
        m = int(sizes[i])
        if i < half:
            pairs.append(indoor_pair(config, 1 + i, m))
        else:
            # LiDAR-like: voxel scaled so the kept count is about m; denser sweeps for small voxels
            v = float(np.clip(0.3 * math.sqrt(25000.0 / m), 0.12, 1.2))
            n_az = int(round(1875 * max(1.0, 2.0 * m / 25000.0)))
            d = lidar_pair(config, 1 + i, v, n_az=n_az)
            d["m_target"] = m
            pairs.append(d)
    return pairs


# ---------------------------------------------------------------------------
# Noiseless lattice pair (exact transform recovery)
# ---------------------------------------------------------------------------

def lattice_pair(item: int = 0, spacing: float = 0.05, config: int = 90) -> dict:
    """Planes+spheres sampled on a jittered parametric lattice (about one point per
    spacing^2), and its exact rigid image, permuted.  No noise, no outliers."""
    rng = rng_for(config, item)
    side = 2.0
    k = int(side / spacing)
    g = (np.arange(k) + 0.5) * spacing
    U, V = np.meshgrid(g, g, indexing="ij")
    U = U.ravel() + rng.uniform(-0.2, 0.2, U.size) * spacing
    V = V.ravel() + rng.uniform(-0.2, 0.2, V.size) * spacing
    pts = []
    for s in range(3):
        p = np.zeros((U.size, 3))
        cols = [c for c in range(3) if c != s]
        p[:, cols[0]] = U
        p[:, cols[1]] = V
        pts.append(p)
    centres = _sphere_centres(rng, 2, 0.45, 1.55, 0.7)
    radius = 0.3
    n_s = int(round(4 * math.pi * radius * radius / (spacing * spacing)))
    i = np.arange(n_s) + 0.5
    phi = np.arccos(1 - 2 * i / n_s)
    th = math.pi * (1 + 5 ** 0.5) * i
    fib = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    for c in centres:
        pts.append(c + radius * fib)
    src = np.concatenate(pts).astype(np.float32).astype(np.float64)
    R = random_rotation(rng)
    t = rng.uniform(-1.0, 1.0, 3)
    perm = rng.permutation(src.shape[0])
    tgt = (src @ R.T + t)[perm]
    vp = np.array([3.0, 3.0, 3.0])
    return dict(
        src=_soa(src),
        tgt=_soa(tgt),
        perm=perm,
        vp_src=vp,
        vp_tgt=R @ vp + t,
        R=R,
        t=t,
        params=Params(voxel=spacing, r_normal=2.0 * spacing, r_fpfh=5.0 * spacing),
        name=f"lattice planes+spheres s={spacing:g}",
    )


# ---------------------------------------------------------------------------
# FPFH-shaped descriptors (matching at scale)
# ---------------------------------------------------------------------------

def synthetic_descriptors(n_src: int, n_tgt: int, item: int = 0, config: int = 3, n_bins: int = 11,
                          inlier_frac: float = 0.5, jitter: float = 0.02):
    """Non-negative 3*n_bins descriptors shaped like FPFH rows: three sub-histograms,
    each summing to S = 100 (1 + rho) with rho ~ U[0.5, 3].  A fraction of target rows
    are jittered copies of source rows (permuted), the rest are fresh draws."""
    rng = rng_for(config, item)

    def draw(n):
        rho = rng.uniform(0.5, 3.0, (n, 1))
        out = []
        for _ in range(3):
            a = rng.gamma(0.6, 1.0, (n, n_bins))
            a /= a.sum(axis=1, keepdims=True)
            out.append(a * 100.0 * (1.0 + rho))
        return np.concatenate(out, axis=1)

    X = draw(n_src)
    Y = draw(n_tgt)
    k = min(int(inlier_frac * n_tgt), n_src)
    src_rows = rng.choice(n_src, size=k, replace=False)
    tgt_rows = rng.choice(n_tgt, size=k, replace=False)
    Y[tgt_rows] = X[src_rows] * (1.0 + jitter * rng.standard_normal((k, 3 * n_bins)))
    Y = np.maximum(Y, 0.0)
    return X.astype(np.float32), Y.astype(np.float32), (src_rows, tgt_rows)


# ---------------------------------------------------------------------------
# Serving trace
# ---------------------------------------------------------------------------

def c4_trace(rate: float, n_requests: int = 2000, warmup: int = 200, config: int = 4):
    """Open-loop Poisson arrivals; each request is one pair of n raw points each,
    n log-uniform in [1k, 120k], type indoor or LiDAR with probability 1/2."""
    rng = rng_for(config, int(rate))
    total = n_requests + warmup
    gaps = rng.exponential(1.0 / rate, total)
    arrivals = np.cumsum(gaps)
    sizes = np.round(np.exp(rng.uniform(math.log(1000), math.log(120000), total))).astype(int)
    kinds = rng.integers(0, 2, total)  # 0 indoor, 1 lidar
    return arrivals, sizes, kinds


def c4_pool(n_each: int = 6, config: int = 4) -> dict:
    """Base pairs for serving requests: n_each LiDAR pairs (64 x 1,875 rays, voxel
    0.3 m) and n_each indoor room pairs of 120,000 raw points per cloud."""
    return {
        0: [indoor_pair(config, 100 + i, 0, n_raw=120000) for i in range(n_each)],
        1: [lidar_pair(config, 200 + i, 0.3) for i in range(n_each)],
    }


def c4_requests(rate: float, n_requests: int = 2000, warmup: int = 200, config: int = 4, pool=None) -> list:
    """Requests of the Poisson trace at `rate`: request i takes base pair i of its
    kind (cycling through the pool) and keeps a seeded random subset of n_i raw
    points of each cloud, in their original order."""
    pool = c4_pool(config=config) if pool is None else pool
    arrivals, sizes, kinds = c4_trace(rate, n_requests, warmup, config)
    out = []
    for i in range(len(arrivals)):
        base = pool[int(kinds[i])][i % len(pool[int(kinds[i])])]
        rng = rng_for(config, int(rate), 1 + i)
        req = dict(arrival=float(arrivals[i]), kind=int(kinds[i]), params=base["params"],
                   vp_src=base["vp_src"], vp_tgt=base["vp_tgt"], warmup=i < warmup)
        for key in ("src", "tgt"):
            n_all = base[key].shape[1]
            n = int(min(sizes[i], n_all))
            sel = np.sort(rng.choice(n_all, size=n, replace=False))
            req[key] = np.ascontiguousarray(base[key][:, sel])
        out.append(req)
    return out


def c3_pair(item: int = 0, config: int = 3, n_beams: int = 128, n_az: int = 3750, n_poses: int = 4,
            step: float = 8.0, outlier_frac: float = 0.20) -> dict:
    """Submap pair for the large matching workload: each side accumulates
    n_poses scans taken `step` metres apart along the heading of its first
    pose, expressed in that pose's frame; the target's first pose is yawed
    and moved 2-10 m from the source's, and 20% of its points are replaced by
    uniform outliers.  Voxel 0.15 m, r_normal 0.45 m, r_FPFH 0.75 m."""
    rng = rng_for(config, item)
    height = 1.73
    yaw = rng.uniform(0.0, 2 * math.pi)
    dist = rng.uniform(2.0, 10.0)
    ang = rng.uniform(0.0, 2 * math.pi)
    s0 = np.array([0.0, 0.0, height])
    s1 = np.array([dist * math.cos(ang), dist * math.sin(ang), height])
    fwd0 = np.array([1.0, 0.0, 0.0])
    fwd1 = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    track = [s0 + k * step * fwd0 for k in range(n_poses)] + [s1 + k * step * fwd1 for k in range(n_poses)]
    boxes = _boxes(rng, 40, [p[:2] for p in track], height)

    def submap(origin, heading_yaw, fwd):
        cy, sy = math.cos(heading_yaw), math.sin(heading_yaw)
        Rz = np.array([[cy, -sy, 0.0], [sy, cy, 0.0], [0.0, 0.0, 1.0]])
        parts = []
        for k in range(n_poses):
            o = origin + k * step * fwd
            local = lidar_scan(rng, o, heading_yaw, boxes, n_beams, n_az)  # in the frame of pose k
            world = local @ Rz.T + o
            parts.append((world - origin) @ Rz)  # frame of the first pose
        return np.concatenate(parts, axis=0)

    src = submap(s0, 0.0, fwd0)
    tgt = submap(s1, yaw, fwd1)
    n = tgt.shape[0]
    n_out = int(round(outlier_frac * n))
    lo, hi = tgt.min(axis=0), tgt.max(axis=0)
    sel = rng.choice(n, size=n_out, replace=False)
    tgt[sel] = rng.uniform(lo, hi, (n_out, 3))
    cy, sy = math.cos(yaw), math.sin(yaw)
    Rz = np.array([[cy, -sy, 0.0], [sy, cy, 0.0], [0.0, 0.0, 1.0]])
    return dict(src=_soa(src), tgt=_soa(tgt), vp_src=np.zeros(3), vp_tgt=np.zeros(3), R=Rz.T,
                t=Rz.T @ (s0 - s1), params=Params(voxel=0.15, r_normal=0.45, r_fpfh=0.75),
                name=f"submap {n_poses}x({n_beams}x{n_az}) v=0.15")

