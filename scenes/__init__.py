"""Seeded synthetic inputs shaped like the paper's workloads.

This module only *draws inputs*: planar surfaces sampled uniformly by area,
Gaussian noise along each surface normal, uniform outliers, sensor poses.
It holds none of the segmentation method's arithmetic (no voxelisation, no
clustering, no plane fitting, no hulls), so both the HIP path and the CPU
oracle may take their inputs from here.

The paper evaluates on simulated MuJoCo scenes seen through simulated
D435 / Livox / RoboSense sensors (Sec. IV-A); those are not available, so the
scenes below stand in for them with the same structure: a floor, an
open-tread staircase, a tabletop and tilted planar patches inside a
robot-centric box at 0.01 m voxels (Sec. IV-A), plus the cluster-parallel
ablation shape (Sec. IV-C) scaled up to thousands of clusters.

All randomness comes from ``numpy.random.default_rng(seed)``; every array
returned is a fresh float32/float64 numpy array.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Rect", "Scene", "MapGeom",
    "scene_tiny", "scene_tiny_exact", "scene_full_map", "scene_stress",
    "frame_points", "identity_pose", "pose_inverse_apply",
    "random_walk_poses", "batched_clusters", "surface_pool", "stream_frame", "StreamFrame", "served_trace",
    "raycast_frame", "polygon_iou_with_rect", "plane_iou",
]


@dataclasses.dataclass(frozen=True)
class MapGeom:
    """Voxel grid geometry: lower corner, voxel edge, cell counts."""
    origin: Tuple[float, float, float]
    voxel_size: float
    dims: Tuple[int, int, int]

    @property
    def hi(self) -> np.ndarray:
        return np.asarray(self.origin) + self.voxel_size * np.asarray(self.dims, dtype=np.float64)


@dataclasses.dataclass(frozen=True)
class Rect:
    """Planar rectangle: centre, two orthonormal in-plane axes, half-sizes."""
    centre: Tuple[float, float, float]
    axis_a: Tuple[float, float, float]
    axis_b: Tuple[float, float, float]
    half_a: float
    half_b: float

    @property
    def normal(self) -> np.ndarray:
        n = np.cross(np.asarray(self.axis_a), np.asarray(self.axis_b))
        return n / np.linalg.norm(n)

    @property
    def area(self) -> float:
        return 4.0 * self.half_a * self.half_b

    def sample(self, rng: np.random.Generator, n: int, sigma: float) -> np.ndarray:
        s = rng.uniform(-1.0, 1.0, size=(n, 2))
        p = (np.asarray(self.centre)[None, :]
             + (s[:, :1] * self.half_a) * np.asarray(self.axis_a)[None, :]
             + (s[:, 1:] * self.half_b) * np.asarray(self.axis_b)[None, :])
        if sigma > 0:
            p = p + rng.normal(0.0, sigma, size=(n, 1)) * self.normal[None, :]
        return p

    def corners(self) -> np.ndarray:
        c = np.asarray(self.centre)
        a = np.asarray(self.axis_a) * self.half_a
        b = np.asarray(self.axis_b) * self.half_b
        return np.stack([c - a - b, c + a - b, c + a + b, c - a + b])


def _hrect(x0: float, x1: float, y0: float, y1: float, z: float) -> Rect:
    """Horizontal rectangle [x0,x1) x [y0,y1) at height z (normal +z)."""
    return Rect(((x0 + x1) / 2, (y0 + y1) / 2, z), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
                (x1 - x0) / 2, (y1 - y0) / 2)


@dataclasses.dataclass
class Scene:
    """A static scene plus the per-frame sampling recipe."""
    name: str
    geom: MapGeom
    rects: List[Rect]
    n_points: int
    sigma: float
    outlier_frac: float
    n_hyp: int
    eps: float = 0.01
    min_cluster: int = 30
    seed: int = 0
    extra_points: Optional[np.ndarray] = None  # injected exact points (float64)


def scene_tiny(seed: int = 0) -> Scene:
    """1.28 m cube at 0.01 m (128^3): floor z=0 and two 0.30x0.60 m stair
    treads at z=0.18 and z=0.36; 50k points, N(0, 2 mm), 2 % outliers."""
    geom = MapGeom((0.0, 0.0, -0.64), 0.01, (128, 128, 128))
    rects = [
        _hrect(0.0, 1.28, 0.0, 1.28, 0.0),
        _hrect(0.40, 0.70, 0.34, 0.94, 0.18),
        _hrect(0.70, 1.00, 0.34, 0.94, 0.36),
    ]
    return Scene("tiny", geom, rects, 50_000, 0.002, 0.02, n_hyp=256, seed=seed)


def scene_tiny_exact(seed: int = 0) -> Scene:
    """Noise-free, outlier-free variant of :func:`scene_tiny` with each
    rectangle's four corners injected (for exact-recovery checks)."""
    sc = scene_tiny(seed)
    corners = np.concatenate([r.corners() for r in sc.rects[1:]], axis=0)
    # keep the injected corners strictly inside the grid's half-open range
    corners = np.minimum(corners, np.nextafter(sc.geom.hi, -np.inf) - 1e-9)
    return dataclasses.replace(sc, name="tiny_exact", sigma=0.0, outlier_frac=0.0,
                               extra_points=corners)


def _rot_xy(alpha: float, beta: float) -> np.ndarray:
    ca, sa, cb, sb = math.cos(alpha), math.sin(alpha), math.cos(beta), math.sin(beta)
    rx = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]])
    ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    return rx @ ry


def _rect_grid(r: Rect, spacing: float) -> np.ndarray:
    na = max(2, int(2 * r.half_a / spacing) + 1)
    nb = max(2, int(2 * r.half_b / spacing) + 1)
    sa, sb = np.meshgrid(np.linspace(-1, 1, na), np.linspace(-1, 1, nb), indexing="ij")
    return (np.asarray(r.centre)[None, :]
            + (sa.reshape(-1, 1) * r.half_a) * np.asarray(r.axis_a)[None, :]
            + (sb.reshape(-1, 1) * r.half_b) * np.asarray(r.axis_b)[None, :])


def _staircase(n_steps: int, x0: float, y0: float, y1: float, run: float, rise: float) -> List[Rect]:
    return [_hrect(x0 + run * i, x0 + run * (i + 1), y0, y1, rise * (i + 1)) for i in range(n_steps)]


def _place_patches(rng: np.random.Generator, fixed: List[Rect], n: int, side: Tuple[float, float],
                   centre_lo: Sequence[float], centre_hi: Sequence[float], tilt_deg: float,
                   clearance: float, z_range: Tuple[float, float]) -> List[Rect]:
    """Rejection-sample ``n`` tilted square-ish patches keeping ``clearance``
    metres from every other surface (so each stays its own component)."""
    from scipy.spatial import cKDTree
    spacing = 0.02
    placed: List[Rect] = []
    cloud = [_rect_grid(r, spacing) for r in fixed]
    tries = 0
    while len(placed) < n:
        tries += 1
        if tries > 200_000:
            raise RuntimeError("patch placement did not converge")
        ha, hb = rng.uniform(side[0], side[1], size=2) / 2
        c = rng.uniform(centre_lo, centre_hi)
        alpha, beta = np.deg2rad(rng.uniform(-tilt_deg, tilt_deg, size=2))
        rot = _rot_xy(alpha, beta)
        r = Rect(tuple(c), tuple(rot[:, 0]), tuple(rot[:, 1]), float(ha), float(hb))
        g = _rect_grid(r, spacing)
        if g[:, 2].min() < z_range[0] or g[:, 2].max() > z_range[1]:
            continue
        tree = cKDTree(np.concatenate(cloud, axis=0))
        d, _ = tree.query(g, k=1)
        if d.min() < clearance + spacing:
            continue
        placed.append(r)
        cloud.append(g)
    return placed


def scene_full_map(seed: int = 1) -> Scene:
    """4x4x2 m local map at 0.01 m (400x400x200 cells): floor, 12-step
    open-tread staircase (0.18 m rise, 0.28 m run; treads above the map top
    fall outside the grid), a 1.2x0.8 m tabletop at 0.72 m and 20 tilted
    (up to +-30 deg) planar patches with sides 0.2-0.6 m; 1M points per frame,
    N(0, 3 mm), 5 % outliers, 512 hypotheses."""
    geom = MapGeom((-2.0, -2.0, -0.1), 0.01, (400, 400, 200))
    rng = np.random.default_rng(seed)
    fixed = [_hrect(-2.0, 2.0, -2.0, 2.0, 0.0)]
    fixed += _staircase(12, -1.5, -1.9, -0.9, 0.28, 0.18)
    fixed += [_hrect(0.3, 1.5, 0.5, 1.3, 0.72)]
    patches = _place_patches(rng, fixed, 20, (0.2, 0.6), (-1.8, -1.8, 0.1), (1.8, 1.8, 1.6),
                             30.0, 0.05, (0.05, 1.85))
    return Scene("full_map", geom, fixed + patches, 1_000_000, 0.003, 0.05, n_hyp=512, seed=seed)


class _ClearanceGrid:
    """Occupancy of placed surfaces on a coarse grid (cell = ``cell`` metres),
    each placed sample marking every cell within ``reach`` cells, so that a
    candidate whose samples all fall in unmarked cells keeps roughly
    reach*cell metres from everything placed before it."""

    def __init__(self, lo, hi, cell: float, reach: int):
        self.lo = np.asarray(lo, np.float64)
        self.cell = cell
        self.reach = reach
        self.dims = np.ceil((np.asarray(hi, np.float64) - self.lo) / cell).astype(np.int64) + 1
        self.occ = np.zeros(tuple(self.dims), dtype=bool)
        r = np.arange(-reach, reach + 1)
        self.offsets = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)

    def _cells(self, pts: np.ndarray) -> np.ndarray:
        c = np.floor((pts - self.lo) / self.cell).astype(np.int64)
        return np.clip(c, 0, self.dims - 1)

    def free(self, pts: np.ndarray) -> bool:
        c = self._cells(pts)
        return not self.occ[c[:, 0], c[:, 1], c[:, 2]].any()

    def mark(self, pts: np.ndarray) -> None:
        c = np.unique(self._cells(pts), axis=0)
        for o in self.offsets:
            q = np.clip(c + o, 0, self.dims - 1)
            self.occ[q[:, 0], q[:, 1], q[:, 2]] = True


def scene_stress(seed: int = 5, n_boxes: int = 500) -> Scene:
    """4x4x2 m at 0.005 m (800x800x400 cells): floor, staircase, two tables
    and ``n_boxes`` floating yawed boxes (sides 0.05-0.4 m, all 6 faces,
    about 0.04 m apart from each other and from the fixed surfaces);
    8M points per frame, N(0, 1.5 mm), 5 % outliers, 1024 hypotheses."""
    geom = MapGeom((-2.0, -2.0, -0.1), 0.005, (800, 800, 400))
    rng = np.random.default_rng(seed)
    fixed = [_hrect(-2.0, 2.0, -2.0, 2.0, 0.0)]
    fixed += _staircase(12, -1.5, -1.9, -0.9, 0.28, 0.18)
    fixed += [_hrect(0.3, 1.5, 0.5, 1.3, 0.72), _hrect(-1.2, -0.4, 0.6, 1.4, 0.76)]
    grid = _ClearanceGrid(geom.origin, geom.hi, 0.02, 2)
    for r in fixed:
        grid.mark(_rect_grid(r, 0.02))
    boxes: List[Rect] = []
    tries = 0
    while len(boxes) < 6 * n_boxes:
        tries += 1
        if tries > 500_000:
            raise RuntimeError("box placement did not converge")
        sx, sy, sz = rng.uniform(0.05, 0.4, size=3)
        c = rng.uniform((-1.8, -1.8, 0.1), (1.8, 1.8, 1.7))
        yaw = rng.uniform(0, 2 * math.pi)
        ex = np.array([math.cos(yaw), math.sin(yaw), 0.0])
        ey = np.array([-math.sin(yaw), math.cos(yaw), 0.0])
        ez = np.array([0.0, 0.0, 1.0])
        faces = []
        for ax, (u, v), h, (hu, hv) in ((ez, (ex, ey), sz / 2, (sx / 2, sy / 2)),
                                        (ex, (ey, ez), sx / 2, (sy / 2, sz / 2)),
                                        (ey, (ez, ex), sy / 2, (sz / 2, sx / 2))):
            for sgn in (1.0, -1.0):
                fc = c + sgn * h * ax
                uu, vv = (u, v) if sgn > 0 else (v, u)
                hu_, hv_ = (hu, hv) if sgn > 0 else (hv, hu)
                faces.append(Rect(tuple(fc), tuple(uu), tuple(vv), float(hu_), float(hv_)))
        g = np.concatenate([_rect_grid(f, 0.02) for f in faces])
        if g[:, 2].min() < 0.03 or g[:, 2].max() > 1.85:
            continue
        if not grid.free(g):
            continue
        boxes += faces
        grid.mark(g)
    return Scene("stress", geom, fixed + boxes, 8_000_000, 0.0015, 0.05, n_hyp=1024, seed=seed)


def identity_pose() -> Tuple[np.ndarray, np.ndarray]:
    return np.eye(3), np.zeros(3)


def pose_inverse_apply(R: np.ndarray, t: np.ndarray, pw: np.ndarray) -> np.ndarray:
    """Express map-frame points in the sensor frame of map_from_sensor (R, t)."""
    return (pw - t[None, :]) @ R


def frame_points(scene: Scene, frame_seed: int, n: Optional[int] = None,
                 pose: Optional[Tuple[np.ndarray, np.ndarray]] = None) -> np.ndarray:
    """One sensor frame: ``n`` float32 xyz points (default ``scene.n_points``).

    A fraction ``outlier_frac`` is uniform in the map box; the rest is spread
    over the scene's rectangles proportionally to area with Gaussian noise of
    ``sigma`` along each normal. With ``pose`` = map_from_sensor (R, t), the
    points are returned in the sensor frame (map points pushed through the
    inverse pose, then rounded to float32)."""
    n = scene.n_points if n is None else int(n)
    rng = np.random.default_rng(frame_seed)
    n_out = int(round(n * scene.outlier_frac))
    extra = scene.extra_points if scene.extra_points is not None else np.zeros((0, 3))
    n_surf = n - n_out - len(extra)
    areas = np.array([r.area for r in scene.rects])
    per = rng.multinomial(n_surf, areas / areas.sum())
    parts = [r.sample(rng, int(k), scene.sigma) for r, k in zip(scene.rects, per) if k > 0]
    lo = np.asarray(scene.geom.origin, dtype=np.float64)
    hi = scene.geom.hi
    parts.append(rng.uniform(lo, hi, size=(n_out, 3)))
    parts.append(np.asarray(extra, dtype=np.float64))
    pw = np.concatenate(parts, axis=0)
    pw = pw[rng.permutation(len(pw))]
    if pose is not None:
        pw = pose_inverse_apply(np.asarray(pose[0]), np.asarray(pose[1]), pw)
    return np.ascontiguousarray(pw.astype(np.float32))


def surface_pool(scene: Scene, seed: int, n: int) -> np.ndarray:
    """``n`` noisy surface samples of ``scene`` in the map frame (float32,
    shuffled, no outliers): drawn once per robot, frames of a served stream
    take random windows of it."""
    rng = np.random.default_rng(seed)
    areas = np.array([r.area for r in scene.rects])
    per = rng.multinomial(n, areas / areas.sum())
    pw = np.concatenate([r.sample(rng, int(k), scene.sigma) for r, k in zip(scene.rects, per) if k > 0])
    return np.ascontiguousarray(pw[rng.permutation(len(pw))].astype(np.float32))


def stream_frame(scene: Scene, pool: np.ndarray, frame_seed: int, n: int,
                 pose: Optional[Tuple[np.ndarray, np.ndarray]] = None) -> np.ndarray:
    """One frame of a served stream: a random window of the robot's surface
    pool (the pool is shuffled, so a window is a uniform subsample) plus
    fresh outliers uniform in the map box, ``outlier_frac`` of the ``n``
    points; expressed in the sensor frame of ``pose`` (map_from_sensor) and
    rounded to float32, like :func:`frame_points`."""
    rng = np.random.default_rng(frame_seed)
    n_out = int(round(n * scene.outlier_frac))
    n_surf = n - n_out
    if n_surf > len(pool):
        raise ValueError("surface pool smaller than the frame")
    start = int(rng.integers(0, len(pool) - n_surf + 1))
    lo = np.asarray(scene.geom.origin, dtype=np.float64)
    pw = np.empty((n, 3), np.float64)
    pw[:n_surf] = pool[start:start + n_surf]
    pw[n_surf:] = rng.uniform(lo, scene.geom.hi, size=(n_out, 3))
    if pose is not None:
        pw = pose_inverse_apply(np.asarray(pose[0]), np.asarray(pose[1]), pw)
    return np.ascontiguousarray(pw.astype(np.float32))


def raycast_frame(scene: Scene, sensor, frame_seed: int, n: int,
                  pose: Optional[Tuple[np.ndarray, np.ndarray]] = None, rects: Optional[List[Rect]] = None,
                  outlier_frac: Optional[float] = None, max_range: float = 8.0) -> np.ndarray:
    """A frame that a sensor at ``sensor`` (map frame) could have seen: ``n``
    returns of rays with directions uniform on the sphere, each the first hit
    among the scene's rectangles (``rects`` overrides them, e.g. for a moved
    object) within ``max_range``, moved by N(0, sigma) along the ray; rays
    that hit nothing return nothing.  A fraction ``outlier_frac`` (default:
    the scene's) are spurious early returns at a uniform fraction in
    [0.05, 0.95) of their ray's hit range.  With ``pose`` (map_from_sensor,
    its translation normally ``sensor``) the points are returned in the
    sensor frame; float32."""
    rng = np.random.default_rng(frame_seed)
    rs = scene.rects if rects is None else rects
    o = np.asarray(sensor, dtype=np.float64)
    C = np.array([r.centre for r in rs], np.float64)
    A = np.array([r.axis_a for r in rs], np.float64)
    B = np.array([r.axis_b for r in rs], np.float64)
    N = np.cross(A, B)
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    ha = np.array([r.half_a for r in rs])
    hb = np.array([r.half_b for r in rs])
    of = scene.outlier_frac if outlier_frac is None else float(outlier_frac)
    out, have = [], 0
    while have < n:
        m = max(2 * (n - have), 4096)
        d = rng.normal(size=(m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        best = np.full(m, np.inf)
        for j in range(len(rs)):
            den = d @ N[j]
            with np.errstate(divide="ignore", invalid="ignore"):
                t = ((C[j] - o) @ N[j]) / den
            ok = (np.abs(den) > 1e-12) & (t > 1e-6) & (t < best) & (t <= max_range)
            if not ok.any():
                continue
            q = o[None, :] + t[ok, None] * d[ok] - C[j][None, :]
            inside = (np.abs(q @ A[j]) <= ha[j]) & (np.abs(q @ B[j]) <= hb[j])
            idx = np.nonzero(ok)[0][inside]
            best[idx] = t[idx]
        hit = np.isfinite(best)
        d, t = d[hit], best[hit]
        k = min(len(t), n - have)
        d, t = d[:k], t[:k]
        r = t + rng.normal(0.0, scene.sigma, size=k)
        spur = rng.uniform(size=k) < of
        r[spur] = t[spur] * rng.uniform(0.05, 0.95, size=int(spur.sum()))
        out.append(o[None, :] + r[:, None] * d)
        have += k
    pw = np.concatenate(out, axis=0)
    if pose is not None:
        pw = pose_inverse_apply(np.asarray(pose[0]), np.asarray(pose[1]), pw)
    return np.ascontiguousarray(pw.astype(np.float32))


@dataclasses.dataclass
class StreamFrame:
    robot: int
    seq: int                 # the robot's own frame number
    arrival: float           # seconds from the start of the stream
    n_points: int
    frame_seed: int
    pose: Tuple[np.ndarray, np.ndarray]


def served_trace(n_robots: int = 8, seconds: float = 4.0, rate_hz: float = 30.0, n_min: int = 200_000,
                 n_max: int = 2_000_000, seed: int = 20) -> List[StreamFrame]:
    """Arrivals of a multi-robot stream: per robot r, a Poisson process at
    ``rate_hz`` (exponential gaps, seed + r), frame sizes uniform in
    [n_min, n_max] and a 6-DoF random-walk pose per frame (sigma_t = 0.01 m,
    sigma_rot = 0.5 deg, seed + 100 + r).  Sorted by arrival."""
    out: List[StreamFrame] = []
    for r in range(n_robots):
        rng = np.random.default_rng(seed + r)
        t, arr = 0.0, []
        while True:
            t += rng.exponential(1.0 / rate_hz)
            if t >= seconds:
                break
            arr.append(t)
        sizes = rng.integers(n_min, n_max + 1, size=len(arr))
        poses = random_walk_poses(seed + 100 + r, len(arr), sigma_t=0.01, sigma_rot_deg=0.5)
        for k, (ta, nk) in enumerate(zip(arr, sizes)):
            out.append(StreamFrame(r, k, float(ta), int(nk), 1_000_000 * (r + 1) + k, poses[k]))
    out.sort(key=lambda f: (f.arrival, f.robot, f.seq))
    return out


def _so3_exp(w: np.ndarray) -> np.ndarray:
    th = float(np.linalg.norm(w))
    k = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-12:
        return np.eye(3) + k
    return np.eye(3) + math.sin(th) / th * k + (1 - math.cos(th)) / th ** 2 * (k @ k)


def random_walk_poses(seed: int, n_frames: int, sigma_t: float = 0.01,
                      sigma_rot_deg: float = 0.5) -> List[Tuple[np.ndarray, np.ndarray]]:
    """6-DoF random walk from the identity: per frame dt ~ N(0, sigma_t)^3 and
    a rotation increment exp(N(0, sigma_rot)^3), composed in float64."""
    rng = np.random.default_rng(seed)
    R, t = np.eye(3), np.zeros(3)
    out = []
    for _ in range(n_frames):
        out.append((R.copy(), t.copy()))
        dR = _so3_exp(np.deg2rad(rng.normal(0.0, sigma_rot_deg, size=3)))
        R = R @ dR
        t = t + rng.normal(0.0, sigma_t, size=3)
    return out


def batched_clusters(seed: int = 3, n_clusters: int = 2000, n_min: int = 50, n_max: int = 200_000,
                     sigma: float = 0.002, outlier_frac: float = 0.10,
                     cap_deg: float = 40.0) -> Tuple[np.ndarray, np.ndarray]:
    """Thousands of noisy plane patches of log-uniform size, as a CSR.

    Cluster k holds n_k = floor(exp(U(ln n_min, ln n_max))) points: a square of
    side 0.01*sqrt(n_k) m (one point per cm^2, like 0.01 m voxel means) with
    normal uniform on the ``cap_deg`` cap around +z and centre uniform in
    [-2,2]^2 x [0,2]; (1-outlier_frac) of the points lie on it with N(0, sigma)
    along the normal, the rest are uniform in the square x [-0.1, 0.1] m
    along the normal. Returns (off uint32[K+1], xyz float32[sum n_k, 3])."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_clusters))).astype(np.int64)
    off = np.zeros(n_clusters + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    xyz = np.empty((int(off[-1]), 3), dtype=np.float32)
    cos_cap = math.cos(math.radians(cap_deg))
    for k in range(n_clusters):
        n = int(sizes[k])
        ct = rng.uniform(cos_cap, 1.0)
        st = math.sqrt(max(0.0, 1 - ct * ct))
        ph = rng.uniform(0, 2 * math.pi)
        nrm = np.array([st * math.cos(ph), st * math.sin(ph), ct])
        a = np.cross(nrm, [1.0, 0.0, 0.0])
        a /= np.linalg.norm(a)
        b = np.cross(nrm, a)
        c = rng.uniform((-2, -2, 0), (2, 2, 2))
        half = 0.005 * math.sqrt(n)
        n_out = int(round(n * outlier_frac))
        n_in = n - n_out
        s = rng.uniform(-half, half, size=(n, 2))
        h = np.concatenate([rng.normal(0.0, sigma, size=n_in), rng.uniform(-0.1, 0.1, size=n_out)])
        p = c[None, :] + s[:, :1] * a[None, :] + s[:, 1:] * b[None, :] + h[:, None] * nrm[None, :]
        p = p[rng.permutation(n)]
        xyz[off[k]:off[k + 1]] = p.astype(np.float32)
    return off.astype(np.uint32), xyz


# ---------------------------------------------------------------------------
# accuracy against the generator's ground truth (the analogue of Table I's IoU)
# ---------------------------------------------------------------------------
def _clip_convex(poly: np.ndarray, a: float, b: float) -> np.ndarray:
    """Sutherland-Hodgman: the part of the convex polygon ``poly`` (k x 2,
    either orientation) inside the box [-a, a] x [-b, b]."""
    out = np.asarray(poly, np.float64)
    for axis, lim, sign in ((0, a, 1.0), (0, a, -1.0), (1, b, 1.0), (1, b, -1.0)):
        if len(out) == 0:
            break
        inp, out = out, []
        for i in range(len(inp)):
            p, q = inp[i - 1], inp[i]
            pin, qin = sign * p[axis] <= lim, sign * q[axis] <= lim
            if qin:
                if not pin:
                    t = (lim - sign * p[axis]) / (sign * (q[axis] - p[axis]))
                    out.append(p + t * (q - p))
                out.append(q)
            elif pin:
                t = (lim - sign * p[axis]) / (sign * (q[axis] - p[axis]))
                out.append(p + t * (q - p))
        out = np.asarray(out, np.float64).reshape(-1, 2)
    return out


def _area(poly: np.ndarray) -> float:
    if len(poly) < 3:
        return 0.0
    x, y = poly[:, 0], poly[:, 1]
    return 0.5 * abs(float(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1))))


def polygon_iou_with_rect(rect: Rect, vertices_xyz: np.ndarray) -> float:
    """Intersection over union of a convex polygon (vertices in 3D, lying in
    or near the rectangle's plane) and the rectangle, both taken in the
    rectangle's own 2D frame."""
    v = np.asarray(vertices_xyz, np.float64).reshape(-1, 3)
    if len(v) < 3:
        return 0.0
    c, a, b = np.asarray(rect.centre), np.asarray(rect.axis_a), np.asarray(rect.axis_b)
    uv = np.c_[(v - c) @ a, (v - c) @ b]
    inter = _area(_clip_convex(uv, rect.half_a, rect.half_b))
    union = rect.area + _area(uv) - inter
    return inter / union if union > 0 else 0.0


def plane_iou(rects: List[Rect], planes: np.ndarray, polygons: List[np.ndarray], max_angle_deg: float = 10.0,
              max_offset: float = 0.05) -> np.ndarray:
    """For each ground-truth rectangle, the best IoU among the detected planes
    (n, d: n.x + d = 0) whose normal is within ``max_angle_deg`` of the
    rectangle's (either sign) and which pass within ``max_offset`` m of its
    centre; 0 when none qualifies."""
    out = np.zeros(len(rects))
    P = np.asarray(planes, np.float64).reshape(-1, 4)
    cos_max = np.cos(np.deg2rad(max_angle_deg))
    fin = np.all(np.isfinite(P), axis=1)
    Pf = np.where(fin[:, None], P, 0.0)
    for i, r in enumerate(rects):
        c = np.asarray(r.centre)
        ok = fin & (np.abs(Pf[:, :3] @ r.normal) >= cos_max) & (np.abs(Pf[:, :3] @ c + Pf[:, 3]) <= max_offset)
        for j in np.nonzero(ok)[0]:
            out[i] = max(out[i], polygon_iou_with_rect(r, polygons[j]))
    return out

