"""Seeded synthetic RGB-D inputs: analytic scenes, camera paths, a depth/colour
renderer and the depth noise model.

This module is the only code shared by the CPU oracle side and the HIP side of
the tests and the benchmark.  It simulates a depth camera; it contains none of
the mapping method's arithmetic (no TSDF, no raycast through a volume, no
placement rule).

Conventions
-----------
* World frame: right-handed, z up.  Units: metres.
* Camera frame: OpenCV axes (x right, y down, z forward).
* A pose ``T_wc`` is a 3x4 float64 array [R | t] mapping camera-frame points
  to world points: x_w = R x_c + t.
* Depth maps hold z-depth (the camera-frame z of the first surface hit along
  the pixel-centre ray), float32 metres; 0 marks "no measurement".
* Pixel (u, v) has its centre at integer coordinates (u, v); the ray through
  it is K^-1 [u, v, 1]^T (the depth-to-vertex map of the paper's Depth Map
  Conversion section).

The paper measured on ICL-NUIM sequences and its own Xtion recordings, none of
which are available here; these scenes stand in for them with the same frame
shape (640x480, 30 fps, float depth in metres, uint8 RGB).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Scene description
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Sphere:
    center: np.ndarray  # (3,)
    radius: float
    color: np.ndarray  # (3,) uint8


@dataclasses.dataclass
class Box:
    center: np.ndarray  # (3,)
    half: np.ndarray  # (3,) half extents
    color: np.ndarray  # (3,) uint8


@dataclasses.dataclass
class Scene:
    """A room (the inside of an axis-aligned box) plus solid spheres and boxes."""

    room_lo: np.ndarray
    room_hi: np.ndarray
    wall_colors: np.ndarray  # (6, 3) uint8: -x, +x, -y, +y, -z, +z walls
    spheres: List[Sphere]
    boxes: List[Box]

    @property
    def n_objects(self) -> int:
        return len(self.spheres) + len(self.boxes)


@dataclasses.dataclass
class Intrinsics:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def as_array(self) -> np.ndarray:
        return np.array([self.fx, self.fy, self.cx, self.cy], dtype=np.float32)


K_QVGA = Intrinsics(262.5, 262.5, 160.0, 120.0, 320, 240)
K_VGA = Intrinsics(525.0, 525.0, 319.5, 239.5, 640, 480)


def _rand_color(rng: np.random.Generator) -> np.ndarray:
    return rng.integers(16, 256, size=3).astype(np.uint8)


# --------------------------------------------------------------------------
# Poses
# --------------------------------------------------------------------------


def look_at(eye: Sequence[float], target: Sequence[float],
            up: Sequence[float] = (0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world pose at ``eye`` looking at ``target`` (OpenCV axes)."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    nr = np.linalg.norm(right)
    if nr < 1e-9:  # looking straight up/down: pick any right vector
        right = np.cross(fwd, np.array([1.0, 0.0, 0.0]))
        nr = np.linalg.norm(right)
    right /= nr
    down = np.cross(fwd, right)
    T = np.zeros((3, 4))
    T[:, 0], T[:, 1], T[:, 2], T[:, 3] = right, down, fwd, eye
    return T


def so3_exp(w: np.ndarray) -> np.ndarray:
    th = float(np.linalg.norm(w))
    Wx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]], np.float64)
    if th < 1e-12:
        return np.eye(3) + Wx
    return (np.eye(3) + np.sin(th) / th * Wx
            + (1 - np.cos(th)) / th ** 2 * (Wx @ Wx))


def perturb_pose(T: np.ndarray, rng: np.random.Generator, trans_m: float,
                 rot_deg: float) -> np.ndarray:
    """Right-multiply ``T`` by a random rigid motion with translation norm
    ``trans_m`` and rotation angle ``rot_deg`` (random axes)."""
    a = rng.normal(size=3)
    a *= trans_m / np.linalg.norm(a)
    b = rng.normal(size=3)
    b *= np.deg2rad(rot_deg) / np.linalg.norm(b)
    dR = so3_exp(b)
    out = np.zeros((3, 4))
    out[:, :3] = T[:, :3] @ dR
    out[:, 3] = T[:, :3] @ a + T[:, 3]
    return out


# --------------------------------------------------------------------------
# Trajectories
# --------------------------------------------------------------------------


def circle_trajectory(seed: int, n_frames: int, radius: float = 1.0,
                      center=(0.0, 0.0, 0.0)) -> List[np.ndarray]:
    """Camera on a horizontal circle of ``radius`` around ``center``, looking
    at the centre; frames spaced evenly over one turn from a seeded phase."""
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    phase = rng.uniform(0, 2 * np.pi)
    c = np.asarray(center, np.float64)
    poses = []
    for i in range(n_frames):
        a = phase + 2 * np.pi * i / n_frames
        eye = c + radius * np.array([np.cos(a), np.sin(a), 0.0])
        poses.append(look_at(eye, c))
    return poses


def _catmull_rom(P: np.ndarray, n_dense: int) -> np.ndarray:
    """Dense samples of a centripetal-free (uniform) Catmull-Rom spline."""
    pts = np.vstack([P[0], P, P[-1]])
    out = []
    segs = len(P) - 1
    per = max(2, n_dense // segs)
    for s in range(segs):
        p0, p1, p2, p3 = pts[s], pts[s + 1], pts[s + 2], pts[s + 3]
        for j in range(per):
            t = j / per
            t2, t3 = t * t, t * t * t
            out.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t2
                              + (-p0 + 3 * p1 - 3 * p2 + p3) * t3))
    out.append(P[-1])
    return np.asarray(out)


def _retime(curve: np.ndarray, n_frames: int, step: float) -> np.ndarray:
    seg = np.linalg.norm(np.diff(curve, axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    want = np.arange(n_frames) * step
    want = np.minimum(want, s[-1])
    return np.stack([np.interp(want, s, curve[:, a]) for a in range(3)], axis=1)


def handheld_trajectory(seed: int, n_frames: int, speed: float = 0.5,
                        fps: float = 30.0, ring=(1.0, 1.3), zr=0.3,
                        center=(0.0, 0.0, 0.0)) -> List[np.ndarray]:
    """Smooth handheld path: a Catmull-Rom spline through seeded waypoints on
    a ring around ``center``, re-timed to ``speed`` m/s at ``fps``, looking at
    a slowly drifting seeded target near the centre."""
    rng = np.random.Generator(np.random.PCG64([seed, 11]))
    c = np.asarray(center, np.float64)
    total = speed * n_frames / fps
    mean_r = 0.5 * (ring[0] + ring[1])
    n_way = 10
    sweep = 1.3 * total / mean_r  # radians covered, with slack for wiggles
    a0 = rng.uniform(0, 2 * np.pi)
    ang = a0 + np.linspace(0, sweep, n_way) + rng.uniform(-0.1, 0.1, n_way)
    rad = rng.uniform(ring[0], ring[1], n_way)
    zz = rng.uniform(-zr, zr, n_way)
    P = np.stack([c[0] + rad * np.cos(ang), c[1] + rad * np.sin(ang), c[2] + zz], axis=1)
    curve = _catmull_rom(P, 4000)
    pos = _retime(curve, n_frames, speed / fps)
    ph = rng.uniform(0, 2 * np.pi, 3)
    poses = []
    for i in range(n_frames):
        tt = i / max(1, n_frames - 1)
        tgt = c + 0.25 * np.sin(2 * np.pi * 0.5 * tt + ph)
        poses.append(look_at(pos[i], tgt))
    return poses


def corridor_trajectory(seed: int, n_frames: int, length: float = 20.0,
                        speed: float = 0.3, fps: float = 30.0,
                        sway: float = 0.2, yaw_deg: float = 20.0,
                        height: float = 1.3) -> List[np.ndarray]:
    """Walk along +x down a corridor with seeded lateral sway and yaw
    oscillation."""
    rng = np.random.Generator(np.random.PCG64([seed, 13]))
    f1, f2 = rng.uniform(0.05, 0.12), rng.uniform(0.08, 0.2)
    p1, p2 = rng.uniform(0, 2 * np.pi, 2)
    poses = []
    for i in range(n_frames):
        t = i / fps
        x = 0.3 + min(speed * t, length - 0.6)
        y = sway * np.sin(2 * np.pi * f1 * t + p1)
        yaw = np.deg2rad(yaw_deg) * np.sin(2 * np.pi * f2 * t + p2)
        eye = np.array([x, y, height])
        tgt = eye + np.array([np.cos(yaw), np.sin(yaw), -0.1])
        poses.append(look_at(eye, tgt))
    return poses


# --------------------------------------------------------------------------
# Scene builders
# --------------------------------------------------------------------------


def _dist_to_path(p: np.ndarray, path: np.ndarray) -> float:
    return float(np.min(np.linalg.norm(path - p[None, :], axis=1)))


def room_scene(seed: int, n_spheres: int, n_boxes: int = 0,
               half_room: float = 2.0, obj_box=1.2,
               r_range=(0.2, 0.5), box_half_range=(0.1, 0.4),
               keep_clear: Optional[np.ndarray] = None,
               clearance: float = 0.3) -> Scene:
    """A 2*half_room cube room with seeded spheres and axis-aligned boxes whose
    centres lie in the box [-obj_box, obj_box] (a scalar or per-axis half
    extents).  Objects do not overlap each other
    and stay ``clearance`` away (surface distance) from the points of
    ``keep_clear`` (the camera path)."""
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    obj_box = np.broadcast_to(np.asarray(obj_box, np.float64), (3,))
    lo = -half_room * np.ones(3)
    hi = half_room * np.ones(3)
    walls = np.stack([_rand_color(rng) for _ in range(6)])
    spheres: List[Sphere] = []
    boxes: List[Box] = []
    placed: List[Tuple[np.ndarray, float]] = []  # bounding spheres

    def ok(c, rb):
        if np.any(c - rb < lo + 0.05) or np.any(c + rb > hi - 0.05):
            return False
        for (c2, r2) in placed:
            if np.linalg.norm(c - c2) < rb + r2 + 0.02:
                return False
        if keep_clear is not None and _dist_to_path(c, keep_clear) < rb + clearance:
            return False
        return True

    tries = 0
    while len(spheres) < n_spheres:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place spheres")
        c = rng.uniform(-obj_box, obj_box, 3)
        r = rng.uniform(*r_range)
        if ok(c, r):
            spheres.append(Sphere(c, float(r), _rand_color(rng)))
            placed.append((c, r))
    tries = 0
    while len(boxes) < n_boxes:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place boxes")
        c = rng.uniform(-obj_box, obj_box, 3)
        h = rng.uniform(*box_half_range, 3)
        rb = float(np.linalg.norm(h))
        if ok(c, rb):
            boxes.append(Box(c, h, _rand_color(rng)))
            placed.append((c, rb))
    return Scene(lo, hi, walls, spheres, boxes)


def corridor_scene(seed: int, length: float = 20.0, width: float = 2.0,
                   height: float = 2.5, n_objects: int = 40) -> Scene:
    """A corridor [0, length] x [-width/2, width/2] x [0, height] with seeded
    boxes and spheres along the two side walls."""
    rng = np.random.Generator(np.random.PCG64([seed, 5]))
    lo = np.array([0.0, -width / 2, 0.0])
    hi = np.array([length, width / 2, height])
    walls = np.stack([_rand_color(rng) for _ in range(6)])
    spheres, boxes = [], []
    xs = np.sort(rng.uniform(0.5, length - 0.5, n_objects))
    for i, x in enumerate(xs):
        side = -1.0 if rng.uniform() < 0.5 else 1.0
        if rng.uniform() < 0.5:
            r = rng.uniform(0.1, 0.3)
            c = np.array([x, side * (width / 2 - r), rng.uniform(r, height - r)])
            spheres.append(Sphere(c, float(r), _rand_color(rng)))
        else:
            h = np.array([rng.uniform(0.1, 0.3), rng.uniform(0.05, 0.25), rng.uniform(0.1, 0.6)])
            c = np.array([x, side * (width / 2 - h[1]), rng.uniform(h[2], height - h[2])])
            boxes.append(Box(c, h, _rand_color(rng)))
    return Scene(lo, hi, walls, spheres, boxes)


# --------------------------------------------------------------------------
# Rendering
# --------------------------------------------------------------------------


def pixel_rays(K: Intrinsics) -> np.ndarray:
    """Camera-frame rays K^-1 [u, v, 1] for every pixel centre, (H, W, 3) f64."""
    u = np.arange(K.width, dtype=np.float64)
    v = np.arange(K.height, dtype=np.float64)
    uu, vv = np.meshgrid(u, v)
    return np.stack([(uu - K.cx) / K.fx, (vv - K.cy) / K.fy, np.ones_like(uu)], axis=-1)


def render(scene: Scene, K: Intrinsics, T_wc: np.ndarray,
           rays_c: Optional[np.ndarray] = None):
    """Ray-trace the analytic scene.  Returns (depth f32 (H,W) z-depth metres,
    rgb u8 (H,W,3), object id i32 (H,W): 0..5 walls, 6.. spheres, then boxes).
    The camera must be inside the room."""
    if rays_c is None:
        rays_c = pixel_rays(K)
    R = T_wc[:, :3]
    C = T_wc[:, 3]
    # world direction (camera z component 1).  Products are written out
    # element-wise: a BLAS call may round differently depending on how it
    # splits the work over threads, which would make frames irreproducible.
    rc = rays_c.reshape(-1, 3)
    d = np.stack([rc[:, 0] * R[a, 0] + rc[:, 1] * R[a, 1] + rc[:, 2] * R[a, 2] for a in range(3)], axis=1)
    n = d.shape[0]
    best = np.full(n, np.inf)
    obj = np.full(n, -1, np.int32)
    # room interior: exit distance along each axis
    with np.errstate(divide="ignore", invalid="ignore"):
        for a in range(3):
            da = d[:, a]
            tpos = (scene.room_hi[a] - C[a]) / da
            tneg = (scene.room_lo[a] - C[a]) / da
            t = np.where(da > 0, tpos, np.where(da < 0, tneg, np.inf))
            wall = np.where(da > 0, 2 * a + 1, 2 * a)
            m = t < best
            best = np.where(m, t, best)
            obj = np.where(m, wall, obj)
    base = 6
    a2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    for si, s in enumerate(scene.spheres):
        oc = C - s.center
        b = d[:, 0] * oc[0] + d[:, 1] * oc[1] + d[:, 2] * oc[2]
        c = (oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2]) - s.radius ** 2
        disc = b * b - a2 * c
        ok = disc >= 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t = (-b - sq) / a2
        m = ok & (t > 1e-9) & (t < best)
        best = np.where(m, t, best)
        obj = np.where(m, base + si, obj)
    base += len(scene.spheres)
    with np.errstate(divide="ignore", invalid="ignore"):
        for bi, bx in enumerate(scene.boxes):
            lo = bx.center - bx.half
            hi = bx.center + bx.half
            t1 = (lo[None, :] - C[None, :]) / d
            t2 = (hi[None, :] - C[None, :]) / d
            # axis-parallel rays: the slab test degenerates to a containment test
            par = d == 0
            inside = (C[None, :] >= lo[None, :]) & (C[None, :] <= hi[None, :])
            tmin = np.where(par, np.where(inside, -np.inf, np.inf), np.minimum(t1, t2))
            tmax = np.where(par, np.where(inside, np.inf, -np.inf), np.maximum(t1, t2))
            tn = tmin.max(axis=1)
            tf = tmax.min(axis=1)
            m = (tn <= tf) & (tn > 1e-9) & (tn < best)
            best = np.where(m, tn, best)
            obj = np.where(m, base + bi, obj)
    depth = np.where(np.isfinite(best), best, 0.0).reshape(K.height, K.width)
    obj = obj.reshape(K.height, K.width)
    palette = np.concatenate([scene.wall_colors]
                             + [s.color[None] for s in scene.spheres]
                             + [b.color[None] for b in scene.boxes], axis=0)
    rgb = palette[np.maximum(obj, 0)]
    return depth.astype(np.float32), rgb.astype(np.uint8), obj


def add_depth_noise(depth: np.ndarray, seed: int, frame: int,
                    sigma_coeff: float = 0.0015) -> np.ndarray:
    """z-dependent Gaussian noise sigma = sigma_coeff * z^2, seeded by
    (seed, frame) with PCG64; zeros (no measurement) stay zero."""
    rng = np.random.Generator(np.random.PCG64([seed, 1000 + frame]))
    z = depth.astype(np.float64)
    noisy = z + rng.normal(size=z.shape) * sigma_coeff * z * z
    noisy = np.where(z > 0, np.maximum(noisy, 1e-3), 0.0)
    return noisy.astype(np.float32)


def scene_sdf(scene: Scene, pts: np.ndarray) -> np.ndarray:
    """Signed distance (metres) to the scene surface, positive in free space
    (inside the room and outside every object).  ``pts``: (..., 3)."""
    p = np.asarray(pts, np.float64)
    d_room = np.minimum((p - scene.room_lo).min(axis=-1), (scene.room_hi - p).min(axis=-1))
    out = d_room
    for s in scene.spheres:
        out = np.minimum(out, np.linalg.norm(p - s.center, axis=-1) - s.radius)
    for b in scene.boxes:
        q = np.abs(p - b.center) - b.half
        outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
        inside = np.minimum(q.max(axis=-1), 0.0)
        out = np.minimum(out, outside + inside)
    return out


# --------------------------------------------------------------------------
# Workloads shaped like the paper's experiments
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Sequence_:
    scene: Scene
    K: Intrinsics
    poses: List[np.ndarray]
    seed: int
    noise: bool = True

    def frame(self, i: int, rays_c: Optional[np.ndarray] = None):
        depth, rgb, obj = render(self.scene, self.K, self.poses[i], rays_c)
        if self.noise:
            depth = add_depth_noise(depth, self.seed, i)
        return depth, rgb

    def frames(self, idx: Sequence[int], threads: int = 8):
        """Render several frames (numpy releases the GIL, so threads help)."""
        from concurrent.futures import ThreadPoolExecutor
        rays = pixel_rays(self.K)
        with ThreadPoolExecutor(max_workers=threads) as ex:
            return list(ex.map(lambda i: self.frame(i, rays), idx))


def small_room_sequence(seed: int = 1, n_frames: int = 10, K: Intrinsics = K_QVGA,
                        noise: bool = True) -> Sequence_:
    """4 m room with 3 spheres (r in 0.2-0.5 m), camera on a 1 m circle
    looking at the centre (320x240, f = 262.5 by default)."""
    poses = circle_trajectory(seed, n_frames, radius=1.0)
    a = np.linspace(0, 2 * np.pi, 720, endpoint=False)
    circle = np.stack([np.cos(a), np.sin(a), np.zeros_like(a)], axis=1)
    # centres kept within +-0.5 m of the camera plane so the spheres are seen
    scene = room_scene(seed, 3, 0, obj_box=(1.6, 1.6, 0.5), keep_clear=circle,
                       clearance=0.3)
    return Sequence_(scene, K, poses, seed, noise)


def large_room_sequence(seed: int = 2, n_frames: int = 300, noise: bool = True) -> Sequence_:
    """4 m room with 6 spheres + 6 boxes, handheld 0.5 m/s path, 640x480."""
    poses = handheld_trajectory(seed, n_frames)
    path = np.stack([T[:, 3] for T in poses])
    scene = room_scene(seed, 6, 6, obj_box=1.5, keep_clear=path, clearance=0.3)
    return Sequence_(scene, K_VGA, poses, seed, noise)


def corridor_sequence(seed: int = 3, n_frames: int = 2000, noise: bool = True) -> Sequence_:
    poses = corridor_trajectory(seed, n_frames)
    scene = corridor_scene(seed)
    return Sequence_(scene, K_VGA, poses, seed, noise)


def room_volumes(seed: int, voxel_size: float, room: float = 4.0,
                 dims_choices=(128, 192, 256, 320, 384), max_volumes: int = 4):
    """Seeded volume layout of one room for the many-scene batched workload:
    1..max_volumes cubic volumes with dims drawn from dims_choices, at seeded
    integer offsets inside the room on a grid whose origin is the room's
    lower corner.  Returns [(offset (3,), dims (3,))]."""
    rng = np.random.Generator(np.random.PCG64([seed, 17]))
    n_room = int(round(room / voxel_size))
    out = []
    for _ in range(int(rng.integers(1, max_volumes + 1))):
        d = int(rng.choice(dims_choices))
        span = max(1, n_room - d)
        off = rng.integers(0, span, 3)
        out.append((tuple(int(x) for x in off), (d, d, d)))
    return out


def multi_room_workload(n_rooms: int = 32, n_frames: int = 100, seed0: int = 1000):
    """Independent 4 m rooms (3 spheres + 2 boxes each) with handheld paths at
    640x480, seeds seed0 + i."""
    out = []
    for i in range(n_rooms):
        seed = seed0 + i
        poses = handheld_trajectory(seed, n_frames)
        path = np.stack([T[:, 3] for T in poses])
        scene = room_scene(seed, 3, 2, obj_box=1.5, keep_clear=path, clearance=0.3)
        out.append(Sequence_(scene, K_VGA, poses, seed, True))
    return out
