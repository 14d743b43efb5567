"""Seeded synthetic inputs shaped like the paper's indoor sequences.

This module only draws random numbers and lays them out in arrays.  It holds
none of the rendering method's arithmetic (no projection, no compositing, no
gradients), so both the CPU oracle's tests and the GPU path may consume it.

Every generator draws from ``numpy.random.default_rng([config_id, seed])`` and
returns float32 arrays in planar structure-of-arrays layout:

    mean [3][N], log_scale [3][N], quat [4][N] (w, x, y, z, unit length),
    opacity_logit [N], rgb [3][N]

Cameras are pinhole, OpenCV axes (x right, y down, z forward), with a
world-to-camera rotation ``R`` (row-major 3x3) and translation ``t`` so that a
world point X maps to ``R @ X + t``.  Pixel (u, v) is sampled at integer
coordinates, so a centred principal point is ((W-1)/2, (H-1)/2).

The workloads stand in for the Replica and TUM-RGBD sequences the paper
evaluates on (Experiments section); those datasets are not used.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Axis-aligned synthetic room (metres): x in [-3, 3], y in [-1.5, 1.5],
# z in [-2.5, 2.5].
ROOM_LO = np.array([-3.0, -1.5, -2.5])
ROOM_HI = np.array([3.0, 1.5, 2.5])


@dataclass
class Gaussians:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity_logit: np.ndarray
    rgb: np.ndarray
    # Optional view-dependent colour coefficients [K-1][3][n] of degree
    # sqrt(K) - 1 (None: view-independent colour).
    sh: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @property
    def sh_degree(self) -> int:
        return 0 if self.sh is None else int(round(np.sqrt(self.sh.shape[0] + 1))) - 1

    def subset(self, idx) -> "Gaussians":
        idx = np.asarray(idx)
        return Gaussians(*(np.ascontiguousarray(a[..., idx]) for a in
                           (self.mean, self.log_scale, self.quat,
                            self.opacity_logit, self.rgb)),
                         None if self.sh is None else
                         np.ascontiguousarray(self.sh[..., idx]))

    def copy(self) -> "Gaussians":
        return Gaussians(self.mean.copy(), self.log_scale.copy(),
                         self.quat.copy(), self.opacity_logit.copy(),
                         self.rgb.copy(),
                         None if self.sh is None else self.sh.copy())


@dataclass
class Camera:
    R: np.ndarray            # float32 [3,3] world -> camera
    t: np.ndarray            # float32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2

    def crop(self, u0: int, v0: int, w: int, h: int) -> "Camera":
        """Camera seeing the window [u0, u0+w) x [v0, v0+h) of this one."""
        return Camera(self.R.copy(), self.t.copy(), self.fx, self.fy,
                      float(np.float32(self.cx - u0)),
                      float(np.float32(self.cy - v0)), w, h, self.near)


@dataclass
class Workload:
    name: str
    gaussians: Gaussians
    cameras: list
    targets: np.ndarray      # float32 [V][3][H][W]
    bg: tuple = (0.0, 0.0, 0.0)
    extra: dict = field(default_factory=dict)


def _rng(config_id: int, seed: int) -> np.random.Generator:
    return np.random.default_rng([config_id, seed])


def _attributes(rng, n):
    """Per-Gaussian attribute distributions shared by every workload."""
    log_scale = rng.normal(-3.0, 0.5, size=(3, n))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity_logit = rng.normal(0.0, 1.0, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(3, n))
    return log_scale, q, opacity_logit, rgb


def sh_coefficients(seed: int, degree: int, n: int, scale: float = 0.1,
                    config_id: int = 95) -> np.ndarray:
    """View-dependent colour coefficients [(degree+1)^2 - 1][3][n], FP32,
    normal with standard deviation `scale` (the higher-order coefficients
    of a fitted map are small next to the base colour)."""
    rng = _rng(config_id, seed)
    k = (degree + 1) ** 2 - 1
    return np.ascontiguousarray(rng.normal(0.0, scale, size=(k, 3, n)),
                                dtype=np.float32)


def with_sh(g: Gaussians, seed: int, degree: int, scale: float = 0.1) -> Gaussians:
    """A copy of g carrying coefficients from sh_coefficients."""
    out = g.copy()
    out.sh = sh_coefficients(seed, degree, g.n, scale) if degree > 0 else None
    return out


def _f32(*arrays):
    return tuple(np.ascontiguousarray(a, dtype=np.float32) for a in arrays)


def identity_camera(fx, fy, width, height, position=(0.0, 0.0, 0.0)):
    R = np.eye(3, dtype=np.float32)
    c = np.asarray(position, dtype=np.float64)
    t = (-(R.astype(np.float64) @ c)).astype(np.float32)
    return Camera(R, t, float(fx), float(fy), (width - 1) / 2.0,
                  (height - 1) / 2.0, int(width), int(height))


def frustum_gaussians(rng, n, cam: Camera, zmin=1.0, zmax=5.0) -> Gaussians:
    """Means uniform in volume inside the camera frustum between zmin and zmax.

    Depth follows the z^2 density (inverse CDF of z^3), image position is
    uniform over the pixel rectangle [-0.5, W-0.5] x [-0.5, H-0.5]; the point
    is then placed on that pixel's ray (camera at the origin, identity
    rotation).
    """
    z = np.cbrt(zmin ** 3 + rng.uniform(size=n) * (zmax ** 3 - zmin ** 3))
    u = rng.uniform(-0.5, cam.width - 0.5, size=n)
    v = rng.uniform(-0.5, cam.height - 0.5, size=n)
    mean = np.stack([(u - cam.cx) / cam.fx * z, (v - cam.cy) / cam.fy * z, z])
    ls, q, ol, rgb = _attributes(rng, n)
    return Gaussians(*_f32(mean, ls, q, ol, rgb))


def room_gaussians(rng, n, wall_frac=0.8, noise=0.02) -> Gaussians:
    """80% of means on the six walls of the room (counts proportional to wall
    area, N(0, noise) along the wall normal), 20% uniform inside the room."""
    lo, hi = ROOM_LO, ROOM_HI
    ext = hi - lo
    walls = []   # (axis, value, area)
    for ax in range(3):
        o1, o2 = [a for a in range(3) if a != ax]
        area = ext[o1] * ext[o2]
        walls.append((ax, lo[ax], area))
        walls.append((ax, hi[ax], area))
    areas = np.array([w[2] for w in walls])
    n_wall = int(round(wall_frac * n))
    which = rng.choice(len(walls), size=n_wall, p=areas / areas.sum())
    pts = rng.uniform(lo, hi, size=(n_wall, 3))
    for i, (ax, val, _) in enumerate(walls):
        sel = which == i
        pts[sel, ax] = val + rng.normal(0.0, noise, size=int(sel.sum()))
    clutter = rng.uniform(lo, hi, size=(n - n_wall, 3))
    mean = np.concatenate([pts, clutter], axis=0).T
    perm = rng.permutation(n)
    mean = mean[:, perm]
    ls, q, ol, rgb = _attributes(rng, n)
    return Gaussians(*_f32(mean, ls, q, ol, rgb))


def _rodrigues(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]],
                  [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def random_walk_poses(rng, n_views, start=(0.0, 0.0, -0.5), step_m=0.05,
                      step_deg=3.0, margin=0.5):
    """Smooth random walk of camera poses inside the room.

    Each step moves ``step_m`` metres and turns ``step_deg`` degrees; the
    rotation axis and the travel direction drift smoothly, and the travel
    direction is reflected when the camera comes within ``margin`` of a wall.
    Returns a list of (R_world_to_cam float32 [3,3], t float32 [3]).
    """
    pos = np.asarray(start, dtype=np.float64)
    Rwc = np.eye(3)                       # camera-to-world
    axis = np.array([0.0, 1.0, 0.0]) + 0.3 * rng.normal(size=3)
    dirn = np.array([0.0, 0.0, 1.0]) + 0.5 * rng.normal(size=3)
    dirn /= np.linalg.norm(dirn)
    lo, hi = ROOM_LO + margin, ROOM_HI - margin
    poses = []
    for _ in range(n_views):
        Rcw = Rwc.T
        poses.append((Rcw.astype(np.float32),
                      (-(Rcw @ pos)).astype(np.float32)))
        axis = axis / np.linalg.norm(axis) + 0.3 * rng.normal(size=3)
        Rwc = _rodrigues(axis, math.radians(step_deg)) @ Rwc
        dirn = dirn + 0.3 * rng.normal(size=3)
        dirn /= np.linalg.norm(dirn)
        new = pos + step_m * dirn
        for ax in range(3):
            if new[ax] < lo[ax] or new[ax] > hi[ax]:
                dirn[ax] = -dirn[ax]
        pos = pos + step_m * dirn
        pos = np.clip(pos, ROOM_LO + 0.05, ROOM_HI - 0.05)
    return poses


def uniform_targets(rng, n_views, width, height):
    return rng.uniform(0.0, 1.0, size=(n_views, 3, height, width)).astype(
        np.float32)


# ---------------------------------------------------------------------------
# The workloads.
# ---------------------------------------------------------------------------

def config0(seed: int = 0, n: int = 10_000) -> Workload:
    """Single view 160x120, N Gaussians uniform in the frustum at 1-5 m,
    fx = fy = 128, centred principal point, U(0,1) target."""
    rng = _rng(0, seed)
    cam = identity_camera(128.0, 128.0, 160, 120)
    g = frustum_gaussians(rng, n, cam)
    tgt = uniform_targets(rng, 1, cam.width, cam.height)
    return Workload("plain-160x120-10k", g, [cam], tgt)


def room_camera(width=1200, height=680, f=600.0, position=(0.0, 0.0, -0.5)):
    return identity_camera(f, f, width, height, position)


def config1(seed: int = 0, n: int = 300_000) -> Workload:
    """Room scene, single view 1200x680, fx = fy = 600, camera at
    (0, 0, -0.5) looking along +z, U(0,1) target."""
    rng = _rng(1, seed)
    g = room_gaussians(rng, n)
    cam = room_camera()
    tgt = uniform_targets(rng, 1, cam.width, cam.height)
    return Workload("room-1200x680-300k", g, [cam], tgt)


def config2(seed: int = 0, n_views: int = 10, variant: str = "1200x680"
            ) -> Workload:
    """Keyframe window over the room scene: ``n_views`` poses on a smooth
    random walk (0.05 m, 3 degrees per step).  Variant "640x480" uses
    N = 150k and fx = fy = 525."""
    if variant == "1200x680":
        n, w, h, f = 300_000, 1200, 680, 600.0
    elif variant == "640x480":
        n, w, h, f = 150_000, 640, 480, 525.0
    else:
        raise ValueError(variant)
    rng = _rng(2, seed)
    g = room_gaussians(rng, n)
    cams = []
    for R, t in random_walk_poses(rng, n_views):
        cams.append(Camera(R, t, f, f, (w - 1) / 2.0, (h - 1) / 2.0, w, h))
    tgt = uniform_targets(rng, n_views, w, h)
    return Workload(f"window{n_views}-{variant}-{n // 1000}k", g, cams, tgt)


def config3_crop(seed: int = 0, n: int = 300_000, size: int = 64,
                 u0: int = 568, v0: int = 308) -> Workload:
    """A size x size crop camera of the room view (principal point shifted)
    for full gradient checks."""
    base = config1(seed, n)
    cam = base.cameras[0].crop(u0, v0, size, size)
    rng = _rng(3, seed)
    tgt = uniform_targets(rng, 1, size, size)
    return Workload(f"crop{size}-room-{n // 1000}k", base.gaussians, [cam], tgt)


@dataclass
class KeyframePoints:
    camera: Camera
    image: np.ndarray        # float32 [3][H][W]
    pts_uvd: np.ndarray      # float32 [K][3]: patch centre (u, v), inverse depth


def insertion_stream(seed: int = 0, n_kf: int = 200, n_patches: int = 96,
                     width: int = 1200, height: int = 680, f: float = 600.0,
                     zmin: float = 1.0, zmax: float = 5.0):
    """Keyframes on the random walk, each with ``n_patches`` sparse patch
    centres at integer pixels (the 3x3 patch stays inside the image) and a
    depth drawn from U(zmin, zmax), given as inverse depth, plus a U(0,1)
    keyframe image.  Stands in for the visual-odometry front end."""
    rng = _rng(3, seed)
    out = []
    for R, t in random_walk_poses(rng, n_kf):
        cam = Camera(R, t, f, f, (width - 1) / 2.0, (height - 1) / 2.0,
                     width, height)
        u = rng.integers(1, width - 1, size=n_patches)
        v = rng.integers(1, height - 1, size=n_patches)
        z = rng.uniform(zmin, zmax, size=n_patches)
        pts = np.stack([u, v, 1.0 / z], axis=1).astype(np.float32)
        img = rng.uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)
        out.append(KeyframePoints(cam, img, pts))
    return out


def tiny_scene(seed: int, n: int = 40, width: int = 33, height: int = 29,
               f: float = 40.0, zmin: float = 1.0, zmax: float = 3.0,
               log_scale_mu: float = -2.0, config_id: int = 90) -> Workload:
    """Small scenes for brute force and finite differences: a handful of
    Gaussians in a small frustum, large enough on screen to overlap."""
    rng = _rng(config_id, seed)
    cam = identity_camera(f, f, width, height)
    g = frustum_gaussians(rng, n, cam, zmin, zmax)
    g.log_scale[:] = rng.normal(log_scale_mu, 0.4, size=(3, n)).astype(np.float32)
    tgt = uniform_targets(rng, 1, width, height)
    return Workload(f"tiny{width}x{height}-{n}", g, [cam], tgt)


# ---------------------------------------------------------------------------
# Synthetic visual-odometry stand-in for mapping runs.
# ---------------------------------------------------------------------------

def wall_depth(cam: Camera, u, v):
    """Camera-space depth z at which the rays through pixels (u, v) leave the
    room box (the true surface depth of the room's walls)."""
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    centre = -R.T @ t
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    dirs_cam = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy,
                         np.ones_like(u)])                      # z = 1
    dirs = R.T @ dirs_cam                                       # world
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = np.where(dirs > 0, (ROOM_HI[:, None] - centre[:, None]) / dirs,
                      np.where(dirs < 0,
                               (ROOM_LO[:, None] - centre[:, None]) / dirs,
                               np.inf))
    return tx.min(0)                 # ray parameter = camera z (dirs_cam z = 1)


@dataclass
class MappingStream:
    cameras: list            # keyframe cameras
    pts: list                # per keyframe float32 [K][3] (u, v, inverse depth)
    gt: Gaussians            # ground-truth scene the keyframe images show


def mapping_stream(seed: int, n_kf: int, width: int = 320, height: int = 240,
                   f: float = 260.0, n_gt: int = 100_000, n_patches: int = 96,
                   wall_frac: float = 1.0, config_id: int = 4):
    """A mapping run: keyframes on the random walk, a ground-truth room scene
    to render their images from, and per keyframe ``n_patches`` patch centres
    (integer pixels, the 3x3 patch inside the image) with the true inverse
    depth of the wall they see."""
    rng = _rng(config_id, seed)
    gt = room_gaussians(rng, n_gt, wall_frac=wall_frac)
    cams, pts = [], []
    for R, t in random_walk_poses(rng, n_kf):
        cam = Camera(R, t, f, f, (width - 1) / 2.0, (height - 1) / 2.0,
                     width, height)
        u = rng.integers(1, width - 1, size=n_patches)
        v = rng.integers(1, height - 1, size=n_patches)
        z = wall_depth(cam, u, v)
        cams.append(cam)
        pts.append(np.stack([u, v, 1.0 / z], 1).astype(np.float32))
    return MappingStream(cams, pts, gt)
