"""Seeded synthetic inputs for the superquadric renderer.

This module only *draws* inputs: superquadric scenes, pinhole camera rigs and
upstream gradients.  It contains none of the renderer's arithmetic (no
occupancy, no voxel lookup, no compositing), so both the FP64 oracle and the
HIP path can consume its arrays without sharing any of the method.

Every array handed to either side is float32 (or int32) and C-contiguous.
Scenes stand in for nuScenes surround-camera frames on the Occ3D grid
(Sec. "Datasets and Metrics": [-40,40]^2 x [-1,5.4] m at 0.4 m); no dataset
or trained primitives are needed or used.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SEED_BASE = 17361


@dataclass
class Grid:
    """Axis-aligned voxel grid.  Voxel (ix, iy, iz) covers
    [lo + i*voxel, lo + (i+1)*voxel); linear id v = (ix*Y + iy)*Z + iz."""
    lo: tuple
    voxel: float
    dims: tuple
    nv: int = 5  # neighbourhood half-width N_v (Sec. "Implementation Details")
    theta: float = 0.0  # influence threshold of the index (0: the N_v cube)

    @property
    def n_voxels(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])


@dataclass
class Prims:
    """N superquadrics S_i = {m, s, r, eps, sigma, c} (Sec. "SuperQuadrics")."""
    means: np.ndarray      # [N,3] f32 centre m
    quats: np.ndarray      # [N,4] f32 quaternion r, (w, x, y, z)
    scales: np.ndarray     # [N,3] f32 s = (s_x, s_y, s_z)
    eps: np.ndarray        # [N,2] f32 (eps1, eps2)
    opacity: np.ndarray    # [N]   f32 density sigma
    logits: np.ndarray     # [N,C] f32 semantic logits c

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_classes(self) -> int:
        return int(self.logits.shape[1])

    def subset(self, idx) -> "Prims":
        idx = np.asarray(idx)
        return Prims(*(np.ascontiguousarray(a[idx]) for a in
                       (self.means, self.quats, self.scales, self.eps, self.opacity, self.logits)))


@dataclass
class Rays:
    """Per-pixel rays r(t) = o + t d with |d| = 1 (rounded to f32)."""
    origins: np.ndarray    # [cams,H,W,3] f32
    dirs: np.ndarray       # [cams,H,W,3] f32

    @property
    def shape(self):
        return self.origins.shape[:3]

    @property
    def n_rays(self) -> int:
        c, h, w = self.shape
        return int(c * h * w)


@dataclass
class March:
    """L uniformly spaced samples in [t_near, t_far], endpoints included."""
    n_samples: int
    t_near: float
    t_far: float
    ckpt_every: int = 0
    kappa: float = 0.0     # early ray termination threshold (0 = none)


@dataclass
class Scene:
    grid: Grid
    prims: Prims
    rays: Rays
    march: March
    name: str = ""
    meta: dict = field(default_factory=dict)


def rng_for(config: int, scene: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 100 * config + scene))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def random_quats(rng, n) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def log_uniform(rng, lo, hi, size) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def make_prims(rng, means, scale_lo, scale_hi, n_classes, eps_lo=0.2, eps_hi=1.8) -> Prims:
    n = means.shape[0]
    quats = random_quats(rng, n)
    scales = log_uniform(rng, scale_lo, scale_hi, (n, 3))
    eps = rng.uniform(eps_lo, eps_hi, (n, 2))
    # sigma ~ U(0,1): reject an exact 0 draw so the open interval holds
    opacity = rng.uniform(0.0, 1.0, n)
    opacity[opacity == 0.0] = 0.5
    logits = rng.standard_normal((n, n_classes))
    return Prims(_f32(means), _f32(quats), _f32(scales), _f32(eps), _f32(opacity), _f32(logits))


def pinhole_rig(n_cams, width, height, hfov_deg, position, yaw0_deg=0.0, yaw_step_deg=60.0,
                pitch_deg=0.0) -> Rays:
    """Pinhole cameras with pixel centres at +0.5, f = (W/2)/tan(HFOV/2), principal
    point at the image centre, OpenCV camera axes (x right, y down, z forward).

    The world (ego) frame has x forward, y left, z up; camera k looks along yaw
    yaw0 + k*yaw_step.  Directions are built and normalised in FP64 and then
    rounded to f32; both the oracle and the kernels consume the rounded arrays.
    """
    fx = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    cx, cy = width / 2.0, height / 2.0
    u = (np.arange(width, dtype=np.float64) + 0.5 - cx) / fx
    v = (np.arange(height, dtype=np.float64) + 0.5 - cy) / fx
    uu, vv = np.meshgrid(u, v)                        # [H,W]
    cam = np.stack([uu, vv, np.ones_like(uu)], -1)    # camera frame
    dirs = np.empty((n_cams, height, width, 3))
    pitch = math.radians(pitch_deg)
    for k in range(n_cams):
        yaw = math.radians(yaw0_deg + yaw_step_deg * k)
        fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
        right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
        down = np.cross(fwd, right)
        d = cam[..., 0:1] * right + cam[..., 1:2] * down + cam[..., 2:3] * fwd
        dirs[k] = d / np.linalg.norm(d, axis=-1, keepdims=True)
    origins = np.broadcast_to(np.asarray(position, dtype=np.float64), dirs.shape)
    return Rays(_f32(origins), _f32(dirs))


OCC3D_GRID = dict(lo=(-40.0, -40.0, -1.0), voxel=0.4, dims=(200, 200, 16))


def _ground_heavy_centres(rng, n):
    """x, y ~ U[-40,40]; 70% of z ~ U[-1,0.5], 30% ~ U(0.5,5.4]."""
    xy = rng.uniform(-40.0, 40.0, (n, 2))
    low = rng.uniform(0.0, 1.0, n) < 0.7
    z = np.where(low, rng.uniform(-1.0, 0.5, n), rng.uniform(0.5, 5.4, n))
    return np.concatenate([xy, z[:, None]], 1)


def config(cfg: int, scene: int = 0, n_prims: int | None = None) -> Scene:
    """Five seeded workloads, numbered 0..4:

    0: tiny 16x16x4 grid at 0.5 m, 64 SQs, 1 camera 64x48, L=32 to 12 m, C=4.
    1: Occ3D-shaped grid, 6,400 SQs, 6 cameras 352x200, L=100 to 45 m, C=17.
    2: as 1 (forward+backward).
    3: as 1 with per-scene counts {2k,4k,6.4k,8k,12k,16k,20k,25.6k} (scene = 0..7).
    4: 25,600 SQs (40% in 64 blobs of radius 2 m), 6 cameras 1600x900, L=200 to 50 m.
    """
    rng = rng_for(cfg, scene)
    if cfg == 0:
        grid = Grid(lo=(-4.0, -4.0, -1.0), voxel=0.5, dims=(16, 16, 4), nv=5)
        n = 64 if n_prims is None else n_prims
        hi = np.array(grid.lo) + np.array(grid.dims) * grid.voxel
        means = rng.uniform(np.array(grid.lo), hi, (n, 3))
        prims = make_prims(rng, means, 0.2, 1.5, 4)
        rays = pinhole_rig(1, 64, 48, 90.0, (0.0, 0.0, 0.0))
        march = March(32, 0.1, 12.0)
    elif cfg in (1, 2, 3):
        grid = Grid(**OCC3D_GRID, nv=5)
        if cfg == 3:
            counts = (2000, 4000, 6400, 8000, 12000, 16000, 20000, 25600)
            n = counts[scene] if n_prims is None else n_prims
        else:
            n = 6400 if n_prims is None else n_prims
        means = _ground_heavy_centres(rng, n)
        prims = make_prims(rng, means, 0.2, 3.0, 17)
        rays = pinhole_rig(6, 352, 200, 90.0, (0.0, 0.0, 1.5))
        march = March(100, 0.1, 45.0)
    elif cfg == 4:
        grid = Grid(**OCC3D_GRID, nv=5)
        n = 25600 if n_prims is None else n_prims
        n_bg = int(round(0.6 * n))
        n_blob_total = n - n_bg
        n_blobs = 64
        bg = _ground_heavy_centres(rng, n_bg)
        blob_c = np.concatenate([rng.uniform(-38.0, 38.0, (n_blobs, 2)),
                                 rng.uniform(-1.0, 3.0, (n_blobs, 1))], 1)
        per = np.full(n_blobs, n_blob_total // n_blobs)
        per[: n_blob_total - per.sum()] += 1
        owner = np.repeat(np.arange(n_blobs), per)
        # uniform in a ball of radius 2 m
        dvec = rng.standard_normal((n_blob_total, 3))
        dvec /= np.linalg.norm(dvec, axis=1, keepdims=True)
        rad = 2.0 * rng.uniform(0.0, 1.0, n_blob_total) ** (1.0 / 3.0)
        members = blob_c[owner] + dvec * rad[:, None]
        lo = np.array(grid.lo)
        hi = lo + np.array(grid.dims) * grid.voxel
        members = np.clip(members, lo, hi - 1e-3)
        means = np.concatenate([bg, members], 0)
        prims = make_prims(rng, means, 0.2, 3.0, 17)
        rays = pinhole_rig(6, 1600, 900, 90.0, (0.0, 0.0, 1.5))
        march = March(200, 0.1, 50.0)
    else:
        raise ValueError(f"unknown config {cfg}")
    return Scene(grid, prims, rays, march, name=f"cfg{cfg}_s{scene}")


def paper_render_scene(seed: int = 0) -> Scene:
    """The render setting of the paper's implementation details (Sec. 4,
    "Implementation Details"), whose render time Table tab:ablation_render_occ
    reports: 6 surround cameras at 704x256, N = 1,600 superquadrics, N_v = 5,
    L = 100 samples in [0.1, 40] m without early termination, on the Occ3D
    grid (200x200x16 at 0.4 m), C = 17.  The primitives are drawn like those of
    workloads 1-3 (ground-heavy centres, scales 0.2-3 m), not trained ones; the
    cameras have a 70 degree horizontal field of view, 60 degrees apart."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 900 + seed))
    grid = Grid(**OCC3D_GRID, nv=5)
    prims = make_prims(rng, _ground_heavy_centres(rng, 1600), 0.2, 3.0, 17)
    rays = pinhole_rig(6, 704, 256, 70.0, (0.0, 0.0, 1.5))
    return Scene(grid, prims, rays, March(100, 0.1, 40.0), name=f"paper_render_s{seed}")


def upstream_grads(rng, rays: Rays, n_classes: int):
    """g_D ~ N(0,1) per pixel, g_S ~ N(0,1) per pixel and class; layouts
    [cams,H,W] and [cams,C,H,W]."""
    c, h, w = rays.shape
    g_d = _f32(rng.standard_normal((c, h, w)))
    g_s = _f32(rng.standard_normal((c, n_classes, h, w)))
    return g_d, g_s


def pseudo_labels(rng, rays: Rays, n_classes: int, t_near: float, t_far: float, unlabelled: float = 0.15):
    """Stand-ins for the 2D pseudo-labels of the training loss (semantic
    class per pixel, metric depth per pixel), layouts [cams,H,W]: classes
    uniform in [0, C) with a fraction `unlabelled` set to -1, depths uniform in
    [t_near, t_far] with a fraction `unlabelled` set to 0 (no depth)."""
    c, h, w = rays.shape
    sem = rng.integers(0, n_classes, (c, h, w)).astype(np.int32)
    sem[rng.random((c, h, w)) < unlabelled] = -1
    depth = _f32(rng.uniform(t_near, t_far, (c, h, w)))
    depth[rng.random((c, h, w)) < unlabelled] = 0.0
    return sem, depth


def sub_rays(rays: Rays, cams=None, rows=None, cols=None) -> Rays:
    """A rectangular window of the rig (same layout, smaller H/W)."""
    o, d = rays.origins, rays.dirs
    if cams is not None:
        o, d = o[cams], d[cams]
    if rows is not None:
        o, d = o[:, rows], d[:, rows]
    if cols is not None:
        o, d = o[:, :, cols], d[:, :, cols]
    return Rays(np.ascontiguousarray(o), np.ascontiguousarray(d))
