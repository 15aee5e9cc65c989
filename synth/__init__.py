"""Seeded synthetic inputs shared by the HIP path's tests, the oracle and the benchmark.

This module holds no arithmetic of the rendering method itself: it only draws raw
parameters, places cameras and draws upstream gradients. Everything is numpy
``default_rng`` seeded, so both sides of a parity test see bit-identical float32
inputs.

Parameter layout (float32, structure of arrays, shape ``[76, N]``):

====== ===== ==========================================================
rows   count meaning
====== ===== ==========================================================
0-2    3     spatial mean mu_p (x, y, z)
3-5    3     direction mean mu_d
6-26   21    raw lower-triangular 6x6 Cholesky entries, row-major
             packed: entry (i, j), j <= i, sits at row 6 + i(i+1)/2 + j
27-74  48    SH coefficients, row 27 + 3*k + c for basis k, channel c
75     1     opacity logit
====== ===== ==========================================================

The 6D Gaussian parameter set (position, direction, 6x6 covariance through a
Cholesky factor, opacity, colour) is the paper's Sec. 3.1; the SH colour with
48 coefficients is Sec. 4.2. Raw values are drawn here; activations belong to
the method and are applied by the renderer and the oracle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NROWS = 76
ROW_MU_P = 0
ROW_MU_D = 3
ROW_L = 6
ROW_SH = 27
ROW_OPACITY = 75

# Packed index of Cholesky entry (i, j), j <= i.
def tri_index(i: int, j: int) -> int:
    return i * (i + 1) // 2 + j


DIAG_SPATIAL = [tri_index(i, i) for i in range(3)]          # 0, 2, 5
DIAG_DIRECTION = [tri_index(i, i) for i in range(3, 6)]     # 9, 14, 20
CROSS_BLOCK = [tri_index(i, j) for i in range(3, 6) for j in range(3)]  # L_dp
OFFDIAG_SPATIAL = [tri_index(1, 0), tri_index(2, 0), tri_index(2, 1)]
OFFDIAG_DIRECTION = [tri_index(4, 3), tri_index(5, 3), tri_index(5, 4)]

SEED_SCENE = 0
SEED_PERTURB = 1
SEED_UPSTREAM = 2
SEED_FD_SUBSET = 3


@dataclass
class Camera:
    """Pinhole camera, world -> camera ``p = R x + t`` with OpenCV axes
    (x right, y down, z forward). Pixel (i, j) has its centre at (i + .5, j + .5)."""

    R: np.ndarray  # (3, 3) float64
    t: np.ndarray  # (3,) float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.t

    def as_float32(self) -> "Camera":
        """The camera as the float32 values the GPU receives (the oracle uses the
        same rounded values, so both render one and the same camera)."""
        return Camera(self.R.astype(np.float32).astype(np.float64),
                      self.t.astype(np.float32).astype(np.float64),
                      float(np.float32(self.fx)), float(np.float32(self.fy)),
                      float(np.float32(self.cx)), float(np.float32(self.cy)),
                      int(self.width), int(self.height))


def look_at_camera(center, width: int, height: int, fov_x_deg: float = 50.0,
                   target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> Camera:
    c = np.asarray(center, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ c
    fx = width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))
    cam = Camera(R, t, fx, fx, width / 2.0, height / 2.0, width, height)
    return cam.as_float32()


def default_camera(width: int, height: int) -> Camera:
    """Radius-4 camera at elevation 20 deg, azimuth 30 deg, looking at the origin."""
    el, az = math.radians(20.0), math.radians(30.0)
    c = 4.0 * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    return look_at_camera(c, width, height)


def fibonacci_cameras(n: int, resolutions, radius: float = 4.0):
    """n cameras on a Fibonacci sphere of the given radius, looking at the origin;
    resolution k is ``resolutions[k % len(resolutions)]``."""
    golden = math.pi * (3.0 - math.sqrt(5.0))
    cams = []
    for i in range(n):
        z = 1.0 - (2.0 * i + 1.0) / n
        r = math.sqrt(max(0.0, 1.0 - z * z))
        phi = golden * i
        c = radius * np.array([r * math.cos(phi), r * math.sin(phi), z])
        w, h = resolutions[i % len(resolutions)]
        cams.append(look_at_camera(c, w, h))
    return cams


def _unit(rng, n):
    v = rng.normal(size=(3, n))
    return v / np.linalg.norm(v, axis=0, keepdims=True)


@dataclass
class SceneSpec:
    """Recipe for one synthetic scene (all draws from one generator, in the order
    means, direction means, 21 Cholesky rows, 48 SH rows, opacity logit)."""

    n: int
    means: str = "cube"            # "cube" U[-1,1]^3, "sphere", "mixed"
    sphere_noise: float = 0.05
    mixed_sphere_frac: float = 0.7
    mixed_cube_half: float = 2.0
    mu_d: str = "random"           # "random" unit vectors or "inward" (-normal)
    l_spatial_diag: tuple = (-3.0, 0.5)
    l_direction_diag: tuple = (-1.0, 0.3)
    l_offdiag_std: float = 0.05
    l_cross_std: float = 0.05
    sh_std: float = 0.3
    logit: tuple = (0.0, 1.0)
    seed: int = SEED_SCENE


def make_scene(spec: SceneSpec) -> np.ndarray:
    """Raw parameters, float32 ``[76, n]``."""
    rng = np.random.default_rng(spec.seed)
    n = spec.n
    out = np.empty((NROWS, n), np.float32)
    normal = None
    if spec.means == "cube":
        mu = rng.uniform(-1.0, 1.0, size=(3, n))
    elif spec.means == "sphere":
        normal = _unit(rng, n)
        mu = normal * (1.0 + rng.normal(0.0, spec.sphere_noise, size=n))
    elif spec.means == "mixed":
        n_s = int(round(spec.mixed_sphere_frac * n))
        normal = _unit(rng, n)
        mu = normal * (1.0 + rng.normal(0.0, spec.sphere_noise, size=n))
        h = spec.mixed_cube_half
        mu[:, n_s:] = rng.uniform(-h, h, size=(3, n - n_s))
    else:
        raise ValueError(spec.means)
    out[ROW_MU_P:ROW_MU_P + 3] = mu
    if spec.mu_d == "random":
        out[ROW_MU_D:ROW_MU_D + 3] = _unit(rng, n)
    elif spec.mu_d == "inward":
        if normal is None:
            normal = mu / np.linalg.norm(mu, axis=0, keepdims=True)
        out[ROW_MU_D:ROW_MU_D + 3] = -normal
    else:
        raise ValueError(spec.mu_d)
    for k in range(21):
        if k in DIAG_SPATIAL:
            m, s = spec.l_spatial_diag
        elif k in DIAG_DIRECTION:
            m, s = spec.l_direction_diag
        elif k in CROSS_BLOCK:
            m, s = 0.0, spec.l_cross_std
        else:
            m, s = 0.0, spec.l_offdiag_std
        out[ROW_L + k] = rng.normal(m, s, size=n)
    out[ROW_SH:ROW_SH + 48] = rng.normal(0.0, spec.sh_std, size=(48, n))
    out[ROW_OPACITY] = rng.normal(spec.logit[0], spec.logit[1], size=n)
    return out


def perturbed(params: np.ndarray, std: float = 0.01, seed: int = SEED_PERTURB) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (params + rng.normal(0.0, std, size=params.shape)).astype(np.float32)


def upstream_gradient(cams, seed: int = SEED_UPSTREAM):
    """dL/dI ~ N(0, 1), one float32 [3, H, W] array per camera."""
    rng = np.random.default_rng(seed)
    return [rng.normal(0.0, 1.0, size=(3, c.height, c.width)).astype(np.float32) for c in cams]


def pixel_subset(width: int, height: int, count: int, seed: int = SEED_FD_SUBSET):
    """Seeded subset of distinct pixel indices (row-major j*W + i), sorted."""
    rng = np.random.default_rng(seed)
    count = min(count, width * height)
    return np.sort(rng.choice(width * height, size=count, replace=False)).astype(np.int64)


# ---------------------------------------------------------------------------
# The workloads (rendering settings lambda_opa = 0.35, background 0, fov 50 deg).
# ---------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    scene: SceneSpec
    cameras: list = field(default_factory=list)
    train: bool = False
    description: str = ""


def workload(name: str, n_override: int | None = None) -> Workload:
    """The synthetic workloads (c0-c4, and the render-only r1, r2);
    ``n_override`` shrinks N for quick tests while keeping the recipe."""
    if name == "c0":
        spec = SceneSpec(n=1000)
        cams = [default_camera(128, 128)]
        desc = "1k 6D Gaussians in U[-1,1]^3, one 128x128 camera, forward only"
    elif name == "c1":
        spec = SceneSpec(n=100_000, means="sphere")
        cams = [default_camera(800, 800)]
        desc = "100k 6D Gaussians on a noisy unit sphere, one 800x800 camera, forward+backward"
    elif name == "c2":
        spec = SceneSpec(n=300_000, means="sphere", mu_d="inward", l_cross_std=0.3)
        cams = [default_camera(800, 800)]
        desc = ("300k 6D Gaussians on a noisy unit sphere, spatial-direction Cholesky entries "
                "N(0,0.3), mu_d = -normal, 800x800, L1 training step with Adam")
    elif name == "c3":
        spec = SceneSpec(n=500_000, means="sphere")
        cams = fibonacci_cameras(16, [(400, 400), (800, 800), (1280, 720), (1600, 900)])
        desc = "500k 6D Gaussians on a noisy sphere, 16 uneven cameras batched"
    elif name == "c4":
        spec = SceneSpec(n=1_000_000, means="mixed", l_direction_diag=(-2.0, 0.5))
        cams = fibonacci_cameras(64, [(1920, 1080)])
        desc = ("1M 6D Gaussians (70% sphere, 30% U[-2,2]^3), direction diagonal exp(N(-2,0.5)), "
                "64-camera 1920x1080 pool, 8 views per step")
    elif name == "r1":
        # render only, shaped like the paper's small volumetric scenes (~10^4 points, 1408^2 views)
        spec = SceneSpec(n=12_657, means="cube", l_spatial_diag=(-2.0, 0.5), logit=(-1.0, 1.0))
        cams = [default_camera(1408, 1408)]
        desc = "12,657 6D Gaussians filling [-1,1]^3 (volumetric), one 1408x1408 camera, forward only"
    elif name == "r2":
        # render only, shaped like the paper's larger object scenes (~1.7e5 points, 1408^2 views)
        spec = SceneSpec(n=174_746, means="sphere")
        cams = [default_camera(1408, 1408)]
        desc = "174,746 6D Gaussians on a noisy unit sphere, one 1408x1408 camera, forward only"
    else:
        raise ValueError(name)
    if n_override is not None:
        spec.n = int(n_override)
    return Workload(name, spec, cams, train=name in ("c2", "c4"), description=desc)


def c4_step_views(step: int, pool: int = 64, per_step: int = 8):
    return [(per_step * step + k) % pool for k in range(per_step)]
