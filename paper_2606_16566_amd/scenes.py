"""Seeded synthetic scenes and cameras for the Gaussian-splatting rasterizer.

This module only draws random inputs and builds camera poses.  It holds none of
the rasterizer's arithmetic, so both the GPU path and the FP64 reference can be
fed from it.  Every array is float32, C-contiguous, in the raw parameterisation
the projection step consumes:

* ``means3d``        [N, 3]   world-space centres
* ``log_scales``     [N, 3]   natural log of the per-axis standard deviations
* ``quats``          [N, 4]   unnormalised rotation quaternions, (w, x, y, z)
* ``opacity_logits`` [N]      logits of the opacity
* ``sh``             [N, K, 3] spherical-harmonic coefficients, K = (deg+1)^2

The five workloads below stand in for the trained scenes of the paper's
experiments (Mip-NeRF 360, Tanks & Temples, Deep Blending), which are not
available: they reproduce the sizes (10k to 10M Gaussians), the resolutions
(256^2 up to 1080p, 16 mixed views) and the overlap structure (uniform clouds
and heavily overlapping anisotropic clusters).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Camera", "Scene", "look_at_camera", "make_config", "make_fd_scene",
           "make_target", "CONFIG_NAMES"]


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    ``viewmat`` is the world-to-camera transform [R | t] (3x4, row-major).
    Pixel (i, j) has its centre at image coordinates (i, j); the principal
    point is the image centre ((W-1)/2, (H-1)/2).
    """
    viewmat: np.ndarray          # (3, 4) float32
    campos: np.ndarray           # (3,) float32, camera centre in world space
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    @property
    def tan_fovx(self) -> float:
        """tan of half the horizontal field of view."""
        return float(np.float32(self.width / (2.0 * self.fx)))

    @property
    def tan_fovy(self) -> float:
        return float(np.float32(self.height / (2.0 * self.fy)))

    @property
    def tiles_x(self) -> int:
        return (self.width + 15) // 16

    @property
    def tiles_y(self) -> int:
        return (self.height + 15) // 16

    @property
    def num_tiles(self) -> int:
        return self.tiles_x * self.tiles_y

    @property
    def num_pixels(self) -> int:
        return self.width * self.height


@dataclass
class Scene:
    name: str
    means3d: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    cameras: list = field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.means3d.shape[0])

    @property
    def sh_degree(self) -> int:
        return int(round(math.sqrt(self.sh.shape[1]))) - 1

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.name + "-subset", *(np.ascontiguousarray(a[idx]) for a in (
            self.means3d, self.log_scales, self.quats, self.opacity_logits, self.sh)),
            cameras=list(self.cameras))


def _focal_for_fov(width: int, fov_x_deg: float) -> float:
    return width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))


def look_at_camera(position, target, width: int, height: int, fov_x_deg: float = 60.0,
                   znear: float = 0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera at ``position`` looking at ``target``; image y points along world +y
    ("down") when the camera looks along +z."""
    pos = np.asarray(position, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, -1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    rot = np.stack([right, down, fwd])              # rows: camera axes in world space
    trans = -rot @ pos
    viewmat = np.concatenate([rot, trans[:, None]], axis=1).astype(np.float32)
    f = np.float32(_focal_for_fov(width, fov_x_deg))
    return Camera(viewmat=viewmat, campos=pos.astype(np.float32), fx=float(f), fy=float(f),
                  cx=(width - 1) / 2.0, cy=(height - 1) / 2.0, width=width, height=height,
                  znear=znear, bg=tuple(float(b) for b in bg))


def _sh_coeffs(rng: np.random.Generator, n: int, degree: int) -> np.ndarray:
    """DC coefficients uniform in [-sqrt(pi), sqrt(pi)] (so the degree-0 colour is
    uniform in [0, 1]); higher-order coefficients N(0, 0.1)."""
    k = (degree + 1) ** 2
    sh = np.empty((n, k, 3), dtype=np.float32)
    sh[:, 0, :] = rng.uniform(-math.sqrt(math.pi), math.sqrt(math.pi), size=(n, 3)).astype(np.float32)
    if k > 1:
        sh[:, 1:, :] = (0.1 * rng.standard_normal(size=(n, k - 1, 3), dtype=np.float32))
    return sh


def _uniform_cloud(rng, n: int, degree: int, centre=(0.0, 0.0, 4.0), log_scale_mu=-4.0,
                   log_scale_sigma=0.5):
    means = (rng.uniform(-1.0, 1.0, size=(n, 3)) + np.asarray(centre)).astype(np.float32)
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, size=(n, 3)).astype(np.float32)
    quats = rng.standard_normal(size=(n, 4), dtype=np.float32)
    logits = rng.standard_normal(size=n, dtype=np.float32)
    sh = _sh_coeffs(rng, n, degree)
    return means, log_scales, quats, logits, sh


def _random_rotations(rng, m: int) -> np.ndarray:
    """m random orthonormal 3x3 matrices (QR of Gaussian matrices)."""
    a = rng.standard_normal(size=(m, 3, 3))
    q, r = np.linalg.qr(a)
    q *= np.sign(np.einsum("bii->bi", r))[:, None, :]
    return q


def _clustered(rng, n: int, blobs: int, degree: int, extent_scale: float = 1.0):
    centres = rng.uniform(-5.0, 5.0, size=(blobs, 3))
    rots = _random_rotations(rng, blobs)
    major = rng.uniform(0.25, 1.0, size=blobs) * extent_scale
    minor = major[:, None] / rng.uniform(1.0, 20.0, size=(blobs, 2))
    stds = np.concatenate([major[:, None], minor], axis=1)          # (blobs, 3)
    owner = np.repeat(np.arange(blobs), -(-n // blobs))[:n]
    offs = rng.standard_normal(size=(n, 3)) * stds[owner]
    offs = np.einsum("nij,nj->ni", rots[owner], offs)
    means = (centres[owner] + offs).astype(np.float32)
    log_scales = rng.normal(-5.0, 1.0, size=(n, 3)).astype(np.float32)
    quats = rng.standard_normal(size=(n, 4), dtype=np.float32)
    logits = rng.normal(-1.0, 1.5, size=n).astype(np.float32)
    sh = _sh_coeffs(rng, n, degree)
    return means, log_scales, quats, logits, sh


CONFIG_NAMES = {
    1: "uniform-10k-256x256-sh0",
    2: "uniform-1M-1920x1080-sh3",
    3: "clustered-6M-1264x832-sh3",
    4: "uniform-3M-1920x1080-sh0-fwdbwd",
    5: "clustered-10M-16views-mixed",
}

_C5_RES = [(640, 480), (1280, 720), (1920, 1080), (1264, 832)]


def make_config(k: int, seed: int | None = None, n: int | None = None) -> Scene:
    """Build workload ``k`` (1..5).  ``n`` overrides the Gaussian count (same
    recipe, used for reduced-size parity cases)."""
    rng = np.random.default_rng(k if seed is None else seed)
    if k == 1:
        arrs = _uniform_cloud(rng, n or 10_000, 0)
        cams = [look_at_camera((0, 0, 0), (0, 0, 1), 256, 256)]
    elif k == 2:
        arrs = _uniform_cloud(rng, n or 1_000_000, 3)
        cams = [look_at_camera((0, 0, 0), (0, 0, 1), 1920, 1080)]
    elif k == 3:
        arrs = _clustered(rng, n or 6_000_000, 200, 3)
        cams = [look_at_camera((0, 0, -9), (0, 0, 0), 1264, 832)]
    elif k == 4:
        arrs = _uniform_cloud(rng, n or 3_000_000, 0)
        cams = [look_at_camera((0, 0, 0), (0, 0, 1), 1920, 1080)]
    elif k == 5:
        arrs = _clustered(rng, n or 10_000_000, 60, 3, extent_scale=2.0)
        cams = []
        for v in range(16):
            th = 2.0 * math.pi * v / 16.0
            w, h = _C5_RES[v % 4]
            cams.append(look_at_camera((12 * math.sin(th), 0.0, -12 * math.cos(th)), (0, 0, 0), w, h))
    else:
        raise ValueError(f"unknown workload {k}")
    return Scene(CONFIG_NAMES[k], *arrs, cameras=cams)


def make_fd_scene(degree: int = 0, n: int = 2000, size: int = 64, seed: int = 404) -> Scene:
    """Small uniform-cloud scene for finite-difference gradient checks."""
    rng = np.random.default_rng(seed)
    arrs = _uniform_cloud(rng, n, degree)
    return Scene(f"fd-{n}-{size}-sh{degree}", *arrs,
                 cameras=[look_at_camera((0, 0, 0), (0, 0, 1), size, size)])


def make_target(height: int, width: int, seed: int) -> np.ndarray:
    """Uniform-random target image [3, H, W] for the L1 loss."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)


def random_projected(rng: np.random.Generator, n: int, width: int, height: int,
                     sigma_px=(0.3, 12.0), margin: float = 20.0):
    """Random screen-space splats for render-only cases: centre [n,2], conic
    [n,3] as (a, b, c) of the quadratic form a*dx^2 + 2b*dx*dy + c*dy^2
    (positive definite by construction: |b| < sqrt(a*c)), opacity [n],
    colour [n,3] and a positive depth [n].  All float32."""
    cen = np.stack([rng.uniform(-margin, width - 1 + margin, n),
                    rng.uniform(-margin, height - 1 + margin, n)], 1)
    sig = np.exp(rng.uniform(np.log(sigma_px[0]), np.log(sigma_px[1]), size=(n, 2)))
    a = 1.0 / sig[:, 0] ** 2
    c = 1.0 / sig[:, 1] ** 2
    b = rng.uniform(-0.95, 0.95, n) * np.sqrt(a * c)
    conic = np.stack([a, b, c], 1)
    opac = rng.uniform(0.02, 0.99, n)
    col = rng.uniform(0, 1, (n, 3))
    depth = rng.uniform(1.0, 10.0, n)
    f = lambda x: np.ascontiguousarray(x, dtype=np.float32)
    return f(cen), f(conic), f(opac), f(col), f(depth)
