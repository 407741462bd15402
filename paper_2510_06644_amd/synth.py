"""Seeded synthetic RGB-D SLAM scenes.

This module only draws random inputs.  It holds none of the rasterizer's
arithmetic (no activation, projection, compositing or gradients), so both the
HIP path and the CPU oracle may consume what it produces.

Every generator uses numpy's PCG64 with an explicit seed.  Scenes are returned
as float32 arrays in the library's layout:

* ``means``          [N, 3]  world-space centres
* ``log_scales``     [N, 3]  per-axis log standard deviations
* ``quats``          [N, 4]  rotation quaternions, (w, x, y, z), not normalised
* ``opacity_logits`` [N]     logits of the opacity
* ``colors``         [N, 3]  RGB (spherical-harmonic degree 0, used as is)

The workloads follow the shapes of the paper's RGB-D datasets (Table 3:
640x480 for TUM-RGBD, 1200x680 for Replica); the datasets themselves are not
used, these random scenes stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Camera", "Scene", "SceneSpec", "CONFIGS", "make_camera", "make_scene",
    "perturb_scene", "pose_offset", "upstream_grads", "fd_crop_spec",
    "SERVING_CLASSES",
]


@dataclasses.dataclass(frozen=True)
class Camera:
    """Pinhole intrinsics; the pose (3x4 world->camera) travels separately."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    colors: np.ndarray

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits,
                self.colors)


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    """Distribution of one synthetic workload."""
    name: str
    width: int
    height: int
    n: int
    seed: int
    log_scale_mean: float = -4.0
    log_scale_std: float = 0.5
    z_near: float = 0.5
    z_far: float = 5.0
    transparent_frac: float = 0.0     # share drawn with opacity U(0.005, 0.05)
    focal_frac: float = 0.8           # fx = fy = focal_frac * width


# The five workloads: a small parity case, tracking at 640x480, mapping at
# 1200x680, the differentiation case at 1200x680, and the serving mix.
CONFIGS = {
    "c0": SceneSpec("c0_128x128_2k", 128, 128, 2_000, 1000),
    "c1": SceneSpec("c1_track_640x480_100k", 640, 480, 100_000, 1001),
    "c2": SceneSpec("c2_map_1200x680_300k", 1200, 680, 300_000, 1002,
                    log_scale_mean=-4.5, log_scale_std=0.7,
                    transparent_frac=0.2),
    "c3": SceneSpec("c3_diff_1200x680_500k", 1200, 680, 500_000, 1003,
                    log_scale_mean=-4.5, log_scale_std=0.7,
                    transparent_frac=0.2),
}

# Serving mix: (count, width, height, gaussians, scene distribution)
SERVING_CLASSES = (
    (6, 320, 240, 20_000, "c0"),
    (6, 640, 480, 100_000, "c0"),
    (4, 1200, 680, 500_000, "c2"),
)


def make_camera(width: int, height: int, focal_frac: float = 0.8) -> Camera:
    f = focal_frac * width
    return Camera(width, height, f, f, width / 2.0, height / 2.0)


def identity_viewmat() -> np.ndarray:
    v = np.zeros((3, 4), np.float32)
    v[0, 0] = v[1, 1] = v[2, 2] = 1.0
    return v


def _logit(p):
    return np.log(p) - np.log1p(-p)


def make_scene(spec: SceneSpec, cam: Camera | None = None,
               n: int | None = None, seed: int | None = None) -> Scene:
    """Draw a scene: centres uniform in the camera frustum (identity pose).

    Depth is volume-uniform on [z_near, z_far] (density proportional to z^2),
    image position uniform over the sensor, so the centre is the back-projection
    of a uniform pixel at that depth.
    """
    cam = cam or make_camera(spec.width, spec.height, spec.focal_frac)
    n = spec.n if n is None else n
    rng = np.random.Generator(np.random.PCG64(spec.seed if seed is None else seed))
    z0, z1 = spec.z_near, spec.z_far
    z = np.cbrt(z0 ** 3 + (z1 ** 3 - z0 ** 3) * rng.random(n))
    px = rng.random(n) * cam.width
    py = rng.random(n) * cam.height
    x = (px - cam.cx) * z / cam.fx
    y = (py - cam.cy) * z / cam.fy
    means = np.stack([x, y, z], 1)
    log_scales = rng.normal(spec.log_scale_mean, spec.log_scale_std, (n, 3))
    q = rng.normal(size=(n, 4))
    quats = q / np.linalg.norm(q, axis=1, keepdims=True)
    eta = rng.normal(0.0, 1.0, n)
    if spec.transparent_frac > 0:
        k = int(round(spec.transparent_frac * n))
        idx = rng.choice(n, size=k, replace=False)
        eta[idx] = _logit(rng.uniform(0.005, 0.05, k))
    colors = rng.random((n, 3))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f32(means), f32(log_scales), f32(quats), f32(eta), f32(colors))


def perturb_scene(scene: Scene, seed: int, mean_sigma=0.01, color_sigma=0.05,
                  logit_sigma=0.2) -> Scene:
    """Seed-perturbed copy used to render a target frame."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = scene.n
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(
        f32(scene.means + rng.normal(0, mean_sigma, (n, 3))),
        scene.log_scales.copy(),
        scene.quats.copy(),
        f32(scene.opacity_logits + rng.normal(0, logit_sigma, n)),
        f32(np.clip(scene.colors + rng.normal(0, color_sigma, (n, 3)), 0, 1)),
    )


def pose_offset(seed: int, trans: float = 0.02, rot_deg: float = 1.0) -> np.ndarray:
    """A tangent vector (rho, phi): `trans` metres along a random unit
    direction and `rot_deg` degrees about a random unit axis."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    return np.concatenate([trans * d, math.radians(rot_deg) * a]).astype(np.float64)


def upstream_grads(width: int, height: int, seed: int, scale: float = 1.0):
    """Random incoming gradients for colour [3,H,W], depth [H,W], alpha [H,W]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g_c = rng.normal(0, scale, (3, height, width)).astype(np.float32)
    g_d = rng.normal(0, scale, (height, width)).astype(np.float32)
    g_a = rng.normal(0, scale, (height, width)).astype(np.float32)
    return g_c, g_d, g_a


def noisy(image: np.ndarray, seed: int, sigma: float = 0.01) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return (image + rng.normal(0, sigma, image.shape)).astype(np.float32)


def fd_crop_spec():
    """The 64x64 window of the 1200x680 camera with 200 Gaussians used for
    finite-difference checks (fx = fy = 960, principal point at the centre)."""
    cam = Camera(64, 64, 960.0, 960.0, 32.0, 32.0)
    spec = SceneSpec("c3_fd_crop_64x64_200", 64, 64, 200, 1003,
                     log_scale_mean=-4.5, log_scale_std=0.7,
                     transparent_frac=0.2)
    return spec, cam
