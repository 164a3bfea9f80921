"""Seeded synthetic scenes and cameras for the Gaussian-splatting render workloads.

This module is the only code shared by the oracle and the HIP path.  It draws
random scene parameters, applies the activations a trained 3D Gaussian
Splatting scene stores them behind (exp for log-scales, sigmoid for opacity
logits, unit normalisation for quaternions), and builds pinhole cameras.  It
contains none of the rendering arithmetic: no projection, culling, colour,
quantisation, key generation, sorting or blending.

The paper measures on trained scenes (Mip-NeRF 360, Tanks & Temples, Deep
Blending) that are not available here; these seeded scenes stand in for them
with the sizes and distributions of the five named workloads:

* ``small`` 10,000 Gaussians in [-1,1]^3, log-scale N(-3.5, 0.5), 256x256, camera
  at distance 3, fovx 60 deg (the small parity case);
* ``1080p`` 1,000,000 Gaussians in [-10,10]^3, log-scale N(-4, 0.6), 1920x1080,
  camera at distance 25, fovx 60 deg;
* ``4k`` 3,000,000 Gaussians in [-20,20]^3, log-scale N(-4, 0.6), 3840x2160,
  64-pose orbit of radius 40 at 20 deg elevation, fovx 50 deg;
* ``serving``: the 1080p and 4k scenes, Poisson arrivals, mixed 720p /
  1080p / 4K orbit poses;
* ``training`` (differentiation): the 1080p scene and camera, target rendered from means
  perturbed by N(0, 0.01).

Draw order for a scene (one ``numpy.random.Generator(PCG64(seed))``):
means U(-h,h)^{Nx3}; log-scales N(mu_s, sigma_s)^{Nx3}; quaternions N(0,1)^{Nx4};
opacity logits N(0,1.5)^N; SH DC N(0,0.5)^{Nx3}; SH rest N(0,0.05)^{Nx15x3}.
Activations run in float64 and the results are stored as float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "Camera", "make_scene", "look_at_camera", "orbit_camera",
    "config_scene", "config_camera", "SCENE_CONFIGS", "CAMERA_CONFIGS", "SERVING_ORBITS", "serving_camera",
    "poisson_requests", "perturbed_means",
]


@dataclass
class Scene:
    """A Gaussian scene as stored by a trained model, activated, float32.

    means [n,3]; scales [n,3] (> 0); quats [n,4] as (w, x, y, z), unit up to
    float32 rounding; opacity [n] in (0, 1); sh [n,16,3] degree-3 coefficients
    (coefficient index l*l + l + m, then RGB channel).
    """
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx], self.scales[idx], self.quats[idx],
                     self.opacity[idx], self.sh[idx])


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    A world point p maps to camera space as R @ p + t.  Pixel (i, j) is sampled
    at image-plane position (i, j): fx = W / (2 tan(fovx/2)), fy = fx,
    cx = (W-1)/2, cy = (H-1)/2, tan(fovy/2) = tan(fovx/2) * H / W.  The depth
    interval [z_near, z_far] is the predefined quantisation interval that
    encloses the scene's bounding cube.
    """
    R: np.ndarray          # [3,3] float64, rows are the camera axes in world space
    t: np.ndarray          # [3] float64
    fx: float
    fy: float
    cx: float
    cy: float
    tan_half_fovx: float
    tan_half_fovy: float
    z_near: float
    z_far: float
    width: int
    height: int
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))


def make_scene(n: int, half_extent: float, log_scale_mean: float,
               log_scale_std: float, seed: int) -> Scene:
    """Draw a seeded scene in the documented order (see module docstring)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(-half_extent, half_extent, size=(n, 3))
    log_scales = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    logits = rng.normal(0.0, 1.5, size=n)
    sh_dc = rng.normal(0.0, 0.5, size=(n, 1, 3))
    sh_rest = rng.normal(0.0, 0.05, size=(n, 15, 3))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    return Scene(
        means=means.astype(np.float32),
        scales=np.exp(log_scales).astype(np.float32),
        quats=quats.astype(np.float32),
        opacity=(1.0 / (1.0 + np.exp(-logits))).astype(np.float32),
        sh=np.concatenate([sh_dc, sh_rest], axis=1).astype(np.float32),
    )


def look_at_camera(eye, target, up, fovx_deg: float, width: int, height: int,
                   z_near: float, z_far: float, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera at ``eye`` looking at ``target``; image y points along -``up``."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    up = np.asarray(up, np.float64)
    zc = target - eye
    zc /= np.linalg.norm(zc)
    xc = np.cross(zc, up)
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    R = np.stack([xc, yc, zc])
    t = -R @ eye
    tanx = math.tan(math.radians(fovx_deg) / 2.0)
    fx = width / (2.0 * tanx)
    return Camera(R=R, t=t, fx=fx, fy=fx, cx=(width - 1) / 2.0, cy=(height - 1) / 2.0,
                  tan_half_fovx=tanx, tan_half_fovy=tanx * height / width,
                  z_near=z_near, z_far=z_far, width=width, height=height,
                  bg=np.asarray(bg, np.float32))


def _depth_interval(distance: float, half_extent: float):
    """Near/far planes enclosing a cube of half-extent h seen from distance D."""
    reach = math.sqrt(3.0) * half_extent
    return max(0.2, distance - reach), distance + reach


def orbit_camera(k: int, n_poses: int, radius: float, elevation_deg: float,
                 fovx_deg: float, width: int, height: int, half_extent: float) -> Camera:
    """Pose k of an orbit around the origin (azimuth 2*pi*k/n_poses, up +y)."""
    az = 2.0 * math.pi * k / n_poses
    el = math.radians(elevation_deg)
    eye = radius * np.array([math.cos(el) * math.sin(az), math.sin(el),
                             -math.cos(el) * math.cos(az)])
    zn, zf = _depth_interval(radius, half_extent)
    return look_at_camera(eye, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), fovx_deg, width, height, zn, zf)


# name -> (n, half_extent, log-scale mean, log-scale std, seed)
SCENE_CONFIGS = {
    "small": (10_000, 1.0, -3.5, 0.5, 0),
    "1080p": (1_000_000, 10.0, -4.0, 0.6, 1),
    "4k": (3_000_000, 20.0, -4.0, 0.6, 2),
}

# name -> camera recipe
CAMERA_CONFIGS = {
    "small": dict(distance=3.0, fovx=60.0, width=256, height=256, half_extent=1.0),
    "1080p": dict(distance=25.0, fovx=60.0, width=1920, height=1080, half_extent=10.0),
    "4k": dict(orbit_radius=40.0, elevation=20.0, n_poses=64, fovx=50.0,
                 width=3840, height=2160, half_extent=20.0),
}


def config_scene(name: str, n: int | None = None) -> Scene:
    """The seeded scene of a named workload (optionally its first n Gaussians)."""
    n_full, h, mu, sd, seed = SCENE_CONFIGS[name]
    return make_scene(n_full if n is None else n, h, mu, sd, seed)


def config_camera(name: str, pose: int = 0, width: int | None = None,
                  height: int | None = None) -> Camera:
    """The camera of a named workload; 4k takes an orbit pose index.

    ``width``/``height`` override the resolution (the serving mix renders the
    same poses at 720p, 1080p and 4K).
    """
    c = CAMERA_CONFIGS[name]
    W = c["width"] if width is None else width
    H = c["height"] if height is None else height
    if "orbit_radius" in c:
        return orbit_camera(pose, c["n_poses"], c["orbit_radius"], c["elevation"],
                            c["fovx"], W, H, c["half_extent"])
    zn, zf = _depth_interval(c["distance"], c["half_extent"])
    return look_at_camera((0.0, 0.0, -c["distance"]), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0),
                          c["fovx"], W, H, zn, zf)


def poisson_requests(rate_hz: float, n_requests: int, seed: int = 3):
    """Serving workload: arrival times (s), resolutions and orbit poses.

    Resolutions are 50% 1280x720, 35% 1920x1080, 15% 3840x2160; each request
    names one of two resident scenes (0: the 1M scene, 1: the 3M scene) with
    equal probability and a random orbit pose out of 64.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arrivals = np.cumsum(gaps)
    res_choice = rng.choice(3, size=n_requests, p=[0.50, 0.35, 0.15])
    res = np.array([(1280, 720), (1920, 1080), (3840, 2160)])[res_choice]
    scene = rng.integers(0, 2, size=n_requests)
    pose = rng.integers(0, 64, size=n_requests)
    return arrivals, res, scene, pose


# Orbits of the two resident scenes of the serving workload: the 1M scene is
# viewed from its single-frame distance, the 3M scene from its 64-pose orbit.
SERVING_ORBITS = (
    dict(scene="1080p", orbit_radius=25.0, elevation=20.0, n_poses=64, fovx=60.0, half_extent=10.0),
    dict(scene="4k", orbit_radius=40.0, elevation=20.0, n_poses=64, fovx=50.0, half_extent=20.0),
)


def serving_camera(scene_index: int, pose: int, width: int, height: int) -> Camera:
    """Camera of a serving request: orbit pose ``pose`` of resident scene ``scene_index``."""
    o = SERVING_ORBITS[scene_index]
    return orbit_camera(pose, o["n_poses"], o["orbit_radius"], o["elevation"], o["fovx"], width, height,
                        o["half_extent"])


def perturbed_means(scene: Scene, sigma: float = 0.01, seed: int = 4) -> np.ndarray:
    """Means + N(0, sigma) noise: the target scene of the differentiation workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (scene.means.astype(np.float64) + rng.normal(0.0, sigma, size=scene.means.shape)).astype(np.float32)
