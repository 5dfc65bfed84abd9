"""Seeded synthetic inputs for the 3D Gaussian Splatting render/backward path.

This module only draws random numbers and lays them out as fp32 arrays; it
contains none of the rendering arithmetic. Both the HIP path and the fp64
oracle consume exactly the arrays produced here.

Shapes (row-major, fp32):
  means3d        [N,3]
  log_scales     [N,3]
  quats          [N,4]   (w, x, y, z), drawn N(0,1) and normalised
  opacity_logits [N]
  sh             [N,K,3] with K = (degree+1)^2, coefficient k = l*l + l + m

Camera: pinhole, OpenCV axes (+x right, +y down, +z forward), horizontal
field of view 60 degrees, square pixels, principal point at the image centre,
world_to_cam is the row-major 3x4 [R|t].

Workloads follow the paper's evaluation scenes in shape only (Table of
workloads and datasets): object-centred scenes like the NeRF-Synthetic ones
and a large indoor-like scene with the camera inside the cloud. Random draws
happen in a fixed order per workload: means, log-scales, quaternions,
opacity logits, SH DC, SH rest, camera(s), then the target or the
perturbation noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F32 = np.float32


@dataclass
class Scene:
    means3d: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means3d.shape[0])

    def arrays(self):
        return (self.means3d, self.log_scales, self.quats, self.opacity_logits, self.sh)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(*(np.ascontiguousarray(a[idx]) for a in self.arrays()), sh_degree=self.sh_degree)


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    world_to_cam: np.ndarray  # (3,4) fp32
    znear: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def with_bg(self, bg) -> "Camera":
        return Camera(self.width, self.height, self.fx, self.fy, self.cx, self.cy,
                      self.world_to_cam.copy(), self.znear, tuple(float(b) for b in bg))

    def crop(self, x0: int, y0: int, w: int, h: int) -> "Camera":
        """Camera seeing only the window [x0,x0+w) x [y0,y0+h) of this one."""
        return Camera(w, h, self.fx, self.fy, self.cx - x0, self.cy - y0,
                      self.world_to_cam.copy(), self.znear, self.bg)


def focal_for_fov(width: int, fov_deg: float = 60.0) -> float:
    return float(F32(width / (2.0 * math.tan(math.radians(fov_deg) / 2.0))))


def look_at(eye, target=(0.0, 0.0, 0.0)) -> np.ndarray:
    """World-to-camera [R|t] for a camera at `eye` looking at `target`.

    Rows of R are the camera axes x_c, y_c, z_c in world coordinates:
    z_c = normalise(target - eye), x_c = normalise(up x z_c) with up = +y
    (or +z when the view direction is parallel to +y), y_c = z_c x x_c.
    """
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    up = np.array([0.0, 1.0, 0.0])
    x = np.cross(up, z)
    if np.linalg.norm(x) < 1e-6:
        x = np.cross(np.array([0.0, 0.0, 1.0]), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ eye
    return np.concatenate([R, t[:, None]], axis=1).astype(F32)


def make_camera(width: int, height: int, eye, target=(0.0, 0.0, 0.0), bg=(0.0, 0.0, 0.0)) -> Camera:
    f = focal_for_fov(width)
    return Camera(width, height, f, f, width / 2.0, height / 2.0, look_at(eye, target), 0.2, tuple(bg))


def _quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(F32)


def _clustered(rng, n, half, n_clusters=20, sigma=0.2):
    centres = rng.uniform(-half, half, size=(n_clusters, 3))
    which = rng.integers(0, n_clusters, size=n)
    return (centres[which] + sigma * rng.standard_normal((n, 3))).astype(F32)


def _sh(rng, n, degree, rest_sigma):
    k = (degree + 1) ** 2
    sh = np.zeros((n, k, 3), F32)
    sh[:, 0, :] = rng.uniform(0.0, 1.0, size=(n, 3))
    if k > 1:
        sh[:, 1:, :] = rest_sigma * rng.standard_normal((n, k - 1, 3))
    return sh


def random_scene(rng, n, *, means="uniform", half=1.0, log_scale=(-3.0, 0.5),
                 opacity=(0.0, 1.0), sh_degree=0, sh_rest_sigma=0.1) -> Scene:
    if means == "uniform":
        m = rng.uniform(-half, half, size=(n, 3)).astype(F32)
    else:
        m = _clustered(rng, n, half)
    ls = rng.normal(log_scale[0], log_scale[1], size=(n, 3)).astype(F32)
    q = _quats(rng, n)
    op = rng.normal(opacity[0], opacity[1], size=n).astype(F32)
    sh = _sh(rng, n, sh_degree, sh_rest_sigma)
    return Scene(m, ls, q, op, sh, sh_degree)


@dataclass
class Workload:
    name: str
    scene: Scene
    camera: Camera
    tile: int = 16
    target: np.ndarray | None = None          # [3,H,W] fp32, when drawn directly
    perturbed: Scene | None = None            # scene whose render (+ noise) is the target
    loss: str = "l1"
    extra: dict = field(default_factory=dict)


def tiny_1k(seed: int = 1) -> Workload:
    """1,000 Gaussians, means U[-1,1]^3, 64x64, camera at z=-3 looking +z, SH degree 0, L1."""
    rng = np.random.default_rng(seed)
    sc = random_scene(rng, 1000, means="uniform", half=1.0, log_scale=(-3.0, 0.5),
                      opacity=(0.0, 1.0), sh_degree=0)
    cam = make_camera(64, 64, (0.0, 0.0, -3.0))
    target = rng.uniform(0.0, 1.0, size=(3, 64, 64)).astype(F32)
    return Workload("tiny_1k_64x64_sh0", sc, cam, 16, target=target, loss="l1")


def _perturb(rng, sc: Scene, sigma=0.01) -> Scene:
    arrs = [a + sigma * rng.standard_normal(a.shape) for a in sc.arrays()]
    return Scene(*(a.astype(F32) for a in arrs), sh_degree=sc.sh_degree)


def object_100k(seed: int = 2, n: int = 100_000, width: int = 800, height: int = 800) -> Workload:
    """100k Gaussians in 20 clusters (sigma 0.2) in [-2,2]^3, 800x800, SH degree 3.

    Loss is L1 + 0.2 D-SSIM against the render of the parameters perturbed by
    N(0, 0.01) on every raw tensor.
    """
    rng = np.random.default_rng(seed)
    sc = random_scene(rng, n, means="clustered", half=2.0, log_scale=(-4.0, 0.5),
                      opacity=(0.0, 1.0), sh_degree=3, sh_rest_sigma=0.1)
    cam = make_camera(width, height, (0.0, 0.0, -4.0))
    pert = _perturb(rng, sc)
    return Workload(f"object_{n // 1000}k_{width}x{height}_sh3", sc, cam, 16, perturbed=pert, loss="l1_dssim")


def large_3m(seed: int = 3, n: int = 3_000_000, width: int = 1920, height: int = 1080) -> Workload:
    """3M Gaussians in 20 clusters in [-5,5]^3, 1920x1080, SH degree 3, camera inside the cloud."""
    rng = np.random.default_rng(seed)
    sc = random_scene(rng, n, means="clustered", half=5.0, log_scale=(-4.5, 0.7),
                      opacity=(-1.0, 1.5), sh_degree=3, sh_rest_sigma=0.1)
    g = rng.standard_normal(3)
    eye = 4.0 * g / np.linalg.norm(g)
    cam = make_camera(width, height, eye)
    target = rng.uniform(0.0, 1.0, size=(3, height, width)).astype(F32)
    return Workload(f"large_{n // 1_000_000}m_{width}x{height}_sh3", sc, cam, 16, target=target, loss="l1")


def tiny_scene(seed: int, n: int, width: int = 32, height: int = 32, sh_degree: int = 0,
               log_scale=(-2.0, 0.3), eye=(0.0, 0.0, -3.0), half=0.6) -> Workload:
    """Small scenes for finite-difference and edge-case checks."""
    rng = np.random.default_rng(seed)
    sc = random_scene(rng, n, means="uniform", half=half, log_scale=log_scale,
                      opacity=(0.0, 1.0), sh_degree=sh_degree, sh_rest_sigma=0.2)
    cam = make_camera(width, height, eye)
    target = rng.uniform(0.0, 1.0, size=(3, height, width)).astype(F32)
    return Workload(f"tiny_{n}_{width}x{height}_sh{sh_degree}", sc, cam, 16, target=target, loss="l1")


def single_gaussian_at_pixel(px: int, py: int, width=32, height=32, log_scale=-2.5,
                             opacity_logit=0.3, dc=(0.7, 0.2, 0.4), depth=3.0) -> Workload:
    """One isotropic Gaussian whose mean projects exactly onto the sample point of pixel (px,py).

    The camera sits at the origin looking +z (R = I, t = 0) with its principal
    point on the sample point (px+0.5, py+0.5); the mean lies on the optical axis.
    """
    f = focal_for_fov(width)
    m = np.array([[0.0, 0.0, depth]], F32)
    sc = Scene(m, np.full((1, 3), log_scale, F32), np.array([[1, 0, 0, 0]], F32),
               np.array([opacity_logit], F32), np.array(dc, F32).reshape(1, 1, 3), 0)
    w2c = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(F32)
    cam = Camera(width, height, f, f, px + 0.5, py + 0.5, w2c, 0.2, (0.0, 0.0, 0.0))
    return Workload("single", sc, cam, 16)


@dataclass
class MultiView:
    """Several scenes, each seen by several cameras: views[i] = (scene index, camera, target)."""
    name: str
    scenes: list
    views: list
    loss: str = "l1"


C4_RESOLUTIONS = ((512, 512), (800, 800), (1280, 720), (1600, 1200), (1920, 1080))


def multi_view(seed: int = 4, sizes=(50_000, 200_000, 500_000, 1_500_000), views_per_scene: int = 4,
               resolutions=C4_RESOLUTIONS, sh_degree: int = 3, radius: float = 4.0) -> MultiView:
    """Scenes of uneven size (clustered in [-2,2]^3 like object_100k), each seen from
    `views_per_scene` eyes drawn uniformly on the sphere of `radius`, each view at a
    resolution drawn uniformly from `resolutions`; targets U(0,1), L1. The defaults are
    the 16-view, four-scene batch workload."""
    rng = np.random.default_rng(seed)
    scenes = [random_scene(rng, n, means="clustered", half=2.0, log_scale=(-4.0, 0.5), opacity=(0.0, 1.0),
                           sh_degree=sh_degree, sh_rest_sigma=0.1) for n in sizes]
    views = []
    for si in range(len(scenes)):
        for _ in range(views_per_scene):
            w, h = resolutions[int(rng.integers(len(resolutions)))]
            g = rng.standard_normal(3)
            cam = make_camera(w, h, radius * g / np.linalg.norm(g))
            views.append((si, cam, rng.uniform(0.0, 1.0, size=(3, h, w)).astype(F32)))
    tag = "_".join(f"{n // 1000}k" if n >= 1000 else str(n) for n in sizes)
    return MultiView(f"multi_view_{len(views)}v_{tag}", scenes, views)


def multi_view_small(seed: int = 5) -> MultiView:
    """A small instance of the batch workload for parity against the oracle: four scenes of
    uneven size (one empty), two views each, ragged resolutions."""
    return multi_view(seed, sizes=(600, 2500, 6000, 0), views_per_scene=2,
                      resolutions=((64, 64), (100, 75), (128, 72), (160, 120)), radius=4.0)


WORKLOADS = {
    "tiny_1k": tiny_1k,
    "object_100k": object_100k,
    "large_3m": large_3m,
}


# ---------------------------------------------------------------- device-drawn targets

_GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, index: np.ndarray) -> np.ndarray:
    """SplitMix64 (Steele, Lea and Flood, 2014): output number index+1 of the generator
    started at `seed` (state seed + (index+1) * golden gamma, then the variant-13 mix)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (index.astype(np.uint64) + np.uint64(1)) * _GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def request_target(seed: int, height: int, width: int) -> np.ndarray:
    """The [3,H,W] U[0,1) target a serving request draws on the device: value i is the top 24
    bits of SplitMix64 output i, times 2^-24."""
    i = np.arange(3 * height * width, dtype=np.uint64)
    return ((splitmix64(seed, i) >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)).reshape(
        3, height, width)


def serving_scenes(seed: int = 6, count: int = 10, n_min: int = 100_000, n_max: int = 2_000_000,
                   sh_degree: int = 3) -> list:
    """Resident scenes of the serving stream: sizes log-uniform in [n_min, n_max], clustered
    in [-2,2]^3 like object_100k."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=count)).astype(np.int64)
    return [random_scene(rng, int(n), means="clustered", half=2.0, log_scale=(-4.0, 0.5), opacity=(0.0, 1.0),
                         sh_degree=sh_degree, sh_rest_sigma=0.1) for n in sizes]


def serving_requests(seed: int, n_scenes: int, count: int, rate_hz: float, resolutions=C4_RESOLUTIONS,
                     radius: float = 4.0):
    """Poisson arrivals at rate_hz: (arrival seconds, scene index, Camera, target seed) per
    request, each with a uniform scene, a random eye on the sphere and a resolution drawn
    uniformly from `resolutions`."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=count))
    out = []
    for k in range(count):
        si = int(rng.integers(n_scenes))
        w, h = resolutions[int(rng.integers(len(resolutions)))]
        g = rng.standard_normal(3)
        cam = make_camera(w, h, radius * g / np.linalg.norm(g))
        out.append((float(t[k]), si, cam, int(rng.integers(0, 2 ** 63))))
    return out
