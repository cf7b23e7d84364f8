"""Seeded synthetic scenes, cameras and upstream gradients.

This module only draws inputs.  It holds none of the splatting arithmetic, so
that both the HIP path and the CPU oracle can consume the very same FP32
arrays.  Every array is drawn in FP64 from ``numpy.random.default_rng(seed)``
(PCG64) and cast to FP32, in the fixed order means -> log-scales -> quats ->
logits -> SH (-> latents).

Layouts (structure of arrays, index-minor so that consecutive Gaussians are
consecutive in memory):
  means       float32[3][n]
  log_scales  float32[3][n]
  quats       float32[4][n]   (w, x, y, z), not necessarily unit length
  logits      float32[n]      opacity = sigmoid(logit)
  sh          float32[(D+1)^2][3][n]   coefficient j, channel c at sh[j, c, :]

The paper (Sec. II-A) parameterises each Gaussian by a centre, a covariance
that sets extent and orientation, an opacity and SH colour; the value
distributions follow the five workloads of the scaling study (tiny, skewed,
main, heavy, learned colour).  The 100x cluster-weight skew stands in for the
density skew the paper measures on real scenes (Sec. I).  No dataset is used.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TILE = 16


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    near_z: float
    tan_half_fov_x: float
    tan_half_fov_y: float
    R_cw: np.ndarray          # float32[3][3], world -> camera rotation (rows = camera axes)
    t_cw: np.ndarray          # float32[3]
    bg: np.ndarray            # float32[3]

    @property
    def tiles_x(self) -> int:
        return (self.width + TILE - 1) // TILE

    @property
    def tiles_y(self) -> int:
        return (self.height + TILE - 1) // TILE

    @property
    def n_tiles(self) -> int:
        return self.tiles_x * self.tiles_y

    def with_bg(self, bg) -> "Camera":
        return dataclasses.replace(self, bg=np.asarray(bg, np.float32).copy())


@dataclasses.dataclass
class Scene:
    n: int
    sh_degree: int
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    logits: np.ndarray
    sh: np.ndarray
    latents: np.ndarray | None = None   # uint16 bf16 bits [n][16] (learned colour only)

    def arrays(self):
        return dict(means=self.means, log_scales=self.log_scales, quats=self.quats,
                    logits=self.logits, sh=self.sh)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(len(idx), self.sh_degree,
                     np.ascontiguousarray(self.means[:, idx]),
                     np.ascontiguousarray(self.log_scales[:, idx]),
                     np.ascontiguousarray(self.quats[:, idx]),
                     np.ascontiguousarray(self.logits[idx]),
                     np.ascontiguousarray(self.sh[:, :, idx]),
                     None if self.latents is None else np.ascontiguousarray(self.latents[idx]))


def pinhole(width: int, height: int, fov_x_deg: float, R_cw, t_cw, bg=(0.0, 0.0, 0.0),
            near_z: float = 0.2) -> Camera:
    """Pinhole camera: horizontal field of view, square pixels, principal point at
    the image centre, pixel (x, y) sampled at (x + 0.5, y + 0.5)."""
    fx = width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))
    fy = fx
    return Camera(width=int(width), height=int(height),
                  fx=float(np.float32(fx)), fy=float(np.float32(fy)),
                  cx=float(np.float32(width / 2.0)), cy=float(np.float32(height / 2.0)),
                  near_z=float(np.float32(near_z)),
                  tan_half_fov_x=float(np.float32(width / (2.0 * fx))),
                  tan_half_fov_y=float(np.float32(height / (2.0 * fy))),
                  R_cw=np.asarray(R_cw, np.float64).astype(np.float32),
                  t_cw=np.asarray(t_cw, np.float64).astype(np.float32),
                  bg=np.asarray(bg, np.float32).copy())


def front_camera(width: int, height: int, distance: float = 3.0, fov_x_deg: float = 60.0,
                 bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera on the -z axis looking at the origin: R = I, t = (0, 0, distance)."""
    return pinhole(width, height, fov_x_deg, np.eye(3), (0.0, 0.0, distance), bg)


def orbit_camera(k: int, count: int, width: int, height: int, radius: float = 4.0,
                 fov_x_deg: float = 60.0, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera k of `count` on a horizontal circle of the given radius, looking at
    the origin; camera axes x right, y down (world +y), z forward."""
    th = 2.0 * math.pi * k / count
    c = np.array([radius * math.sin(th), 0.0, -radius * math.cos(th)])
    z = -c / np.linalg.norm(c)
    y = np.array([0.0, 1.0, 0.0])
    x = np.cross(y, z)
    R = np.stack([x, y, z])
    t = -R @ c
    return pinhole(width, height, fov_x_deg, R, t, bg)


# --------------------------------------------------------------------------- draws

def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _sh(rng, n, degree, dc_std, rest_std):
    nc = (degree + 1) ** 2
    sh = np.empty((nc, 3, n))
    sh[0] = rng.normal(0.0, dc_std, (3, n))
    if nc > 1:
        sh[1:] = rng.normal(0.0, rest_std, (nc - 1, 3, n))
    return sh


def _cluster_means(rng, n, n_clusters, skew=100.0, spread=0.1):
    """Mixture of isotropic clusters; cluster c has weight proportional to
    skew**(c/(C-1)), so the heaviest/lightest weight ratio is `skew`."""
    w = skew ** (np.arange(n_clusters) / (n_clusters - 1))
    w /= w.sum()
    centres = rng.uniform(-1.0, 1.0, (n_clusters, 3))
    labels = rng.choice(n_clusters, size=n, p=w)
    offs = spread * rng.standard_normal((n, 3))
    return (centres[labels] + offs).T.copy()


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))


def uniform_scene(n: int, seed: int, log_scale_mean=-3.5, log_scale_std=0.5, sh_degree=0,
                  dc_std=0.3, rest_std=0.05) -> Scene:
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (3, n))
    log_scales = rng.normal(log_scale_mean, log_scale_std, (3, n))
    quats = _unit_quats(rng, n)
    logits = rng.standard_normal(n)
    sh = _sh(rng, n, sh_degree, dc_std, rest_std)
    return Scene(n, sh_degree, _f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh))


def skewed_scene(n: int, seed: int, n_clusters=64, log_scale_mean=-4.5, log_scale_std=0.7,
                 sh_degree=3, anisotropic=False, max_ratio=20.0) -> Scene:
    rng = np.random.default_rng(seed)
    means = _cluster_means(rng, n, n_clusters)
    if anisotropic:
        base = rng.normal(log_scale_mean, log_scale_std, n)
        ln_rho = np.log(max_ratio) * rng.uniform(0.0, 1.0, n)
        axis = rng.integers(0, 3, n)
        log_scales = np.repeat((base - ln_rho / 3.0)[None, :], 3, axis=0)
        log_scales[axis, np.arange(n)] = base + 2.0 * ln_rho / 3.0
    else:
        log_scales = rng.normal(log_scale_mean, log_scale_std, (3, n))
    quats = _unit_quats(rng, n)
    logits = rng.standard_normal(n)
    sh = _sh(rng, n, sh_degree, 0.5, 0.05)
    return Scene(n, sh_degree, _f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh))


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 (nearest-even) and return the raw 16-bit patterns."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32)


# ------------------------------------------------------------------------ workloads

CONFIG_NAMES = {1: "tiny", 2: "skewed", 3: "main", 4: "heavy", 5: "learned"}


def config_scene(cfg: int, n: int | None = None) -> Scene:
    """Scene of workload `cfg` (1 tiny, 2 skewed, 3 main, 4 heavy, 5 learned colour).
    `n` overrides the Gaussian count (same distributions, same seed)."""
    seed = 1000 * cfg
    if cfg == 1:
        return uniform_scene(n or 4096, seed)
    if cfg in (2, 5):
        s = skewed_scene(n or 200_000, seed)
        if cfg == 5:
            rng = np.random.default_rng(seed + 7)
            s.latents = bf16_bits(rng.normal(0.0, 0.1, (s.n, 16)).astype(np.float32))
        return s
    if cfg == 3:
        return skewed_scene(n or 1_000_000, seed)
    if cfg == 4:
        return skewed_scene(n or 3_000_000, seed, n_clusters=256, anisotropic=True)
    raise ValueError(f"unknown workload {cfg}")


def low_rank_colour(scene: Scene, rank: int, seed: int) -> Scene:
    """The same scene with view-dependent colour of low rank: the SH
    coefficients of degree >= 1 are a_i B for per-Gaussian factors a_i ~
    N(0, I_rank) and one scene-wide basis B (rank x 3 ((D+1)^2 - 1)) with
    N(0, 0.05^2 / rank) entries, so each coefficient keeps the std 0.05 of the
    independent draw while the whole view dependence spans `rank` dimensions
    (as correlated highlights do).  DC coefficients are kept."""
    rng = np.random.default_rng(seed)
    nb = (scene.sh_degree + 1) ** 2
    basis = rng.normal(0.0, 0.05 / np.sqrt(rank), (rank, 3 * (nb - 1)))
    a = rng.standard_normal((scene.n, rank))
    sh = scene.sh.astype(np.float64).copy()
    sh[1:] = (a @ basis).T.reshape(nb - 1, 3, scene.n)
    return dataclasses.replace(scene, sh=_f32(sh))


def coherent_colour(scene: Scene, seed: int, noise: float = 0.03) -> Scene:
    """The same scene with spatially coherent base colour, as in captured
    scenes where neighbouring Gaussians of a dense region share a colour: the
    degree-0 coefficient of channel k is 1.2 sin(2.5 <w_k, mu> + phi_k) +
    N(0, noise^2), a smooth field over space (w_k unit directions, phi_k
    phases, both seeded).  Higher-degree coefficients are kept."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((3, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    phi = rng.uniform(0.0, 2.0 * np.pi, 3)
    mu = scene.means.astype(np.float64)
    sh = scene.sh.astype(np.float64).copy()
    sh[0] = 1.2 * np.sin(2.5 * (w @ mu) + phi[:, None]) + rng.normal(0.0, noise, (3, scene.n))
    return dataclasses.replace(scene, sh=_f32(sh))


def density_noise(n: int, seed: int) -> np.ndarray:
    """Random draws of one density-control round, float32[6][n]: rows 0-2
    N(0, 1) (the Gaussian spread), rows 3-5 U(-1, 1) (the perturbation)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((3, n))
    e = rng.uniform(-1.0, 1.0, (3, n))
    return _f32(np.concatenate([z, e]))


# neighbour radius of the density control per workload: about 20 other
# centres within it on average (skewed 200k: 0.03; main 1M: 0.0175)
DENSITY_RADIUS = {1: 0.08, 2: 0.03, 3: 0.0175, 4: 0.012, 5: 0.03}


def config_camera(cfg: int, k: int = 0, bg=(0.0, 0.0, 0.0)) -> Camera:
    if cfg == 1:
        return front_camera(128, 128, 3.0, 60.0, bg)
    if cfg in (2, 5):
        return front_camera(800, 800, 3.0, 60.0, bg)
    if cfg == 3:
        return orbit_camera(k, 32, 1600, 1064, 4.0, 60.0, bg)
    if cfg == 4:
        return orbit_camera(0, 32, 1920, 1080, 4.0, 60.0, bg)
    raise ValueError(f"unknown workload {cfg}")


def upstream_grad(cam: Camera, seed: int) -> np.ndarray:
    """dL/dimage ~ N(0, 1), float32[3][H][W]."""
    rng = np.random.default_rng(seed)
    return _f32(rng.standard_normal((3, cam.height, cam.width)))


def target_image(cam: Camera, seed: int) -> np.ndarray:
    """Seeded L1 target, U(0,1), float32[3][H][W]."""
    rng = np.random.default_rng(seed)
    return _f32(rng.uniform(0.0, 1.0, (3, cam.height, cam.width)))


def view_dirs(n: int, per: int, seed: int) -> np.ndarray:
    """`per` fixed directions uniform on the sphere for each of n Gaussians,
    float32[n][per][3]."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, per, 3))
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    return _f32(d)
