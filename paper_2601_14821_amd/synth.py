"""Seeded synthetic scenes and cameras.

This module only draws inputs. It holds none of the rasterizer's arithmetic
(no projection, compositing or removal effect), so both the FP64 oracle and
the HIP path can take their inputs from it.

Splat layout (one row per splat, FP32, 236 bytes per splat as in the paper's
uncompressed property table, Sec. 5.5):
  means      [N, 3]      world-space centre
  scales     [N, 3]      activated scale (exp of the log-scale)
  quats      [N, 4]      rotation quaternion (w, x, y, z), unit norm
  opacities  [N]         activated base opacity o in (0, 1)
  sh         [N, 16, 3]  real SH coefficients, coefficient-major, channel-minor

Cameras are pinhole with OpenCV axes (x right, y down, z forward); R and t map
world to camera coordinates.

Draw order inside one scene is fixed: means, log-scales, quaternions, opacity
logits, SH DC, SH AC.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray
    sh: np.ndarray

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(*(np.ascontiguousarray(a[idx]) for a in
                       (self.means, self.scales, self.quats, self.opacities, self.sh)))


@dataclasses.dataclass
class Camera:
    R: np.ndarray          # [3, 3] float32, world -> camera rotation
    t: np.ndarray          # [3] float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def eye(self) -> np.ndarray:
        return (-self.R.astype(np.float64).T @ self.t.astype(np.float64))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def random_scene(n: int, seed: int, log_scale_mu: float = -3.5, log_scale_sigma: float = 0.5,
                 clustered: bool = False, n_clusters: int = 64, cluster_sigma: float = 0.15,
                 background_frac: float = 0.2, dc_sigma: float = 0.5, ac_sigma: float = 0.05,
                 opacity_logit_sigma: float = 1.5) -> Scene:
    """Draw a scene with the distributions of the benchmark workloads.

    Uniform means lie in [-1, 1]^3. Clustered means draw 64 centres uniformly in
    [-1, 1]^3; a `1 - background_frac` share of the splats picks a centre and
    adds isotropic N(0, cluster_sigma^2) offsets, the rest is uniform.
    """
    rng = np.random.default_rng(seed)
    if clustered:
        centres = rng.uniform(-1.0, 1.0, size=(n_clusters, 3))
        is_bg = rng.uniform(size=n) < background_frac
        pick = rng.integers(0, n_clusters, size=n)
        offs = rng.normal(0.0, cluster_sigma, size=(n, 3))
        unif = rng.uniform(-1.0, 1.0, size=(n, 3))
        means = np.where(is_bg[:, None], unif, centres[pick] + offs)
    else:
        means = rng.uniform(-1.0, 1.0, size=(n, 3))
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.normal(0.0, opacity_logit_sigma, size=n)
    sh = np.empty((n, 16, 3))
    sh[:, 0, :] = rng.normal(0.0, dc_sigma, size=(n, 3))
    sh[:, 1:, :] = rng.normal(0.0, ac_sigma, size=(n, 15, 3))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f32(means), f32(np.exp(log_scales)), f32(q), f32(_sigmoid(logits)), f32(sh))


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), width=128, height=128,
            fov_deg: float = 60.0) -> Camera:
    """Pinhole camera at `eye` looking at `target`; `fov_deg` is horizontal."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f])
    t = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Camera(R.astype(np.float32), t.astype(np.float32), float(np.float32(fx)), float(np.float32(fx)),
                  width / 2.0, height / 2.0, int(width), int(height))


def ring_cameras(n_views: int, width: int, height: int, radius: float = 3.0, fov_deg: float = 60.0,
                 height_offset: float = 0.0):
    """Views on a ring in the y = 0 plane, azimuth 2*pi*v/n_views, looking at the origin."""
    cams = []
    for v in range(n_views):
        a = 2.0 * math.pi * v / n_views
        eye = (radius * math.sin(a), height_offset, radius * math.cos(a))
        cams.append(look_at(eye, width=width, height=height, fov_deg=fov_deg))
    return cams


def hemisphere_cameras(n_views: int, width: int, height: int, seed: int, r_lo: float = 3.0,
                       r_hi: float = 4.0, min_elev_deg: float = 10.0, jitter_deg: float = 3.0,
                       fov_deg: float = 60.0):
    """Fibonacci-lattice directions on the upper (+y) hemisphere above `min_elev_deg`,
    jittered in azimuth and elevation, radius uniform in [r_lo, r_hi]."""
    rng = np.random.default_rng(seed)
    golden = math.pi * (3.0 - math.sqrt(5.0))
    s_lo = math.sin(math.radians(min_elev_deg))
    cams = []
    for v in range(n_views):
        s = s_lo + (1.0 - s_lo) * (v + 0.5) / n_views          # sin(elevation), area-uniform
        elev = math.asin(s) + math.radians(rng.normal(0.0, jitter_deg))
        elev = min(max(elev, math.radians(min_elev_deg)), math.radians(85.0))
        az = golden * v + math.radians(rng.normal(0.0, jitter_deg))
        r = rng.uniform(r_lo, r_hi)
        eye = (r * math.cos(elev) * math.sin(az), r * math.sin(elev), r * math.cos(elev) * math.cos(az))
        cams.append(look_at(eye, width=width, height=height, fov_deg=fov_deg))
    return cams


def perturbed(scene: Scene, seed: int, mean_sigma: float = 0.01, sh_sigma: float = 0.02) -> Scene:
    """Copy of `scene` with means + N(0, mean_sigma^2) and SH + N(0, sh_sigma^2)."""
    rng = np.random.default_rng(seed)
    m = scene.means + rng.normal(0.0, mean_sigma, size=scene.means.shape)
    s = scene.sh + rng.normal(0.0, sh_sigma, size=scene.sh.shape)
    return Scene(np.ascontiguousarray(m, np.float32), scene.scales.copy(), scene.quats.copy(),
                 scene.opacities.copy(), np.ascontiguousarray(s, np.float32))


# --------------------------------------------------------------------------------------------
# The benchmark workloads. Each returns (scene, cameras); c4 also returns the perturbed scene.
# --------------------------------------------------------------------------------------------

RESOLUTIONS = ((640, 480), (1280, 720), (1600, 1064))


def workload_small():
    """2,000 uniform splats, log-scale N(-3.5, 0.5), 4 ring views at 128x128."""
    return random_scene(2000, 1001), ring_cameras(4, 128, 128)


def workload_single_view(n: int = 500_000):
    """500k clustered splats, log-scale N(-3.5, 0.5), one 1280x720 view at azimuth 0."""
    return random_scene(n, 2001, clustered=True), ring_cameras(1, 1280, 720)


def workload_full_scene(n: int = 3_000_000, n_views: int = 200):
    """3M clustered splats, log-scale N(-4, 0.7), 200 hemisphere views at 1600x1064."""
    scene = random_scene(n, 3001, log_scale_mu=-4.0, log_scale_sigma=0.7, clustered=True)
    return scene, hemisphere_cameras(n_views, 1600, 1064, seed=3002)


def workload_differentiation(n: int = 1_000_000, n_views: int = 4):
    """1M clustered splats, 4 hemisphere views at 1280x720, plus the perturbed target scene."""
    scene = random_scene(n, 4001, clustered=True)
    cams = hemisphere_cameras(n_views, 1280, 720, seed=4003)
    return scene, cams, perturbed(scene, 4002)


def workload_fd_case():
    """64 splats at 32x32 for the finite-difference check: one ring view."""
    scene = random_scene(64, 4100, log_scale_mu=-2.5, log_scale_sigma=0.3)
    return scene, ring_cameras(1, 32, 32)


def workload_batched(n_scenes: int = 16, n_lo: int = 50_000, n_hi: int = 2_000_000,
                     v_lo: int = 8, v_hi: int = 32, scale: float = 1.0):
    """Uneven batch: per scene s (seed 5000+s), N log-uniform in [n_lo, n_hi], 8..32 views,
    one resolution out of RESOLUTIONS. `scale` shrinks N for quick runs."""
    out = []
    for s in range(n_scenes):
        rng = np.random.default_rng(5000 + s)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))) * scale))
        v = int(rng.integers(v_lo, v_hi + 1))
        w, h = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
        scene = random_scene(max(n, 1), 50000 + s, clustered=True)
        out.append((scene, hemisphere_cameras(v, w, h, seed=60000 + s)))
    return out


@dataclasses.dataclass
class RenderSettings:
    """Run settings handed to the rasterizer (and to any checker) as plain inputs.

    tile_w x tile_h: screen tile; lds_batch: splat records staged per batch;
    eps2d: low-pass added to the 2D covariance diagonal (px^2); near: camera-z cull;
    jclamp: Jacobian clamp in units of the half field of view; a splat counts at a
    pixel iff q <= q_max and o*exp(-q/2) >= alpha_min, alpha = min(alpha_max, .);
    t_min: early-stop transmittance (0 = exact mode); bg: background colour.
    """
    tile_w: int = 16
    tile_h: int = 16
    lds_batch: int = 320
    eps2d: float = 0.3
    near: float = 0.2
    jclamp: float = 1.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    q_max: float = 9.0
    t_min: float = 1e-4
    bg: tuple = (0.0, 0.0, 0.0)
    sh_degree: int = 3

    def replace(self, **kw) -> "RenderSettings":
        return dataclasses.replace(self, **kw)

    def tiles(self, cam: Camera):
        return (cam.width + self.tile_w - 1) // self.tile_w, (cam.height + self.tile_h - 1) // self.tile_h


def random_tile_records(n: int, tiles_x: int, tiles_y: int, seed: int, n_depths: int = 64,
                        max_w: int = 5, max_h: int = 4, empty_frac: float = 0.1):
    """Seeded stand-ins for projected splats, for testing tile binning on its own:
    tile rectangles (x0, y0, x1, y1, half-open; a share of them empty) and
    positive FP32 depths drawn from `n_depths` values so that equal keys occur."""
    rng = np.random.default_rng(seed)
    x0 = rng.integers(0, tiles_x, n)
    y0 = rng.integers(0, tiles_y, n)
    x1 = np.minimum(tiles_x, x0 + rng.integers(1, max_w + 1, n))
    y1 = np.minimum(tiles_y, y0 + rng.integers(1, max_h + 1, n))
    empty = rng.uniform(size=n) < empty_frac
    x1 = np.where(empty, x0, x1)
    rect = np.stack([x0, y0, x1, y1], 1).astype(np.int16)
    depths = np.float32(rng.uniform(0.5, 8.0, n_depths))[rng.integers(0, n_depths, n)]
    return rect, depths
