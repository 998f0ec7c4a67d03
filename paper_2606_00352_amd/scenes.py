"""Seeded synthetic scenes and cameras.

This module only draws inputs: it holds none of the renderer's arithmetic and
is shared by the GPU path, the tests and the benchmark.  The scenes stand in
for the trained Mip-NeRF 360 / nvcampus models the paper measures on (sec. 5.1,
Experimental setup), which are not available: they take the paper's scale
(5.8M gaussians as its "garden" scene, 1080p and 4K frames, degree-3 SH) and a
clustered layout whose dense screen regions hold thousands of gaussians per
8x8 render tile, as the paper's teaser scene does (peak 2,485, Fig. 1).

Conventions of every scene array (all float32, C-contiguous):
  means [N,3]; scales [N,3] (linear, already exponentiated); quats [N,4] as
  (w, x, y, z), unit length; opacities [N] (already through the sigmoid);
  sh [N,16,3] (coefficient-major, RGB-minor; degree 3).
Cameras are pinhole with OpenCV axes (x right, y down, z forward) and a
world-to-camera [R | t] matrix.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SH_COEFFS = 16  # degree 3


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    world_to_cam: np.ndarray  # float32 [3, 4], row-major [R | t]
    background: tuple = (0.0, 0.0, 0.0)

    def __post_init__(self):
        self.world_to_cam = np.ascontiguousarray(self.world_to_cam, dtype=np.float32).reshape(3, 4)


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

    def arrays(self):
        return self.means, self.scales, self.quats, self.opacities, self.sh


def _finish(rng, means, n, log_scale_mean, log_scale_std, logit_std=1.5):
    """Draws the per-gaussian attributes after the means, in a fixed order:
    log-scales, quaternions, opacity logits, SH DC, SH rest."""
    log_s = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logit = rng.normal(0.0, logit_std, size=n)
    dc = rng.uniform(0.0, 1.0, size=(n, 1, 3))
    rest = rng.normal(0.0, 0.1, size=(n, SH_COEFFS - 1, 3))
    return Scene(
        means=np.ascontiguousarray(means, dtype=np.float32),
        scales=np.ascontiguousarray(np.exp(log_s), dtype=np.float32),
        quats=np.ascontiguousarray(q, dtype=np.float32),
        opacities=np.ascontiguousarray(1.0 / (1.0 + np.exp(-logit)), dtype=np.float32),
        sh=np.ascontiguousarray(np.concatenate([dc, rest], axis=1), dtype=np.float32),
    )


def uniform_scene(n: int = 10_000, seed: int = 0, log_scale_mean: float = math.log(0.02),
                  log_scale_std: float = 0.5) -> Scene:
    """Small parity scene: means uniform in x, y in [-1, 1], z in [2, 6]."""
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-1.0, 1.0, size=(n, 2))
    z = rng.uniform(2.0, 6.0, size=(n, 1))
    return _finish(rng, np.concatenate([xy, z], axis=1), n, log_scale_mean, log_scale_std)


def _random_rotation(rng) -> np.ndarray:
    # QR of a gaussian matrix, sign-fixed: a uniformly random orthogonal matrix
    a = rng.normal(size=(3, 3))
    qm, r = np.linalg.qr(a)
    qm = qm * np.sign(np.diag(r))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


# Base standard deviation (world units) of the clusters.  With it the dense
# screen regions of the 5.8M-gaussian 1080p orbit views hold ~2,900-4,000
# opacity-level boxes per 8x8 render tile (99th percentile of tiles; the
# busiest tile of a view holds 3,700-10,000).  Wider clusters do not get the
# peak lower: past ~5 units they fill the 20-unit box and the peak settles
# near 7,000 from depth stacking alone.
CLUSTER_SPREAD = 4.0


def clustered_scene(n: int = 5_800_000, seed: int = 1, n_clusters: int = 200, box: float = 10.0,
                    spread: float = CLUSTER_SPREAD, log_scale_mean: float = math.log(0.02),
                    log_scale_std: float = 0.5) -> Scene:
    """Mixture of anisotropic clusters inside [-box, box]^3 with Pareto
    (alpha = 1.2, x_m = 1) cluster weights; gaussian order shuffled."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box, box, size=(n_clusters, 3))
    weights = 1.0 + rng.pareto(1.2, size=n_clusters)
    counts = rng.multinomial(n, weights / weights.sum())
    pts = np.empty((n, 3), dtype=np.float64)
    at = 0
    for k in range(n_clusters):
        m = int(counts[k])
        if m == 0:
            continue
        rot = _random_rotation(rng)
        std = spread * np.exp(rng.normal(0.0, 0.5, size=3))
        got = np.empty((0, 3))
        while got.shape[0] < m:
            need = m - got.shape[0]
            cand = centres[k] + (rng.normal(size=(need + need // 4 + 16, 3)) * std) @ rot.T
            cand = cand[np.all(np.abs(cand) <= box, axis=1)]
            got = np.concatenate([got, cand[:need]], axis=0)
        pts[at:at + m] = got
        at += m
    pts = pts[rng.permutation(n)]
    return _finish(rng, pts, n, log_scale_mean, log_scale_std)


def camera_at_origin(width: int = 256, height: int = 256, f: float = 256.0,
                     background=(0.0, 0.0, 0.0)) -> Camera:
    """Camera at the world origin looking down +z, principal point centred."""
    m = np.zeros((3, 4), dtype=np.float32)
    m[0, 0] = m[1, 1] = m[2, 2] = 1.0
    return Camera(width, height, f, f, width / 2.0, height / 2.0, m, tuple(background))


def look_at_origin(eye, width: int, height: int, f: float, background=(0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera at `eye` looking at the world origin, with world -y up."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = -eye / np.linalg.norm(eye)
    right = np.cross(fwd, np.array([0.0, -1.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    rot = np.stack([right, down, fwd], axis=0)
    t = -rot @ eye
    m = np.concatenate([rot, t[:, None]], axis=1).astype(np.float32)
    return Camera(width, height, f, f, width / 2.0, height / 2.0, m, tuple(background))


def orbit_cameras(n_views: int = 60, seed: int = 101, width: int = 1920, height: int = 1080,
                  f: float = 1100.0, radius: float = 25.0, elevation_deg: float = 20.0,
                  background=(0.0, 0.0, 0.0)):
    """Evenly spaced views on a circular orbit around the origin; the starting
    azimuth is drawn from `seed`."""
    rng = np.random.default_rng(seed)
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    e = math.radians(elevation_deg)
    cams = []
    for i in range(n_views):
        th = phi0 + 2.0 * math.pi * i / n_views
        eye = (radius * math.cos(e) * math.sin(th), -radius * math.sin(e),
               -radius * math.cos(e) * math.cos(th))
        cams.append(look_at_origin(eye, width, height, f, background))
    return cams


# Named workloads --------------------------------------------------------------

def config0():
    """10,000 gaussians, 256x256, camera at the origin looking +z, f = 256."""
    return uniform_scene(10_000, seed=0), [camera_at_origin(256, 256, 256.0)]


def config1(n: int = 5_800_000, n_views: int = 60):
    """5.8M clustered gaussians, 1920x1080, 60-view orbit, f = 1100."""
    return clustered_scene(n, seed=1), orbit_cameras(n_views, 101, 1920, 1080, 1100.0)


def config2(n: int = 6_000_000, n_views: int = 60):
    """6M clustered gaussians with larger splats, 3840x2160, f = 2200."""
    scene = clustered_scene(n, seed=2, log_scale_mean=math.log(0.05), log_scale_std=0.7)
    return scene, orbit_cameras(n_views, 102, 3840, 2160, 2200.0)


# Serving workload ---------------------------------------------------------------

SERVING_SIZES = (500_000, 1_500_000, 3_000_000, 5_800_000)
SERVING_RESOLUTIONS = ((1280, 720), (1920, 1080), (3840, 2160))


def serving_scenes(sizes=SERVING_SIZES, first_seed: int = 31):
    """Resident scenes of the serving workload: clustered scenes (the 1080p
    benchmark generator) of the given sizes, seeds first_seed, first_seed + 1, ..."""
    return [clustered_scene(n, seed=first_seed + k) for k, n in enumerate(sizes)]


@dataclasses.dataclass
class Request:
    id: int
    arrival: float      # seconds from the start of the trace
    scene: int          # index into the resident scenes
    cls: int            # index into the resolutions
    camera: Camera


def serving_trace(duration: float, rate: float = 2000.0, seed: int = 35, n_scenes: int = 4,
                  resolutions=SERVING_RESOLUTIONS, radius: float = 25.0):
    """Poisson arrivals at `rate` per second over `duration` seconds; each
    request picks a scene and a resolution uniformly and an orbit camera with
    azimuth ~ U(0, 2 pi), elevation ~ U(10, 30) degrees at `radius`, focal
    length 1100 * W / 1920 (the 1080p field of view at every size)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        scene = int(rng.integers(n_scenes))
        cls = int(rng.integers(len(resolutions)))
        th = rng.uniform(0.0, 2.0 * math.pi)
        e = math.radians(rng.uniform(10.0, 30.0))
        w, h = resolutions[cls]
        eye = (radius * math.cos(e) * math.sin(th), -radius * math.sin(e), -radius * math.cos(e) * math.cos(th))
        out.append(Request(len(out), t, scene, cls, look_at_origin(eye, w, h, 1100.0 * w / 1920.0)))
    return out
