"""Seeded synthetic inputs: scenes of disentangled 4D Gaussians, pinhole cameras and
request streams, shaped like the paper's workloads (Sec. 4: Plenoptic Video at
1352x1014, D-NeRF-like random point clouds, Tab. 5's 100,000-Gaussian speed test).

This module holds no arithmetic of the rendering method.  It only draws numbers
and builds camera poses; both the GPU path and the CPU oracle consume what it
returns.  All arrays are float32 in the planar layout the library expects:

    mean      (3, N)   world-space spatial mean mu_xyz
    scale     (3, N)   activated spatial scales s_xyz = exp(log-scale)
    quat      (4, N)   rotation quaternion, scalar first (w, x, y, z), unnormalised
    opacity   (N,)     activated opacity o = sigmoid(logit)
    t_mean    (N,)     temporal mean mu_t
    t_scale   (N,)     activated temporal scale s_t = exp(log s_t)
    velocity  (3, N)   velocity of the mean V_3D
    sh        (K, 3, N) spherical-harmonic coefficients, K = (degree + 1)^2

The disentangled representation is the paper's Eq. 8 (s_4D, mu_4D, q, V_3D) plus
opacity and colour.  Raw (pre-activation) parameters are kept alongside so that a
perturbed copy can be drawn the way a training target would be.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TILE = 16


@dataclass
class Scene:
    n: int
    sh_degree: int
    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    t_mean: np.ndarray
    t_scale: np.ndarray
    velocity: np.ndarray
    sh: np.ndarray
    raw: dict = field(default_factory=dict, repr=False)

    FIELDS = ("mean", "scale", "quat", "opacity", "t_mean", "t_scale", "velocity", "sh")

    def arrays(self):
        return {k: getattr(self, k) for k in self.FIELDS}

    def subset(self, idx):
        idx = np.asarray(idx)
        kw = {k: np.ascontiguousarray(getattr(self, k)[..., idx]) for k in self.FIELDS}
        return Scene(n=int(idx.size), sh_degree=self.sh_degree, **kw)

    def nbytes(self):
        return sum(getattr(self, k).nbytes for k in self.FIELDS)


@dataclass
class Camera:
    """Pinhole camera; R is world-to-camera (row major), the camera looks along +z,
    x to the right and y down in the image.  Intrinsics in pixels."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    tan_fovx: float
    tan_fovy: float
    znear: float
    R: np.ndarray  # (9,) float32
    T: np.ndarray  # (3,) float32
    campos: np.ndarray  # (3,) float32

    @property
    def tiles(self):
        return ((self.width + TILE - 1) // TILE) * ((self.height + TILE - 1) // TILE)


def _f32(x):
    return float(np.float32(x))


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), width=128, height=128,
            fovx_deg=60.0, znear=0.2, cx=None, cy=None) -> Camera:
    """Camera at `eye` looking at `target`.  Horizontal field of view `fovx_deg`,
    square pixels, principal point at the image centre unless given."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.asarray(up, np.float64)
    if abs(float(fwd @ up)) > 0.999:
        up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32)
    T = (-(R.astype(np.float64) @ eye)).astype(np.float32)
    fx = _f32(width / (2.0 * math.tan(math.radians(fovx_deg) / 2.0)))
    fy = fx
    cx = _f32(width / 2.0) if cx is None else _f32(cx)
    cy = _f32(height / 2.0) if cy is None else _f32(cy)
    return Camera(width=int(width), height=int(height), fx=fx, fy=fy, cx=cx, cy=cy,
                  tan_fovx=_f32(width / (2.0 * fx)), tan_fovy=_f32(height / (2.0 * fy)),
                  znear=_f32(znear), R=R.reshape(9).copy(), T=T.copy(),
                  campos=eye.astype(np.float32))


def _log_uniform(rng, lo, hi, n):
    return rng.uniform(math.log(lo), math.log(hi), n)


def make_scene(seed, n, sh_degree, *, box=None, clusters=None, cluster_box=None, cluster_std=0.8,
               log_scale=(-3.0, 0.3), dc=(0.5, 0.2), rest_std=0.05, t_scale_range=(0.05, 0.5),
               vel_std=0.2, morton=True) -> Scene:
    """Draw a scene.  Draw order (fixed): cluster centres, cluster assignment,
    offsets (or uniform means), log-scales, quaternions, opacity logits, SH,
    temporal means, log temporal scales, velocities.  The Gaussians are then stored in
    3D Morton order of their means (a storage order; any order renders the same set)."""
    rng = np.random.default_rng(seed)
    if clusters:
        lo, hi = cluster_box
        centres = rng.uniform(lo, hi, (clusters, 3))
        assign = rng.integers(0, clusters, n)
        offs = rng.normal(0.0, cluster_std, (n, 3))
        mean = (centres[assign] + offs).T
    else:
        lo, hi = box
        mean = rng.uniform(lo, hi, (n, 3)).T
    log_s = rng.normal(log_scale[0], log_scale[1], (3, n))
    quat = rng.normal(0.0, 1.0, (4, n))
    quat /= np.linalg.norm(quat, axis=0, keepdims=True)
    logit = rng.normal(0.0, 1.0, n)
    K = (sh_degree + 1) ** 2
    sh = np.empty((K, 3, n))
    sh[0] = rng.normal(dc[0], dc[1], (3, n))
    if K > 1:
        sh[1:] = rng.normal(0.0, rest_std, (K - 1, 3, n))
    t_mean = rng.uniform(0.0, 1.0, n)
    log_st = _log_uniform(rng, t_scale_range[0], t_scale_range[1], n)
    vel = rng.normal(0.0, vel_std, (3, n))
    raw = dict(mean=mean, log_scale=log_s, quat=quat, logit=logit, sh=sh, t_mean=t_mean,
               log_t_scale=log_st, velocity=vel)
    if morton:
        order = morton_order(mean)
        raw = {k: np.ascontiguousarray(v[..., order]) for k, v in raw.items()}
    return scene_from_raw(raw, sh_degree)


def _spread10(x):
    """Spread the low 10 bits of x to every third bit."""
    x = x.astype(np.uint64) & np.uint64(0x3FF)
    x = (x | (x << np.uint64(16))) & np.uint64(0x030000FF)
    x = (x | (x << np.uint64(8))) & np.uint64(0x0300F00F)
    x = (x | (x << np.uint64(4))) & np.uint64(0x030C30C3)
    x = (x | (x << np.uint64(2))) & np.uint64(0x09249249)
    return x


def morton_order(mean):
    """Indices that sort points (3, N) along a 3D Morton (Z-order) curve over their
    bounding box, 10 bits per axis.  Storing a scene in this order keeps Gaussians that
    are close in space close in memory: a block of consecutive Gaussians then covers a
    small part of the screen from any viewpoint."""
    lo = mean.min(axis=1, keepdims=True)
    span = np.maximum(mean.max(axis=1, keepdims=True) - lo, 1e-12)
    q = np.clip(((mean - lo) / span * 1023.0).astype(np.int64), 0, 1023)
    code = _spread10(q[0]) | (_spread10(q[1]) << np.uint64(1)) | (_spread10(q[2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


def scene_from_raw(raw, sh_degree) -> Scene:
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    n = raw["mean"].shape[1]
    return Scene(n=n, sh_degree=sh_degree, mean=f(raw["mean"]), scale=f(np.exp(raw["log_scale"])),
                 quat=f(raw["quat"]), opacity=f(1.0 / (1.0 + np.exp(-raw["logit"]))),
                 t_mean=f(raw["t_mean"]), t_scale=f(np.exp(raw["log_t_scale"])),
                 velocity=f(raw["velocity"]), sh=f(raw["sh"]), raw=raw)


def perturb_raw(scene: Scene, seed, std=0.01) -> Scene:
    """Copy of `scene` with N(0, std) noise on every raw parameter."""
    rng = np.random.default_rng(seed)
    raw = {k: v + rng.normal(0.0, std, v.shape) for k, v in scene.raw.items()}
    return scene_from_raw(raw, scene.sh_degree)


# ----------------------------------------------------------------------------- workloads
def small_case():
    """2,000 Gaussians, 128x128, SH0, t = 0.5 (correctness case)."""
    sc = make_scene(1, 2000, 0, box=(-2.0, 2.0), log_scale=(-3.0, 0.3), dc=(0.5, 0.2),
                    t_scale_range=(0.05, 0.5), vel_std=0.2)
    cam = look_at((0.0, 0.0, -6.0), width=128, height=128, fovx_deg=60.0)
    return sc, cam, np.float32(0.5)


def clustered_scene(n=300_000, seed=2, sh_degree=3, morton=True):
    """Plenoptic-like: 32-cluster mixture in [-5,5]^3, SH3.  morton=False keeps the draw
    order (Gaussians of all clusters interleaved, as a trained scene may store them)."""
    return make_scene(seed, n, sh_degree, clusters=32, cluster_box=(-5.0, 5.0), cluster_std=0.8,
                      log_scale=(-4.5, 0.6), dc=(0.5, 0.2), rest_std=0.05,
                      t_scale_range=(0.02, 0.5), vel_std=0.1, morton=morton)


def arc_camera(j, n_cams=20, radius=10.0, width=1352, height=1014):
    th = math.radians(-60.0 + 120.0 * j / (n_cams - 1))
    return look_at((radius * math.sin(th), 0.0, -radius * math.cos(th)), width=width, height=height)


def arc_cameras(width=1352, height=1014):
    return [arc_camera(j, 20, 10.0, width, height) for j in range(20)]


def sweep_times(k=300):
    return [np.float32(i / (k - 1)) for i in range(k)]


def sphere_camera(rng, radius, width, height):
    d = rng.normal(0.0, 1.0, 3)
    d /= np.linalg.norm(d)
    return look_at(radius * d, width=width, height=height)


def fit_case(n=100_000):
    """Differentiation case: clustered-scene distributions with SH1, 8 random (camera, t) views
    at 800x800, target = the same scene with N(0, 0.01) noise on raw parameters."""
    sc = clustered_scene(n=n, seed=3, sh_degree=1)
    rng = np.random.default_rng(1003)
    views = []
    for _ in range(8):
        cam = sphere_camera(rng, 10.0, 800, 800)
        views.append((cam, np.float32(rng.uniform(0.0, 1.0))))
    target_scene = perturb_raw(sc, 2003, 0.01)
    return sc, views, target_scene


RES_CHOICES = ((640, 480), (1352, 1014), (1920, 1080))
RES_PROBS = (0.5, 0.3, 0.2)


def serving_scene(n=500_000):
    return clustered_scene(n=n, seed=4, sh_degree=3)


def serving_requests(rate=200.0, duration=60.0, seed=1004):
    """Poisson arrivals; each request: camera on the radius-10 sphere, t ~ U[0,1],
    resolution from {640x480: 0.5, 1352x1014: 0.3, 1920x1080: 0.2}."""
    rng = np.random.default_rng(seed)
    reqs = []
    at = 0.0
    while True:
        at += rng.exponential(1.0 / rate)
        if at >= duration:
            break
        w, h = RES_CHOICES[rng.choice(3, p=RES_PROBS)]
        cam = sphere_camera(rng, 10.0, w, h)
        reqs.append((at, cam, np.float32(rng.uniform(0.0, 1.0))))
    return reqs


def large_scene(n=2_000_000):
    return make_scene(5, n, 3, clusters=128, cluster_box=(-10.0, 10.0), cluster_std=0.8,
                      log_scale=(-5.0, 0.7), dc=(0.5, 0.2), rest_std=0.05,
                      t_scale_range=(0.01, 0.5), vel_std=0.15)


def large_views(width=2704, height=2028):
    out = []
    for th, t in zip((-45.0, -15.0, 15.0, 45.0), (0.125, 0.375, 0.625, 0.875)):
        r = math.radians(th)
        out.append((look_at((25.0 * math.sin(r), 0.0, -25.0 * math.cos(r)), width=width, height=height),
                    np.float32(t)))
    return out


def upstream_grad(seed, width, height):
    """A seeded dL/dimage of shape (3, H, W) (a fixed random linear functional)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1.0, (3, height, width)).astype(np.float32)
