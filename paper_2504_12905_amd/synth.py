"""Seeded synthetic inputs: scenes, cameras, initialisations, sample-free request streams.

This module is shared by the FP64 oracle tests and the HIP path. It holds none of
the method's arithmetic (no projection, rendering, derivatives or solver code):
it only draws random numbers and lays them out in the parameter layout below.

Parameter vector beta (float32, length P = n * (11 + 3K), K = (d+1)^2, d = SH
degree). The paper's per-Gaussian parameters are opacity, colour, mean, scale and
quaternion (Sec. 4.1); spherical-harmonic colour of degree d replaces the plain
colour. Segments are component-major (all Gaussians' x, then all y, ...):

    [0n, 3n)          mean x, y, z
    [3n, 6n)          log-scale x, y, z
    [6n, 10n)         quaternion w, x, y, z (not normalised)
    [10n, 11n)        opacity logit
    [11n + (3k + c) n]  SH coefficient k (0..K-1) of colour channel c

Cameras are float32 rows of 16: R (3x3 world-to-camera, row-major), t (3),
fx, fy, cx, cy. Axes follow the usual computer-vision convention: x right,
y down, z forward; the pixel (i, j) has its centre at (i + 0.5, j + 0.5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CAM_FLOATS = 16
# 1 / (2 sqrt(pi)): value of the degree-0 real spherical harmonic. Used here only
# to express "RGB drawn uniformly in [0, 1]" as a DC coefficient of a colour that
# is 0.5 + Y00 * f (the colour model whose range the paper quotes in Sec. 4.5).
_Y00 = 0.28209479177387814


def n_params(n: int, sh_degree: int) -> int:
    return n * (11 + 3 * (sh_degree + 1) ** 2)


def seg(n: int, name: str, sh_degree: int = 0) -> slice:
    """Slice of beta holding one parameter group (component-major)."""
    K = (sh_degree + 1) ** 2
    table = {
        "mean": (0, 3), "log_scale": (3, 6), "quat": (6, 10), "opacity": (10, 11),
        "sh": (11, 11 + 3 * K), "sh_dc": (11, 14),
    }
    a, b = table[name]
    return slice(a * n, b * n)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def make_scene(n: int, sh_degree: int, seed: int, means: str = "cube", extent: float = 1.0,
               log_scale_mu: float = -3.0, log_scale_sd: float = 0.3,
               sh_rest_sd: float = 0.1) -> np.ndarray:
    """Ground-truth scene with the priors shared by the synthetic workloads.

    means: 'cube' = uniform in [-extent, extent]^3; 'ball' = uniform in the ball of
    radius extent; 'logradius' = radius exp(U[ln 0.05, ln 10]) times a uniform
    direction (dense toward the centre; used for the unbounded-scene workload).
    """
    g = _rng(seed, 0)
    K = (sh_degree + 1) ** 2
    beta = np.zeros(n_params(n, sh_degree), dtype=np.float64)
    if means == "cube":
        mu = g.uniform(-extent, extent, size=(3, n))
    elif means == "ball":
        d = g.normal(size=(3, n))
        d /= np.linalg.norm(d, axis=0, keepdims=True)
        r = extent * g.uniform(size=n) ** (1.0 / 3.0)
        mu = d * r
    elif means == "logradius":
        d = g.normal(size=(3, n))
        d /= np.linalg.norm(d, axis=0, keepdims=True)
        r = np.exp(g.uniform(math.log(0.05), math.log(10.0), size=n))
        mu = d * r
    else:
        raise ValueError(means)
    beta[seg(n, "mean")] = mu.reshape(-1)
    beta[seg(n, "log_scale")] = g.normal(log_scale_mu, log_scale_sd, size=3 * n)
    q = g.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    beta[seg(n, "quat")] = q.reshape(-1)
    beta[seg(n, "opacity")] = g.normal(0.0, 1.0, size=n)
    rgb = g.uniform(0.0, 1.0, size=(3, n))
    sh = np.zeros((K, 3, n))
    sh[0] = (rgb - 0.5) / _Y00
    if K > 1:
        sh[1:] = g.normal(0.0, sh_rest_sd, size=(K - 1, 3, n))
    beta[seg(n, "sh", sh_degree)] = sh.reshape(-1)
    return beta.astype(np.float32)


def perturb_init(beta: np.ndarray, n: int, sh_degree: int, seed: int,
                 mean_sd: float = 0.05, log_scale_sd: float = 0.2, rgb_sd: float = 0.1) -> np.ndarray:
    """Initialisation = ground truth + noise on means, log-scales and DC colour.

    The colour noise is drawn in RGB units and expressed on the DC coefficient;
    higher SH orders, opacity and quaternions are left at the ground truth.
    """
    g = _rng(seed, 1)
    out = beta.astype(np.float64).copy()
    out[seg(n, "mean")] += g.normal(0.0, mean_sd, size=3 * n)
    out[seg(n, "log_scale")] += g.normal(0.0, log_scale_sd, size=3 * n)
    out[seg(n, "sh_dc")] += g.normal(0.0, rgb_sd, size=3 * n) / _Y00
    return out.astype(np.float32)


def look_at(center: np.ndarray, target: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """World-to-camera (R, t) for a camera at `center` looking at `target`, world up +z."""
    f = target - center
    f = f / np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0])
    if abs(float(f @ up)) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f], axis=0)
    t = -R @ center
    return R, t


def pack_camera(R: np.ndarray, t: np.ndarray, width: int, height: int, fov_deg: float) -> np.ndarray:
    fx = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    row = np.zeros(CAM_FLOATS, dtype=np.float64)
    row[0:9] = R.reshape(-1)
    row[9:12] = t
    row[12:16] = [fx, fx, width / 2.0, height / 2.0]
    return row.astype(np.float32)


def sphere_cameras(n_views: int, radius: float, width: int, height: int, fov_deg: float,
                   seed: int) -> np.ndarray:
    """Cameras with directions uniform on the sphere, looking at the origin."""
    g = _rng(seed, 2)
    out = np.zeros((n_views, CAM_FLOATS), dtype=np.float32)
    for i in range(n_views):
        d = g.normal(size=3)
        d /= np.linalg.norm(d)
        R, t = look_at(radius * d, np.zeros(3))
        out[i] = pack_camera(R, t, width, height, fov_deg)
    return out


def ellipse_cameras(n_views: int, width: int, height: int, fov_deg: float, seed: int,
                    ax: float = 3.0, ay: float = 2.0, z: float = 0.5) -> np.ndarray:
    """Cameras on a noisy horizontal ellipse at height z, looking near the origin."""
    g = _rng(seed, 3)
    out = np.zeros((n_views, CAM_FLOATS), dtype=np.float32)
    for i in range(n_views):
        th = 2.0 * math.pi * i / n_views + g.normal(0.0, 0.02)
        c = np.array([ax * math.cos(th), ay * math.sin(th), z]) + g.normal(0.0, 0.1, size=3)
        tgt = g.normal(0.0, 0.05, size=3)
        R, t = look_at(c, tgt)
        out[i] = pack_camera(R, t, width, height, fov_deg)
    return out


@dataclass
class Workload:
    """One synthetic fitting problem: ground truth, init and cameras."""
    name: str
    n: int
    sh_degree: int
    width: int
    height: int
    cams: np.ndarray              # [V_total, 16] float32
    beta_gt: np.ndarray           # [P] float32
    beta_init: np.ndarray         # [P] float32
    views_per_step: int
    sample_frac: float            # fraction of pixels per 16x16 tile (1.0 = all)
    cg_iters: int
    lm_iters: int
    lam: float
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def samples_per_tile(self) -> int:
        return 256 if self.sample_frac >= 1.0 else max(1, int(round(self.sample_frac * 256)))


def config0(seed: int = 0) -> Workload:
    """1,000 Gaussians in [-1,1]^3, SH degree 0, 4 views 64x64, all pixels."""
    n, d = 1000, 0
    gt = make_scene(n, d, seed, means="cube")
    return Workload("lm-run-1k-sh0-4x64", n, d, 64, 64,
                    sphere_cameras(4, 3.0, 64, 64, 60.0, seed), gt,
                    perturb_init(gt, n, d, seed), 4, 1.0, 10, 20, 1e-3, seed)


def config1(seed: int = 0, n: int = 100_000) -> Workload:
    """100k Gaussians in the unit ball, SH degree 3, 64 views 800x800, 8 views and
    10 % of pixels per LM step, 8 CG steps."""
    d = 3
    gt = make_scene(n, d, seed, means="ball")
    return Workload("object-100k-sh3-8of64x800", n, d, 800, 800,
                    sphere_cameras(64, 4.0, 800, 800, 60.0, seed), gt,
                    perturb_init(gt, n, d, seed), 8, 0.10, 8, 20, 0.1, seed)


def config2(seed: int = 0, n: int = 1_500_000) -> Workload:
    """1.5M Gaussians, SH degree 3, 150 views 1264x832 on a noisy ellipse, 16 views
    and 5 % residual-weighted pixels per LM step, 10 CG steps."""
    d = 3
    gt = make_scene(n, d, seed, means="logradius")
    return Workload("unbounded-1.5M-sh3-16of150x1264x832", n, d, 1264, 832,
                    ellipse_cameras(150, 1264, 832, 70.0, seed), gt,
                    perturb_init(gt, n, d, seed), 16, 0.05, 10, 20, 0.1, seed)


def config3(seed: int = 0, n: int = 200_000) -> Workload:
    """Differentiation check: 200k Gaussians, SH degree 3, 16 views 512x512."""
    d = 3
    gt = make_scene(n, d, seed, means="ball")
    return Workload("autograd-200k-sh3-16x512", n, d, 512, 512,
                    sphere_cameras(16, 4.0, 512, 512, 60.0, seed), gt,
                    perturb_init(gt, n, d, seed), 16, 1.0, 8, 1, 0.1, seed)


def tiny(n: int = 3, sh_degree: int = 0, n_views: int = 1, size: int = 32, seed: int = 0,
         log_scale_mu: float = -1.6, extent: float = 0.5) -> Workload:
    """Small scenes for dense-Jacobian checks (a few Gaussians, one or two views)."""
    gt = make_scene(n, sh_degree, seed, means="cube", extent=extent, log_scale_mu=log_scale_mu,
                    log_scale_sd=0.2)
    return Workload(f"tiny-{n}-sh{sh_degree}-{n_views}x{size}", n, sh_degree, size, size,
                    sphere_cameras(n_views, 3.0, size, size, 60.0, seed), gt,
                    perturb_init(gt, n, sh_degree, seed), n_views, 1.0, 10, 5, 1e-3, seed)


def request_stream(n_requests: int = 256, rate_hz: float = 20.0, seed: int = 0) -> list[dict]:
    """Serving workload: Poisson arrivals; per-request sizes drawn log-uniform."""
    g = _rng(seed, 4)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += g.exponential(1.0 / rate_hz)
        n = int(round(math.exp(g.uniform(math.log(2000), math.log(200_000)))))
        out.append(dict(id=i, seed=i, arrival_s=t, n=n, sh_degree=int(g.integers(0, 4)),
                        n_views=int(g.integers(4, 33)), res=int(g.choice([256, 512, 800])),
                        lm_iters=30, cg_iters=8, lam=0.1))
    return out
