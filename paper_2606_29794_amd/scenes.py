"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers: Gaussian parameters (already
activated: positive scales, opacities in (0, 1), unit quaternions), camera
poses, target images and request streams.  It contains none of the
rasterizer's arithmetic, so both the FP64 oracle and the HIP path can take
their inputs from it without sharing any computation.

All arrays are float32, structure-of-arrays ``[component][P]``:

* ``mean``    [3][P]  world-space centres
* ``scale``   [3][P]  per-axis standard deviations (exp of the drawn log-scale)
* ``rot``     [4][P]  unit quaternions (w, x, y, z)
* ``opacity`` [P]     sigmoid of a standard normal draw
* ``sh``      [K][3][P] real spherical-harmonic coefficients, K = (deg+1)^2

A camera is ``dict(W=[3][3] world->camera rotation (row-major), b=[3],
center=[3], cam_type, fov_x, fov_y, order)``.  ``b = -W @ center``.

Draw order within one seed follows a fixed sequence: means, log-scales,
quaternions, opacity logits, SH, cameras, targets, arrival times.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CAM_FULL = 0
CAM_FISHEYE = 1
CAM_PINHOLE = 2

# sqrt(4*pi): a constant function c on the sphere has degree-0 SH coefficient
# c*sqrt(4*pi) in the orthonormal real basis.  Used only to express a drawn
# final colour as a degree-0 coefficient (config 0 draws colours, not SH).
_SQRT_4PI = math.sqrt(4.0 * math.pi)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Haar-uniform rotation matrix via QR of a Gaussian matrix."""
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _unit_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((3, n))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    return v


@dataclass
class Scene:
    mean: np.ndarray
    scale: np.ndarray
    rot: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def P(self) -> int:
        return int(self.mean.shape[1])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.mean[:, idx].copy(), self.scale[:, idx].copy(),
                     self.rot[:, idx].copy(), self.opacity[idx].copy(),
                     self.sh[:, :, idx].copy(), self.sh_degree)


def make_scene(P: int, sh_degree: int, radial: str, r_lo: float, r_hi: float,
               seed: int, log_scale_mu: float = -3.0, log_scale_sigma: float = 0.5,
               sh_sigma: float = 0.2, rgb_dc: bool = False,
               rng: np.random.Generator | None = None) -> Scene:
    """Gaussians around the origin.

    radial = "volume": r^3 uniform in [r_lo^3, r_hi^3] (uniform density in a shell)
    radial = "log":    log r uniform in [log r_lo, log r_hi]
    rgb_dc: draw the final colour U[0,1]^3 and store it as a degree-0 coefficient
    (only meaningful with sh_degree 0); otherwise every coefficient ~ N(0, sh_sigma).
    """
    rng = rng or _rng(seed)
    d = _unit_dirs(rng, P)
    u = rng.random(P)
    if radial == "volume":
        r = (r_lo ** 3 + u * (r_hi ** 3 - r_lo ** 3)) ** (1.0 / 3.0)
    elif radial == "log":
        r = np.exp(np.log(r_lo) + u * (np.log(r_hi) - np.log(r_lo)))
    else:
        raise ValueError(radial)
    mean = (d * r[None, :]).astype(np.float32)
    log_s = rng.normal(log_scale_mu, log_scale_sigma, size=(3, P))
    scale = np.exp(log_s).astype(np.float32)
    q = rng.standard_normal((4, P))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    rot = q.astype(np.float32)
    logit = rng.standard_normal(P)
    opacity = (1.0 / (1.0 + np.exp(-logit))).astype(np.float32)
    K = (sh_degree + 1) ** 2
    if rgb_dc:
        assert sh_degree == 0
        rgb = rng.random((3, P))
        sh = ((rgb - 0.5) * _SQRT_4PI)[None].astype(np.float32)
    else:
        sh = rng.normal(0.0, sh_sigma, size=(K, 3, P)).astype(np.float32)
    return Scene(np.ascontiguousarray(mean), np.ascontiguousarray(scale),
                 np.ascontiguousarray(rot), np.ascontiguousarray(opacity),
                 np.ascontiguousarray(sh), sh_degree)


def axis_rotation(axis: int, angle: float) -> np.ndarray:
    """Rotation by `angle` radians about coordinate axis 0, 1 or 2."""
    c, s = math.cos(angle), math.sin(angle)
    i, j = [(1, 2), (2, 0), (0, 1)][axis]
    R = np.eye(3)
    R[i, i] = c; R[i, j] = -s; R[j, i] = s; R[j, j] = c
    return R


def make_camera(rng: np.random.Generator, order: int, cam_type: int = CAM_FULL,
                fov_x: float = 2 * math.pi, fov_y: float = math.pi,
                center_radius: float = 0.0, rotate: bool = True, W: np.ndarray | None = None) -> dict:
    """Camera with uniform random rotation (or the given W) and centre
    uniform in a ball."""
    if W is None:
        W = random_rotation(rng) if rotate else np.eye(3)
    if center_radius > 0:
        c = _unit_dirs(rng, 1)[:, 0] * center_radius * rng.random() ** (1.0 / 3.0)
    else:
        c = np.zeros(3)
    b = -W @ c
    return dict(W=W.astype(np.float32), b=b.astype(np.float32),
                center=c.astype(np.float32), cam_type=int(cam_type),
                fov_x=float(fov_x), fov_y=float(fov_y), order=int(order))


def pinhole_fov_y(fov_x: float, aspect_w: float = 16.0, aspect_h: float = 9.0) -> float:
    """Vertical FoV of a pinhole with square pixels and the given aspect."""
    return 2.0 * math.atan(math.tan(fov_x / 2.0) * aspect_h / aspect_w)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    scene: Scene
    cameras: list
    targets: list = field(default_factory=list)   # per view: [3][n_active] drawn lazily
    seed: int = 0
    extra: dict = field(default_factory=dict)


def config0(P: int = 2000) -> Workload:
    """2,000 SH-0 Gaussians in a volume-uniform shell r in [2, 6], camera at
    the origin with identity pose, full sphere at Nside 64 (order 6)."""
    seed = 1000
    rng = _rng(seed)
    sc = make_scene(P, 0, "volume", 2.0, 6.0, seed, rgb_dc=True, rng=rng)
    cam = make_camera(rng, 6, CAM_FULL, rotate=False)
    return Workload("cfg0_fwd_2k_sh0_nside64", sc, [cam], seed=seed)


def config1(P: int = 100_000, order: int = 8) -> Workload:
    """100K SH-3 Gaussians (config-0 spatial law), a 180-degree fisheye with a
    random optical axis at Nside 256 (order 8)."""
    seed = 1001
    rng = _rng(seed)
    sc = make_scene(P, 3, "volume", 2.0, 6.0, seed, rng=rng)
    cam = make_camera(rng, order, CAM_FISHEYE, fov_x=math.pi, fov_y=math.pi)
    return Workload("cfg1_fwdbwd_100k_sh3_fisheye180_nside256", sc, [cam], seed=seed)


def config1_fd(variant: str = "literal") -> Workload:
    """64-Gaussian, Nside 16 gradient-check scenes.

    literal: the config-1 laws at 64 Gaussians.
    overlap: log-scales shifted by +1.4 and means in a 60-degree cap around the
    optical axis so that footprints overlap at this coarse grid."""
    seed = 1101 if variant == "literal" else 1102
    rng = _rng(seed)
    if variant == "literal":
        sc = make_scene(64, 3, "volume", 2.0, 6.0, seed, rng=rng)
    else:
        sc = make_scene(64, 3, "volume", 2.0, 6.0, seed, log_scale_mu=-1.6, rng=rng)
        # fold directions into a 60-degree cap around +z (camera optical axis)
        m = sc.mean.astype(np.float64)
        r = np.linalg.norm(m, axis=0)
        cz = np.cos(np.deg2rad(30.0))
        u = rng.random(64)
        z = cz + u * (1 - cz)
        phi = rng.random(64) * 2 * np.pi
        s = np.sqrt(1 - z * z)
        sc.mean = np.ascontiguousarray(np.stack([s * np.cos(phi), s * np.sin(phi), z]) * r).astype(np.float32)
    # a fixed small tilt keeps the optical axis near world +z while no pixel
    # centre falls exactly on the 90-degree mask boundary
    W = axis_rotation(0, 0.11) @ axis_rotation(1, 0.23)
    cam = make_camera(rng, 4, CAM_FISHEYE, fov_x=math.pi, fov_y=math.pi, W=W)
    return Workload(f"cfg1fd_{variant}_64_sh3_nside16", sc, [cam], seed=seed)


def config2(P: int = 1_000_000, n_views: int = 4, order: int = 9) -> Workload:
    """1M SH-3 Gaussians, log-uniform radius in [1, 20]; four full-sphere
    views at Nside 512 (order 9) from centres in a ball of radius 0.5."""
    seed = 1002
    rng = _rng(seed)
    sc = make_scene(P, 3, "log", 1.0, 20.0, seed, rng=rng)
    cams = [make_camera(rng, order, CAM_FULL, center_radius=0.5) for _ in range(n_views)]
    return Workload("cfg2_train_1m_sh3_4x_full_nside512", sc, cams, seed=seed)


def config3(P: int = 3_000_000, order: int = 11) -> Workload:
    """3M SH-3 Gaussians (config-2 spatial law); one 60-degree 16:9 pinhole
    at Nside 2048 (order 11)."""
    seed = 1003
    rng = _rng(seed)
    sc = make_scene(P, 3, "log", 1.0, 20.0, seed, rng=rng)
    fx = math.radians(60.0)
    cam = make_camera(rng, order, CAM_PINHOLE, fov_x=fx, fov_y=pinhole_fov_y(fx), center_radius=0.5)
    return Workload("cfg3_pinhole60_3m_sh3_nside2048", sc, [cam], seed=seed)


def config4(P: int = 2_000_000, n_requests: int = 2000, rate_hz: float = 200.0) -> Workload:
    """Serving trace: resident 2M SH-3 scene; Poisson arrivals; random pose,
    camera type and Nside in {128, 256, 512, 1024} per request."""
    seed = 1004
    rng = _rng(seed)
    sc = make_scene(P, 3, "log", 1.0, 20.0, seed, rng=rng)
    cams = []
    for _ in range(n_requests):
        kind = int(rng.integers(0, 3))
        order = int(rng.integers(7, 11))
        if kind == 0:
            fx = math.radians(rng.uniform(60.0, 90.0))
            cams.append(make_camera(rng, order, CAM_PINHOLE, fov_x=fx, fov_y=pinhole_fov_y(fx), center_radius=0.5))
        elif kind == 1:
            f = math.radians(rng.uniform(180.0, 220.0))
            cams.append(make_camera(rng, order, CAM_FISHEYE, fov_x=f, fov_y=f, center_radius=0.5))
        else:
            cams.append(make_camera(rng, order, CAM_FULL, center_radius=0.5))
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arrivals = np.cumsum(gaps)
    return Workload("cfg4_serve_2m_sh3_mixed", sc, cams, seed=seed, extra=dict(arrivals=arrivals))


def target_image(seed: int, view: int, n_active: int) -> np.ndarray:
    """Seeded U[0,1] noise target, [3][n_active] float32."""
    rng = _rng(seed * 1000 + 17 + view)
    return rng.random((3, n_active)).astype(np.float32)
