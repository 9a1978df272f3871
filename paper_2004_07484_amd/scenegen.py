"""Seeded synthetic scenes, cameras and upstream gradients.

This module only draws random inputs. It holds none of the renderer's
arithmetic, so both the HIP path and the FP64 oracle can be fed from it.
Every value is drawn in float64 with numpy's PCG64 generator and cast to
float32, the precision the renderer consumes.

Workloads follow the shapes the paper uses for its timings and examples:
a scene is a set of spheres with position, radius, opacity and a feature
vector (Sec. 3.1), seen by a pinhole camera with focal length and sensor
width (Sec. 3.2, Lst. 1); sphere counts of 1e3 to 3e6 and images of 64^2
to 1080p bracket Tab. 2 (15k and 234k points at 1000^2) and Fig. 3
(up to 4.4M spheres at 1024^2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Camera:
    """Pinhole camera: x_cam = R @ x_world + t, principal point at the sensor centre.

    ``focal`` and ``sensor_width`` share one unit (Lst. 1 passes them as
    f and s). Pixels are square: pitch = sensor_width / width. ``znear`` and
    ``zfar`` bound the hit distance that maps to the depth z in [0, 1].
    ``orthographic``: parallel rays along +z from the pixel centres on the
    sensor plane z = 0 instead (``focal`` then plays no part).
    """

    R: np.ndarray  # [3, 3] float32, world -> camera
    t: np.ndarray  # [3] float32
    focal: float
    sensor_width: float
    znear: float
    zfar: float
    width: int
    height: int
    orthographic: bool = False


@dataclasses.dataclass
class Scene:
    pos: np.ndarray  # [n, 3] float32
    radius: np.ndarray  # [n] float32
    opacity: Optional[np.ndarray]  # [n] float32 or None (all ones)
    payload: np.ndarray  # [n, C] float32
    bg: np.ndarray  # [C] float32

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def C(self) -> int:
        return int(self.payload.shape[1])


@dataclasses.dataclass
class Params:
    gamma: float = 0.1
    eps: float = 1e-5
    min_radius_px: float = 0.0
    K: int = 8
    stop_share: float = 0.0  # early stop threshold (0 = every hit blends)


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    camera: Camera
    params: Params
    seed: int


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def identity_camera(width: int, height: int, focal: float = 1.0,
                    sensor_width: float = 2.0, znear: float = 1.0,
                    zfar: float = 10.0) -> Camera:
    return Camera(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32),
                  focal=float(focal), sensor_width=float(sensor_width),
                  znear=float(znear), zfar=float(zfar),
                  width=int(width), height=int(height))


def look_at_camera(eye, target, up, width: int, height: int, focal: float = 1.0,
                   sensor_width: float = 2.0, znear: float = 1.0,
                   zfar: float = 10.0) -> Camera:
    """Camera at ``eye`` looking at ``target``; x right, y down, z forward."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])  # rows: camera axes in world coordinates
    t = -R @ eye
    return Camera(R=_f32(R), t=_f32(t), focal=float(focal),
                  sensor_width=float(sensor_width), znear=float(znear),
                  zfar=float(zfar), width=int(width), height=int(height))


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def box_scene(rng, n: int, C: int, r_lo: float, r_hi: float,
              z_lo: float = 3.0, z_hi: float = 6.0, xy: float = 1.0,
              payload: str = "uniform", with_opacity: bool = True) -> Scene:
    """Centres uniform in [-xy, xy]^2 x [z_lo, z_hi]; radii log-uniform."""
    x = rng.uniform(-xy, xy, n)
    y = rng.uniform(-xy, xy, n)
    z = rng.uniform(z_lo, z_hi, n)
    r = _log_uniform(rng, r_lo, r_hi, n)
    o = rng.uniform(0.3, 1.0, n)
    if payload == "uniform":
        f = rng.uniform(0.0, 1.0, (n, C))
    else:
        f = rng.standard_normal((n, C))
    return Scene(pos=_f32(np.stack([x, y, z], 1)), radius=_f32(r),
                 opacity=_f32(o) if with_opacity else None, payload=_f32(f),
                 bg=np.zeros(C, np.float32))


def blob_scene(rng, n: int, C: int, n_blobs: int = 20, sigma: float = 0.2,
               r_lo: float = 0.001, r_hi: float = 0.01,
               z_range=(3.0, 8.0)) -> Scene:
    """Centres on ``n_blobs`` isotropic Gaussian blobs, clipped to z_range by rejection."""
    mx = rng.uniform(-1.0, 1.0, n_blobs)
    my = rng.uniform(-1.0, 1.0, n_blobs)
    mz = rng.uniform(3.6, 7.4, n_blobs)
    means = np.stack([mx, my, mz], 1)
    which = rng.integers(0, n_blobs, n)
    pos = means[which] + sigma * rng.standard_normal((n, 3))
    while True:
        bad = (pos[:, 2] < z_range[0]) | (pos[:, 2] > z_range[1])
        nb = int(bad.sum())
        if nb == 0:
            break
        pos[bad] = means[which[bad]] + sigma * rng.standard_normal((nb, 3))
    r = _log_uniform(rng, r_lo, r_hi, n)
    o = rng.uniform(0.3, 1.0, n)
    f = rng.standard_normal((n, C))
    return Scene(pos=_f32(pos), radius=_f32(r), opacity=_f32(o), payload=_f32(f),
                 bg=np.zeros(C, np.float32))


def upstream_grad(seed: int, height: int, width: int, C: int) -> np.ndarray:
    """dLoss/dF ~ N(0, 1) per pixel and channel, [H, W, C] float32."""
    return _f32(np.random.default_rng(seed).standard_normal((height, width, C)))


# --- the five workloads ---------------------------------------------------

def config1() -> Workload:
    """1,000 spheres, 64x64, C=3, K=5, black background, seed 0."""
    rng = np.random.default_rng(0)
    sc = box_scene(rng, 1000, 3, 0.01, 0.1)
    return Workload("spheres1k_64x64_c3", sc, identity_camera(64, 64),
                    Params(gamma=0.1, eps=1e-5, K=5), 0)


def config2() -> Workload:
    """100,000 spheres, 512x512, C=3, K=8, seed 1."""
    rng = np.random.default_rng(1)
    sc = box_scene(rng, 100_000, 3, 0.002, 0.03)
    return Workload("spheres100k_512x512_c3", sc, identity_camera(512, 512),
                    Params(gamma=0.1, eps=1e-5, K=8), 1)


def config3(n: int = 1_000_000) -> Workload:
    """1M spheres on 20 Gaussian blobs, 1024x1024, C=8 latent N(0,1) payload, K=8, seed 2."""
    rng = np.random.default_rng(2)
    sc = blob_scene(rng, n, 8)
    return Workload(f"blobs{n // 1000}k_1024x1024_c8", sc,
                    identity_camera(1024, 1024), Params(gamma=0.1, eps=1e-5, K=8), 2)


def config5(n: int = 3_000_000) -> Workload:
    """3M spheres on blobs, 1920x1080, C=16, K=8, seed 5."""
    rng = np.random.default_rng(5)
    sc = blob_scene(rng, n, 16)
    return Workload(f"blobs{n // 1000}k_1920x1080_c16", sc,
                    identity_camera(1920, 1080), Params(gamma=0.1, eps=1e-5, K=8), 5)


def config4_scenes(B: int = 32, seed: int = 3) -> List[Workload]:
    """Uneven batch: sphere counts log-uniform in [1e3, 5e5], square sizes from
    {256, 512, 768, 1024}, cameras on a radius-5 sphere looking at the origin."""
    out = []
    for b, ss in enumerate(np.random.SeedSequence(seed).spawn(B)):
        rng = np.random.default_rng(ss)
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(5e5)))))
        res = int(rng.choice([256, 512, 768, 1024]))
        up = np.array([0.0, 0.0, 1.0])
        while True:
            v = rng.standard_normal(3)
            v /= np.linalg.norm(v)
            if abs(float(v @ up)) <= 0.99:
                break
        cam = look_at_camera(5.0 * v, np.zeros(3), up, res, res)
        x = rng.uniform(-1.0, 1.0, (n, 3))
        r = _log_uniform(rng, 0.002, 0.03, n)
        o = rng.uniform(0.3, 1.0, n)
        f = rng.uniform(0.0, 1.0, (n, 3))
        sc = Scene(pos=_f32(x), radius=_f32(r), opacity=_f32(o), payload=_f32(f),
                   bg=np.zeros(3, np.float32))
        out.append(Workload(f"batch{b}_{n}_{res}", sc, cam,
                            Params(gamma=0.1, eps=1e-5, K=5), seed))
    return out


def tiny_scene(seed: int, n: int = 5, C: int = 2, W: int = 24, H: int = 24,
               r_lo: float = 0.15, r_hi: float = 0.45, with_opacity: bool = True,
               bg: Optional[np.ndarray] = None) -> Workload:
    """A handful of large spheres filling a small image (finite-difference scale)."""
    rng = np.random.default_rng(seed)
    sc = box_scene(rng, n, C, r_lo, r_hi, z_lo=3.0, z_hi=5.0, xy=0.8,
                   payload="normal", with_opacity=with_opacity)
    if bg is None:
        sc.bg = _f32(rng.uniform(-0.5, 0.5, C))
    else:
        sc.bg = _f32(bg)
    return Workload(f"tiny{seed}", sc, identity_camera(W, H, focal=3.0),
                    Params(gamma=0.5, eps=1e-5, K=n + 1), seed)


WORKLOADS = {
    "cfg1": config1,
    "cfg2": config2,
    "cfg3": config3,
    "cfg5": config5,
}
