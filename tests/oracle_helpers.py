"""Shared helpers for the oracle pins (no renderer arithmetic here)."""
from __future__ import annotations

import copy
import types

import numpy as np

from oracle import reference as ref


def as_f64(scene):
    return types.SimpleNamespace(
        pos=np.array(scene.pos, np.float64), radius=np.array(scene.radius, np.float64),
        opacity=None if scene.opacity is None else np.array(scene.opacity, np.float64),
        payload=np.array(scene.payload, np.float64), bg=np.array(scene.bg, np.float64))


def random_rotation(rng) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def intrinsics(cam) -> np.ndarray:
    """Hartley-Zisserman intrinsic matrix in pixel units, pixel (i, j) spans
    [j, j+1) x [i, i+1) and the principal point is the image centre."""
    fpx = cam.focal * cam.width / cam.sensor_width
    return np.array([[fpx, 0.0, cam.width / 2.0], [0.0, fpx, cam.height / 2.0], [0.0, 0.0, 1.0]])


def pixel_direction(cam, i, j) -> np.ndarray:
    """Unit camera-space ray through the centre of pixel (i, j), via K^-1."""
    v = np.linalg.solve(intrinsics(cam), np.array([j + 0.5, i + 0.5, 1.0]))
    return v / np.linalg.norm(v)


def loss(scene, cam, params, G, rows=None) -> float:
    F = ref.forward(scene, cam, params, rows=rows)["F"]
    if rows is None:
        return float(np.sum(G * F))
    return float(np.sum(G[rows] * F[rows]))


def fd_grads(scene, cam, params, G, rel_h=1e-6, rows=None, which=None):
    """Central finite differences of sum(G * F) for every scene parameter."""
    out = {}
    fields = [("pos", "grad_pos"), ("radius", "grad_radius"), ("opacity", "grad_opacity"),
              ("payload", "grad_payload"), ("bg", "grad_bg")]
    for field, gname in fields:
        base = getattr(scene, field)
        if base is None:
            out[gname] = None
            continue
        g = np.zeros_like(base)
        for idx in np.ndindex(base.shape):
            if which is not None and not which(gname, idx):
                continue
            x = base[idx]
            h = rel_h * max(1.0, abs(x))
            sp, sm = copy.deepcopy(scene), copy.deepcopy(scene)
            getattr(sp, field)[idx] = x + h
            getattr(sm, field)[idx] = x - h
            g[idx] = (loss(sp, cam, params, G, rows) - loss(sm, cam, params, G, rows)) / (2 * h)
        out[gname] = g
    return out


def fd_camera_grads(scene, cam, params, G, rel_h=1e-6, rows=None) -> np.ndarray:
    """Central finite differences of sum(G * F) for the 14 camera values
    [R (3x3 row-major, perturbed entry by entry as a free matrix), t, focal,
    sensor_width]."""
    out = np.zeros(14)
    for k in range(14):
        cp, cm = copy.deepcopy(cam), copy.deepcopy(cam)
        if k < 9:
            x = float(np.asarray(cam.R, np.float64).reshape(9)[k])
        elif k < 12:
            x = float(np.asarray(cam.t, np.float64)[k - 9])
        else:
            x = float(cam.focal if k == 12 else cam.sensor_width)
        h = rel_h * max(1.0, abs(x))
        for c, v in ((cp, x + h), (cm, x - h)):
            if k < 9:
                R = np.array(c.R, np.float64).reshape(9)
                R[k] = v
                c.R = R.reshape(3, 3)
            elif k < 12:
                t = np.array(c.t, np.float64)
                t[k - 9] = v
                c.t = t
            elif k == 12:
                c.focal = v
            else:
                c.sensor_width = v
        out[k] = (loss(scene, cp, params, G, rows) - loss(scene, cm, params, G, rows)) / (2 * h)
    return out
