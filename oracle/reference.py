"""ctypes binding of the FP64 oracle (oracle/pulsar_oracle.c).

Test infrastructure: the tests, the smoke check and the benchmark's CPU
baseline call it; the renderer never does. Inputs are any objects with the
attributes of a scene (pos, radius, opacity, payload, bg), a camera
(R, t, focal, sensor_width, znear, zfar, width, height) and render parameters
(gamma, eps, min_radius_px, K). All arithmetic happens in float64 in C.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)

AMBIGUITY_REL = 1e-5


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.oracle_forward.restype = ctypes.c_int
        lib.oracle_forward.argtypes = [
            ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
            ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            ctypes.c_double, ctypes.c_int, _ip, _dp, _dp, _ip, _dp, _ip, _dp, _u8p,
            ctypes.c_int, ctypes.c_int, ctypes.c_double]
        lib.oracle_backward.restype = ctypes.c_int
        lib.oracle_backward.argtypes = [
            ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
            ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            ctypes.c_int, _ip, _dp, _dp, _dp, _ip, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.oracle_pixel_hits.restype = ctypes.c_int
        lib.oracle_pixel_hits.argtypes = [
            ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
            ctypes.c_int, ctypes.c_int, _u8p, _dp, _dp, _dp, _dp, _dp, _dp]
        _lib = lib
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a, typ=_dp):
    return None if a is None else a.ctypes.data_as(typ)


def camera_vector(cam) -> np.ndarray:
    return _d(np.concatenate([np.asarray(cam.R, np.float64).reshape(9),
                              np.asarray(cam.t, np.float64).reshape(3),
                              [cam.focal, cam.sensor_width, cam.znear, cam.zfar,
                               1.0 if getattr(cam, "orthographic", False) else 0.0]]))


def _rows(rows: Optional[Sequence[int]], H: int):
    if rows is None:
        return 0, None
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int32))
    if r.size and (r.min() < 0 or r.max() >= H):
        raise ValueError("row index out of range")
    return int(r.size), r


def forward(scene, cam, params, rows: Optional[Sequence[int]] = None,
            n_threads: int = 0, blend_topk: bool = False) -> dict:
    """F [H,W,C], L [H,W], nhits, klist_t/klist_id [H,W,K], t_next, ambiguous.
    blend_topk: blend only each pixel's K nearest hits (the other reading of
    the role of K; the backward formulas are then its exact derivative).
    params.stop_share (default 0): the early stop of Sec. 3.2 / App. B with
    that share threshold (the oracle C file states the rule); nhits and the
    K nearest then count the blended hits only.

    Rows that are not listed hold NaN in F and L and -1 in nhits.
    """
    lib = _load()
    pos, rad = _d(scene.pos), _d(scene.radius)
    opa = None if scene.opacity is None else _d(scene.opacity)
    pay, bg = _d(scene.payload), _d(scene.bg)
    n, C = int(pos.shape[0]), int(pay.shape[1])
    W, H, K = int(cam.width), int(cam.height), int(params.K)
    nr, r = _rows(rows, H)
    F = np.full((H, W, C), np.nan)
    L = np.full((H, W), np.nan)
    nh = np.full((H, W), -1, np.int32)
    kt = np.full((H, W, K), np.inf)
    kid = np.full((H, W, K), -1, np.int32)
    tn = np.full((H, W), np.inf)
    amb = np.zeros((H, W), np.uint8)
    rc = lib.oracle_forward(n, C, _ptr(pos), _ptr(rad), _ptr(opa), _ptr(pay), _ptr(bg),
                            _ptr(camera_vector(cam)), W, H, float(params.gamma),
                            float(params.eps), float(params.min_radius_px), K,
                            AMBIGUITY_REL, nr, _ptr(r, _ip), _ptr(F), _ptr(L), _ptr(nh, _ip),
                            _ptr(kt), _ptr(kid, _ip), _ptr(tn), _ptr(amb, _u8p),
                            int(n_threads), int(bool(blend_topk)),
                            float(getattr(params, "stop_share", 0.0)))
    if rc != 0:
        raise ValueError(f"oracle_forward failed with code {rc}")
    return dict(F=F, L=L, nhits=nh, klist_t=kt, klist_id=kid, t_next=tn,
                ambiguous=amb.astype(bool))


def backward(scene, cam, params, G, fwd: dict, rows: Optional[Sequence[int]] = None) -> dict:
    """Gradients of sum(G * F) for the scene parameters, the background and
    the camera: grad_camera = [dR (3x3 row-major), dt (3), df, ds], with
    grad_camera_abs the sum of |term| behind each value and grad_camera_sphere
    [n, 14] the part of grad_camera that comes from each sphere."""
    lib = _load()
    pos, rad = _d(scene.pos), _d(scene.radius)
    opa = None if scene.opacity is None else _d(scene.opacity)
    pay, bg = _d(scene.payload), _d(scene.bg)
    n, C = int(pos.shape[0]), int(pay.shape[1])
    W, H, K = int(cam.width), int(cam.height), int(params.K)
    nr, r = _rows(rows, H)
    G = _d(G)
    assert G.shape == (H, W, C)
    gp = np.zeros((n, 3))
    gr = np.zeros(n)
    go = np.zeros(n) if opa is not None else None
    gf = np.zeros((n, C))
    gb = np.zeros(C)
    gcam = np.zeros(14)
    gabs = np.zeros(14)
    gsph = np.zeros((n, 14))
    F = _d(np.nan_to_num(fwd["F"]))
    L = _d(np.nan_to_num(fwd["L"]))
    kid = np.ascontiguousarray(fwd["klist_id"].astype(np.int32))
    rc = lib.oracle_backward(n, C, _ptr(pos), _ptr(rad), _ptr(opa), _ptr(pay), _ptr(bg),
                             _ptr(camera_vector(cam)), W, H, float(params.gamma),
                             float(params.eps), float(params.min_radius_px), K, nr,
                             _ptr(r, _ip), _ptr(G), _ptr(F), _ptr(L), _ptr(kid, _ip),
                             _ptr(gp), _ptr(gr), _ptr(go), _ptr(gf), _ptr(gb), _ptr(gcam),
                             _ptr(gabs), _ptr(gsph))
    if rc != 0:
        raise ValueError(f"oracle_backward failed with code {rc}")
    return dict(grad_pos=gp, grad_radius=gr, grad_opacity=go, grad_payload=gf, grad_bg=gb,
                grad_camera=gcam, grad_camera_abs=gabs, grad_camera_sphere=gsph)


def paper_normalised(scene, cam, params, fwd: dict, grads: dict,
                     rows: Optional[Sequence[int]] = None) -> dict:
    """The paper's gradients for optimisation, from the exact ones: every
    gradient of sphere k (position, radius, opacity, payload) divided by the
    number of pixels whose K nearest hits include k (App. B, normalisation),
    and no position or radius gradient for a sphere whose projected radius
    R f / (c_z pitch) is at most 3 pixels (Sec. 3.2; Sec. 7, limitation 1),
    R the effective radius (App. B, Step 0). Camera gradients are normalised
    by each sphere's image area (App. B, normalisation of the camera
    gradients; reading: the part of the camera gradient that comes from
    sphere k, grads["grad_camera_sphere"][k], is scaled by 1e-3 / A_k with A_k
    = pi (R f / (c_z pitch))^2 its projected disk area in pixels, then the
    parts are added). The background gradient is returned unchanged. Counts
    run over the evaluated rows."""
    K = int(params.K)
    kid = np.asarray(fwd["klist_id"])
    H = kid.shape[0]
    sel = range(H) if rows is None else rows
    n = int(np.asarray(scene.pos).shape[0])
    count = np.zeros(n)
    for i in sel:
        ids = kid[i].reshape(-1, K)
        ids = ids[ids >= 0]
        np.add.at(count, ids, 1.0)
    pos = np.asarray(scene.pos, np.float64)
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    cz = pos @ R[2] + float(np.asarray(cam.t, np.float64)[2])
    pitch = float(cam.sensor_width) / float(cam.width)
    r = np.asarray(scene.radius, np.float64)
    ortho = bool(getattr(cam, "orthographic", False))
    # projected radius in pixels: R f / (c_z pitch), or R / pitch for the
    # orthographic projection (where the minimum size is min_radius_px pixels)
    rmin = float(params.min_radius_px) * pitch * (1.0 if ortho else cz / float(cam.focal))
    reff = np.maximum(r, rmin) if params.min_radius_px > 0 else r
    rpx = reff / pitch if ortho else reff * float(cam.focal) / (cz * pitch)
    gated = ~(rpx > 3.0)
    scale = np.where(count > 0, 1.0 / np.maximum(count, 1.0), 1.0)
    out = dict(grads)
    out["grad_pos"] = grads["grad_pos"] * (scale * ~gated)[:, None]
    out["grad_radius"] = grads["grad_radius"] * scale * ~gated
    if grads.get("grad_opacity") is not None:
        out["grad_opacity"] = grads["grad_opacity"] * scale
    out["grad_payload"] = grads["grad_payload"] * scale[:, None]
    if grads.get("grad_camera_sphere") is not None:
        area = np.pi * rpx * rpx
        out["grad_camera"] = (grads["grad_camera_sphere"] * (1e-3 / area)[:, None]).sum(0)
        out["grad_camera_abs"] = np.abs(grads["grad_camera_sphere"] *
                                        (1e-3 / area)[:, None]).sum(0)
    out["pixel_count"] = count
    out["projected_radius_px"] = rpx
    return out


def pixel_hits(scene, cam, params, i: int, j: int) -> dict:
    """Per-sphere ray test of pixel (i, j): hit, t, q, b, camera-space centre, radius, ray."""
    lib = _load()
    pos, rad = _d(scene.pos), _d(scene.radius)
    opa = None if scene.opacity is None else _d(scene.opacity)
    n = int(pos.shape[0])
    hit = np.zeros(n, np.uint8)
    t, q, b = np.zeros(n), np.zeros(n), np.zeros(n)
    c = np.zeros((n, 3))
    reff = np.zeros(n)
    u = np.zeros(3)
    rc = lib.oracle_pixel_hits(n, _ptr(pos), _ptr(rad), _ptr(opa), _ptr(camera_vector(cam)),
                               int(cam.width), int(cam.height), float(params.min_radius_px),
                               int(i), int(j), _ptr(hit, _u8p), _ptr(t), _ptr(q), _ptr(b),
                               _ptr(c), _ptr(reff), _ptr(u))
    if rc != 0:
        raise ValueError(f"oracle_pixel_hits failed with code {rc}")
    return dict(hit=hit.astype(bool), t=t, q=q, b=b, c=c, reff=reff, u=u)


def ambiguity_mask(fwd: dict) -> np.ndarray:
    return fwd["ambiguous"]
