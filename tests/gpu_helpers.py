"""Run workloads through the HIP renderer (C ABI) and compare with the oracle."""
from __future__ import annotations

import numpy as np

from paper_2004_07484_amd import _capi

IMAGE_REL = 1e-4   # |d| <= 1e-4 max(|ref|, 1e-2 max|ref|)
GRAD_REL = 1e-3    # |d| <= 1e-3 max(|ref|, 1e-2 max|ref|)
FLOOR = 1e-2


def cam_struct(cam):
    return _capi.make_camera(np.asarray(cam.R, np.float32).reshape(9),
                             np.asarray(cam.t, np.float32).reshape(3), cam.focal,
                             cam.sensor_width, cam.znear, cam.zfar, cam.width, cam.height)


def to_dev(a):
    import torch
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to("cuda:0")


def gpu_render(scene, cam, params, G=None, max_pairs=0, depth_bits=0, need=None,
               stream=None):
    """Forward (and backward when G is given) on cuda:0; numpy results."""
    import torch
    cs = cam_struct(cam)
    ps = _capi.make_params(params.gamma, params.eps, params.min_radius_px, params.K,
                           max_pairs, depth_bits)
    n, C = scene.payload.shape
    pos, rad, opa = to_dev(scene.pos), to_dev(scene.radius), to_dev(scene.opacity)
    pay, bg = to_dev(scene.payload), to_dev(scene.bg)
    ws = torch.empty(_capi.pulsar_workspace_size(n, cam.width, cam.height, C, ps),
                     dtype=torch.uint8, device="cuda:0")
    image = torch.empty((cam.height, cam.width, C), device="cuda:0")
    aux = torch.empty((cam.height, cam.width), device="cuda:0")
    _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux, ws, stream)
    code, pairs = _capi.pulsar_query_status(ws, stream)
    out = dict(F=image.cpu().numpy(), L=aux.cpu().numpy(), status=code, pairs=pairs)
    if G is not None and code == _capi.PULSAR_OK:
        need = need or {"pos", "radius", "opacity", "payload", "bg"}

        def buf(name, shape):
            return torch.full(shape, float("nan"), device="cuda:0") if name in need else None

        gp, gr = buf("pos", (n, 3)), buf("radius", (n,))
        go = buf("opacity", (n,)) if opa is not None else None
        gf, gb = buf("payload", (n, C)), buf("bg", (C,))
        _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, ps, image, aux, to_dev(G), gp, gr, go, gf,
                         gb, ws, stream)
        torch.cuda.synchronize()
        for key, t in [("grad_pos", gp), ("grad_radius", gr), ("grad_opacity", go),
                       ("grad_payload", gf), ("grad_bg", gb)]:
            out[key] = None if t is None else t.cpu().numpy()
    return out


def close_mask(got, ref, rel, floor=FLOOR):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max() if ref.size else 0.0
    tol = rel * np.maximum(np.abs(ref), floor * scale)
    return np.abs(got - ref) <= tol


def assert_close(got, ref, rel, what, floor=FLOOR):
    ok = close_mask(got, ref, rel, floor)
    if not ok.all():
        got = np.asarray(got, np.float64)
        ref = np.asarray(ref, np.float64)
        idx = np.argwhere(~ok)[:5]
        scale = np.abs(ref).max()
        worst = (np.abs(got - ref) / np.maximum(np.abs(ref), floor * scale))[~ok].max()
        raise AssertionError(f"{what}: {int((~ok).sum())} of {ok.size} elements outside "
                             f"{rel} (worst {worst:.3g}); first at {idx.tolist()}: "
                             f"got {got[tuple(idx[0])]} ref {ref[tuple(idx[0])]}")


def masked_G(G, rows, ambiguous):
    """Upstream gradient restricted to the evaluated rows and the pixels whose
    K nearest hits are not sensitive to rounding."""
    Gm = np.zeros_like(G)
    if rows is None:
        Gm[:] = G
    else:
        Gm[rows] = G[rows]
    Gm[ambiguous] = 0.0
    return Gm


def compare_grads(gpu, ref, what=""):
    for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
        if ref.get(key) is None or gpu.get(key) is None:
            continue
        assert_close(gpu[key], ref[key], GRAD_REL, f"{what} {key}")
