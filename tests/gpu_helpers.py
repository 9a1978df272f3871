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
               stream=None, chunk=0, raster_blocks=0, fwd_flags=0, bwd_flags=0,
               workspace=None, bwd_workspace=None, camera_grad=False):
    """Forward (and backward when G is given) on cuda:0; numpy results.
    workspace: a device byte tensor to use instead of a new one. bwd_workspace,
    when given, is called with the forward's workspace and returns the one the
    backward runs on."""
    import torch
    cs = cam_struct(cam)
    share = float(getattr(params, "stop_share", 0.0))
    ps = _capi.make_params(params.gamma, params.eps, params.min_radius_px, params.K,
                           max_pairs, depth_bits, chunk, raster_blocks, fwd_flags, share)
    pb = _capi.make_params(params.gamma, params.eps, params.min_radius_px, params.K,
                           max_pairs, depth_bits, chunk, raster_blocks, bwd_flags, share)
    n, C = scene.payload.shape
    pos, rad, opa = to_dev(scene.pos), to_dev(scene.radius), to_dev(scene.opacity)
    pay, bg = to_dev(scene.payload), to_dev(scene.bg)
    ws = workspace if workspace is not None else torch.empty(
        _capi.pulsar_workspace_size(n, cam.width, cam.height, C, ps), dtype=torch.uint8,
        device="cuda:0")
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
        wsb = ws if bwd_workspace is None else bwd_workspace(ws)
        if camera_grad:
            gcam = torch.full((14,), float("nan"), device="cuda:0")
            _capi.pulsar_bwd_camera(pos, rad, opa, pay, bg, cs, pb, image, aux, to_dev(G), gp, gr,
                                    go, gf, gb, gcam, wsb, stream)
            torch.cuda.synchronize()
            out["grad_camera"] = gcam.cpu().numpy()
        else:
            _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, pb, image, aux, to_dev(G), gp, gr, go,
                             gf, gb, wsb, stream)
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


def gpu_render_batch(workloads, params, Gs=None, depth_bits=0, chunk=0, raster_blocks=0,
                     bgs=None, stream=None, flags=0):
    """One batched forward (and backward when Gs is given) over several
    workloads sharing C and params; returns one result dict per scene."""
    import torch
    B = len(workloads)
    C = workloads[0].scene.payload.shape[1]
    ps = _capi.make_params(params.gamma, params.eps, params.min_radius_px, params.K, 0,
                           depth_bits, chunk, raster_blocks, flags,
                           float(getattr(params, "stop_share", 0.0)))
    scenes = _capi.make_scenes([cam_struct(w.camera) for w in workloads],
                               [w.scene.n for w in workloads])
    cat = lambda xs, shape: np.concatenate([np.asarray(x, np.float32).reshape(shape) for x in xs])
    pos = to_dev(cat([w.scene.pos for w in workloads], (-1, 3)))
    rad = to_dev(cat([w.scene.radius for w in workloads], (-1,)))
    opa = to_dev(cat([w.scene.opacity for w in workloads], (-1,)))
    pay = to_dev(cat([w.scene.payload for w in workloads], (-1, C)))
    bg = to_dev(np.stack([w.scene.bg if bgs is None else bgs[b]
                          for b, w in enumerate(workloads)]).astype(np.float32))
    N, P = _capi.batch_sizes(scenes)
    ws = torch.empty(_capi.pulsar_batch_workspace_size(scenes, C, ps), dtype=torch.uint8,
                     device="cuda:0")
    image = torch.empty((P, C), device="cuda:0")
    aux = torch.empty((P,), device="cuda:0")
    _capi.pulsar_fwd_batched(scenes, pos, rad, opa, pay, bg, ps, image, aux, ws, stream)
    code, pairs = _capi.pulsar_query_status(ws, stream)
    F, L = image.cpu().numpy(), aux.cpu().numpy()
    outs, p0, n0 = [], 0, 0
    for w in workloads:
        H, W, n = w.camera.height, w.camera.width, w.scene.n
        outs.append(dict(F=F[p0:p0 + H * W].reshape(H, W, C), L=L[p0:p0 + H * W].reshape(H, W),
                         status=code, pairs=pairs, sl=(p0, n0)))
        p0 += H * W
        n0 += n
    if Gs is not None and code == _capi.PULSAR_OK:
        G = to_dev(np.concatenate([np.asarray(g, np.float32).reshape(-1, C) for g in Gs]))
        gp = torch.full((N, 3), float("nan"), device="cuda:0")
        gr = torch.full((N,), float("nan"), device="cuda:0")
        go = torch.full((N,), float("nan"), device="cuda:0")
        gf = torch.full((N, C), float("nan"), device="cuda:0")
        gb = torch.full((B, C), float("nan"), device="cuda:0")
        _capi.pulsar_bwd_batched(scenes, pos, rad, opa, pay, bg, ps, image, aux, G, gp, gr, go,
                                 gf, gb, ws, stream)
        torch.cuda.synchronize()
        gp, gr, go, gf, gb = (t.cpu().numpy() for t in (gp, gr, go, gf, gb))
        for b, (w, o) in enumerate(zip(workloads, outs)):
            n0, n = o["sl"][1], w.scene.n
            o.update(grad_pos=gp[n0:n0 + n], grad_radius=gr[n0:n0 + n],
                     grad_opacity=go[n0:n0 + n], grad_payload=gf[n0:n0 + n], grad_bg=gb[b])
    return outs


# Camera gradients are sums over every hit of terms of both signs (the
# derivative of the image with respect to the camera, Sec. 3.1, adds each
# hit's dL/dc p^T, dL/dc and dL/dkappa): a value can cancel to far below its
# terms, so its scale is the larger of |ref| and this fraction of the sum of
# the absolute values of its terms.
CAMERA_FLOOR = 1e-4


def assert_camera_close(got, ref, ref_abs, what, rel=GRAD_REL):
    """|got - ref| <= rel max(|ref|, CAMERA_FLOOR sum of |terms|), per value."""
    got = np.asarray(got, np.float64)
    scale = np.maximum(np.abs(ref), CAMERA_FLOOR * np.asarray(ref_abs, np.float64))
    err = np.abs(got - ref) / np.maximum(scale, 1e-300)
    assert np.all(err <= rel), f"{what}: worst {err.max():.3g} at {int(err.argmax())}: " \
        f"got {got.tolist()} ref {np.asarray(ref).tolist()}"
