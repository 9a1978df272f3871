"""PyTorch front end: torch.autograd.Function and a Renderer module (paper Sec. 4, Lst. 1).

PyTorch only provides device memory, the stream and autograd bookkeeping;
every step of the rendering pass runs in the HIP kernels of libpulsar.so.
The backward recomputes per-pixel hits from the workspace the forward filled
(nothing per pixel is stored beyond the image and its log-normaliser).

Pair capacity: a forward whose (tile, sphere) pairs exceed the capacity has
invalid outputs. check_capacity="sync" waits for every forward and re-renders
with a larger capacity; "lazy" (the default) never waits: the device status
is copied to pinned host memory behind the forward and read once it has
landed (by the backward, by the next call of the same Renderer, or by
Renderer.check_status()), so a render step can be captured in a graph.
"""
from __future__ import annotations

import math
import warnings
from typing import Optional

import torch

from . import _capi


def axis_angle_to_matrix(r) -> list:
    """Rodrigues' formula on the host; returns a row-major 3x3 list."""
    rx, ry, rz = (float(v) for v in r)
    th = math.sqrt(rx * rx + ry * ry + rz * rz)
    if th < 1e-12:
        return [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0]
    kx, ky, kz = rx / th, ry / th, rz / th
    c, s, v = math.cos(th), math.sin(th), 1.0 - math.cos(th)
    return [c + kx * kx * v, kx * ky * v - kz * s, kx * kz * v + ky * s,
            ky * kx * v + kz * s, c + ky * ky * v, ky * kz * v - kx * s,
            kz * kx * v - ky * s, kz * ky * v + kx * s, c + kz * kz * v]


def axis_angle_to_matrix_torch(r: torch.Tensor) -> torch.Tensor:
    """Rodrigues' formula as differentiable torch operations: [3] -> [3, 3]
    (R = I + sin(th) K + (1 - cos(th)) K^2, K the cross-product matrix of the
    unit axis; first order at th = 0 so the derivative there is exact)."""
    r = r.reshape(3)
    th2 = (r * r).sum()
    zero = torch.zeros((), dtype=r.dtype, device=r.device)

    def skew(k):
        return torch.stack([torch.stack([zero, -k[2], k[1]]),
                            torch.stack([k[2], zero, -k[0]]),
                            torch.stack([-k[1], k[0], zero])])

    eye = torch.eye(3, dtype=r.dtype, device=r.device)
    if float(th2.detach()) < 1e-20:
        return eye + skew(r)
    th = torch.sqrt(th2)
    K = skew(r / th)
    return eye + torch.sin(th) * K + (1.0 - torch.cos(th)) * (K @ K)


def rotation_6d_to_matrix(r6) -> list:
    """The continuous 6D rotation parametrisation (Zhou et al., cited in
    Sec. 4 for the camera vector): two 3-vectors a1, a2 are made orthonormal by
    Gram-Schmidt, b1 = a1 / |a1|, b2 = (a2 - (b1 . a2) b1) / |.|, b3 = b1 x b2,
    and R = [b1 b2 b3] by columns. On the host; returns a row-major 3x3 list."""
    a1 = [float(v) for v in r6[0:3]]
    a2 = [float(v) for v in r6[3:6]]
    n1 = math.sqrt(sum(v * v for v in a1))
    b1 = [v / n1 for v in a1]
    d = sum(x * y for x, y in zip(b1, a2))
    u = [y - d * x for x, y in zip(b1, a2)]
    n2 = math.sqrt(sum(v * v for v in u))
    b2 = [v / n2 for v in u]
    b3 = [b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2],
          b1[0] * b2[1] - b1[1] * b2[0]]
    return [b1[0], b2[0], b3[0], b1[1], b2[1], b3[1], b1[2], b2[2], b3[2]]


def rotation_6d_to_matrix_torch(r6: torch.Tensor) -> torch.Tensor:
    """rotation_6d_to_matrix as differentiable torch operations: [6] -> [3, 3]."""
    r6 = r6.reshape(6)
    a1, a2 = r6[0:3], r6[3:6]
    b1 = a1 / torch.linalg.vector_norm(a1)
    u = a2 - (b1 * a2).sum() * b1
    b2 = u / torch.linalg.vector_norm(u)
    b3 = torch.linalg.cross(b1, b2)
    return torch.stack([b1, b2, b3], dim=1)


def camera_struct(cam, width: int, height: int, znear: float, zfar: float):
    """Accepts a pulsar_camera_t, an object with R, t, focal, sensor_width
    (znear/zfar/width/height optional), the 8-vector [t (3), axis-angle (3),
    focal, sensor_width] of Lst. 1, read as x_cam = R(axis-angle) x_world + t,
    or the 11-vector [t (3), 6D rotation (6), focal, sensor_width] (Sec. 4)."""
    if isinstance(cam, _capi.pulsar_camera_t):
        return cam
    if hasattr(cam, "R"):
        return _capi.make_camera(cam.R, cam.t, cam.focal, cam.sensor_width,
                                 getattr(cam, "znear", znear), getattr(cam, "zfar", zfar),
                                 getattr(cam, "width", width), getattr(cam, "height", height))
    v = cam.detach().cpu().reshape(-1).tolist() if hasattr(cam, "detach") else list(cam)
    if len(v) == 8:
        return _capi.make_camera(axis_angle_to_matrix(v[3:6]), v[0:3], v[6], v[7], znear, zfar,
                                 width, height)
    if len(v) == 11:
        return _capi.make_camera(rotation_6d_to_matrix(v[3:9]), v[0:3], v[9], v[10], znear,
                                 zfar, width, height)
    raise ValueError("camera vector must be [t(3), axis-angle(3), focal, sensor_width] or "
                     "[t(3), 6D rotation(6), focal, sensor_width]")


class StatusProbe:
    """A forward's device status (the first PULSAR_STATUS_BYTES bytes of its
    workspace) copied into pinned host memory behind the forward's kernels on
    the current stream, so nothing waits for it; read once it has landed."""

    def __init__(self, ws: torch.Tensor, what: str):
        self.what = what
        self.host = torch.empty(_capi.PULSAR_STATUS_BYTES, dtype=torch.uint8, pin_memory=True)
        self.host.copy_(ws[:_capi.PULSAR_STATUS_BYTES], non_blocking=True)
        self.done = torch.cuda.Event()
        self.done.record(torch.cuda.current_stream(ws.device))

    def result(self, wait: bool = False):
        """(code, pairs), or None while the copy is still in flight (wait=False)."""
        if not wait and not self.done.query():
            return None
        self.done.synchronize()
        return _capi.decode_status(self.host.numpy().tobytes())


def _capturing() -> bool:
    return torch.cuda.is_available() and torch.cuda.is_current_stream_capturing()


def _forward_into(pos, radius, opacity, payload, bg, cam, params, check: bool):
    """Run pulsar_fwd into fresh outputs; grow the pair capacity and re-run
    if the device reports an overflow (only when check is set)."""
    n, C = payload.shape
    dev = payload.device
    image = torch.empty((cam.height, cam.width, C), device=dev, dtype=torch.float32)
    aux = torch.empty((cam.height, cam.width), device=dev, dtype=torch.float32)
    while True:
        ws = torch.empty(_capi.pulsar_workspace_size(n, cam.width, cam.height, C, params),
                         device=dev, dtype=torch.uint8)
        _capi.pulsar_fwd(pos, radius, opacity, payload, bg, cam, params, image, aux, ws)
        if not check:
            return image, aux, ws, params
        code, pairs = _capi.pulsar_query_status(ws)
        if code == _capi.PULSAR_OK:
            return image, aux, ws, params
        # never below twice the capacity that overflowed
        want = max(pairs * 5 // 4 + 1024, 2 * int(params.max_pairs))
        grown = _capi.make_params(params.gamma, params.eps, params.min_radius_px, params.K,
                                  int(min(2**31 - 1, want)), params.depth_bits,
                                  params.chunk, params.raster_blocks, params.flags)
        if grown.max_pairs <= params.max_pairs:
            raise _capi.PulsarError(code, "pulsar_fwd")
        params = grown


def _raise_if_overflowed(probe) -> None:
    """A backward whose forward overflowed the pair capacity has nothing
    valid to differentiate; checked only if the status has already landed."""
    if probe is None:
        return
    res = probe.result(wait=False)
    if res is not None and res[0] != _capi.PULSAR_OK:
        raise _capi.PulsarError(res[0], f"{probe.what} ({res[1]} tile pairs; raise max_pairs)")


class PulsarFunction(torch.autograd.Function):
    """F = R(S, camera) with the hand-written backward of libpulsar.so."""

    @staticmethod
    def forward(ctx, pos, radius, opacity, payload, bg, cam, params, check="lazy", cam_R=None,
                cam_t=None, cam_f=None, cam_s=None, probes=None):
        """cam is the pulsar_camera_t the kernels use; cam_R [3,3], cam_t [3],
        cam_f, cam_s, when given, are tensors holding the same values, and
        receive dLoss/dR (R as a free matrix), dLoss/dt, dLoss/dfocal and
        dLoss/dsensor_width. check: "sync", "lazy" (a StatusProbe, appended
        to the list `probes` when one is given) or False."""
        pos, radius, payload, bg = (t.contiguous() for t in (pos, radius, payload, bg))
        opacity = opacity.contiguous() if opacity is not None else None
        sync = check in (True, "sync") and not _capturing()
        image, aux, ws, params = _forward_into(pos, radius, opacity, payload, bg, cam, params,
                                               sync)
        ctx.probe = None
        if check == "lazy" and not _capturing():
            ctx.probe = StatusProbe(ws, "pulsar_fwd")
            if isinstance(probes, list):
                probes.append(ctx.probe)
        ctx.save_for_backward(pos, radius, opacity, payload, bg, image, aux, ws)
        ctx.cam, ctx.params = cam, params
        ctx.cam_shapes = [None if x is None else x.shape for x in (cam_R, cam_t, cam_f, cam_s)]
        ctx.mark_non_differentiable(aux)
        return image, aux

    @staticmethod
    def backward(ctx, grad_image, grad_aux):
        pos, radius, opacity, payload, bg, image, aux, ws = ctx.saved_tensors
        _raise_if_overflowed(ctx.probe)
        need = ctx.needs_input_grad
        n, C = payload.shape

        def out(flag, shape):
            return torch.empty(shape, device=payload.device, dtype=torch.float32) if flag \
                else None

        gp, gr = out(need[0], (n, 3)), out(need[1], (n,))
        go = out(need[2] and opacity is not None, (n,))
        gf, gb = out(need[3], (n, C)), out(need[4], (C,))
        if grad_image is None:
            grad_image = torch.zeros_like(image)
        cam_grads = [None] * 4
        if any(need[8:12]):
            gcam = torch.empty(14, device=payload.device, dtype=torch.float32)
            _capi.pulsar_bwd_camera(pos, radius, opacity, payload, bg, ctx.cam, ctx.params,
                                    image, aux, grad_image.contiguous(), gp, gr, go, gf, gb,
                                    gcam, ws)
            parts = (gcam[0:9], gcam[9:12], gcam[12], gcam[13])
            for k in range(4):
                if need[8 + k]:
                    cam_grads[k] = parts[k].reshape(ctx.cam_shapes[k])
        else:
            _capi.pulsar_bwd(pos, radius, opacity, payload, bg, ctx.cam, ctx.params, image, aux,
                             grad_image.contiguous(), gp, gr, go, gf, gb, ws)
        return (gp, gr, go, gf, gb, None, None, None, *cam_grads, None)


class PulsarBatchFunction(torch.autograd.Function):
    """Batched F = R(S_b, camera_b) for b = 1..B in one call (packed layout of
    pulsar_fwd_batched), with the batched hand-written backward."""

    @staticmethod
    def forward(ctx, pos, radius, opacity, payload, bg, scenes, params, check="lazy"):
        pos, radius, payload, bg = (t.contiguous() for t in (pos, radius, payload, bg))
        opacity = opacity.contiguous() if opacity is not None else None
        N, P = _capi.batch_sizes(scenes)
        C = payload.shape[1]
        dev = payload.device
        image = torch.empty((P, C), device=dev, dtype=torch.float32)
        aux = torch.empty((P,), device=dev, dtype=torch.float32)
        ws = torch.empty(_capi.pulsar_batch_workspace_size(scenes, C, params), device=dev,
                         dtype=torch.uint8)
        _capi.pulsar_fwd_batched(scenes, pos, radius, opacity, payload, bg, params, image, aux,
                                 ws)
        ctx.probe = None
        if check in (True, "sync") and not _capturing():
            code, _ = _capi.pulsar_query_status(ws)
            if code != _capi.PULSAR_OK:
                raise _capi.PulsarError(code, "pulsar_fwd_batched")
        elif check == "lazy" and not _capturing():
            ctx.probe = StatusProbe(ws, "pulsar_fwd_batched")
        ctx.save_for_backward(pos, radius, opacity, payload, bg, image, aux, ws)
        ctx.scenes, ctx.params = scenes, params
        ctx.mark_non_differentiable(aux)
        return image, aux

    @staticmethod
    def backward(ctx, grad_image, grad_aux):
        pos, radius, opacity, payload, bg, image, aux, ws = ctx.saved_tensors
        _raise_if_overflowed(ctx.probe)
        need = ctx.needs_input_grad
        N, C = payload.shape
        B = bg.shape[0]

        def out(flag, shape):
            return torch.empty(shape, device=payload.device, dtype=torch.float32) if flag \
                else None

        gp, gr = out(need[0], (N, 3)), out(need[1], (N,))
        go = out(need[2] and opacity is not None, (N,))
        gf, gb = out(need[3], (N, C)), out(need[4], (B, C))
        if grad_image is None:
            grad_image = torch.zeros_like(image)
        _capi.pulsar_bwd_batched(ctx.scenes, pos, radius, opacity, payload, bg, ctx.params,
                                 image, aux, grad_image.contiguous(), gp, gr, go, gf, gb, ws)
        return gp, gr, go, gf, gb, None, None, None


def render_batch(cams, counts, pos, radius, payload, opacity=None, bg=None, gamma=0.1,
                 K: int = 5, eps: float = 1e-5, min_radius_px: float = 0.0, widths=None,
                 heights=None, min_depth: float = 1.0, max_depth: float = 10.0,
                 params=None, check_capacity="lazy"):
    """Renders B scenes in one batched call. cams: B cameras (pulsar_camera_t,
    objects with R/t or 8-vectors, the latter two with widths/heights given);
    counts: spheres per scene, the sphere tensors packed in scene order.
    Returns a list of B images [H_b, W_b, C] (views into one packed tensor)."""
    B = len(cams)
    C = payload.shape[1]
    structs = []
    for b, c in enumerate(cams):
        if isinstance(c, _capi.pulsar_camera_t):
            structs.append(c)
        else:
            structs.append(camera_struct(c, int(widths[b]), int(heights[b]), min_depth,
                                         max_depth))
    scenes = _capi.make_scenes(structs, counts)
    if bg is None:
        bg = torch.zeros((B, C), device=payload.device, dtype=torch.float32)
    if params is None:
        params = _capi.make_params(gamma, eps, min_radius_px, K)
    image, _ = PulsarBatchFunction.apply(pos, radius, opacity, payload, bg, scenes, params,
                                         check_capacity)
    out, p0 = [], 0
    for s in structs:
        hw = int(s.width) * int(s.height)
        out.append(image[p0:p0 + hw].view(int(s.height), int(s.width), C))
        p0 += hw
    return out


class Renderer(torch.nn.Module):
    """Lst. 1 style renderer: Renderer(width, height, max_num_spheres)(pos, payload, radius, cam).

    The camera is an 8-vector [t, axis-angle, focal, sensor_width], an
    11-vector [t, 6D rotation, focal, sensor_width] or an object with R, t,
    focal and sensor_width; a vector tensor that requires grad receives
    dLoss/dcamera. ``max_depth`` is the far clip
    zfar and ``min_depth`` the near clip znear of the depth mapping.
    ``min_radius_px=_capi.PULSAR_MIN_RADIUS_PX_PAPER`` draws every sphere at
    least one pixel large, as the paper does.
    """

    def __init__(self, width: int, height: int, max_num_spheres: int, n_channels: int = 3,
                 K: int = 5, max_pairs: int = 0, check_capacity="lazy",
                 autotune: bool = False, tune_cache: Optional[str] = None):
        super().__init__()
        self.width, self.height = int(width), int(height)
        self.max_num_spheres, self.n_channels, self.K = int(max_num_spheres), int(n_channels), \
            int(K)
        self.max_pairs = int(max_pairs)
        if check_capacity is True:
            check_capacity = "sync"
        if check_capacity not in ("sync", "lazy", False):
            raise ValueError('check_capacity must be "sync", "lazy" or False')
        self.check_capacity = check_capacity
        self._probes = []  # status probes of calls not yet checked
        self.autotune = bool(autotune)
        self._tune_cache = None
        self._tune_path = tune_cache
        self._knobs = {}
        _capi.load()

    def check_status(self, wait: bool = True) -> None:
        """Reads the status of earlier lazy-checked calls (waiting for them
        when wait is set). After an overflow the calls from then on use a
        larger pair capacity; the overflowing call's outputs were invalid,
        which a warning reports (or, with wait, an exception)."""
        pending = []
        for pr in self._probes:
            res = pr.result(wait=wait)
            if res is None:
                pending.append(pr)
                continue
            code, pairs = res
            if code != _capi.PULSAR_OK:
                grown = max(pairs * 5 // 4 + 1024, 2 * self.max_pairs)
                self.max_pairs = int(min(2**31 - 1, grown))
                msg = (f"a render produced {pairs} tile pairs, more than its capacity; its "
                       f"outputs were invalid. Later renders use max_pairs={self.max_pairs}.")
                self._probes = pending
                if wait:
                    raise _capi.PulsarError(code, msg)
                warnings.warn(msg, RuntimeWarning, stacklevel=3)
        self._probes = pending[-64:]

    def _tuned(self, params, pos, radius, opacity, payload, bg, cs):
        """Knobs for this workload from the tuning cache, or measured now on
        these inputs (one forward + backward per candidate)."""
        from . import autotune as at
        if self._tune_cache is None:
            self._tune_cache = at.TuneCache(self._tune_path)
        n, C = payload.shape
        key = at.cache_key(at.arch_name(), n, self.width * self.height, C, self.K)
        knobs = self._knobs.get(key)
        if knobs is None:
            with torch.no_grad():
                G = torch.ones((self.height, self.width, C), device=payload.device)
                state = {}

                def run(p):
                    img, aux, ws, _ = _forward_into(pos, radius, opacity, payload, bg, cs, p,
                                                    False)
                    _capi.pulsar_bwd(pos, radius, opacity, payload, bg, cs, p, img, aux, G,
                                     None, None, None, None, None, ws)
                    state["ws"] = ws

                tuned, _ = at.tune(run, params, key=key, cache=self._tune_cache)
            knobs = at.knobs_of(tuned)
            self._knobs[key] = knobs
        return at.with_knobs(params, knobs)

    def forward(self, pos, payload, radius, cam, opacity: Optional[torch.Tensor] = None,
                gamma: float = 0.1, max_depth: float = 10.0, min_depth: float = 1.0,
                bg: Optional[torch.Tensor] = None, eps: float = 1e-5,
                min_radius_px: float = 0.0, return_aux: bool = False,
                orthographic: bool = False, blend_topk: bool = False,
                paper_gradients: bool = False, store_hits: bool = False,
                stop_share: float = 0.0):
        """orthographic: parallel rays along +z (PULSAR_ORTHO; no camera
        gradient). blend_topk: only each pixel's K nearest hits blend
        (PULSAR_BLEND_TOPK). paper_gradients: the paper's gradients for
        optimisation, averaged over each sphere's pixels with the 3-pixel
        position gate (PULSAR_GRAD_PAPER_NORM). store_hits: the forward keeps
        each pixel's K nearest hits for the backward (PULSAR_STORE_HITS).
        stop_share: early ray termination at that share (0 = off)."""
        if pos.shape[0] > self.max_num_spheres:
            raise ValueError("more spheres than the renderer was built for")
        C = payload.shape[1]
        if bg is None:
            bg = torch.zeros(C, device=payload.device, dtype=torch.float32)
        cam_tensors = (None, None, None, None)
        if torch.is_tensor(cam) and cam.requires_grad and torch.is_grad_enabled():
            # the 8-vector [t, axis-angle, focal, sensor_width] as differentiable
            # parts; the kernels get the same values
            v = cam.reshape(-1)
            if v.numel() == 8:
                cam_tensors = (axis_angle_to_matrix_torch(v[3:6]), v[0:3], v[6], v[7])
            elif v.numel() == 11:
                cam_tensors = (rotation_6d_to_matrix_torch(v[3:9]), v[0:3], v[9], v[10])
            else:
                raise ValueError("camera vector must be [t(3), axis-angle(3), focal, "
                                 "sensor_width] or [t(3), 6D rotation(6), focal, sensor_width]")
            Rv = cam_tensors[0].detach().cpu().reshape(9).tolist()
            hv = [float(cam_tensors[k].detach().cpu().reshape(-1)[j]) for k, j in
                  ((1, 0), (1, 1), (1, 2), (2, 0), (3, 0))]
            cs = _capi.make_camera(Rv, hv[0:3], hv[3], hv[4], min_depth, max_depth, self.width,
                                   self.height)
        else:
            cs = camera_struct(cam, self.width, self.height, min_depth, max_depth)
        if self.check_capacity == "lazy" and self._probes and not _capturing():
            self.check_status(wait=False)
        flags = ((_capi.PULSAR_ORTHO if orthographic else 0) |
                 (_capi.PULSAR_BLEND_TOPK if blend_topk else 0) |
                 (_capi.PULSAR_GRAD_PAPER_NORM if paper_gradients else 0) |
                 (_capi.PULSAR_STORE_HITS if store_hits else 0))
        if orthographic and torch.is_tensor(cam) and cam.requires_grad:
            raise ValueError("camera gradients are not available for the orthographic projection")
        params = _capi.make_params(gamma, eps, min_radius_px, self.K, self.max_pairs, flags=flags,
                                   stop_share=stop_share)
        if self.autotune:
            params = self._tuned(params, pos.detach().contiguous(), radius.detach().contiguous(),
                                 None if opacity is None else opacity.detach().contiguous(),
                                 payload.detach().contiguous(), bg.detach().contiguous(), cs)
        if not (torch.is_grad_enabled() and any(
                t is not None and t.requires_grad
                for t in (pos, radius, opacity, payload, bg) + cam_tensors)):
            # no backward can follow: skip keeping its per-pixel state
            params.flags |= _capi.PULSAR_NO_BWD_AUX
        image, aux = PulsarFunction.apply(pos, radius, opacity, payload, bg, cs, params,
                                          self.check_capacity, *cam_tensors, self._probes)
        return (image, aux) if return_aux else image
