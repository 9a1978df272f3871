"""ctypes binding of libpulsar.so: argument marshalling only.

Every entry point of include/pulsar.h is mirrored under the same name. Tensor
arguments must be contiguous float32 CUDA (HIP) tensors; they are passed as
raw device pointers together with the current torch stream. No computation
happens here, and there is no fallback: without the built library every call
raises PulsarLibraryMissing.
"""
from __future__ import annotations

import ctypes
import struct
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpulsar.so")

PULSAR_OK = 0
PULSAR_ERR_INVALID_ARGUMENT = -1
PULSAR_ERR_WORKSPACE = -2
PULSAR_ERR_UNSUPPORTED = -3
PULSAR_ERR_HIP = -4
PULSAR_ERR_CAPACITY = -5
PULSAR_ERR_SCRATCH = -6
PULSAR_NOALLOC_SCRATCH_BYTES = 64 << 20
PULSAR_STATUS_BYTES = 16

EXPORTED = ("pulsar_workspace_size", "pulsar_fwd", "pulsar_bwd", "pulsar_batch_workspace_size",
            "pulsar_fwd_batched", "pulsar_bwd_batched", "pulsar_bwd_camera",
            "pulsar_bwd_camera_batched", "pulsar_query_status",
            "pulsar_status_string", "pulsar_last_hip_error", "pulsar_timing_enable",
            "pulsar_timing_read", "pulsar_stage_name", "pulsar_version", "pulsar_fwd_noalloc",
            "pulsar_fwd_batched_devcam")

PULSAR_NUM_STAGES = 8
PULSAR_NO_BWD_AUX = 0x1   # forward keeps no backward state
PULSAR_REBIN = 0x2        # backward rebuilds its tile lists and thresholds
PULSAR_GRAD_PAPER_NORM = 0x4  # per-pixel averaged gradients, 3-pixel position gate
PULSAR_BLEND_TOPK = 0x8   # blend only each pixel's K nearest hits
PULSAR_ORTHO = 0x10       # orthographic projection
PULSAR_STORE_HITS = 0x20  # forward stores each pixel's K nearest hits for the backward
PULSAR_BWD_TILES = 0x40   # backward always walks the tile lists (per-pair slots)
PULSAR_MIN_RADIUS_PX_PAPER = 0.70710678  # every sphere covers a pixel centre
PULSAR_MAX_SCENES = 4096


class PulsarLibraryMissing(RuntimeError):
    pass


class PulsarError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = f"{where}: {pulsar_status_string(code)} (code {code})"
        if code == PULSAR_ERR_HIP:
            msg += f": {pulsar_last_hip_error()}"
        super().__init__(msg)


class pulsar_camera_t(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("focal", ctypes.c_float),
                ("sensor_width", ctypes.c_float), ("znear", ctypes.c_float),
                ("zfar", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class pulsar_params_t(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_float), ("eps", ctypes.c_float),
                ("min_radius_px", ctypes.c_float), ("K", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("max_pairs", ctypes.c_int32),
                ("depth_bits", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("raster_blocks", ctypes.c_int32), ("stop_share", ctypes.c_float)]


class pulsar_scene_t(ctypes.Structure):
    _fields_ = [("camera", pulsar_camera_t), ("n", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PulsarLibraryMissing(
            f"{LIB_PATH} is not built; run paper_2004_07484_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.pulsar_workspace_size.restype = ctypes.c_size_t
    lib.pulsar_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.POINTER(pulsar_params_t)]
    lib.pulsar_fwd.restype = ctypes.c_int
    lib.pulsar_fwd.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp,
                               ctypes.POINTER(pulsar_camera_t), ctypes.POINTER(pulsar_params_t),
                               _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.pulsar_fwd_noalloc.restype = ctypes.c_int
    lib.pulsar_fwd_noalloc.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp,
                                       ctypes.POINTER(pulsar_camera_t),
                                       ctypes.POINTER(pulsar_params_t), _vp, _vp, _vp]
    lib.pulsar_bwd.restype = ctypes.c_int
    lib.pulsar_bwd.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp,
                               ctypes.POINTER(pulsar_camera_t), ctypes.POINTER(pulsar_params_t),
                               _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.pulsar_batch_workspace_size.restype = ctypes.c_size_t
    lib.pulsar_batch_workspace_size.argtypes = [ctypes.POINTER(pulsar_scene_t), ctypes.c_int32,
                                                ctypes.c_int32, ctypes.POINTER(pulsar_params_t)]
    lib.pulsar_fwd_batched.restype = ctypes.c_int
    lib.pulsar_fwd_batched.argtypes = [ctypes.POINTER(pulsar_scene_t), ctypes.c_int32, _vp, _vp,
                                       _vp, _vp, ctypes.c_int32, _vp,
                                       ctypes.POINTER(pulsar_params_t), _vp, _vp, _vp,
                                       ctypes.c_size_t, _vp]
    lib.pulsar_fwd_batched_devcam.restype = ctypes.c_int
    lib.pulsar_fwd_batched_devcam.argtypes = [ctypes.POINTER(pulsar_scene_t), ctypes.c_int32,
                                              _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp,
                                              ctypes.POINTER(pulsar_params_t), _vp, _vp, _vp,
                                              ctypes.c_size_t, _vp]
    lib.pulsar_bwd_batched.restype = ctypes.c_int
    lib.pulsar_bwd_batched.argtypes = [ctypes.POINTER(pulsar_scene_t), ctypes.c_int32, _vp, _vp,
                                       _vp, _vp, ctypes.c_int32, _vp,
                                       ctypes.POINTER(pulsar_params_t), _vp, _vp, _vp, _vp, _vp,
                                       _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.pulsar_bwd_camera.restype = ctypes.c_int
    lib.pulsar_bwd_camera.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp,
                                      ctypes.POINTER(pulsar_camera_t),
                                      ctypes.POINTER(pulsar_params_t), _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.pulsar_bwd_camera_batched.restype = ctypes.c_int
    lib.pulsar_bwd_camera_batched.argtypes = [ctypes.POINTER(pulsar_scene_t), ctypes.c_int32,
                                              _vp, _vp, _vp, _vp, ctypes.c_int32, _vp,
                                              ctypes.POINTER(pulsar_params_t), _vp, _vp, _vp,
                                              _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                              _vp]
    lib.pulsar_query_status.restype = ctypes.c_int
    lib.pulsar_query_status.argtypes = [_vp, ctypes.c_size_t, _vp,
                                        ctypes.POINTER(ctypes.c_int64)]
    lib.pulsar_status_string.restype = ctypes.c_char_p
    lib.pulsar_status_string.argtypes = [ctypes.c_int]
    lib.pulsar_last_hip_error.restype = ctypes.c_char_p
    lib.pulsar_last_hip_error.argtypes = []
    lib.pulsar_version.restype = ctypes.c_int
    lib.pulsar_version.argtypes = []
    lib.pulsar_timing_enable.restype = ctypes.c_int
    lib.pulsar_timing_enable.argtypes = [ctypes.c_int]
    lib.pulsar_timing_read.restype = ctypes.c_int
    lib.pulsar_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
    lib.pulsar_stage_name.restype = ctypes.c_char_p
    lib.pulsar_stage_name.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def make_camera(R, t, focal, sensor_width, znear, zfar, width, height) -> pulsar_camera_t:
    c = pulsar_camera_t()
    Rf = [float(x) for x in _flat(R)]
    tf = [float(x) for x in _flat(t)]
    if len(Rf) != 9 or len(tf) != 3:
        raise ValueError("R must have 9 entries and t 3")
    c.R[:] = Rf
    c.t[:] = tf
    c.focal, c.sensor_width = float(focal), float(sensor_width)
    c.znear, c.zfar = float(znear), float(zfar)
    c.width, c.height = int(width), int(height)
    return c


def make_params(gamma=0.1, eps=1e-5, min_radius_px=0.0, K=8, max_pairs=0,
                depth_bits=0, chunk=0, raster_blocks=0, flags=0,
                stop_share=0.0) -> pulsar_params_t:
    p = pulsar_params_t()
    p.gamma, p.eps, p.min_radius_px = float(gamma), float(eps), float(min_radius_px)
    p.K, p.flags, p.max_pairs, p.depth_bits = int(K), int(flags), int(max_pairs), \
        int(depth_bits)
    p.chunk, p.raster_blocks, p.stop_share = int(chunk), int(raster_blocks), float(stop_share)
    return p


def make_scenes(cameras, counts):
    """ctypes array of pulsar_scene_t from cameras (pulsar_camera_t) and sphere counts."""
    cameras, counts = list(cameras), [int(c) for c in counts]
    if len(cameras) != len(counts):
        raise ValueError("one sphere count per camera")
    arr = (pulsar_scene_t * len(cameras))()
    for b, (c, n) in enumerate(zip(cameras, counts)):
        arr[b].camera = c
        arr[b].n = n
        arr[b].reserved = 0
    return arr


def batch_sizes(scenes) -> Tuple[int, int]:
    """(total spheres, total pixels) of a scene array."""
    N = sum(int(s.n) for s in scenes)
    P = sum(int(s.camera.width) * int(s.camera.height) for s in scenes)
    return N, P


def _flat(x):
    if hasattr(x, "detach"):
        x = x.detach().cpu().reshape(-1).tolist()
    elif hasattr(x, "reshape"):
        x = x.reshape(-1).tolist()
    return list(x)


def _ptr(t, name: str, required: bool = True, shape: Optional[Tuple[int, ...]] = None):
    if t is None:
        if required:
            raise ValueError(f"{name} is required")
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    import torch
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


# ---------------------------------------------------------------- entry points

def pulsar_version() -> int:
    return load().pulsar_version()


def pulsar_status_string(code: int) -> str:
    return load().pulsar_status_string(int(code)).decode()


def pulsar_last_hip_error() -> str:
    return load().pulsar_last_hip_error().decode()


def pulsar_workspace_size(n: int, width: int, height: int, C: int,
                          params: pulsar_params_t) -> int:
    return int(load().pulsar_workspace_size(int(n), int(width), int(height), int(C),
                                            ctypes.byref(params)))


def pulsar_fwd(pos, radius, opacity, payload, background, cam: pulsar_camera_t,
               params: pulsar_params_t, image, aux, ws, stream=None) -> None:
    n, C = int(payload.shape[0]), int(payload.shape[1])
    H, W = int(cam.height), int(cam.width)
    rc = load().pulsar_fwd(
        _ptr(pos, "pos", n > 0, (n, 3)), _ptr(radius, "radius", n > 0, (n,)),
        _ptr(opacity, "opacity", False, (n,)), _ptr(payload, "payload", n > 0, (n, C)), n, C,
        _ptr(background, "background", True, (C,)), ctypes.byref(cam), ctypes.byref(params),
        _ptr(image, "image", True, (H, W, C)), _ptr(aux, "aux", False, (H, W)),
        _ws_ptr(ws), int(ws.numel()), _stream(stream))
    if rc != PULSAR_OK:
        raise PulsarError(rc, "pulsar_fwd")


def pulsar_fwd_noalloc(pos, radius, opacity, payload, background, cam: pulsar_camera_t,
                       params: pulsar_params_t, image, aux, stream=None) -> None:
    """pulsar_fwd on the library's static scratch buffer (no workspace)."""
    n, C = int(payload.shape[0]), int(payload.shape[1])
    H, W = int(cam.height), int(cam.width)
    rc = load().pulsar_fwd_noalloc(
        _ptr(pos, "pos", n > 0, (n, 3)), _ptr(radius, "radius", n > 0, (n,)),
        _ptr(opacity, "opacity", False, (n,)), _ptr(payload, "payload", n > 0, (n, C)), n, C,
        _ptr(background, "background", True, (C,)), ctypes.byref(cam), ctypes.byref(params),
        _ptr(image, "image", True, (H, W, C)), _ptr(aux, "aux", False, (H, W)),
        _stream(stream))
    if rc != PULSAR_OK:
        raise PulsarError(rc, "pulsar_fwd_noalloc")


def pulsar_bwd(pos, radius, opacity, payload, background, cam: pulsar_camera_t,
               params: pulsar_params_t, image, aux, grad_image, grad_pos, grad_radius,
               grad_opacity, grad_payload, grad_background, ws, stream=None) -> None:
    n, C = int(payload.shape[0]), int(payload.shape[1])
    H, W = int(cam.height), int(cam.width)
    rc = load().pulsar_bwd(
        _ptr(pos, "pos", n > 0, (n, 3)), _ptr(radius, "radius", n > 0, (n,)),
        _ptr(opacity, "opacity", False, (n,)), _ptr(payload, "payload", n > 0, (n, C)), n, C,
        _ptr(background, "background", True, (C,)), ctypes.byref(cam), ctypes.byref(params),
        _ptr(image, "image", True, (H, W, C)), _ptr(aux, "aux", True, (H, W)),
        _ptr(grad_image, "grad_image", True, (H, W, C)),
        _ptr(grad_pos, "grad_pos", False, (n, 3)), _ptr(grad_radius, "grad_radius", False, (n,)),
        _ptr(grad_opacity, "grad_opacity", False, (n,)),
        _ptr(grad_payload, "grad_payload", False, (n, C)),
        _ptr(grad_background, "grad_background", False, (C,)),
        _ws_ptr(ws), int(ws.numel()), _stream(stream))
    if rc != PULSAR_OK:
        raise PulsarError(rc, "pulsar_bwd")


def pulsar_bwd_camera(pos, radius, opacity, payload, background, cam: pulsar_camera_t,
                      params: pulsar_params_t, image, aux, grad_image, grad_pos, grad_radius,
                      grad_opacity, grad_payload, grad_background, grad_camera, ws,
                      stream=None) -> None:
    """pulsar_bwd plus grad_camera [14]: dR (3x3 row-major), dt, dfocal, dsensor_width."""
    n, C = int(payload.shape[0]), int(payload.shape[1])
    H, W = int(cam.height), int(cam.width)
    rc = load().pulsar_bwd_camera(
        _ptr(pos, "pos", n > 0, (n, 3)), _ptr(radius, "radius", n > 0, (n,)),
        _ptr(opacity, "opacity", False, (n,)), _ptr(payload, "payload", n > 0, (n, C)), n, C,
        _ptr(background, "background", True, (C,)), ctypes.byref(cam), ctypes.byref(params),
        _ptr(image, "image", True, (H, W, C)), _ptr(aux, "aux", True, (H, W)),
        _ptr(grad_image, "grad_image", True, (H, W, C)),
        _ptr(grad_pos, "grad_pos", False, (n, 3)), _ptr(grad_radius, "grad_radius", False, (n,)),
        _ptr(grad_opacity, "grad_opacity", False, (n,)),
        _ptr(grad_payload, "grad_payload", False, (n, C)),
        _ptr(grad_background, "grad_background", False, (C,)),
        _ptr(grad_camera, "grad_camera", True, (14,)),
        _ws_ptr(ws), int(ws.numel()), _stream(stream))
    if rc != PULSAR_OK:
        raise PulsarError(rc, "pulsar_bwd_camera")


def pulsar_batch_workspace_size(scenes, C: int, params: pulsar_params_t) -> int:
    return int(load().pulsar_batch_workspace_size(scenes, len(scenes), int(C),
                                                  ctypes.byref(params)))


def pulsar_fwd_batched(scenes, pos, radius, opacity, payload, background,
                       params: pulsar_params_t, image, aux, ws, stream=None) -> None:
    """Packed batch (include/pulsar.h): pos [N,3], background [B,C], image [P,C], aux [P]."""
    B = len(scenes)
    N, P = batch_sizes(scenes)
    C = int(payload.shape[1])
    rc = load().pulsar_fwd_batched(
        scenes, B, _ptr(pos, "pos", N > 0, (N, 3)), _ptr(radius, "radius", N > 0, (N,)),
        _ptr(opacity, "opacity", False, (N,)), _ptr(payload, "payload", N > 0, (N, C)), C,
        _ptr(background, "background", True, (B, C)), ctypes.byref(params),
        _ptr(image, "image", True, (P, C)), _ptr(aux, "aux", False, (P,)),
        _ws_ptr(ws), int(ws.numel()), _stream(stream))
    if rc != PULSAR_OK:
        raise PulsarError(rc, "pulsar_fwd_batched")


def cameras_bytes(cameras) -> bytes:
    """The bytes of B pulsar_camera_t structs, for a device camera array
    (a uint8 tensor of B * sizeof(pulsar_camera_t) bytes)."""
    cams = list(cameras)
    arr = (pulsar_camera_t * len(cams))(*cams)
    return ctypes.string_at(ctypes.addressof(arr), ctypes.sizeof(arr))


def pulsar_fwd_batched_devcam(scenes, d_cameras, pos, radius, opacity, payload, background,
                              params: pulsar_params_t, image, aux, ws, stream=None) -> None:
    """pulsar_fwd_batched with the cameras read from d_cameras (a contiguous
    uint8 device tensor holding B pulsar_camera_t, see cameras_bytes) when
    the work runs; scenes give the image sizes and sphere counts."""
    B = len(scenes)
    N, P = batch_sizes(scenes)
    C = int(payload.shape[1])
    if (not d_cameras.is_cuda or d_cameras.element_size() != 1 or not d_cameras.is_contiguous()
            or d_cameras.numel() != B * ctypes.sizeof(pulsar_camera_t)):
        raise ValueError("d_cameras must hold B pulsar_camera_t in a contiguous uint8 device "
                         "tensor")
    rc = load().pulsar_fwd_batched_devcam(
        scenes, B, d_cameras.data_ptr(), _ptr(pos, "pos", N > 0, (N, 3)),
        _ptr(radius, "radius", N > 0, (N,)), _ptr(opacity, "opacity", False, (N,)),
        _ptr(payload, "payload", N > 0, (N, C)), C,
        _ptr(background, "background", True, (B, C)), ctypes.byref(params),
        _ptr(image, "image", True, (P, C)), _ptr(aux, "aux", False, (P,)),
        _ws_ptr(ws), int(ws.numel()), _stream(stream))
    if rc != PULSAR_OK:
        raise PulsarError(rc, "pulsar_fwd_batched_devcam")


def pulsar_bwd_batched(scenes, pos, radius, opacity, payload, background,
                       params: pulsar_params_t, image, aux, grad_image, grad_pos, grad_radius,
                       grad_opacity, grad_payload, grad_background, ws, stream=None) -> None:
    B = len(scenes)
    N, P = batch_sizes(scenes)
    C = int(payload.shape[1])
    rc = load().pulsar_bwd_batched(
        scenes, B, _ptr(pos, "pos", N > 0, (N, 3)), _ptr(radius, "radius", N > 0, (N,)),
        _ptr(opacity, "opacity", False, (N,)), _ptr(payload, "payload", N > 0, (N, C)), C,
        _ptr(background, "background", True, (B, C)), ctypes.byref(params),
        _ptr(image, "image", True, (P, C)), _ptr(aux, "aux", True, (P,)),
        _ptr(grad_image, "grad_image", True, (P, C)),
        _ptr(grad_pos, "grad_pos", False, (N, 3)), _ptr(grad_radius, "grad_radius", False, (N,)),
        _ptr(grad_opacity, "grad_opacity", False, (N,)),
        _ptr(grad_payload, "grad_payload", False, (N, C)),
        _ptr(grad_background, "grad_background", False, (B, C)),
        _ws_ptr(ws), int(ws.numel()), _stream(stream))
    if rc != PULSAR_OK:
        raise PulsarError(rc, "pulsar_bwd_batched")


def pulsar_bwd_camera_batched(scenes, pos, radius, opacity, payload, background,
                              params: pulsar_params_t, image, aux, grad_image, grad_pos,
                              grad_radius, grad_opacity, grad_payload, grad_background,
                              grad_camera, ws, stream=None) -> None:
    B = len(scenes)
    N, P = batch_sizes(scenes)
    C = int(payload.shape[1])
    rc = load().pulsar_bwd_camera_batched(
        scenes, B, _ptr(pos, "pos", N > 0, (N, 3)), _ptr(radius, "radius", N > 0, (N,)),
        _ptr(opacity, "opacity", False, (N,)), _ptr(payload, "payload", N > 0, (N, C)), C,
        _ptr(background, "background", True, (B, C)), ctypes.byref(params),
        _ptr(image, "image", True, (P, C)), _ptr(aux, "aux", True, (P,)),
        _ptr(grad_image, "grad_image", True, (P, C)),
        _ptr(grad_pos, "grad_pos", False, (N, 3)), _ptr(grad_radius, "grad_radius", False, (N,)),
        _ptr(grad_opacity, "grad_opacity", False, (N,)),
        _ptr(grad_payload, "grad_payload", False, (N, C)),
        _ptr(grad_background, "grad_background", False, (B, C)),
        _ptr(grad_camera, "grad_camera", True, (B, 14)),
        _ws_ptr(ws), int(ws.numel()), _stream(stream))
    if rc != PULSAR_OK:
        raise PulsarError(rc, "pulsar_bwd_camera_batched")


def pulsar_query_status(ws, stream=None) -> Tuple[int, int]:
    """Synchronises the stream; returns (status code, number of tile pairs)."""
    pairs = ctypes.c_int64(0)
    rc = load().pulsar_query_status(_ws_ptr(ws), int(ws.numel()), _stream(stream),
                                    ctypes.byref(pairs))
    if rc not in (PULSAR_OK, PULSAR_ERR_CAPACITY, PULSAR_ERR_INVALID_ARGUMENT):
        raise PulsarError(rc, "pulsar_query_status")
    return rc, int(pairs.value)


def decode_status(raw: bytes) -> Tuple[int, int]:
    """(status code, tile pairs) from the first PULSAR_STATUS_BYTES bytes of a
    workspace (the layout the header documents)."""
    flag, _stored, pairs = struct.unpack("<IIQ", bytes(raw[:PULSAR_STATUS_BYTES]))
    return -int(flag), int(pairs)


def _ws_ptr(ws) -> int:
    if not ws.is_cuda or ws.element_size() != 1 or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 device tensor")
    return ws.data_ptr()


def pulsar_timing_enable(on: bool) -> bool:
    return bool(load().pulsar_timing_enable(1 if on else 0))


def pulsar_timing_read() -> dict:
    """{stage name: (total ms, launches)} for the stage timings recorded so far."""
    lib = load()
    ms = (ctypes.c_double * PULSAR_NUM_STAGES)()
    cnt = (ctypes.c_int64 * PULSAR_NUM_STAGES)()
    rc = lib.pulsar_timing_read(ms, cnt)
    if rc != PULSAR_OK:
        raise PulsarError(rc, "pulsar_timing_read")
    return {pulsar_stage_name(i): (float(ms[i]), int(cnt[i])) for i in range(PULSAR_NUM_STAGES)}


def pulsar_stage_name(stage: int) -> str:
    return load().pulsar_stage_name(int(stage)).decode()
