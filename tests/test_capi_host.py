"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, plans workspaces and rejects bad arguments before any launch.
None of these calls touches a GPU."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

from paper_2004_07484_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pulsar.h")

FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first


def _lib():
    if not os.path.exists(_capi.LIB_PATH):
        from paper_2004_07484_amd import build
        build.build()
    return _capi.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\**\s+\**(pulsar_\w+)\s*\(", text, re.M)))


def test_header_declarations_are_exported():
    lib = _lib()
    names = declared_functions()
    assert set(_capi.EXPORTED) <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _capi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pulsar_\w+)", out))
    assert set(names) <= exported


def test_version_and_status_strings():
    _lib()
    assert _capi.pulsar_version() == 3
    for code in [0, -1, -2, -3, -4, -5, -6, -99]:
        assert len(_capi.pulsar_status_string(code)) > 5
    assert "capacity" in _capi.pulsar_status_string(_capi.PULSAR_ERR_CAPACITY)


def test_workspace_size_plan():
    _lib()
    p = _capi.make_params(K=8)
    s1 = _capi.pulsar_workspace_size(1000, 64, 64, 3, p)
    s2 = _capi.pulsar_workspace_size(100_000, 64, 64, 3, p)
    s0 = _capi.pulsar_workspace_size(0, 64, 64, 3, p)
    assert 0 < s0 < s1 < s2
    assert s1 % 256 == 0
    # explicit pair capacity grows the workspace by 16 bytes per pair
    big = _capi.pulsar_workspace_size(1000, 64, 64, 3, _capi.make_params(K=8, max_pairs=10**6))
    small = _capi.pulsar_workspace_size(1000, 64, 64, 3, _capi.make_params(K=8, max_pairs=10**5))
    assert big - small >= 16 * 9 * 10**5
    # invalid requests plan nothing
    assert _capi.pulsar_workspace_size(-1, 64, 64, 3, p) == 0
    assert _capi.pulsar_workspace_size(10, 0, 64, 3, p) == 0
    assert _capi.pulsar_workspace_size(10, 64, 70000, 3, p) == 0
    assert _capi.pulsar_workspace_size(10, 64, 64, 0, p) == 0
    assert _capi.pulsar_workspace_size(10, 64, 64, 3, _capi.make_params(K=0)) == 0
    assert _capi.pulsar_workspace_size(10, 64, 64, 3, _capi.make_params(K=33)) == 0


def _call_fwd(cam, params, n=10, C=3, ws_bytes=1 << 30, image=FAKE, bg=FAKE, pos=FAKE):
    lib = _lib()
    return lib.pulsar_fwd(pos, FAKE, None, FAKE, n, C, bg, ctypes.byref(cam),
                          ctypes.byref(params), image, None, FAKE, ws_bytes, None)


def _cam(**kw):
    d = dict(R=[1, 0, 0, 0, 1, 0, 0, 0, 1], t=[0, 0, 0], focal=1.0, sensor_width=2.0, znear=1.0,
             zfar=10.0, width=64, height=64)
    d.update(kw)
    return _capi.make_camera(**d)


@pytest.mark.parametrize("cam_kw", [dict(focal=0.0), dict(focal=-1.0),
                                    dict(sensor_width=0.0), dict(znear=0.0),
                                    dict(znear=5.0, zfar=5.0), dict(width=0),
                                    dict(height=65536), dict(t=[0, float("nan"), 0]),
                                    dict(focal=float("inf"))])
def test_bad_camera_is_rejected(cam_kw):
    assert _call_fwd(_cam(**cam_kw), _capi.make_params()) == _capi.PULSAR_ERR_INVALID_ARGUMENT


@pytest.mark.parametrize("par_kw,code", [
    (dict(gamma=0.0), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(gamma=2.0), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(gamma=1e-6), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(eps=-1.0), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(min_radius_px=-0.5), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(K=0), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(K=33), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(max_pairs=-5), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(depth_bits=17), _capi.PULSAR_ERR_UNSUPPORTED),
    (dict(depth_bits=8), _capi.PULSAR_ERR_UNSUPPORTED),
    (dict(chunk=32), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(chunk=100), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(chunk=2048), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(raster_blocks=100), _capi.PULSAR_ERR_INVALID_ARGUMENT),
    (dict(raster_blocks=70000), _capi.PULSAR_ERR_INVALID_ARGUMENT),
])
def test_bad_params_are_rejected(par_kw, code):
    assert _call_fwd(_cam(), _capi.make_params(**par_kw)) == code


def test_reserved_flags_are_unsupported():
    for bit in [0x80, 0x100, 0x80000000]:
        p = _capi.make_params(flags=bit | _capi.PULSAR_REBIN)
        assert _call_fwd(_cam(), p) == _capi.PULSAR_ERR_UNSUPPORTED


def test_known_flags_pass_validation():
    # validation accepts them and stops at the next check, the workspace size
    for flags in [_capi.PULSAR_NO_BWD_AUX, _capi.PULSAR_REBIN, _capi.PULSAR_GRAD_PAPER_NORM,
                  _capi.PULSAR_BLEND_TOPK, _capi.PULSAR_ORTHO,
                  _capi.PULSAR_NO_BWD_AUX | _capi.PULSAR_REBIN | _capi.PULSAR_GRAD_PAPER_NORM]:
        p = _capi.make_params(flags=flags)
        assert _call_fwd(_cam(), p, ws_bytes=1024) == _capi.PULSAR_ERR_WORKSPACE
        # flags change no workspace size
        assert _capi.pulsar_workspace_size(10, 64, 64, 3, p) == \
            _capi.pulsar_workspace_size(10, 64, 64, 3, _capi.make_params())


def test_pair_slots_are_planned_for_every_backward():
    """Every plan with backward state holds one gradient slot per pair (the
    default backward may take the tile walk for scenes with very large
    spheres, decided on the device), 16 bytes per float4 of a slot; the
    stored hits come on top of that."""
    _lib()
    cap = 10**5
    plain = _capi.pulsar_workspace_size(1000, 64, 64, 3, _capi.make_params(max_pairs=cap))
    small = _capi.pulsar_workspace_size(1000, 64, 64, 3, _capi.make_params(max_pairs=cap // 2))
    tiles = _capi.pulsar_workspace_size(1000, 64, 64, 3, _capi.make_params(
        max_pairs=cap, flags=_capi.PULSAR_BWD_TILES))
    store = _capi.pulsar_workspace_size(1000, 64, 64, 3, _capi.make_params(
        max_pairs=cap, flags=_capi.PULSAR_STORE_HITS))
    # per pair: tile and sphere index twice (16 bytes) and a slot of two
    # float4 at C = 3 (dL/dc, dL/dR | dL/df[4], dL/do, ...)
    assert plain - small >= (16 + 32) * (cap - cap // 2)
    assert tiles == plain
    assert store > plain
    p = _capi.make_params(flags=_capi.PULSAR_BWD_TILES)
    assert _call_fwd(_cam(), p, ws_bytes=1024) == _capi.PULSAR_ERR_WORKSPACE


def test_missing_pointers_and_small_workspace():
    p = _capi.make_params()
    assert _call_fwd(_cam(), p, image=None) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    assert _call_fwd(_cam(), p, bg=None) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    assert _call_fwd(_cam(), p, pos=None) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    assert _call_fwd(_cam(), p, n=-1) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    assert _call_fwd(_cam(), p, C=0) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    need = _capi.pulsar_workspace_size(10, 64, 64, 3, p)
    assert _call_fwd(_cam(), p, ws_bytes=need - 1) == _capi.PULSAR_ERR_WORKSPACE


def test_backward_argument_checks():
    lib = _lib()
    cam, p = _cam(), _capi.make_params()
    args = [FAKE, FAKE, None, FAKE, 10, 3, FAKE, ctypes.byref(cam), ctypes.byref(p), FAKE, FAKE,
            FAKE, FAKE, FAKE, None, FAKE, FAKE, FAKE, 1 << 30, None]
    bad_aux = list(args)
    bad_aux[10] = None
    assert lib.pulsar_bwd(*bad_aux) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    op_grad_without_opacity = list(args)
    op_grad_without_opacity[14] = FAKE
    assert lib.pulsar_bwd(*op_grad_without_opacity) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    small = list(args)
    small[18] = 1024
    assert lib.pulsar_bwd(*small) == _capi.PULSAR_ERR_WORKSPACE
    # a forward without backward state leaves nothing to reuse: only a rebin
    # may follow it
    no_state = _capi.make_params(flags=_capi.PULSAR_NO_BWD_AUX)
    args_ns = list(args)
    args_ns[8] = ctypes.byref(no_state)
    assert lib.pulsar_bwd(*args_ns) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    # the camera variant needs its output and otherwise checks like pulsar_bwd
    cam_args = args[:17] + [None] + args[17:]
    assert lib.pulsar_bwd_camera(*cam_args) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    cam_small = small[:17] + [FAKE] + small[17:]
    assert lib.pulsar_bwd_camera(*cam_small) == _capi.PULSAR_ERR_WORKSPACE
    cam_bad_aux = bad_aux[:17] + [FAKE] + bad_aux[17:]
    assert lib.pulsar_bwd_camera(*cam_bad_aux) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    # no focal / sensor-width terms for parallel rays
    ortho = _capi.make_params(flags=_capi.PULSAR_ORTHO)
    cam_ortho = list(cam_args)
    cam_ortho[8] = ctypes.byref(ortho)
    cam_ortho[17] = FAKE
    assert lib.pulsar_bwd_camera(*cam_ortho) == _capi.PULSAR_ERR_UNSUPPORTED
    rebin = _capi.make_params(flags=_capi.PULSAR_NO_BWD_AUX | _capi.PULSAR_REBIN)
    args_rb = list(small)
    args_rb[8] = ctypes.byref(rebin)
    assert lib.pulsar_bwd(*args_rb) == _capi.PULSAR_ERR_WORKSPACE


def test_launch_without_device_reports_hip_error():
    """With no GPU present a well-formed call fails cleanly with PULSAR_ERR_HIP.
    Runs in a child process so HIP runtime state stays out of this one."""
    code = r"""
import ctypes, sys
sys.path.insert(0, %r)
from paper_2004_07484_amd import _capi
lib = _capi.load()
cnt = ctypes.c_int(0)
ctypes.CDLL("libamdhip64.so").hipGetDeviceCount(ctypes.byref(cnt))
if cnt.value > 0:
    print("HAS_GPU")
    sys.exit(0)
cam = _capi.make_camera([1,0,0,0,1,0,0,0,1], [0,0,0], 1.0, 2.0, 1.0, 10.0, 16, 16)
p = _capi.make_params()
f = ctypes.c_void_p(0x10000)
rc = lib.pulsar_fwd(f, f, None, f, 4, 3, f, ctypes.byref(cam), ctypes.byref(p), f, None, f,
                    1 << 30, None)
print("RC", rc, lib.pulsar_last_hip_error().decode())
""" % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    if "HAS_GPU" in out.stdout:
        pytest.skip("a GPU is present; this checks the no-device path")
    assert f"RC {_capi.PULSAR_ERR_HIP}" in out.stdout, out.stdout + out.stderr



# ---------------------------------------------------------------- batched calls

def _scenes(specs):
    """specs: list of (width, height, n)."""
    return _capi.make_scenes([_cam(width=w, height=h) for w, h, _ in specs],
                             [n for _, _, n in specs])


def _call_fwd_batched(scenes, params, C=3, ws_bytes=1 << 34, pos=FAKE, image=FAKE, B=None):
    lib = _lib()
    return lib.pulsar_fwd_batched(scenes, len(scenes) if B is None else B, pos, FAKE, None, FAKE,
                                  C, FAKE, ctypes.byref(params), image, None, FAKE, ws_bytes,
                                  None)


def test_batch_workspace_matches_single_scene_and_grows():
    _lib()
    p = _capi.make_params(K=5)
    one = _scenes([(256, 256, 5000)])
    assert _capi.pulsar_batch_workspace_size(one, 3, p) == \
        _capi.pulsar_workspace_size(5000, 256, 256, 3, p)
    two = _scenes([(256, 256, 5000), (512, 384, 20000)])
    three = _scenes([(256, 256, 5000), (512, 384, 20000), (1024, 1024, 0)])
    s1 = _capi.pulsar_batch_workspace_size(one, 3, p)
    s2 = _capi.pulsar_batch_workspace_size(two, 3, p)
    s3 = _capi.pulsar_batch_workspace_size(three, 3, p)
    assert 0 < s1 < s2 < s3
    # the same scenes in another order need the same space
    rev = _scenes([(512, 384, 20000), (256, 256, 5000)])
    assert _capi.pulsar_batch_workspace_size(rev, 3, p) == s2
    # the tuning knobs only resize work-item buffers
    assert _capi.pulsar_batch_workspace_size(two, 3, _capi.make_params(K=5, chunk=64)) > s2
    assert _capi.pulsar_batch_workspace_size(two, 3, _capi.make_params(K=5, raster_blocks=512)) \
        == s2


def test_batched_argument_checks():
    _lib()
    p = _capi.make_params(K=5)
    good = _scenes([(64, 64, 10), (32, 48, 7)])
    assert _capi.pulsar_batch_workspace_size(good, 3, p) > 0
    # B out of range
    assert _call_fwd_batched(good, p, B=0) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    many = _scenes([(8, 8, 1)] * (_capi.PULSAR_MAX_SCENES + 1))
    assert _call_fwd_batched(many, p) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    assert _capi.pulsar_batch_workspace_size(many, 3, p) == 0
    # a bad camera or count anywhere in the batch
    bad = _scenes([(64, 64, 10), (0, 48, 7)])
    assert _call_fwd_batched(bad, p) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    neg = _scenes([(64, 64, 10), (32, 48, -1)])
    assert _call_fwd_batched(neg, p) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    res = _scenes([(64, 64, 10), (32, 48, 7)])
    res[1].reserved = 3
    assert _call_fwd_batched(res, p) == _capi.PULSAR_ERR_UNSUPPORTED
    # more than 2^31 - 1 spheres in total
    huge = _scenes([(64, 64, 2**30), (64, 64, 2**30)])
    assert _call_fwd_batched(huge, p) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    # pointers and workspace
    assert _call_fwd_batched(good, p, pos=None) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    assert _call_fwd_batched(good, p, image=None) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    need = _capi.pulsar_batch_workspace_size(good, 3, p)
    assert _call_fwd_batched(good, p, ws_bytes=need - 1) == _capi.PULSAR_ERR_WORKSPACE
    # all-empty batches need no sphere pointers
    empty = _scenes([(64, 64, 0), (32, 48, 0)])
    need0 = _capi.pulsar_batch_workspace_size(empty, 3, p)
    assert _call_fwd_batched(empty, p, pos=None, ws_bytes=need0 - 1) == _capi.PULSAR_ERR_WORKSPACE


def test_batched_backward_argument_checks():
    lib = _lib()
    p = _capi.make_params(K=5)
    sc = _scenes([(64, 64, 10), (32, 48, 7)])
    args = [sc, 2, FAKE, FAKE, None, FAKE, 3, FAKE, ctypes.byref(p), FAKE, FAKE, FAKE, FAKE,
            FAKE, None, FAKE, FAKE, FAKE, 1 << 34, None]
    no_grad_image = list(args)
    no_grad_image[11] = None
    assert lib.pulsar_bwd_batched(*no_grad_image) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    op_grad_without_opacity = list(args)
    op_grad_without_opacity[14] = FAKE
    assert lib.pulsar_bwd_batched(*op_grad_without_opacity) == _capi.PULSAR_ERR_INVALID_ARGUMENT
    small = list(args)
    small[18] = 4096
    assert lib.pulsar_bwd_batched(*small) == _capi.PULSAR_ERR_WORKSPACE


def test_flag_constants_mirror_the_header():
    """Every PULSAR_* flag and preset the header defines has the same value
    in the Python binding."""
    text = open(HEADER).read()
    defs = dict(re.findall(r"^#define (PULSAR_[A-Z0-9_]+) (0x[0-9a-fA-F]+)u$", text, re.M))
    assert {"PULSAR_NO_BWD_AUX", "PULSAR_REBIN", "PULSAR_GRAD_PAPER_NORM", "PULSAR_BLEND_TOPK",
            "PULSAR_ORTHO"} <= set(defs)
    for name, val in defs.items():
        assert getattr(_capi, name) == int(val, 16), name
    vals = [int(v, 16) for v in defs.values()]
    assert all(v & (v - 1) == 0 for v in vals) and len(set(vals)) == len(vals)  # distinct bits
    preset = re.search(r"^#define PULSAR_MIN_RADIUS_PX_PAPER ([0-9.]+)f$", text, re.M)
    assert preset and abs(float(preset.group(1)) - _capi.PULSAR_MIN_RADIUS_PX_PAPER) < 1e-8
    assert abs(_capi.PULSAR_MIN_RADIUS_PX_PAPER - 0.5 * 2 ** 0.5) < 1e-8


def test_noalloc_forward_rejects_what_its_scratch_cannot_hold():
    """pulsar_fwd_noalloc checks its static scratch size on the host, before
    any HIP call; invalid requests get pulsar_fwd's own validation error."""
    lib = _lib()
    p = _capi.make_params(K=8)
    cam = _cam(width=4096, height=4096)
    need = _capi.pulsar_workspace_size(2_000_000, 4096, 4096, 3, p)
    assert need > _capi.PULSAR_NOALLOC_SCRATCH_BYTES
    rc = lib.pulsar_fwd_noalloc(FAKE, FAKE, None, FAKE, 2_000_000, 3, FAKE, ctypes.byref(cam),
                                ctypes.byref(p), FAKE, FAKE, None)
    assert rc == _capi.PULSAR_ERR_SCRATCH
    assert "scratch" in _capi.pulsar_status_string(rc)
    rc = lib.pulsar_fwd_noalloc(FAKE, FAKE, None, FAKE, 10, 0, FAKE, ctypes.byref(_cam()),
                                ctypes.byref(p), FAKE, FAKE, None)
    assert rc == _capi.PULSAR_ERR_INVALID_ARGUMENT
    assert lib.pulsar_fwd_noalloc(FAKE, FAKE, None, FAKE, 10, 3, FAKE, None, ctypes.byref(p),
                                  FAKE, FAKE, None) == _capi.PULSAR_ERR_INVALID_ARGUMENT


def test_stage_names_match_the_header():
    """Every timing stage the header defines has its own name, and the binding
    reads as many stages as the header declares."""
    _lib()
    text = open(HEADER).read()
    stages = {m[0]: int(m[1]) for m in re.findall(r"#define PULSAR_STAGE_(\w+) (\d+)", text)}
    n = int(re.search(r"#define PULSAR_NUM_STAGES (\d+)", text).group(1))
    assert n == _capi.PULSAR_NUM_STAGES
    assert sorted(stages.values()) == list(range(n))
    for name, i in stages.items():
        assert _capi.pulsar_stage_name(i) == name.lower(), (name, i)
    assert _capi.pulsar_stage_name(n) == "unknown"
    assert _capi.pulsar_stage_name(-1) == "unknown"
