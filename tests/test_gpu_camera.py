"""Camera gradients of the HIP backward (pulsar_bwd_camera and its batched
form) against the FP64 oracle: dLoss/dR, dLoss/dt, dLoss/dfocal and
dLoss/dsensor_width on rotated, clamped and larger scenes, with the scene
gradients of the same call unchanged."""
import copy

import numpy as np
import pytest

from oracle import reference as ref
from paper_2004_07484_amd import _capi
from paper_2004_07484_amd import scenegen as sg
from tests.gpu_helpers import (assert_camera_close, compare_grads, cam_struct, gpu_render,
                               masked_G, to_dev)
from tests.oracle_helpers import random_rotation

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _rotated(wl, seed):
    """The same camera-space scene seen through a random rigid camera pose."""
    rng = np.random.default_rng(seed)
    Rq = random_rotation(rng)
    tq = rng.uniform(-1, 1, 3)
    sc = copy.deepcopy(wl.scene)
    sc.pos = ((sc.pos.astype(np.float64) - tq) @ Rq).astype(np.float32)
    cam = copy.deepcopy(wl.camera)
    cam.R = Rq.astype(np.float32)
    cam.t = tq.astype(np.float32)
    return sc, cam


def _check(sc, cam, par, what, rows=None, G_seed=500, flags=0):
    _say(f"[camera] {what} n={sc.n} {cam.width}x{cam.height} C={sc.C} K={par.K}")
    fwd = ref.forward(sc, cam, par, rows=rows)
    G = sg.upstream_grad(G_seed, cam.height, cam.width, sc.C)
    Gm = masked_G(G, rows, fwd["ambiguous"])
    out = gpu_render(sc, cam, par, Gm, camera_grad=True, fwd_flags=flags, bwd_flags=flags)
    assert out["status"] == _capi.PULSAR_OK
    g = ref.backward(sc, cam, par, Gm, fwd, rows=rows)
    assert np.isfinite(out["grad_camera"]).all()
    compare_grads(out, g, what)
    assert_camera_close(out["grad_camera"], g["grad_camera"], g["grad_camera_abs"], what)
    return out


@pytest.mark.parametrize("seed", [1, 2])
def test_camera_gradients_small_rotated(seed):
    wl = sg.config1()
    sc, cam = _rotated(wl, seed)
    _check(sc, cam, wl.params, f"1k spheres, pose {seed}")


def test_camera_gradients_tile_order():
    """The same through the backward that walks the tile lists."""
    wl = sg.config1()
    sc, cam = _rotated(wl, 3)
    _check(sc, cam, wl.params, "1k spheres, tile order", flags=_capi.PULSAR_BWD_TILES)


def test_camera_gradients_large_spheres():
    """Spheres wider than 16 tiles send the default backward to the tile walk
    (decided on the device); its camera terms go through the per-pair slots."""
    wl = sg.tiny_scene(142, n=24, C=3, W=96, H=80, r_lo=0.3, r_hi=0.9)
    wl.params = sg.Params(gamma=0.3, eps=1e-5, K=6)
    sc, cam = _rotated(wl, 4)
    _check(sc, cam, wl.params, "large spheres, tile walk chosen on the device")


def test_camera_gradients_identity_pose():
    wl = sg.config1()
    _check(wl.scene, wl.camera, wl.params, "1k spheres, identity pose")


def test_camera_gradients_minimum_size():
    """Clamped spheres' radius follows the focal length and sensor width."""
    wl = sg.config1()
    sc, cam = _rotated(wl, 3)
    par = sg.Params(gamma=0.1, eps=1e-5, min_radius_px=1.5, K=5)
    _check(sc, cam, par, "1k spheres, minimum size 1.5 px")


def test_camera_gradients_tiny_scenes_all_hits():
    """K above the hit count: the full derivative of Eq. 1."""
    for seed in (3, 4):
        wl = sg.tiny_scene(seed, n=6, C=3)
        sc, cam = _rotated(wl, seed)
        _check(sc, cam, wl.params, f"tiny {seed}")


def test_camera_gradients_100k_rows():
    wl = sg.config2()
    sc, cam = _rotated(wl, 5)
    rows = sorted(np.random.default_rng(81).choice(cam.height, 3, replace=False).tolist())
    _check(sc, cam, wl.params, "100k spheres, 3 rows", rows=rows)


def test_camera_gradients_wide_payload():
    """C > 32 takes the wide backward kernel."""
    rng = np.random.default_rng(17)
    sc = sg.box_scene(rng, 300, 40, 0.02, 0.12)
    cam = sg.identity_camera(40, 40)
    par = sg.Params(gamma=0.1, eps=1e-5, K=4)
    _check(sc, cam, par, "C=40 wide path")


def test_scene_gradients_unchanged_by_camera_request():
    wl = sg.config1()
    sc, cam = _rotated(wl, 6)
    G = sg.upstream_grad(6, cam.height, cam.width, sc.C)
    a = gpu_render(sc, cam, wl.params, G)
    b = gpu_render(sc, cam, wl.params, G, camera_grad=True)
    for key in ["F", "L", "grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
        assert np.array_equal(a[key], b[key]), key
    c = gpu_render(sc, cam, wl.params, G, camera_grad=True, need={"payload"})
    assert np.array_equal(c["grad_camera"], b["grad_camera"])


def test_batched_camera_gradients_match_single_scenes():
    import torch
    wls = [sg.config1(), sg.tiny_scene(7, n=6, C=3, W=40, H=24)]
    wls[1] = sg.Workload(wls[1].name, sg.box_scene(np.random.default_rng(7), 700, 3, 0.01, 0.1),
                         sg.look_at_camera([0.3, -0.2, -1.0], [0.0, 0.0, 4.5], [0, 1, 0], 48, 40),
                         wls[0].params, 7)
    par = wls[0].params
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    scenes = _capi.make_scenes([cam_struct(w.camera) for w in wls], [w.scene.n for w in wls])
    C = 3
    cat = lambda f: np.concatenate([f(w) for w in wls], 0)
    pos, rad = to_dev(cat(lambda w: w.scene.pos)), to_dev(cat(lambda w: w.scene.radius))
    opa, pay = to_dev(cat(lambda w: w.scene.opacity)), to_dev(cat(lambda w: w.scene.payload))
    bg = to_dev(np.stack([w.scene.bg for w in wls]))
    P = sum(w.camera.width * w.camera.height for w in wls)
    N = sum(w.scene.n for w in wls)
    Gs = [sg.upstream_grad(60 + i, w.camera.height, w.camera.width, C) for i, w in enumerate(wls)]
    G = to_dev(np.concatenate([g.reshape(-1, C) for g in Gs], 0))
    ws = torch.empty(_capi.pulsar_batch_workspace_size(scenes, C, ps), dtype=torch.uint8,
                     device="cuda:0")
    image = torch.empty((P, C), device="cuda:0")
    aux = torch.empty((P,), device="cuda:0")
    _capi.pulsar_fwd_batched(scenes, pos, rad, opa, pay, bg, ps, image, aux, ws)
    gcam = torch.full((len(wls), 14), float("nan"), device="cuda:0")
    gp = torch.empty((N, 3), device="cuda:0")
    _capi.pulsar_bwd_camera_batched(scenes, pos, rad, opa, pay, bg, ps, image, aux, G, gp, None,
                                    None, None, None, gcam, ws)
    torch.cuda.synchronize()
    got = gcam.cpu().numpy()
    for i, w in enumerate(wls):
        single = gpu_render(w.scene, w.camera, w.params, Gs[i], camera_grad=True)
        scale = np.abs(single["grad_camera"]).max()
        np.testing.assert_allclose(got[i], single["grad_camera"], rtol=1e-4, atol=1e-5 * scale)


def test_renderer_camera_vector_gradient():
    """Renderer with the 8-vector camera [t, axis-angle, focal, sensor_width]
    requiring grad: its gradient is the oracle's dLoss/d(R, t, f, s) chained
    through Rodrigues' formula (Jacobian taken in FP64 on the CPU)."""
    import torch
    from paper_2004_07484_amd.renderer import Renderer, axis_angle_to_matrix_torch
    wl = sg.config1()
    sc, par = wl.scene, wl.params
    vec = np.array([0.05, -0.1, 0.3, 0.2, -0.15, 0.1, wl.camera.focal,
                    wl.camera.sensor_width], np.float32)
    cam_v = torch.tensor(vec, device="cuda:0", requires_grad=True)
    # the rotation the kernels receive, and the same camera for the oracle
    R32 = axis_angle_to_matrix_torch(cam_v.detach()[3:6]).cpu().numpy().astype(np.float32)
    cam = copy.deepcopy(wl.camera)
    cam.R, cam.t = R32, vec[0:3].copy()
    fwd = ref.forward(sc, cam, par)
    Gm = masked_G(sg.upstream_grad(91, cam.height, cam.width, sc.C), None, fwd["ambiguous"])
    g = ref.backward(sc, cam, par, Gm, fwd)
    r = Renderer(cam.width, cam.height, sc.n, n_channels=sc.C, K=par.K)
    img = r(to_dev(sc.pos), to_dev(sc.payload), to_dev(sc.radius), cam_v,
            opacity=to_dev(sc.opacity), gamma=par.gamma, max_depth=cam.zfar,
            min_depth=cam.znear, bg=to_dev(sc.bg))
    img.backward(to_dev(Gm))
    got = cam_v.grad.cpu().numpy()
    aa = torch.tensor(vec[3:6].astype(np.float64))
    J = torch.autograd.functional.jacobian(lambda a: axis_angle_to_matrix_torch(a).reshape(9),
                                           aa).numpy()  # [9, 3]
    want = np.concatenate([g["grad_camera"][9:12], J.T @ g["grad_camera"][0:9],
                           g["grad_camera"][12:14]])
    scale = np.concatenate([g["grad_camera_abs"][9:12], np.abs(J).T @ g["grad_camera_abs"][0:9],
                            g["grad_camera_abs"][12:14]])
    assert_camera_close(got, want, scale, "Renderer camera vector")


@pytest.mark.parametrize("case", ["rotated", "min_radius"])
def test_paper_normalised_camera_gradients(case):
    """PULSAR_GRAD_PAPER_NORM on pulsar_bwd_camera: each sphere's part of the
    camera gradient scaled by 1e-3 over its projected disk area, beside the
    averaged and gated scene gradients (oracle paper_normalised)."""
    wl = sg.config1()
    par = wl.params
    if case == "rotated":
        sc, cam = _rotated(wl, 3)
    else:
        sc, cam = wl.scene, wl.camera
        par = sg.Params(gamma=par.gamma, eps=par.eps, min_radius_px=0.9, K=par.K)
    _say(f"[camera] paper normalisation, {case}")
    fwd = ref.forward(sc, cam, par)
    G = masked_G(sg.upstream_grad(501, cam.height, cam.width, sc.C), None, fwd["ambiguous"])
    out = gpu_render(sc, cam, par, G, camera_grad=True, bwd_flags=_capi.PULSAR_GRAD_PAPER_NORM)
    assert out["status"] == _capi.PULSAR_OK
    pn = ref.paper_normalised(sc, cam, par, fwd, ref.backward(sc, cam, par, G, fwd))
    compare_grads(out, pn, f"paper norm {case}")
    assert_camera_close(out["grad_camera"], pn["grad_camera"], pn["grad_camera_abs"],
                        f"paper norm {case} camera")


def test_renderer_6d_camera_vector_gradient():
    """Renderer with the 11-vector camera [t, 6D rotation, focal,
    sensor_width] requiring grad: its gradient is the oracle's dLoss/d(R, t,
    f, s) chained through the 6D parametrisation (Jacobian in FP64 on the
    CPU)."""
    import torch
    from paper_2004_07484_amd.renderer import Renderer, rotation_6d_to_matrix_torch
    wl = sg.config1()
    sc, par = wl.scene, wl.params
    vec = np.array([0.05, -0.1, 0.3, 0.98, 0.1, -0.12, -0.08, 0.97, 0.15, wl.camera.focal,
                    wl.camera.sensor_width], np.float32)
    cam_v = torch.tensor(vec, device="cuda:0", requires_grad=True)
    R32 = rotation_6d_to_matrix_torch(cam_v.detach()[3:9]).cpu().numpy().astype(np.float32)
    cam = copy.deepcopy(wl.camera)
    cam.R, cam.t = R32, vec[0:3].copy()
    fwd = ref.forward(sc, cam, par)
    Gm = masked_G(sg.upstream_grad(92, cam.height, cam.width, sc.C), None, fwd["ambiguous"])
    g = ref.backward(sc, cam, par, Gm, fwd)
    r = Renderer(cam.width, cam.height, sc.n, n_channels=sc.C, K=par.K)
    img = r(to_dev(sc.pos), to_dev(sc.payload), to_dev(sc.radius), cam_v,
            opacity=to_dev(sc.opacity), gamma=par.gamma, max_depth=cam.zfar,
            min_depth=cam.znear, bg=to_dev(sc.bg))
    img.backward(to_dev(Gm))
    got = cam_v.grad.cpu().numpy()
    r6 = torch.tensor(vec[3:9].astype(np.float64))
    J = torch.autograd.functional.jacobian(lambda a: rotation_6d_to_matrix_torch(a).reshape(9),
                                           r6).numpy()  # [9, 6]
    want = np.concatenate([g["grad_camera"][9:12], J.T @ g["grad_camera"][0:9],
                           g["grad_camera"][12:14]])
    scale = np.concatenate([g["grad_camera_abs"][9:12], np.abs(J).T @ g["grad_camera_abs"][0:9],
                            g["grad_camera_abs"][12:14]])
    assert_camera_close(got, want, scale, "Renderer 6D camera vector")
