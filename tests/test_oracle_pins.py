"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
textbook ray-sphere quadratic (numpy.roots), closed forms of Eq. 1,
invariants the paper states (commutativity, App. A), the gamma limits
(Sec. 3.2), the background weight (Sec. 3.2), central finite differences,
and Python's own sort for the K nearest hits (App. B, Step 2).
The paper prints no per-pixel values, so there is no worked example to match.
"""
import copy
import math
import types

import numpy as np
import pytest

from oracle import reference as ref
from paper_2004_07484_amd import scenegen as sg
from tests.oracle_helpers import as_f64, fd_camera_grads, fd_grads, pixel_direction, \
    random_rotation


def _rotated_world(wl, rng):
    """Same camera-space scene seen through a random rigid camera pose."""
    Rq = random_rotation(rng)
    tq = rng.uniform(-1, 1, 3)
    sc = as_f64(wl.scene)
    sc.pos = (sc.pos - tq) @ Rq  # rows of R^T (c - t)
    cam = copy.deepcopy(wl.camera)
    cam.R = Rq
    cam.t = tq
    return sc, cam


# ---------------------------------------------------------------- geometry

def test_hit_distance_matches_quadratic_roots():
    """t is the smaller root of |t u - c|^2 = R^2 (textbook quadratic), and a
    hit happens exactly when that root is real, distinct and <= far."""
    rng = np.random.default_rng(11)
    wl = sg.tiny_scene(3, n=40, W=32, H=24, r_lo=0.2, r_hi=0.9)
    sc, cam = _rotated_world(wl, rng)
    checked = 0
    for (i, j) in [(i, j) for i in range(0, 24, 2) for j in range(0, 32, 2)]:
        hits = ref.pixel_hits(sc, cam, wl.params, i, j)
        u = pixel_direction(cam, i, j)
        np.testing.assert_allclose(hits["u"], u, rtol=0, atol=1e-15)
        for k in range(sc.pos.shape[0]):
            c = cam.R @ sc.pos[k] + cam.t
            np.testing.assert_allclose(hits["c"][k], c, rtol=0, atol=1e-13)
            R = sc.radius[k]
            roots = np.roots([1.0, -2.0 * (u @ c), c @ c - R * R])
            real = np.all(np.abs(np.imag(roots)) == 0) and abs(roots[0] - roots[1]) > 1e-9
            takes_part = c[2] - R >= cam.znear
            if real and takes_part:
                t1 = float(np.min(np.real(roots)))
                expect = t1 <= cam.zfar
            else:
                expect = False
            assert bool(hits["hit"][k]) == expect, (i, j, k)
            if expect:
                assert abs(hits["t"][k] - t1) <= 1e-10 * t1
                checked += 1
    assert checked > 50


def test_pixel_convention_matches_intrinsics():
    """A sphere centred on the ray of pixel (i, j) built from K^-1 is hit at its
    centre (q = 0) at that pixel and nowhere outside its projected disc."""
    cam = sg.identity_camera(40, 30, focal=1.3, sensor_width=1.7)
    params = sg.Params(gamma=0.2, K=4)
    for (i, j) in [(0, 0), (29, 39), (14, 20), (3, 31)]:
        c = 6.0 * pixel_direction(cam, i, j)
        sc = types.SimpleNamespace(pos=c[None, :], radius=np.array([1e-3]),
                                   opacity=np.array([0.8]), payload=np.ones((1, 1)),
                                   bg=np.zeros(1))
        out = ref.forward(sc, cam, params)
        assert out["nhits"][i, j] == 1
        assert out["nhits"].sum() == 1  # 1e-3 at depth 6 is far below one pixel
        hits = ref.pixel_hits(sc, cam, params, i, j)
        assert hits["q"][0] < 1e-14


# ---------------------------------------------------------------- Eq. 1

@pytest.mark.parametrize("gamma", [1.0, 0.1, 1e-2, 1e-5])
def test_single_sphere_closed_form(gamma):
    """One sphere centred on a pixel ray: q = 0, d = 1, t = |c| - R, and Eq. 1
    reduces to F = (o e^{oz/g} f + e^{eps/g} bg) / (o e^{oz/g} + e^{eps/g})."""
    rng = np.random.default_rng(5)
    cam = sg.identity_camera(24, 20, focal=1.1, sensor_width=2.0, znear=1.0, zfar=12.0)
    Rq = random_rotation(rng)
    tq = rng.uniform(-2, 2, 3)
    cam.R, cam.t = Rq, tq
    i, j = 7, 11
    lam, rad, o = 4.0, 0.3, 0.7
    c = lam * pixel_direction(cam, i, j)
    p = Rq.T @ (c - tq)
    C = 3
    f = rng.standard_normal(C)
    bg = rng.standard_normal(C)
    eps = 1e-5
    sc = types.SimpleNamespace(pos=p[None, :], radius=np.array([rad]), opacity=np.array([o]),
                               payload=f[None, :], bg=bg)
    out = ref.forward(sc, cam, sg.Params(gamma=gamma, eps=eps, K=2))
    t = lam - rad
    z = (cam.zfar - t) / (cam.zfar - cam.znear)
    la, lb = math.log(o) + o * z / gamma, eps / gamma  # log weights of sphere and background
    M = max(la, lb)
    wa, wb = math.exp(la - M), math.exp(lb - M)
    F = (wa * f + wb * bg) / (wa + wb)
    L = M + math.log(wa + wb)
    np.testing.assert_allclose(out["F"][i, j], F, rtol=1e-13, atol=1e-13)
    assert abs(out["L"][i, j] - L) <= 1e-13 * abs(L)
    assert out["nhits"][i, j] == 1
    assert abs(out["klist_t"][i, j, 0] - t) <= 1e-13 * t


def test_empty_pixels_are_background():
    """With no hit, only the background weight exp(eps/gamma) remains: F = bg, L = eps/gamma."""
    wl = sg.config1()
    sc = as_f64(wl.scene)
    sc.bg = np.array([0.25, -0.5, 0.75])
    out = ref.forward(sc, wl.camera, wl.params)
    empty = out["nhits"] == 0
    assert empty.sum() > 1000
    assert np.array_equal(out["F"][empty], np.broadcast_to(sc.bg, (int(empty.sum()), 3)))
    assert np.all(out["L"][empty] == wl.params.eps / wl.params.gamma)


def test_hard_limit_selects_largest_opacity_depth():
    """gamma -> 1e-5: Eq. 1 becomes an argmax over o*z (not necessarily the nearest)."""
    wl = sg.tiny_scene(7, n=6, C=3, W=20, H=20, r_lo=0.3, r_hi=0.6)
    sc = as_f64(wl.scene)
    params = sg.Params(gamma=1e-5, eps=1e-5, K=8)
    out = ref.forward(sc, wl.camera, params)
    cam = wl.camera
    n_checked = 0
    for i in range(cam.height):
        for j in range(cam.width):
            hits = ref.pixel_hits(sc, cam, params, i, j)
            ks = np.nonzero(hits["hit"])[0]
            if len(ks) == 0:
                continue
            z = (cam.zfar - hits["t"][ks]) / (cam.zfar - cam.znear)
            oz = sc.opacity[ks] * z
            order = np.argsort(-oz)
            gap = oz[order[0]] - (oz[order[1]] if len(ks) > 1 else params.eps)
            if gap / params.gamma < 60:  # e^-60 ~ 1e-26 below: winner takes all
                continue
            win = ks[order[0]]
            np.testing.assert_allclose(out["F"][i, j], sc.payload[win], rtol=1e-12, atol=1e-12)
            n_checked += 1
    assert n_checked > 100


def test_soft_limit_is_smooth_average():
    """gamma = 1: exp(o z) stays within [1, e], so every hit keeps a share of
    at least o d / (e * sum) of the blend; F lies in the convex hull of the hit
    payloads and the background."""
    wl = sg.tiny_scene(8, n=6, C=1, W=16, H=16, r_lo=0.3, r_hi=0.6)
    sc = as_f64(wl.scene)
    params = sg.Params(gamma=1.0, eps=1e-5, K=8)
    out = ref.forward(sc, wl.camera, params)
    for i in range(16):
        for j in range(16):
            hits = ref.pixel_hits(sc, wl.camera, params, i, j)
            ks = np.nonzero(hits["hit"])[0]
            vals = np.concatenate([sc.payload[ks, 0], sc.bg])
            assert vals.min() - 1e-12 <= out["F"][i, j, 0] <= vals.max() + 1e-12


# ---------------------------------------------------------------- invariants

def test_permutation_invariance():
    """The blend is commutative in the sphere order (App. A)."""
    wl = sg.config1()
    sc = as_f64(wl.scene)
    perm = np.random.default_rng(3).permutation(sc.pos.shape[0])
    sp = types.SimpleNamespace(pos=sc.pos[perm], radius=sc.radius[perm],
                               opacity=sc.opacity[perm], payload=sc.payload[perm], bg=sc.bg)
    params = sg.Params(gamma=0.1, K=64)  # no truncation: gradients permute too
    a = ref.forward(sc, wl.camera, params)
    b = ref.forward(sp, wl.camera, params)
    np.testing.assert_allclose(b["F"], a["F"], rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(b["L"], a["L"], rtol=1e-14, atol=0)
    G = sg.upstream_grad(5, 64, 64, 3)
    ga = ref.backward(sc, wl.camera, params, G, a)
    gb = ref.backward(sp, wl.camera, params, G, b)
    for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload"]:
        ref_v = ga[key][perm]
        np.testing.assert_allclose(gb[key], ref_v, rtol=1e-9, atol=1e-12 * np.abs(ref_v).max())
    np.testing.assert_allclose(gb["grad_bg"], ga["grad_bg"], rtol=1e-12)


def test_spheres_that_cannot_be_seen_change_nothing():
    """Spheres behind the camera, beside the frustum, crossing the near plane or
    beyond the far plane leave F and L bitwise unchanged and get zero gradients;
    a zero-opacity sphere leaves F and L unchanged and only gets d/do."""
    wl = sg.tiny_scene(4, n=5, C=2)
    base = as_f64(wl.scene)
    params = sg.Params(gamma=0.3, K=16)
    extra_pos = np.array([[0.0, 0.0, -3.0],    # behind the camera
                          [50.0, 0.0, 4.0],    # beside the frustum
                          [0.1, 0.0, 1.1],     # crosses the near plane (c_z - R < near)
                          [0.0, 0.1, 12.0],    # entirely beyond far (t >= 11.5)
                          [0.05, -0.05, 3.5]])  # in view, opacity 0
    extra_r = np.array([0.5, 0.5, 0.3, 0.5, 0.4])
    extra_o = np.array([0.9, 0.9, 0.9, 0.9, 0.0])
    rng = np.random.default_rng(0)
    ext = types.SimpleNamespace(
        pos=np.concatenate([base.pos, extra_pos]), radius=np.concatenate([base.radius, extra_r]),
        opacity=np.concatenate([base.opacity, extra_o]),
        payload=np.concatenate([base.payload, rng.standard_normal((5, 2))]), bg=base.bg)
    a = ref.forward(base, wl.camera, params)
    b = ref.forward(ext, wl.camera, params)
    assert np.array_equal(a["F"], b["F"]) and np.array_equal(a["L"], b["L"])
    assert b["nhits"].sum() > a["nhits"].sum()  # the zero-opacity sphere is hit
    G = sg.upstream_grad(9, wl.camera.height, wl.camera.width, 2)
    ga = ref.backward(base, wl.camera, params, G, a)
    gb = ref.backward(ext, wl.camera, params, G, b)
    n = base.pos.shape[0]
    for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload"]:
        assert np.array_equal(gb[key][:n], ga[key])
        assert np.all(gb[key][n:n + 4] == 0.0)
    assert np.all(gb["grad_pos"][n + 4] == 0) and gb["grad_radius"][n + 4] == 0
    assert np.all(gb["grad_payload"][n + 4] == 0) and gb["grad_opacity"][n + 4] != 0
    assert np.array_equal(gb["grad_bg"], ga["grad_bg"])


def test_rigid_camera_motion_invariance():
    """Moving world and camera together changes nothing in the image."""
    rng = np.random.default_rng(21)
    wl = sg.tiny_scene(2, n=6, C=3)
    a = ref.forward(wl.scene, wl.camera, wl.params)
    sc, cam = _rotated_world(wl, rng)
    b = ref.forward(sc, cam, wl.params)
    np.testing.assert_allclose(b["F"], a["F"], rtol=1e-9, atol=1e-11)
    assert np.array_equal(a["nhits"], b["nhits"])


def test_klist_is_k_smallest_hits():
    """The gradient set is the K nearest hits in ascending (t, index) order."""
    wl = sg.tiny_scene(6, n=12, C=1, W=16, H=16, r_lo=0.3, r_hi=0.7)
    params = sg.Params(gamma=0.1, K=3)
    out = ref.forward(wl.scene, wl.camera, params)
    deep = 0
    for i in range(16):
        for j in range(16):
            h = ref.pixel_hits(wl.scene, wl.camera, params, i, j)
            ks = np.nonzero(h["hit"])[0]
            order = sorted(ks, key=lambda k: (h["t"][k], k))
            assert out["nhits"][i, j] == len(ks)
            want = list(order[:3]) + [-1] * (3 - min(3, len(ks)))
            assert list(out["klist_id"][i, j]) == want
            if len(ks) > 3:
                deep += 1
                assert out["t_next"][i, j] == h["t"][order[3]]
    assert deep > 10


# ---------------------------------------------------------------- gradients

def _assert_grads_close(an, fd, rtol, floor_frac=1e-4):
    for key, v in fd.items():
        if v is None:
            assert an[key] is None
            continue
        a = an[key]
        scale = max(np.abs(v).max(), 1e-300)
        err = np.abs(a - v)
        tol = rtol * np.maximum(np.abs(v), floor_frac * scale)
        assert np.all(err <= tol), (key, float((err / np.maximum(np.abs(v), floor_frac * scale)).max()))


@pytest.mark.parametrize("seed,with_opacity,rotate", [(1, True, False), (2, True, True),
                                                      (3, False, True)])
def test_gradients_match_finite_differences(seed, with_opacity, rotate):
    """Analytic gradients (K above the hit count: the exact derivative of Eq. 1)
    against FP64 central differences, world-space chain rule included."""
    wl = sg.tiny_scene(seed, n=5, C=2, with_opacity=with_opacity)
    if rotate:
        sc, cam = _rotated_world(wl, np.random.default_rng(seed))
    else:
        sc, cam = as_f64(wl.scene), wl.camera
    params = wl.params
    G = sg.upstream_grad(100 + seed, cam.height, cam.width, 2).astype(np.float64)
    fwd = ref.forward(sc, cam, params)
    assert fwd["nhits"].max() <= params.K
    an = ref.backward(sc, cam, params, G, fwd)
    fd = fd_grads(sc, cam, params, G)
    _assert_grads_close(an, fd, rtol=2e-6)


def test_minimum_size_gradients_match_finite_differences():
    """With the one-pixel minimum size on, clamped spheres take R = rho c_z / f:
    their radius gradient is zero and the depth picks up dR/dc_z."""
    wl = sg.tiny_scene(12, n=4, C=2, W=24, H=24, r_lo=0.02, r_hi=0.06)
    sc = as_f64(wl.scene)
    params = sg.Params(gamma=0.5, eps=1e-5, min_radius_px=2.5, K=8)
    fwd = ref.forward(sc, wl.camera, params)
    assert fwd["nhits"].sum() > 10
    G = sg.upstream_grad(7, 24, 24, 2).astype(np.float64)
    an = ref.backward(sc, wl.camera, params, G, fwd)
    pitch = wl.camera.sensor_width / wl.camera.width
    clamped = params.min_radius_px * pitch * sc.pos[:, 2] / wl.camera.focal > sc.radius
    assert clamped.any()
    assert np.all(an["grad_radius"][clamped] == 0)
    fd = fd_grads(sc, wl.camera, params, G)
    _assert_grads_close(an, fd, rtol=2e-6)


@pytest.mark.parametrize("seed,rotate,min_radius_px", [(1, False, 0.0), (2, True, 0.0),
                                                       (12, True, 2.5)])
def test_camera_gradients_match_finite_differences(seed, rotate, min_radius_px):
    """dLoss/d(R, t, f, s) against FP64 central differences of the forward
    with the camera perturbed (R entry by entry as a free matrix). The third
    case has clamped minimum-size spheres, whose radius follows f and s."""
    if min_radius_px > 0:
        wl = sg.tiny_scene(seed, n=4, C=2, W=24, H=24, r_lo=0.02, r_hi=0.06)
        params = sg.Params(gamma=0.5, eps=1e-5, min_radius_px=min_radius_px, K=8)
    else:
        wl = sg.tiny_scene(seed, n=5, C=2)
        params = wl.params
    if rotate:
        sc, cam = _rotated_world(wl, np.random.default_rng(seed))
    else:
        sc, cam = as_f64(wl.scene), wl.camera
    G = sg.upstream_grad(200 + seed, cam.height, cam.width, 2).astype(np.float64)
    fwd = ref.forward(sc, cam, params)
    assert fwd["nhits"].max() <= params.K and fwd["nhits"].sum() > 10
    an = ref.backward(sc, cam, params, G, fwd)["grad_camera"]
    fd = fd_camera_grads(sc, cam, params, G)
    scale = np.abs(fd).max()
    assert np.all(np.abs(an - fd) <= 2e-6 * np.maximum(np.abs(fd), 1e-4 * scale)), \
        (an.tolist(), fd.tolist())
    # the focal length and the sensor width act only through their ratio
    # (rays and the minimum-size radius): f df + s ds = 0
    assert abs(cam.focal * an[12] + cam.sensor_width * an[13]) <= 1e-9 * (
        abs(cam.focal * an[12]) + 1e-300)


def test_camera_gradient_parts_per_sphere_and_area_normalisation():
    """Each sphere's part of the camera gradient: with spheres whose images do
    not overlap, every pixel sees one sphere at most, so the loss is a sum of
    one term per sphere and sphere k's part equals the FP64 central
    differences of the camera for a scene holding sphere k alone (the parts
    also add up to the total). The paper-normalised camera gradient scales
    each part by 1e-3 over the sphere's projected disk area pi rpx^2 (App. B,
    normalisation of the camera gradients), rpx = R f / (c_z pitch), which
    the number of pixel centres the larger sphere covers confirms."""
    rng = np.random.default_rng(17)
    cam = sg.identity_camera(40, 36, focal=1.2, sensor_width=2.0)
    pitch = cam.sensor_width / cam.width
    # three spheres apart in the image, at different depths, one large
    pos = np.array([[-0.45, -0.35, 3.2], [0.5, 0.3, 4.5], [0.02, 0.03, 3.8]])
    radius = np.array([0.12, 0.09, 0.35])
    C = 2
    sc = types.SimpleNamespace(pos=pos, radius=radius, opacity=rng.uniform(0.4, 1.0, 3),
                               payload=rng.uniform(-1, 1, (3, C)), bg=np.array([0.1, -0.2]))
    params = sg.Params(gamma=0.4, eps=1e-5, K=4)
    fwd = ref.forward(sc, cam, params)
    assert fwd["nhits"].max() == 1  # no pixel sees two spheres
    G = sg.upstream_grad(18, cam.height, cam.width, C).astype(np.float64)
    g = ref.backward(sc, cam, params, G, fwd)
    parts = g["grad_camera_sphere"]
    np.testing.assert_allclose(parts.sum(0), g["grad_camera"], rtol=1e-12,
                               atol=1e-12 * np.abs(parts).sum())
    fd_parts = []
    for k in range(3):
        one = types.SimpleNamespace(pos=pos[k:k + 1], radius=radius[k:k + 1],
                                    opacity=sc.opacity[k:k + 1], payload=sc.payload[k:k + 1],
                                    bg=sc.bg)
        fd = fd_camera_grads(one, cam, params, G)
        scale = np.abs(fd).max()
        assert np.all(np.abs(parts[k] - fd) <= 2e-6 * np.maximum(np.abs(fd), 1e-4 * scale)), \
            (k, parts[k].tolist(), fd.tolist())
        fd_parts.append(fd)
    pn = ref.paper_normalised(sc, cam, params, fwd, g)
    rpx = pn["projected_radius_px"]
    np.testing.assert_allclose(rpx, radius * cam.focal / (pos[:, 2] * pitch), rtol=1e-12)
    covered = int(fwd["nhits"].sum())  # every hit pixel belongs to one sphere
    big = int(np.argmax(rpx))
    mask = np.zeros_like(fwd["nhits"], bool)
    for i in range(cam.height):
        for j in range(cam.width):
            mask[i, j] = ref.pixel_hits(sc, cam, params, i, j)["hit"][big]
    assert covered >= mask.sum() > 0
    assert abs(mask.sum() - np.pi * rpx[big] ** 2) <= 0.1 * np.pi * rpx[big] ** 2 + \
        2 * np.pi * rpx[big], (int(mask.sum()), rpx[big])
    want = sum(1e-3 / (np.pi * rpx[k] ** 2) * fd_parts[k] for k in range(3))
    scale = np.abs(want).max()
    assert np.all(np.abs(pn["grad_camera"] - want) <= 2e-6 * np.maximum(np.abs(want),
                                                                        1e-4 * scale))
    np.testing.assert_array_equal(pn["grad_bg"], g["grad_bg"])


def test_camera_pose_gradient_is_the_rotated_position_sum():
    """Moving the camera by dt moves every centre by dt in camera space, the
    same as moving every sphere by R^T dt: dLoss/dt = R sum_i dLoss/dp_i, and
    likewise dLoss/dR = sum_i (R dLoss/dp_i) p_i^T."""
    wl = sg.tiny_scene(4, n=6, C=2)
    sc, cam = _rotated_world(wl, np.random.default_rng(4))
    params = wl.params
    G = sg.upstream_grad(44, cam.height, cam.width, 2).astype(np.float64)
    g = ref.backward(sc, cam, params, G, ref.forward(sc, cam, params))
    R = np.asarray(cam.R, np.float64)
    gc = g["grad_pos"] @ R.T  # rows R dLoss/dp_i
    np.testing.assert_allclose(g["grad_camera"][9:12], gc.sum(0), rtol=1e-9,
                               atol=1e-12 * np.abs(gc).sum())
    np.testing.assert_allclose(g["grad_camera"][:9].reshape(3, 3), gc.T @ sc.pos, rtol=1e-9,
                               atol=1e-12 * np.abs(gc).sum())


def test_paper_normalisation_counts_and_gate():
    """The optimisation variant of the gradients: the pixel count of every
    sphere equals a brute-force count from per-pixel ray tests (its rank in
    (t, index) order below K), small spheres lose exactly their position and
    radius gradients, and the rest is the exact gradient over the count."""
    wl = sg.tiny_scene(21, n=8, C=2, W=32, H=32, r_lo=0.05, r_hi=0.5)
    sc, cam = as_f64(wl.scene), wl.camera
    params = sg.Params(gamma=0.3, eps=1e-5, K=3)
    fwd = ref.forward(sc, cam, params)
    G = sg.upstream_grad(55, 32, 32, 2).astype(np.float64)
    exact = ref.backward(sc, cam, params, G, fwd)
    pn = ref.paper_normalised(sc, cam, params, fwd, exact)
    n = sc.pos.shape[0]
    brute = np.zeros(n)
    for i in range(32):
        for j in range(32):
            h = ref.pixel_hits(sc, cam, params, i, j)
            ks = sorted(np.nonzero(h["hit"])[0], key=lambda k: (h["t"][k], k))[:params.K]
            brute[ks] += 1
    np.testing.assert_array_equal(pn["pixel_count"], brute)
    # projected radius against the pinhole intrinsics: f in pixels times R / c_z
    fpx = cam.focal * cam.width / cam.sensor_width
    np.testing.assert_allclose(pn["projected_radius_px"], fpx * sc.radius / sc.pos[:, 2],
                               rtol=1e-12)
    small = pn["projected_radius_px"] <= 3.0
    assert small.any() and (~small).any() and (brute > 1).any()
    seen = brute > 0
    for key in ["grad_opacity", "grad_payload"]:
        want = exact[key][seen] / (brute[seen][:, None] if exact[key].ndim == 2 else brute[seen])
        np.testing.assert_allclose(pn[key][seen], want, rtol=1e-12)
    assert np.all(pn["grad_pos"][small] == 0) and np.all(pn["grad_radius"][small] == 0)
    big = seen & ~small
    np.testing.assert_allclose(pn["grad_pos"][big], exact["grad_pos"][big] / brute[big][:, None],
                               rtol=1e-12)
    np.testing.assert_array_equal(pn["grad_bg"], exact["grad_bg"])


def _ortho_hits_numpy(sc, cam, reff):
    """Orthographic ray test written out in numpy, independent of the oracle:
    the ray of pixel (i, j) leaves (x_s, y_s, 0) along +z; it hits sphere k
    iff the centre lies less than R_k from the ray and the front intersection
    c_z - sqrt(R^2 - q^2) is at most zfar (with c_z - R >= znear). Returns
    hit [H, W, n] and t [H, W, n]."""
    pitch = cam.sensor_width / cam.width
    xs = (np.arange(cam.width) + 0.5) * pitch - 0.5 * cam.sensor_width
    ys = (np.arange(cam.height) + 0.5) * pitch - 0.5 * cam.sensor_width * cam.height / cam.width
    c = sc.pos @ np.asarray(cam.R, np.float64).reshape(3, 3).T + np.asarray(cam.t, np.float64)
    q2 = (c[None, None, :, 0] - xs[None, :, None]) ** 2 + \
        (c[None, None, :, 1] - ys[:, None, None]) ** 2
    inside = q2 < reff[None, None, :] ** 2
    t = c[None, None, :, 2] - np.sqrt(np.maximum(reff[None, None, :] ** 2 - q2, 0.0))
    seen = (c[:, 2] - reff >= cam.znear)[None, None, :]
    return inside & (t <= cam.zfar) & seen, t


@pytest.mark.parametrize("min_radius_px", [0.0, 2.5])
def test_paper_normalisation_orthographic(min_radius_px):
    """The optimisation variant under the orthographic projection: pixel
    counts equal a brute-force count over an independent numpy ray test, the
    projected radius is R / pitch at any depth (checked against the number of
    pixel centres a large sphere covers, about pi rpx^2), the minimum size is
    the constant min_radius_px pixels, and the 3-pixel gate and the averaging
    follow (Sec. 3.1 orthographic model; App. B normalisation; Sec. 3.2 gate)."""
    rng = np.random.default_rng(31)
    n, W, H, C = 9, 40, 36, 2
    cam = sg.identity_camera(W, H, focal=1.3)
    cam.orthographic = True
    pitch = cam.sensor_width / W
    # depths far apart, so a pinhole radius R f / (c_z pitch) would differ
    z = rng.uniform(2.0, 9.0, n)
    r = np.exp(rng.uniform(np.log(0.3 * pitch), np.log(7.0 * pitch), n))
    r[0] = 8.0 * pitch  # one sphere large enough to count its pixel centres
    r[1] = 0.2 * pitch  # one well below the minimum size when it is on
    xy = rng.uniform(-0.6, 0.6, (n, 2))
    xy[0] = [0.013, -0.021]
    sc = types.SimpleNamespace(pos=np.column_stack([xy, z]), radius=r,
                               opacity=rng.uniform(0.3, 1.0, n),
                               payload=rng.uniform(0, 1, (n, C)), bg=np.zeros(C))
    params = sg.Params(gamma=0.3, eps=1e-5, K=3, min_radius_px=min_radius_px)
    fwd = ref.forward(sc, cam, params)
    G = sg.upstream_grad(56, H, W, C).astype(np.float64)
    exact = ref.backward(sc, cam, params, G, fwd)
    pn = ref.paper_normalised(sc, cam, params, fwd, exact)
    reff = np.maximum(r, min_radius_px * pitch) if min_radius_px > 0 else r
    hit, t = _ortho_hits_numpy(sc, cam, reff)
    brute = np.zeros(n)
    for i in range(H):
        for j in range(W):
            ks = sorted(np.nonzero(hit[i, j])[0], key=lambda k: (t[i, j, k], k))[:params.K]
            brute[ks] += 1
    np.testing.assert_array_equal(pn["pixel_count"], brute)
    rpx = pn["projected_radius_px"]
    # the covered pixel centres of the big sphere: a lattice disk of radius rpx
    covered = hit[:, :, 0].sum()
    assert abs(covered - np.pi * rpx[0] ** 2) <= 2.0 * np.pi * rpx[0] + 1.0, (covered, rpx[0])
    # independent of depth and of the focal length, in pixel units
    np.testing.assert_allclose(rpx, reff * W / cam.sensor_width, rtol=1e-12)
    if min_radius_px > 0:
        assert rpx[1] == pytest.approx(min_radius_px, rel=1e-12)
    small = rpx <= 3.0
    assert small.any() and (~small).any()
    seen = brute > 0
    assert seen[0] and (brute > 1).any()
    for key in ["grad_opacity", "grad_payload"]:
        want = exact[key][seen] / (brute[seen][:, None] if exact[key].ndim == 2 else brute[seen])
        np.testing.assert_allclose(pn[key][seen], want, rtol=1e-12)
    assert np.all(pn["grad_pos"][small] == 0) and np.all(pn["grad_radius"][small] == 0)
    big = seen & ~small
    assert big.any()
    np.testing.assert_allclose(pn["grad_pos"][big], exact["grad_pos"][big] / brute[big][:, None],
                               rtol=1e-12)
    np.testing.assert_allclose(pn["grad_radius"][big], exact["grad_radius"][big] / brute[big],
                               rtol=1e-12)
    np.testing.assert_array_equal(pn["grad_bg"], exact["grad_bg"])


def test_paper_minimum_size_reaches_a_pixel_centre():
    """With min_radius_px = sqrt(2)/2 (the one-pixel rule of App. B, Step 0)
    every sphere far too small to be seen is still hit by at least one pixel
    ray: brute force over every pixel of a 24 x 24 image."""
    from paper_2004_07484_amd import _capi
    rng = np.random.default_rng(77)
    n = 40
    cam = sg.identity_camera(24, 24, focal=1.5)
    z = rng.uniform(2.0, 8.0, n)
    half = 0.5 * cam.sensor_width / cam.focal * 0.95  # inside the field of view
    sc = types.SimpleNamespace(
        pos=np.stack([rng.uniform(-half, half, n) * z, rng.uniform(-half, half, n) * z, z], 1),
        radius=np.full(n, 1e-5), opacity=None, payload=np.ones((n, 1)), bg=np.zeros(1))
    hit_any = np.zeros(n, bool)
    missed = np.zeros(n, bool)
    for mr, out in [(_capi.PULSAR_MIN_RADIUS_PX_PAPER, hit_any), (0.3, missed)]:
        params = sg.Params(gamma=0.5, eps=1e-5, min_radius_px=mr, K=4)
        for i in range(24):
            for j in range(24):
                out |= ref.pixel_hits(sc, cam, params, i, j)["hit"]
    assert hit_any.all()
    assert not missed.all()  # a smaller minimum loses some spheres between rays


def test_topk_blend_against_brute_force_and_derivative():
    """The top-K blend: (a) with K above every pixel's hit count it is the
    full blend; (b) per pixel it equals Eq. 1 written out over the K nearest
    hits of a brute-force ray test; (c) the backward, given its F and L, is
    its exact derivative (central differences; the scene has no pixel whose
    K nearest change under the step)."""
    wl = sg.tiny_scene(31, n=10, C=2, W=20, H=20, r_lo=0.3, r_hi=0.6)
    sc, cam = as_f64(wl.scene), wl.camera
    full = ref.forward(sc, cam, sg.Params(gamma=0.3, eps=1e-5, K=8))
    top8 = ref.forward(sc, cam, sg.Params(gamma=0.3, eps=1e-5, K=8), blend_topk=True)
    assert full["nhits"].max() <= 8
    np.testing.assert_array_equal(top8["F"], full["F"])
    params = sg.Params(gamma=0.3, eps=1e-5, K=2)
    top = ref.forward(sc, cam, params, blend_topk=True)
    assert top["nhits"].max() > 2
    for i in range(0, 20, 3):
        for j in range(0, 20, 3):
            h = ref.pixel_hits(sc, cam, params, i, j)
            ks = sorted(np.nonzero(h["hit"])[0], key=lambda k: (h["t"][k], k))[:params.K]
            z = (cam.zfar - h["t"][ks]) / (cam.zfar - cam.znear)
            o = sc.opacity[ks]
            w = o * (1.0 - h["q"][ks] / h["reff"][ks]) * np.exp(o * z / params.gamma)
            wb = np.exp(params.eps / params.gamma)
            F = (w @ sc.payload[ks] + wb * sc.bg) / (w.sum() + wb)
            np.testing.assert_allclose(top["F"][i, j], F, rtol=1e-12, atol=1e-14)
    G = sg.upstream_grad(66, 20, 20, 2).astype(np.float64)
    an = ref.backward(sc, cam, params, G, top)
    def loss_topk(s):
        return float(np.sum(G * ref.forward(s, cam, params, blend_topk=True)["F"]))
    for field, gname in [("pos", "grad_pos"), ("radius", "grad_radius"),
                         ("opacity", "grad_opacity"), ("payload", "grad_payload")]:
        base = getattr(sc, field)
        fd = np.zeros_like(base)
        for idx in np.ndindex(base.shape):
            x = base[idx]
            hstep = 1e-6 * max(1.0, abs(x))
            sp, sm = copy.deepcopy(sc), copy.deepcopy(sc)
            getattr(sp, field)[idx] = x + hstep
            getattr(sm, field)[idx] = x - hstep
            fd[idx] = (loss_topk(sp) - loss_topk(sm)) / (2 * hstep)
        scale = np.abs(fd).max()
        np.testing.assert_allclose(an[gname], fd, rtol=2e-6, atol=1e-5 * scale)


def _ortho(wl):
    cam = copy.deepcopy(wl.camera)
    cam.orthographic = True
    return cam


def test_orthographic_rays_closed_form_and_shift():
    """Orthographic projection (Sec. 3.1): the ray of pixel (i, j) starts at
    its centre on the sensor plane and runs along +z, so a sphere's hit is
    t = c_z - sqrt(R^2 - q^2) with q its distance in x, y from the pixel
    centre, the covered pixels do not depend on depth, and moving every
    sphere by a whole number of pixels in x shifts the image by as many."""
    wl = sg.tiny_scene(41, n=6, C=2, W=32, H=32, r_lo=0.1, r_hi=0.3)
    sc, cam = as_f64(wl.scene), _ortho(wl)
    params = sg.Params(gamma=0.4, eps=1e-5, K=8)
    pitch = cam.sensor_width / cam.width
    for (i, j) in [(5, 7), (16, 16), (20, 11)]:
        h = ref.pixel_hits(sc, cam, params, i, j)
        xs = (j + 0.5) * pitch - cam.sensor_width / 2
        ys = (i + 0.5) * pitch - cam.sensor_width * cam.height / cam.width / 2
        q = np.hypot(sc.pos[:, 0] - xs, sc.pos[:, 1] - ys)
        want = q < sc.radius
        np.testing.assert_array_equal(h["hit"], want)
        np.testing.assert_allclose(h["t"][want], sc.pos[want, 2] -
                                   np.sqrt(sc.radius[want] ** 2 - q[want] ** 2), rtol=1e-13)
    base = ref.forward(sc, cam, params)
    assert base["nhits"].max() >= 2
    deeper = copy.deepcopy(sc)
    deeper.pos[:, 2] += 1.5
    np.testing.assert_array_equal(ref.forward(deeper, cam, params)["nhits"], base["nhits"])
    moved = copy.deepcopy(sc)
    moved.pos[:, 0] += 3 * pitch
    F = ref.forward(moved, cam, params)["F"]
    np.testing.assert_allclose(F[:, 3:], base["F"][:, :-3], rtol=1e-9, atol=1e-12)


def test_orthographic_gradients_match_finite_differences():
    wl = sg.tiny_scene(42, n=5, C=2, W=24, H=24, r_lo=0.15, r_hi=0.4)
    sc, cam = as_f64(wl.scene), _ortho(wl)
    for params in [wl.params, sg.Params(gamma=0.5, eps=1e-5, min_radius_px=2.5, K=8)]:
        G = sg.upstream_grad(43, cam.height, cam.width, 2).astype(np.float64)
        fwd = ref.forward(sc, cam, params)
        assert fwd["nhits"].max() <= params.K and fwd["nhits"].sum() > 10
        an = ref.backward(sc, cam, params, G, fwd)
        _assert_grads_close(an, fd_grads(sc, cam, params, G), rtol=2e-6)


def test_truncated_gradient_is_masked_derivative():
    """With K below the hit count, sphere j's gradient is the derivative of
    sum over pixels where j is among the K nearest of G * F (App. B, Step 2):
    central differences with G masked per sphere. The background gradient is
    not truncated."""
    wl = sg.tiny_scene(9, n=6, C=2, W=20, H=20, r_lo=0.35, r_hi=0.7)
    sc = as_f64(wl.scene)
    params = sg.Params(gamma=0.3, eps=1e-5, K=2)
    fwd = ref.forward(sc, wl.camera, params)
    assert fwd["nhits"].max() > params.K
    G = sg.upstream_grad(31, 20, 20, 2).astype(np.float64)
    an = ref.backward(sc, wl.camera, params, G, fwd)
    n = sc.pos.shape[0]
    for jsph in range(n):
        member = np.any(fwd["klist_id"] == jsph, axis=2)
        Gj = G * member[:, :, None]
        fd = fd_grads(sc, wl.camera, params, Gj,
                      which=lambda name, idx, j=jsph: name != "grad_bg" and idx[0] == j)
        for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload"]:
            v, a = fd[key][jsph], an[key][jsph]
            np.testing.assert_allclose(a, v, rtol=2e-6, atol=2e-6 * np.abs(an[key]).max())
    fdb = fd_grads(sc, wl.camera, params, G, which=lambda name, idx: name == "grad_bg")
    np.testing.assert_allclose(an["grad_bg"], fdb["grad_bg"], rtol=2e-6)


def test_row_subset_matches_full_frame():
    """Row subsets evaluate exactly the same pixels, and the subset backward is
    the backward of the full frame with G zero off the subset."""
    wl = sg.tiny_scene(13, n=8, C=2, W=20, H=18)
    full = ref.forward(wl.scene, wl.camera, wl.params)
    rows = [0, 5, 6, 17]
    sub = ref.forward(wl.scene, wl.camera, wl.params, rows=rows)
    assert np.array_equal(sub["F"][rows], full["F"][rows])
    assert np.array_equal(sub["L"][rows], full["L"][rows])
    G = sg.upstream_grad(3, 18, 20, 2)
    Gm = np.zeros_like(G)
    Gm[rows] = G[rows]
    a = ref.backward(wl.scene, wl.camera, wl.params, G, sub, rows=rows)
    b = ref.backward(wl.scene, wl.camera, wl.params, Gm, full)
    for key in a:
        np.testing.assert_allclose(a[key], b[key], rtol=1e-12, atol=1e-14)


def test_negative_opacity_is_rejected():
    wl = sg.tiny_scene(1, n=3)
    sc = as_f64(wl.scene)
    sc.opacity[1] = -0.1
    with pytest.raises(ValueError):
        ref.forward(sc, wl.camera, wl.params)


def test_exact_depth_ties_break_by_sphere_index():
    """Coincident spheres tie exactly in t; the K-list then orders them by
    index (the tie-break reading)."""
    wl = sg.tiny_scene(14, n=4, C=2, W=16, H=16)
    sc = as_f64(wl.scene)
    dup = types.SimpleNamespace(
        pos=np.concatenate([sc.pos[2:3], sc.pos]), radius=np.concatenate([sc.radius[2:3], sc.radius]),
        opacity=np.concatenate([sc.opacity[2:3], sc.opacity]),
        payload=np.concatenate([sc.payload[2:3] + 1.0, sc.payload]), bg=sc.bg)
    params = sg.Params(gamma=0.3, K=6)
    out = ref.forward(dup, wl.camera, params)
    both = 0
    for i in range(16):
        for j in range(16):
            h = ref.pixel_hits(dup, wl.camera, params, i, j)
            if h["hit"][0]:
                assert h["hit"][3] and h["t"][0] == h["t"][3]
                ids = list(out["klist_id"][i, j])
                assert ids.index(0) + 1 == ids.index(3)
                both += 1
    assert both > 3


# ---------------------------------------------------------------- early stop

def _early_stop_brute(sc, cam, gamma, eps, s):
    """Early stop written out with numpy, independent of the oracle: per
    pixel the pinhole ray test, the hits ordered by (float32(|c| - R), index),
    and the walk that stops at the first hit whose largest possible weight
    exp(z(|c| - R) / gamma) is below s / (1 - s) of the running denominator.
    Returns F, L, the blended count and, per pixel, the exact weights and
    shares of the skipped hits."""
    H, W = cam.height, cam.width
    C = sc.payload.shape[1]
    pitch = cam.sensor_width / W
    c = np.asarray(sc.pos, np.float64)  # identity camera
    R = np.asarray(sc.radius, np.float64)
    o = np.asarray(sc.opacity, np.float64)
    tmin = (np.linalg.norm(c, axis=1) - R).astype(np.float32)
    span = cam.zfar - cam.znear
    F = np.zeros((H, W, C))
    L = np.zeros((H, W))
    nb = np.zeros((H, W), int)
    skipped = []
    for i in range(H):
        for j in range(W):
            v = np.array([(j + 0.5) * pitch - cam.sensor_width / 2,
                          (i + 0.5) * pitch - cam.sensor_width * H / W / 2, cam.focal])
            u = v / np.linalg.norm(v)
            b = c @ u
            q = np.sqrt(np.maximum((c * c).sum(1) - b * b, 0.0))
            t = b - np.sqrt(np.maximum(R * R - q * q, 0.0))
            hit = (q < R) & (t <= cam.zfar) & (c[:, 2] - R >= cam.znear)
            ks = sorted(np.nonzero(hit)[0], key=lambda k: (tmin[k], k))
            lw = np.log(o * np.maximum(1 - q / R, 1e-300)) + o * (cam.zfar - t) / span / gamma
            logs = [eps / gamma]
            used = []
            for k in ks:
                bound = (cam.zfar - float(tmin[k])) / span / gamma
                if bound < np.log(s / (1 - s)) + np.logaddexp.reduce(logs):
                    break
                logs.append(lw[k])
                used.append(k)
            Lp = np.logaddexp.reduce(logs)
            w = np.exp(np.array(logs) - Lp)
            F[i, j] = w[0] * sc.bg + (w[1:, None] * sc.payload[used]).sum(0)
            L[i, j] = Lp
            nb[i, j] = len(used)
            rest = [k for k in ks if k not in used]
            skipped.append([(np.exp(lw[k]), np.exp(lw[k]) / (np.exp(Lp) + np.exp(lw[k])))
                            for k in rest])
    return F, L, nb, skipped


def _early_stop_scene():
    """Spheres stacked in depth over one image region, so near ones dominate
    and far ones fall below the share."""
    rng = np.random.default_rng(41)
    n = 30
    z = rng.uniform(2.0, 9.0, n)
    xy = rng.uniform(-0.2, 0.2, (n, 2)) * z[:, None] / 3.0
    sc = types.SimpleNamespace(pos=np.column_stack([xy, z]),
                               radius=rng.uniform(0.3, 0.6, n) * z / 3.0,
                               opacity=rng.uniform(0.5, 1.0, n),
                               payload=rng.standard_normal((n, 2)), bg=np.array([0.2, -0.3]))
    cam = sg.identity_camera(20, 18, focal=2.0)
    return sc, cam


def test_early_stop_matches_brute_force_and_bounds_the_skipped_share():
    """Sec. 3.2 / App. B early stop: the oracle equals an independent brute
    force (image, log-normaliser, blended counts), and every skipped hit's
    share of its pixel, w / (D + w) with D the final denominator, is below
    the threshold: no farther sphere could have reached it."""
    sc, cam = _early_stop_scene()
    s = 0.03
    params = sg.Params(gamma=0.08, eps=1e-5, K=20, stop_share=s)
    out = ref.forward(sc, cam, params)
    F, L, nb, skipped = _early_stop_brute(sc, cam, params.gamma, params.eps, s)
    np.testing.assert_allclose(out["F"], F, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["L"], L, rtol=1e-12)
    np.testing.assert_array_equal(out["nhits"], nb)
    shares = [sh for px in skipped for _, sh in px]
    assert len(shares) > 50  # the stop happens, and often
    assert max(shares) < s
    exact = ref.forward(sc, cam, sg.Params(gamma=0.08, eps=1e-5, K=20))
    assert (exact["nhits"] > out["nhits"]).sum() > 20
    # a share of zero keeps every hit: exactly the plain blend
    zero = ref.forward(sc, cam, sg.Params(gamma=0.08, eps=1e-5, K=20, stop_share=0.0))
    assert np.array_equal(zero["F"], exact["F"]) and np.array_equal(zero["L"], exact["L"])


def test_early_stop_gradients_match_finite_differences():
    """With the stop decisions fixed (pixels near a decision carry no
    upstream gradient), the backward over the blended hits is the derivative
    of the early-stopped image: FP64 central differences."""
    sc, cam = _early_stop_scene()
    params = sg.Params(gamma=0.08, eps=1e-5, K=20, stop_share=0.03)
    fwd = ref.forward(sc, cam, params)
    G = sg.upstream_grad(43, cam.height, cam.width, 2).astype(np.float64)
    G[fwd["ambiguous"]] = 0.0
    an = ref.backward(sc, cam, params, G, fwd)
    fd = fd_grads(sc, cam, params, G)
    _assert_grads_close(an, fd, rtol=1e-5, floor_frac=1e-3)
