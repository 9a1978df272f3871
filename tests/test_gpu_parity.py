"""Parity of the HIP renderer (through the C ABI) with the FP64 oracle.

Images: |d| <= 1e-4 max(|ref|, 1e-2 max|ref|). Gradients: 1e-3 on the same
scale. Upstream gradients are zero on pixels whose K nearest hits the oracle
flags as rounding-sensitive, and off the evaluated rows for large workloads.
"""
import sys
import types

import numpy as np
import pytest

from oracle import reference as ref
from paper_2004_07484_amd import _capi
from paper_2004_07484_amd import scenegen as sg
from tests.gpu_helpers import (GRAD_REL, IMAGE_REL, assert_close, compare_grads, gpu_render,
                               masked_G)

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _parity(wl, rows=None, G_seed=1000, what="", grads=True, max_pairs=0, knobs=None,
            oracle=None):
    """GPU (C ABI) against the oracle on wl; `knobs` are launch knobs
    (chunk, raster_blocks); `oracle` is a cached (fwd, G, grads)."""
    sc, cam, par = wl.scene, wl.camera, wl.params
    knobs = knobs or {}
    _say(f"[parity] {what} n={sc.n} {cam.width}x{cam.height} C={sc.C} K={par.K} rows="
         f"{None if rows is None else len(rows)} knobs={knobs}")
    if oracle is None:
        fwd = ref.forward(sc, cam, par, rows=rows)
        G = sg.upstream_grad(wl.seed + G_seed, cam.height, cam.width, sc.C)
        Gm = masked_G(G, rows, fwd["ambiguous"])
        g = ref.backward(sc, cam, par, Gm, fwd, rows=rows) if grads else None
    else:
        fwd, Gm, g = oracle
    out = gpu_render(sc, cam, par, Gm if grads else None, max_pairs=max_pairs, **knobs)
    assert out["status"] == _capi.PULSAR_OK
    sel = slice(None) if rows is None else rows
    assert_close(out["F"][sel], fwd["F"][sel], IMAGE_REL, f"{what} image")
    assert_close(out["L"][sel], fwd["L"][sel], IMAGE_REL, f"{what} log-normaliser")
    if grads:
        compare_grads(out, g, what)
    return fwd, out


def test_config1_full_frame():
    _parity(sg.config1(), what="1k spheres 64x64")


def test_config2_row_subset():
    wl = sg.config2()
    rows = sorted(np.random.default_rng(77).choice(512, 12, replace=False).tolist())
    _parity(wl, rows=rows, what="100k spheres 512x512")


_CFG3 = {}


def _config3_oracle():
    """1M spheres at 1024x1024 (C=8, K=8) on 6 seeded rows: the oracle's
    forward and gradients, computed once for every launch configuration."""
    if not _CFG3:
        wl = sg.config3()
        rows = sorted(np.random.default_rng(78).choice(1024, 6, replace=False).tolist())
        fwd = ref.forward(wl.scene, wl.camera, wl.params, rows=rows)
        G = sg.upstream_grad(wl.seed + 1000, wl.camera.height, wl.camera.width, wl.scene.C)
        Gm = masked_G(G, rows, fwd["ambiguous"])
        g = ref.backward(wl.scene, wl.camera, wl.params, Gm, fwd, rows=rows)
        _CFG3.update(wl=wl, rows=rows, oracle=(fwd, Gm, g))
    return _CFG3


# the default launch and every configuration the autotuner can pick at this
# workload, the benchmark's among them (knob ranges of autotune.KNOBS)
@pytest.mark.parametrize("knobs", [
    {}, dict(chunk=192, raster_blocks=16384), dict(chunk=256, raster_blocks=16384),
    dict(chunk=320, raster_blocks=16384), dict(chunk=512, raster_blocks=16384),
    dict(chunk=64, raster_blocks=1024), dict(chunk=256, raster_blocks=8192)])
def test_config3_full_size_row_subset(knobs):
    """1M spheres at 1024x1024, C=8, K=8: the benchmark workload, in the
    default launch configuration and the tuned ones, checked on 6 seeded rows
    (G zero elsewhere)."""
    c = _config3_oracle()
    fwd, out = _parity(c["wl"], rows=c["rows"], what="1M blobs 1024x1024", knobs=knobs,
                       oracle=c["oracle"])
    assert np.isfinite(out["F"]).all()


TILES = dict(fwd_flags=_capi.PULSAR_BWD_TILES, bwd_flags=_capi.PULSAR_BWD_TILES)


@pytest.mark.parametrize("case", ["config1", "config2_rows", "config3_rows", "rotated",
                                  "min_radius_K1", "ragged_split"])
def test_tile_order_backward(case):
    """The backward that walks the tile lists (PULSAR_BWD_TILES) against the
    oracle, like the default walk in sphere order."""
    if case == "config1":
        _parity(sg.config1(), what="tiles: 1k spheres", knobs=TILES)
    elif case == "config2_rows":
        rows = sorted(np.random.default_rng(79).choice(512, 8, replace=False).tolist())
        _parity(sg.config2(), rows=rows, what="tiles: 100k spheres", knobs=TILES)
    elif case == "config3_rows":
        c = _config3_oracle()
        _parity(c["wl"], rows=c["rows"], what="tiles: 1M blobs", oracle=c["oracle"],
                knobs=dict(chunk=256, raster_blocks=16384, **TILES))
    else:
        kw = dict(n=40, C=3, W=40, H=32, r_lo=0.05, r_hi=0.4)
        if case == "ragged_split":
            kw.update(n=400, W=37, H=29)
        wl = sg.tiny_scene(131 + len(case), **kw)
        wl.params = sg.Params(gamma=0.2, eps=1e-5, K=1 if case == "min_radius_K1" else 5,
                              min_radius_px=2.0 if case == "min_radius_K1" else 0.0)
        if case == "rotated":
            rng = np.random.default_rng(9)
            q, r = np.linalg.qr(rng.standard_normal((3, 3)))
            q = q * np.sign(np.diag(r))
            if np.linalg.det(q) < 0:
                q[:, 0] = -q[:, 0]
            tq = rng.uniform(-1, 1, 3)
            wl.scene.pos = ((wl.scene.pos.astype(np.float64) - tq) @ q).astype(np.float32)
            wl.camera.R, wl.camera.t = q.astype(np.float32), tq.astype(np.float32)
        knobs = dict(TILES)
        if case == "ragged_split":
            knobs.update(chunk=64)
        _parity(wl, what=f"tiles: {case}", knobs=knobs)


def test_large_spheres_take_the_tile_walk():
    """Spheres wider than 16 tiles (their pixels would all fall to one wave
    of the walk in sphere order): the default backward takes the walk over
    the tile lists, decided on the device, so it gives bit for bit what
    asking for that walk gives, and the oracle's gradients."""
    wl = sg.tiny_scene(141, n=30, C=3, W=96, H=80, r_lo=0.3, r_hi=0.9)
    wl.params = sg.Params(gamma=0.3, eps=1e-5, K=6)
    sc, cam, par = wl.scene, wl.camera, wl.params
    _say("[parity] large spheres (up to 11x11 tiles), default vs tile-order backward")
    fwd = ref.forward(sc, cam, par)
    G = masked_G(sg.upstream_grad(1411, cam.height, cam.width, sc.C), None, fwd["ambiguous"])
    g = ref.backward(sc, cam, par, G, fwd)
    a = gpu_render(sc, cam, par, G)
    b = gpu_render(sc, cam, par, G, **TILES)
    assert a["status"] == _capi.PULSAR_OK and b["status"] == _capi.PULSAR_OK
    assert_close(a["F"], fwd["F"], IMAGE_REL, "large spheres image")
    compare_grads(a, g, "large spheres")
    for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
        assert np.array_equal(a[key], b[key]), key


def test_sphere_and_tile_order_backwards_agree():
    """Both backward walks compute the same per-(pixel, sphere) terms and only
    add them in another order: on the 100k-sphere workload (every pixel) they
    agree to float32 summation error, and the images are identical."""
    wl = sg.config2()
    sc, cam, par = wl.scene, wl.camera, wl.params
    G = sg.upstream_grad(wl.seed + 1000, cam.height, cam.width, sc.C)
    _say("[parity] sphere-order vs tile-order backward, 100k spheres")
    a = gpu_render(sc, cam, par, G)
    b = gpu_render(sc, cam, par, G, **TILES)
    assert np.array_equal(a["F"], b["F"]) and np.array_equal(a["L"], b["L"])
    for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
        assert_close(a[key], b[key], 1e-4, f"sphere vs tile order {key}")


@pytest.mark.parametrize("case", ["truncated_K2", "K1", "K32", "no_opacity", "rotated",
                                  "ragged", "one_channel", "forty_channels", "min_radius"])
def test_small_scene_variants(case):
    kw = dict(n=12, C=3, W=40, H=32, r_lo=0.2, r_hi=0.6)
    if case == "ragged":
        kw.update(W=37, H=29)
    if case == "one_channel":
        kw.update(C=1)
    if case == "forty_channels":
        kw.update(C=40)
    if case == "no_opacity":
        kw.update(with_opacity=False)
    if case == "min_radius":
        kw.update(r_lo=0.01, r_hi=0.05, n=30)
    wl = sg.tiny_scene(101 + len(case), **kw)
    wl.params = sg.Params(gamma=0.2, eps=1e-5, K={"truncated_K2": 2, "K1": 1, "K32": 32}.get(
        case, 5), min_radius_px=2.0 if case == "min_radius" else 0.0)
    if case == "rotated":
        rng = np.random.default_rng(5)
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        tq = rng.uniform(-1, 1, 3)
        sc = wl.scene
        sc.pos = ((sc.pos.astype(np.float64) - tq) @ q).astype(np.float32)
        wl.camera.R = q.astype(np.float32)
        wl.camera.t = tq.astype(np.float32)
    fwd, _ = _parity(wl, what=case)
    if case in ("truncated_K2", "K1"):
        assert fwd["nhits"].max() > wl.params.K  # the truncation is exercised


@pytest.mark.parametrize("K", [3, 5, 8, 13])
def test_dense_tiles_with_short_klists(K):
    """Tiles split into several work items whose K-lists are merged, with K
    below the register list size (fixed leading entries) and at it: the
    merged K-th nearest hit must be that of one pass over the whole list."""
    wl = sg.config1()
    sc = wl.scene
    sc.radius = (sc.radius * 8.0).astype(np.float32)
    par = sg.Params(gamma=0.1, eps=1e-5, K=K)
    cam = wl.camera
    _say(f"[parity] dense tiles K={K} chunk=64")
    fwd = ref.forward(sc, cam, par)
    assert fwd["nhits"].max() > 64  # several work items per tile
    G = sg.upstream_grad(300 + K, cam.height, cam.width, sc.C)
    Gm = masked_G(G, None, fwd["ambiguous"])
    out = gpu_render(sc, cam, par, Gm, chunk=64)
    assert out["status"] == _capi.PULSAR_OK
    assert_close(out["F"], fwd["F"], IMAGE_REL, "dense image")
    g = ref.backward(sc, cam, par, Gm, fwd)
    compare_grads(out, g, f"dense K={K}")


def test_near_plane_deep_stack():
    """Large spheres whose nearest points sit just beyond the near plane,
    stacked deep with a small K: the backward skips a sphere at pixels whose
    K-th nearest hit lies before the sphere's nearest point (|c| - R, lowered
    by a margin), and that skip must never drop a gradient, also where |c| - R
    is small against |c|."""
    rng = np.random.default_rng(77)
    n, C = 40, 3
    r = rng.uniform(0.15, 0.5, n)
    z = 1.0 + r + rng.uniform(1e-4, 0.3, n)  # nearest point just past znear = 1
    x = rng.uniform(-0.4, 0.4, n)
    y = rng.uniform(-0.3, 0.3, n)
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    sc = sg.Scene(pos=f32(np.stack([x, y, z], 1)), radius=f32(r),
                  opacity=f32(rng.uniform(0.3, 1.0, n)), payload=f32(rng.standard_normal((n, C))),
                  bg=f32(rng.uniform(-0.5, 0.5, C)))
    wl = sg.Workload("near_stack", sc, sg.identity_camera(48, 40, focal=1.0),
                     sg.Params(gamma=0.3, eps=1e-5, K=3), 77)
    fwd, _ = _parity(wl, what="near-plane deep stack")
    assert fwd["nhits"].max() > 3 * wl.params.K  # deep pixels: most hits lie behind the K-th


def test_many_tiles_per_sphere():
    """Spheres covering dozens of tiles, deep pixels, several sort blocks."""
    wl = sg.tiny_scene(55, n=300, C=4, W=160, H=120, r_lo=0.05, r_hi=0.4)
    wl.params = sg.Params(gamma=0.1, K=6)
    fwd, out = _parity(wl, what="large spheres 160x120")
    assert out["pairs"] > 3000


def test_hard_blend_limit():
    """gamma = 1e-5: pixels with a clear winner in o z show its payload."""
    wl = sg.tiny_scene(7, n=10, C=3, W=32, H=32, r_lo=0.3, r_hi=0.6)
    wl.params = sg.Params(gamma=1e-5, eps=1e-5, K=4)
    fwd = ref.forward(wl.scene, wl.camera, wl.params)
    out = gpu_render(wl.scene, wl.camera, wl.params)
    checked = 0
    for i in range(32):
        for j in range(32):
            h = ref.pixel_hits(wl.scene, wl.camera, wl.params, i, j)
            ks = np.nonzero(h["hit"])[0]
            if len(ks) == 0:
                continue
            z = (wl.camera.zfar - h["t"][ks]) / (wl.camera.zfar - wl.camera.znear)
            oz = np.sort(wl.scene.opacity[ks].astype(np.float64) * z)[::-1]
            if len(ks) > 1 and (oz[0] - oz[1]) / 1e-5 < 200:
                continue
            np.testing.assert_allclose(out["F"][i, j], fwd["F"][i, j], rtol=1e-4, atol=1e-5)
            checked += 1
    assert checked > 100


def test_empty_scene_is_background():
    cam = sg.identity_camera(24, 20)
    sc = sg.Scene(pos=np.zeros((0, 3), np.float32), radius=np.zeros(0, np.float32),
                  opacity=np.zeros(0, np.float32), payload=np.zeros((0, 2), np.float32),
                  bg=np.array([0.5, -2.0], np.float32))
    par = sg.Params(gamma=0.1, K=3)
    G = sg.upstream_grad(3, 20, 24, 2)
    out = gpu_render(sc, cam, par, G)
    assert np.array_equal(out["F"], np.broadcast_to(sc.bg, (20, 24, 2)))
    np.testing.assert_allclose(out["L"], 1e-4, rtol=1e-6)
    np.testing.assert_allclose(out["grad_bg"], G.astype(np.float64).sum((0, 1)), rtol=1e-5)


def test_invisible_spheres_change_nothing():
    wl = sg.config1()
    base = gpu_render(wl.scene, wl.camera, wl.params, sg.upstream_grad(5, 64, 64, 3))
    sc = wl.scene
    extra = np.array([[0, 0, -3], [50, 0, 4], [0.1, 0, 1.1], [0, 0.1, 12.0]], np.float32)
    ext = sg.Scene(pos=np.concatenate([sc.pos, extra]),
                   radius=np.concatenate([sc.radius, np.array([0.5, 0.5, 0.3, 0.5], np.float32)]),
                   opacity=np.concatenate([sc.opacity, np.full(4, 0.9, np.float32)]),
                   payload=np.concatenate([sc.payload, np.ones((4, 3), np.float32)]), bg=sc.bg)
    nan_sphere = sg.Scene(pos=np.concatenate([ext.pos, np.array([[np.nan, 0, 4]], np.float32)]),
                          radius=np.concatenate([ext.radius, np.array([0.5], np.float32)]),
                          opacity=np.concatenate([ext.opacity, np.array([0.5], np.float32)]),
                          payload=np.concatenate([ext.payload, np.ones((1, 3), np.float32)]),
                          bg=sc.bg)
    got = gpu_render(nan_sphere, wl.camera, wl.params, sg.upstream_grad(5, 64, 64, 3))
    assert np.array_equal(got["F"], base["F"]) and np.array_equal(got["L"], base["L"])
    assert got["pairs"] == base["pairs"]
    for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload"]:
        assert np.all(got[key][1000:] == 0.0)


def test_forward_is_deterministic_and_permutation_invariant():
    wl = sg.config1()
    a = gpu_render(wl.scene, wl.camera, wl.params)
    b = gpu_render(wl.scene, wl.camera, wl.params)
    assert np.array_equal(a["F"], b["F"]) and np.array_equal(a["L"], b["L"])
    perm = np.random.default_rng(9).permutation(wl.scene.n)
    sc = wl.scene
    sp = sg.Scene(pos=sc.pos[perm], radius=sc.radius[perm], opacity=sc.opacity[perm],
                  payload=sc.payload[perm], bg=sc.bg)
    c = gpu_render(sp, wl.camera, wl.params)
    assert_close(c["F"], a["F"], 1e-5, "permuted image")


def test_backward_is_bitwise_reproducible():
    """With C <= 32 every gradient is summed in a fixed order (per-pair slots
    added per sphere in emission order, background block sums in block
    order), so two runs agree bit for bit."""
    wl = sg.config1()
    G = sg.upstream_grad(4, 64, 64, 3)
    a = gpu_render(wl.scene, wl.camera, wl.params, G)
    b = gpu_render(wl.scene, wl.camera, wl.params, G, raster_blocks=1024)
    for key in ["F", "L", "grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
        assert np.array_equal(a[key], b[key], equal_nan=False), key


@pytest.mark.parametrize("make", [sg.config1, sg.config2])
def test_rebin_backward_on_another_workspace(make):
    """A forward with PULSAR_NO_BWD_AUX writes the same image and
    log-normaliser as one that keeps its backward state; a backward with
    PULSAR_REBIN on another workspace, whose bytes an unrelated render left
    behind, gives bitwise the gradients of the backward that reuses the
    forward's workspace."""
    import torch
    wl = make()
    cam = wl.camera
    _say(f"[rebin] {wl.name}")
    G = sg.upstream_grad(wl.seed + 77, cam.height, cam.width, wl.scene.C)
    a = gpu_render(wl.scene, cam, wl.params, G)
    # fewer spheres, same image and parameters: fits the same workspace size
    other = sg.box_scene(np.random.default_rng(99), wl.scene.n // 2, wl.scene.C, 0.002, 0.03)

    def dirty(ws):
        fresh = torch.full_like(ws, 0xA5)
        # an unrelated scene's forward and backward on the new workspace
        r = gpu_render(other, cam, wl.params, np.ones((cam.height, cam.width, wl.scene.C),
                                                      np.float32), workspace=fresh)
        assert r["status"] == _capi.PULSAR_OK
        return fresh

    b = gpu_render(wl.scene, cam, wl.params, G, fwd_flags=_capi.PULSAR_NO_BWD_AUX,
                   bwd_flags=_capi.PULSAR_NO_BWD_AUX | _capi.PULSAR_REBIN, bwd_workspace=dirty)
    assert a["status"] == _capi.PULSAR_OK and b["status"] == _capi.PULSAR_OK
    for key in ["F", "L", "grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
        assert np.array_equal(a[key], b[key]), key


def test_capacity_overflow_is_reported_then_recovers():
    wl = sg.config1()
    small = gpu_render(wl.scene, wl.camera, wl.params, max_pairs=100)
    assert small["status"] == _capi.PULSAR_ERR_CAPACITY and small["pairs"] > 100
    _parity(wl, what="1k spheres, exact capacity", max_pairs=small["pairs"])


def test_work_item_size_only_changes_rounding():
    """Cutting the tile lists into work items of another size changes only
    the order of the blend's sums."""
    wl = sg.config2()
    G = sg.upstream_grad(4, 512, 512, 3)
    a = gpu_render(wl.scene, wl.camera, wl.params, G, chunk=64)
    b = gpu_render(wl.scene, wl.camera, wl.params, G, chunk=1024)
    assert_close(b["F"], a["F"], 1e-5, "image")
    for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
        assert_close(b[key], a[key], 1e-4, key)


def test_only_requested_gradients_are_written():
    wl = sg.config1()
    G = sg.upstream_grad(8, 64, 64, 3)
    full = gpu_render(wl.scene, wl.camera, wl.params, G)
    part = gpu_render(wl.scene, wl.camera, wl.params, G, need={"payload", "bg"})
    assert part["grad_pos"] is None and part["grad_radius"] is None
    assert_close(part["grad_payload"], full["grad_payload"], 1e-5, "payload")
    assert_close(part["grad_bg"], full["grad_bg"], 1e-5, "bg")


@pytest.mark.parametrize("case", ["plain", "rotated", "min_radius", "dense_K3", "ortho"])
def test_paper_normalised_gradients(case):
    """PULSAR_GRAD_PAPER_NORM: gradients averaged over each sphere's pixel
    count and the 3-pixel position gate, against the oracle's definition.
    Full frames without rounding-sensitive pixels, so the counts are exact."""
    wl = sg.config1()
    sc, cam, par = wl.scene, wl.camera, wl.params
    # radii x4: some spheres wider than 3 pixels, no rounding-sensitive pixel
    sc.radius = (sc.radius * 4.0).astype(np.float32)
    if case == "rotated":
        rng = np.random.default_rng(8)
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        tq = rng.uniform(-1, 1, 3)
        sc.pos = ((sc.pos.astype(np.float64) - tq) @ q).astype(np.float32)
        cam.R, cam.t = q.astype(np.float32), tq.astype(np.float32)
    if case == "min_radius":
        par = sg.Params(gamma=0.1, eps=1e-5, min_radius_px=0.7071, K=5)
    if case == "dense_K3":
        sc.radius = (sc.radius * 1.25).astype(np.float32)
        par = sg.Params(gamma=0.1, eps=1e-5, K=3)
    flags = 0
    if case == "ortho":
        # orthographic spheres look larger: the unscaled radii (x4 / 4 is exact)
        sc.radius = (sc.radius / 4.0).astype(np.float32)
        cam.orthographic = True
        par = sg.Params(gamma=0.1, eps=1e-5, min_radius_px=0.7071, K=5)
        flags = _capi.PULSAR_ORTHO
    _say(f"[parity] paper-normalised gradients, {case}")
    fwd = ref.forward(sc, cam, par)
    assert not fwd["ambiguous"].any()
    G = sg.upstream_grad(700, cam.height, cam.width, sc.C)
    g = ref.paper_normalised(sc, cam, par, fwd, ref.backward(sc, cam, par, G, fwd))
    pr = g["projected_radius_px"]
    assert (pr <= 3.0).any() and (pr > 3.0).any()
    assert np.all(np.abs(pr - 3.0) > 1e-4)  # gate decisions are not rounding-sensitive
    out = gpu_render(sc, cam, par, G, fwd_flags=flags,
                     bwd_flags=flags | _capi.PULSAR_GRAD_PAPER_NORM)
    assert out["status"] == _capi.PULSAR_OK
    compare_grads(out, g, f"paper-normalised {case}")


def test_paper_normalisation_wide_payload():
    """C > 32 takes the wide backward, whose payload gradients are added per
    hit and averaged afterwards."""
    rng = np.random.default_rng(23)
    sc = sg.box_scene(rng, 120, 40, 0.15, 0.7)
    cam = sg.identity_camera(40, 40)
    par = sg.Params(gamma=0.1, eps=1e-5, K=4)
    _say("[parity] paper-normalised gradients, C=40")
    fwd = ref.forward(sc, cam, par)
    assert not fwd["ambiguous"].any()
    G = sg.upstream_grad(701, cam.height, cam.width, sc.C)
    g = ref.paper_normalised(sc, cam, par, fwd, ref.backward(sc, cam, par, G, fwd))
    pr = g["projected_radius_px"]
    assert (pr <= 3.0).any() and (pr > 3.0).any() and np.all(np.abs(pr - 3.0) > 1e-4)
    out = gpu_render(sc, cam, par, G, bwd_flags=_capi.PULSAR_GRAD_PAPER_NORM)
    assert out["status"] == _capi.PULSAR_OK
    compare_grads(out, g, "paper-normalised C=40")


@pytest.mark.parametrize("case", ["spheres1k", "dense_split_tiles", "rotated_rebin"])
def test_topk_blend(case):
    """PULSAR_BLEND_TOPK: only each pixel's K nearest hits enter Eq. 1 (image
    and log-normaliser), and the unchanged backward is its derivative;
    against the oracle's top-K forward. Pixels whose K nearest the oracle
    flags as rounding-sensitive are left out of the image comparison and get
    no upstream gradient."""
    wl = sg.config1()
    sc, cam, par = wl.scene, wl.camera, wl.params
    chunk, bwd_flags = 0, 0
    if case == "dense_split_tiles":
        sc.radius = (sc.radius * 8.0).astype(np.float32)
        chunk = 64
    if case == "rotated_rebin":
        rng = np.random.default_rng(9)
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        tq = rng.uniform(-1, 1, 3)
        sc.pos = ((sc.pos.astype(np.float64) - tq) @ q).astype(np.float32)
        cam.R, cam.t = q.astype(np.float32), tq.astype(np.float32)
        bwd_flags = _capi.PULSAR_REBIN
    _say(f"[parity] top-K blend, {case}")
    fwd = ref.forward(sc, cam, par, blend_topk=True)
    assert fwd["nhits"].max() > par.K
    G = sg.upstream_grad(800, cam.height, cam.width, sc.C)
    Gm = masked_G(G, None, fwd["ambiguous"])
    out = gpu_render(sc, cam, par, Gm, chunk=chunk, fwd_flags=_capi.PULSAR_BLEND_TOPK,
                     bwd_flags=bwd_flags)
    assert out["status"] == _capi.PULSAR_OK
    ok = ~fwd["ambiguous"]
    assert_close(out["F"][ok], fwd["F"][ok], IMAGE_REL, f"top-K image {case}")
    assert_close(out["L"][ok], fwd["L"][ok], IMAGE_REL, f"top-K log-normaliser {case}")
    full = ref.forward(sc, cam, par)
    deep = (fwd["nhits"] > par.K) & ok
    assert np.abs(full["F"][deep] - fwd["F"][deep]).max() > 1e-5  # the variant matters
    g = ref.backward(sc, cam, par, Gm, fwd)
    compare_grads(out, g, f"top-K {case}")


@pytest.mark.parametrize("case", ["spheres1k", "rotated", "min_radius", "dense_split_tiles"])
def test_orthographic_projection(case):
    """PULSAR_ORTHO against the oracle's orthographic rays: image,
    log-normaliser and every scene gradient."""
    import copy as _copy
    wl = sg.config1()
    sc, par = wl.scene, wl.params
    cam = _copy.deepcopy(wl.camera)
    cam.orthographic = True
    chunk = 0
    if case == "rotated":
        rng = np.random.default_rng(12)
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        tq = rng.uniform(-1, 1, 3)
        sc.pos = ((sc.pos.astype(np.float64) - tq) @ q).astype(np.float32)
        cam.R, cam.t = q.astype(np.float32), tq.astype(np.float32)
    if case == "min_radius":
        par = sg.Params(gamma=0.1, eps=1e-5, min_radius_px=1.5, K=5)
    if case == "dense_split_tiles":
        sc.radius = (sc.radius * 6.0).astype(np.float32)
        chunk = 64
    _say(f"[parity] orthographic, {case}")
    fwd = ref.forward(sc, cam, par)
    assert fwd["nhits"].max() > 1
    G = sg.upstream_grad(900, cam.height, cam.width, sc.C)
    Gm = masked_G(G, None, fwd["ambiguous"])
    flags = _capi.PULSAR_ORTHO
    out = gpu_render(sc, cam, par, Gm, chunk=chunk, fwd_flags=flags, bwd_flags=flags)
    assert out["status"] == _capi.PULSAR_OK
    assert_close(out["F"], fwd["F"], IMAGE_REL, f"orthographic image {case}")
    assert_close(out["L"], fwd["L"], IMAGE_REL, f"orthographic log-normaliser {case}")
    g = ref.backward(sc, cam, par, Gm, fwd)
    compare_grads(out, g, f"orthographic {case}")
