"""PULSAR_STORE_HITS: the forward keeps every pixel's K nearest hits and the
backward walks them pixel by pixel (App. B, preparation for the backward
pass), against the oracle and against the default (recomputing) backward."""
import sys

import numpy as np
import pytest

from oracle import reference as ref
from paper_2004_07484_amd import _capi
from paper_2004_07484_amd import scenegen as sg
from tests.gpu_helpers import (IMAGE_REL, assert_close, compare_grads, gpu_render,
                               gpu_render_batch, masked_G)

pytestmark = pytest.mark.gpu
STORE = _capi.PULSAR_STORE_HITS


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("case", ["config1", "config2_rows", "dense_K3", "rebin", "topk",
                                  "early_stop", "wide_payload", "orthographic"])
def test_stored_hits_match_oracle(case):
    wl = sg.config1()
    sc, cam, par = wl.scene, wl.camera, wl.params
    rows, fwd_flags, bwd_flags, topk = None, STORE, STORE, False
    if case == "config2_rows":
        wl = sg.config2()
        sc, cam, par = wl.scene, wl.camera, wl.params
        rows = sorted(np.random.default_rng(79).choice(512, 10, replace=False).tolist())
    if case == "dense_K3":
        sc.radius = (sc.radius * 6.0).astype(np.float32)
        par = sg.Params(gamma=0.1, eps=1e-5, K=3)
    if case == "rebin":
        fwd_flags, bwd_flags = STORE | _capi.PULSAR_NO_BWD_AUX, STORE | _capi.PULSAR_REBIN
    if case == "topk":
        fwd_flags |= _capi.PULSAR_BLEND_TOPK
        topk = True
    if case == "early_stop":
        from tests.test_gpu_early_stop import stacked
        sc, cam, par = stacked()
    if case == "wide_payload":
        rng = np.random.default_rng(5)
        sc.payload = rng.standard_normal((sc.n, 40)).astype(np.float32)
        sc.bg = np.zeros(40, np.float32)
    if case == "orthographic":
        import copy
        cam = copy.deepcopy(cam)
        cam.orthographic = True
        fwd_flags |= _capi.PULSAR_ORTHO
        bwd_flags |= _capi.PULSAR_ORTHO
    _say(f"[store hits] {case}")
    fwd = ref.forward(sc, cam, par, rows=rows, blend_topk=topk)
    G = sg.upstream_grad(600, cam.height, cam.width, sc.C)
    Gm = masked_G(G, rows, fwd["ambiguous"])
    out = gpu_render(sc, cam, par, Gm, fwd_flags=fwd_flags, bwd_flags=bwd_flags)
    assert out["status"] == _capi.PULSAR_OK
    sel = slice(None) if rows is None else rows
    ok = ~fwd["ambiguous"][sel]
    assert_close(out["F"][sel][ok], fwd["F"][sel][ok], IMAGE_REL, f"{case} image")
    g = ref.backward(sc, cam, par, Gm, fwd, rows=rows)
    compare_grads(out, g, f"store hits {case}")


def test_stored_hits_equal_recompute_up_to_order():
    """Same forward; the two backwards differ only in summation order (FP32
    sums of terms of both signs: 1e-4 on the parity scale, ten times tighter
    than the oracle tolerance)."""
    wl = sg.config1()
    sc, cam, par = wl.scene, wl.camera, wl.params
    fwd = ref.forward(sc, cam, par)
    G = masked_G(sg.upstream_grad(601, 64, 64, 3), None, fwd["ambiguous"])
    a = gpu_render(sc, cam, par, G)
    b = gpu_render(sc, cam, par, G, fwd_flags=STORE, bwd_flags=STORE)
    assert np.array_equal(a["F"], b["F"]) and np.array_equal(a["L"], b["L"])
    for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
        assert_close(b[key], a[key], 1e-4, f"{key} store vs recompute")


def test_backward_without_stored_hits_is_reported():
    """A stored-hits backward on a workspace whose forward kept none writes
    zeros and reports an invalid argument instead of reading stale hits."""
    import torch
    from tests.gpu_helpers import cam_struct, to_dev
    wl = sg.config1()
    sc, cam, par = wl.scene, wl.camera, wl.params
    cs = cam_struct(cam)
    pf = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    pb = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K, flags=STORE)
    n, C = sc.payload.shape
    ws = torch.empty(_capi.pulsar_workspace_size(n, 64, 64, C, pb), dtype=torch.uint8,
                     device="cuda:0")
    d = [to_dev(x) for x in (sc.pos, sc.radius, sc.opacity, sc.payload, sc.bg)]
    image, aux = torch.empty((64, 64, C), device="cuda:0"), torch.empty((64, 64), device="cuda:0")
    _capi.pulsar_fwd(*d, cs, pf, image, aux, ws)
    gp = torch.full((n, 3), float("nan"), device="cuda:0")
    _capi.pulsar_bwd(*d, cs, pb, image, aux, torch.ones((64, 64, C), device="cuda:0"), gp, None,
                     None, None, None, ws)
    code, _ = _capi.pulsar_query_status(ws)
    assert code == _capi.PULSAR_ERR_INVALID_ARGUMENT
    assert bool((gp == 0).all())


def test_stored_hits_batched():
    from tests.test_gpu_batched import PARAMS, _small_batch
    wls = _small_batch()
    par = PARAMS
    fwds, Gs = [], []
    for w in wls:
        f = ref.forward(w.scene, w.camera, par)
        fwds.append(f)
        Gs.append(masked_G(sg.upstream_grad(w.seed + 9, w.camera.height, w.camera.width,
                                            w.scene.C), None, f["ambiguous"]))
    outs = gpu_render_batch(wls, par, Gs=Gs, flags=STORE)
    for w, f, G, o in zip(wls, fwds, Gs, outs):
        assert o["status"] == _capi.PULSAR_OK
        assert_close(o["F"], f["F"], IMAGE_REL, f"{w.name} image")
        compare_grads(o, ref.backward(w.scene, w.camera, par, G, f), f"batched {w.name}")
