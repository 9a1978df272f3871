"""Batched rendering of uneven scenes in one call (pulsar_fwd_batched /
pulsar_bwd_batched): each scene matches its own single-scene call and the
FP64 oracle, and the captured batch replays like eager launches."""
import sys

import numpy as np
import pytest

from oracle import reference as ref
from paper_2004_07484_amd import _capi
from paper_2004_07484_amd import scenegen as sg
from tests.gpu_helpers import (GRAD_REL, IMAGE_REL, assert_close, compare_grads, gpu_render,
                               gpu_render_batch, masked_G)

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _small_batch():
    """Five small scenes: ragged sizes, different cameras and backgrounds, one empty."""
    rng = np.random.default_rng(404)
    specs = [(40, 32, 14), (37, 29, 9), (24, 24, 0), (64, 48, 25), (33, 41, 12)]
    out = []
    for b, (W, H, n) in enumerate(specs):
        wl = sg.tiny_scene(500 + b, n=max(n, 1), C=3, W=W, H=H, r_lo=0.15, r_hi=0.5)
        if n == 0:
            sc = wl.scene
            wl.scene = sg.Scene(pos=sc.pos[:0], radius=sc.radius[:0], opacity=sc.opacity[:0],
                                payload=sc.payload[:0], bg=sc.bg)
        if b == 3:
            # move the spheres rigidly (w' = q w + tq) and the camera with them
            # (R' = q^T, t' = -q^T tq), so the view is unchanged
            q, r = np.linalg.qr(rng.standard_normal((3, 3)))
            q = q * np.sign(np.diag(r))
            if np.linalg.det(q) < 0:
                q[:, 0] = -q[:, 0]
            tq = rng.uniform(-0.5, 0.5, 3)
            sc = wl.scene
            sc.pos = (np.asarray(sc.pos, np.float64) @ q.T + tq).astype(np.float32)
            wl.camera.R = q.T.astype(np.float32)
            wl.camera.t = (-(q.T @ tq)).astype(np.float32)
        wl.scene.bg = rng.uniform(-0.5, 0.5, 3).astype(np.float32)
        out.append(wl)
    return out


PARAMS = sg.Params(gamma=0.2, eps=1e-5, K=5)


def test_batched_small_scenes_match_oracle():
    wls = _small_batch()
    Gs, fwds = [], []
    for b, wl in enumerate(wls):
        fwd = ref.forward(wl.scene, wl.camera, PARAMS)
        G = sg.upstream_grad(900 + b, wl.camera.height, wl.camera.width, 3)
        Gs.append(masked_G(G, None, fwd["ambiguous"]))
        fwds.append(fwd)
    _say(f"[batched] {len(wls)} small scenes vs oracle")
    outs = gpu_render_batch(wls, PARAMS, Gs)
    for b, (wl, fwd, G, out) in enumerate(zip(wls, fwds, Gs, outs)):
        assert out["status"] == _capi.PULSAR_OK
        assert_close(out["F"], fwd["F"], IMAGE_REL, f"scene {b} image")
        assert_close(out["L"], fwd["L"], IMAGE_REL, f"scene {b} log-normaliser")
        g = ref.backward(wl.scene, wl.camera, PARAMS, G, fwd)
        compare_grads(out, g, f"scene {b}")


def _cfg4_batch(extra=True):
    wls = sg.config4_scenes()
    if extra:
        # a ragged image and an empty scene inside the batch
        t = sg.tiny_scene(77, n=40, C=3, W=61, H=45, r_lo=0.1, r_hi=0.4)
        e = sg.tiny_scene(78, n=1, C=3, W=16, H=8)
        sc = e.scene
        e.scene = sg.Scene(pos=sc.pos[:0], radius=sc.radius[:0], opacity=sc.opacity[:0],
                           payload=sc.payload[:0], bg=sc.bg)
        wls = wls[:16] + [t, e] + wls[16:]
    return wls


def test_batched_equals_looped_uneven_batch():
    """The 32-scene uneven batch (1k-500k spheres, 256^2-1024^2, random
    cameras) plus a ragged and an empty scene: every tile list holds its
    spheres in index order in both calls, so the forward is bitwise equal to
    per-scene calls; gradients agree to float summation order."""
    wls = _cfg4_batch()
    par = wls[0].params
    Gs = [sg.upstream_grad(1000 + b, w.camera.height, w.camera.width, 3)
          for b, w in enumerate(wls)]
    _say(f"[batched] uneven batch of {len(wls)} scenes, {sum(w.scene.n for w in wls)} spheres")
    outs = gpu_render_batch(wls, par, Gs)
    for b, (wl, G, out) in enumerate(zip(wls, Gs, outs)):
        assert out["status"] == _capi.PULSAR_OK
        one = gpu_render(wl.scene, wl.camera, par, G)
        assert np.array_equal(out["F"], one["F"]), b
        assert np.array_equal(out["L"], one["L"]), b
        for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
            assert_close(out[key], one[key], 1e-4, f"scene {b} {key}", floor=1e-2)


_CFG4 = {}


def _cfg4_oracle_rows():
    """The 32-scene batch with oracle rows of three scenes (smallest, median,
    largest): upstream gradients masked to those rows, computed once."""
    if not _CFG4:
        wls = _cfg4_batch(extra=False)
        par = wls[0].params
        rng = np.random.default_rng(4242)
        order = np.argsort([w.scene.n for w in wls])
        check = {int(order[0]): None, int(order[len(order) // 2]): None, int(order[-1]): None}
        Gs = []
        for b, w in enumerate(wls):
            G = sg.upstream_grad(2000 + b, w.camera.height, w.camera.width, 3)
            if b in check:
                rows = sorted(rng.choice(w.camera.height, 2, replace=False).tolist())
                fwd = ref.forward(w.scene, w.camera, par, rows=rows)
                G = masked_G(G, rows, fwd["ambiguous"])
                g = ref.backward(w.scene, w.camera, par, G, fwd, rows=rows)
                check[b] = (rows, fwd, g)
            Gs.append(G)
        _CFG4.update(wls=wls, check=check, Gs=Gs)
    return _CFG4


# the default launch and the batch configurations the autotuner picks at
# the largest grid
@pytest.mark.parametrize("knobs", [{}, dict(chunk=192, raster_blocks=16384),
                                   dict(chunk=320, raster_blocks=16384),
                                   dict(chunk=512, raster_blocks=16384),
                                   dict(chunk=64, raster_blocks=4096)])
def test_batched_default_key_width_and_oracle_rows(knobs):
    """Default depth key width (the batch has other tile numbers, so the key
    layout differs from single calls): images agree to 1e-6, and sampled rows
    of three scenes match the oracle, in each launch configuration."""
    c = _cfg4_oracle_rows()
    wls, check, Gs = c["wls"], c["check"], c["Gs"]
    par = wls[0].params
    _say(f"[batched] default key width, oracle rows of scenes {sorted(check)}, knobs {knobs}")
    outs = gpu_render_batch(wls, par, Gs, **knobs)
    for b, (rows, fwd, g) in check.items():
        out = outs[b]
        assert out["status"] == _capi.PULSAR_OK
        assert_close(out["F"][rows], fwd["F"][rows], IMAGE_REL, f"scene {b} image")
        compare_grads(out, g, f"scene {b}")
    for b in (0, 7, 31):
        one = gpu_render(wls[b].scene, wls[b].camera, par)
        assert_close(outs[b]["F"], one["F"], 1e-6, f"scene {b} batched vs single")


def test_batched_graph_replay_matches_eager():
    import torch
    wls = _cfg4_batch(extra=False)[:12]
    par = wls[0].params
    C = 3
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    scenes = _capi.make_scenes([sg_cam(w) for w in wls], [w.scene.n for w in wls])
    N, P = _capi.batch_sizes(scenes)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to("cuda:0")
    pos = dev(np.concatenate([w.scene.pos for w in wls]))
    rad = dev(np.concatenate([w.scene.radius for w in wls]))
    opa = dev(np.concatenate([w.scene.opacity for w in wls]))
    pay = dev(np.concatenate([w.scene.payload for w in wls]))
    bg = dev(np.stack([w.scene.bg for w in wls]))
    G = dev(np.concatenate([sg.upstream_grad(3000 + b, w.camera.height, w.camera.width, C)
                            .reshape(-1, C) for b, w in enumerate(wls)]))
    ws = torch.empty(_capi.pulsar_batch_workspace_size(scenes, C, ps), dtype=torch.uint8,
                     device="cuda:0")
    img = torch.empty((P, C), device="cuda:0")
    aux = torch.empty((P,), device="cuda:0")
    outs = [torch.empty((N, 3), device="cuda:0"), torch.empty(N, device="cuda:0"),
            torch.empty(N, device="cuda:0"), torch.empty((N, C), device="cuda:0"),
            torch.empty((len(wls), C), device="cuda:0")]

    def step(stream):
        _capi.pulsar_fwd_batched(scenes, pos, rad, opa, pay, bg, ps, img, aux, ws, stream)
        _capi.pulsar_bwd_batched(scenes, pos, rad, opa, pay, bg, ps, img, aux, G, *outs, ws,
                                 stream)

    def snapshot():
        torch.cuda.synchronize()
        return [img.cpu().numpy().copy(), aux.cpu().numpy().copy()] + \
            [o.cpu().numpy().copy() for o in outs]

    _say(f"[batched] graph capture of {len(wls)} scenes")
    step(torch.cuda.current_stream())
    eager = snapshot()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(torch.cuda.current_stream())
    for rep in range(3):
        img.zero_()
        for o in outs:
            o.fill_(float("nan"))
        graph.replay()
        got = snapshot()
        assert np.array_equal(got[0], eager[0]) and np.array_equal(got[1], eager[1]), rep
        for g, e, name in zip(got[2:], eager[2:], ["pos", "radius", "opacity", "payload", "bg"]):
            assert_close(g, e, 1e-5, f"replay {rep} grad {name}")
        step(torch.cuda.current_stream())
        torch.cuda.synchronize()
    code, _ = _capi.pulsar_query_status(ws)
    assert code == _capi.PULSAR_OK


def sg_cam(w):
    from tests.gpu_helpers import cam_struct
    return cam_struct(w.camera)


@pytest.mark.parametrize("knob", [dict(chunk=64), dict(chunk=256), dict(chunk=1024),
                                  dict(raster_blocks=256), dict(raster_blocks=16384)])
def test_tuning_knobs_keep_results(knob):
    """Work-item size and persistent grid size are result-neutral: the grid
    size leaves the image bitwise unchanged, the work-item size only changes
    the blend's summation order."""
    wl = sg.config2()
    G = sg.upstream_grad(1001, wl.camera.height, wl.camera.width, wl.scene.C)
    _say(f"[tuning] {knob}")
    base = gpu_render(wl.scene, wl.camera, wl.params, G)
    got = gpu_render(wl.scene, wl.camera, wl.params, G, **knob)
    assert got["status"] == _capi.PULSAR_OK
    if "raster_blocks" in knob:
        assert np.array_equal(got["F"], base["F"])
        assert np.array_equal(got["L"], base["L"])
    else:
        assert_close(got["F"], base["F"], 2e-6, "image", floor=1e-2)
        assert_close(got["L"], base["L"], 2e-6, "log-normaliser", floor=1e-2)
    # a bitwise-equal forward leaves only float atomic order to the gradients;
    # a changed summation order moves F in its last bits, which h = G . (f - F)
    # amplifies where f is close to F, so those are held to the parity bar
    rel = 1e-4 if "raster_blocks" in knob else GRAD_REL
    for key in ["grad_pos", "grad_radius", "grad_opacity", "grad_payload", "grad_bg"]:
        assert_close(got[key], base[key], rel, key, floor=1e-2)


@pytest.mark.parametrize("flags", [_capi.PULSAR_ORTHO, _capi.PULSAR_BLEND_TOPK,
                                   _capi.PULSAR_ORTHO | _capi.PULSAR_BLEND_TOPK,
                                   _capi.PULSAR_BWD_TILES])
def test_batched_variants_match_oracle(flags):
    """The orthographic projection, the top-K blend and the tile-order
    backward in a batched call of small scenes, against the oracle per
    scene."""
    import copy
    ortho = bool(flags & _capi.PULSAR_ORTHO)
    topk = bool(flags & _capi.PULSAR_BLEND_TOPK)
    wls = [copy.deepcopy(w) for w in _small_batch()]
    Gs, fwds = [], []
    for b, wl in enumerate(wls):
        wl.camera.orthographic = ortho
        fwd = ref.forward(wl.scene, wl.camera, PARAMS, blend_topk=topk)
        G = sg.upstream_grad(950 + b, wl.camera.height, wl.camera.width, 3)
        Gs.append(masked_G(G, None, fwd["ambiguous"]))
        fwds.append(fwd)
    _say(f"[batched] {len(wls)} small scenes, flags {flags}")
    outs = gpu_render_batch(wls, PARAMS, Gs, flags=flags)
    for b, (wl, fwd, G, out) in enumerate(zip(wls, fwds, Gs, outs)):
        assert out["status"] == _capi.PULSAR_OK
        ok = ~fwd["ambiguous"]
        assert_close(out["F"][ok], fwd["F"][ok], IMAGE_REL, f"scene {b} image")
        assert_close(out["L"][ok], fwd["L"][ok], IMAGE_REL, f"scene {b} log-normaliser")
        g = ref.backward(wl.scene, wl.camera, PARAMS, G, fwd)
        compare_grads(out, g, f"scene {b}")


def _packed(wls):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()
    C = wls[0].scene.C
    return dict(pos=t(np.concatenate([w.scene.pos for w in wls])),
                rad=t(np.concatenate([w.scene.radius for w in wls])),
                opa=t(np.concatenate([w.scene.opacity for w in wls])),
                pay=t(np.concatenate([w.scene.payload for w in wls])),
                bg=t(np.stack([w.scene.bg for w in wls])),
                G=t(np.concatenate([sg.upstream_grad(70 + b, w.camera.height, w.camera.width, C)
                                    .reshape(-1, C) for b, w in enumerate(wls)])))


def test_device_cameras_in_a_graph():
    """pulsar_fwd_batched_devcam reads the cameras from device memory when the
    work runs: a batched forward + backward captured once renders, at each
    replay, with the cameras then in the array, bitwise equal to
    pulsar_fwd_batched / pulsar_bwd_batched with those cameras on the host."""
    import torch
    wls = sorted(sg.config4_scenes(), key=lambda w: w.scene.n)[:3]
    par = wls[0].params
    C = wls[0].scene.C
    B = len(wls)
    _say(f"[batch] device cameras, {B} scenes {[w.scene.n for w in wls]}")
    d = _packed(wls)
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    cams0 = [sg_cam(w) for w in wls]
    scenes = _capi.make_scenes(cams0, [w.scene.n for w in wls])
    N, P = _capi.batch_sizes(scenes)
    ws = torch.empty(_capi.pulsar_batch_workspace_size(scenes, C, ps), dtype=torch.uint8,
                     device="cuda:0")
    d_cams = torch.from_numpy(np.frombuffer(_capi.cameras_bytes(cams0), np.uint8).copy()).cuda()

    def outs():
        return [torch.empty(s, device="cuda:0") for s in
                ((P, C), (P,), (N, 3), (N,), (N,), (N, C), (B, C))]

    og = outs()

    def step(o, s, devcam):
        if devcam:
            _capi.pulsar_fwd_batched_devcam(scenes, d_cams, d["pos"], d["rad"], d["opa"],
                                            d["pay"], d["bg"], ps, o[0], o[1], ws, s)
        else:
            _capi.pulsar_fwd_batched(host_scenes, d["pos"], d["rad"], d["opa"], d["pay"],
                                     d["bg"], ps, o[0], o[1], ws, s)
        _capi.pulsar_bwd_batched(scenes if devcam else host_scenes, d["pos"], d["rad"], d["opa"],
                                 d["pay"], d["bg"], ps, o[0], o[1], d["G"], *o[2:], ws, s)

    host_scenes = scenes
    step(og, torch.cuda.current_stream(), True)  # warm-up outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(og, torch.cuda.current_stream(), True)
    rng = np.random.default_rng(17)
    oe = outs()
    for k in range(4):
        cams = []
        for w in wls:
            v = rng.standard_normal(3)
            v /= np.linalg.norm(v)
            c = sg.look_at_camera(4.0 * v, rng.uniform(-0.2, 0.2, 3), [0.0, 0.0, 1.0],
                                  w.camera.width, w.camera.height,
                                  focal=float(rng.uniform(0.8, 1.2)))
            cams.append(sg_cam(types_ns(c)))
        d_cams.copy_(torch.from_numpy(np.frombuffer(_capi.cameras_bytes(cams), np.uint8).copy()))
        graph.replay()
        torch.cuda.synchronize()
        code, _ = _capi.pulsar_query_status(ws)
        assert code == _capi.PULSAR_OK
        got = [x.clone() for x in og]
        # eager work between replays: the same cameras through the host table
        host_scenes = _capi.make_scenes(cams, [w.scene.n for w in wls])
        step(oe, torch.cuda.current_stream(), False)
        torch.cuda.synchronize()
        for name, a, b in zip(["image", "aux", "pos", "radius", "opacity", "payload", "bg"],
                              got, oe):
            assert torch.equal(a, b), f"replay {k}: {name} differs from the host-camera call"


def types_ns(cam):
    """A Workload-like holder for sg_cam."""
    import types
    return types.SimpleNamespace(camera=cam)


def test_invalid_device_camera_is_reported():
    import torch
    wls = sorted(sg.config4_scenes(), key=lambda w: w.scene.n)[:2]
    par = wls[0].params
    C = wls[0].scene.C
    d = _packed(wls)
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    cams = [sg_cam(w) for w in wls]
    scenes = _capi.make_scenes(cams, [w.scene.n for w in wls])
    N, P = _capi.batch_sizes(scenes)
    bad = _capi.make_camera(cams[1].R, cams[1].t, -1.0, cams[1].sensor_width, cams[1].znear,
                            cams[1].zfar, cams[1].width, cams[1].height)
    d_cams = torch.from_numpy(np.frombuffer(_capi.cameras_bytes([cams[0], bad]),
                                            np.uint8).copy()).cuda()
    ws = torch.empty(_capi.pulsar_batch_workspace_size(scenes, C, ps), dtype=torch.uint8,
                     device="cuda:0")
    image, aux = torch.empty((P, C), device="cuda:0"), torch.empty((P,), device="cuda:0")
    _capi.pulsar_fwd_batched_devcam(scenes, d_cams, d["pos"], d["rad"], d["opa"], d["pay"],
                                    d["bg"], ps, image, aux, ws)
    code, _ = _capi.pulsar_query_status(ws)
    assert code == _capi.PULSAR_ERR_INVALID_ARGUMENT
    # the same workspace with valid cameras is fine again
    d_cams.copy_(torch.from_numpy(np.frombuffer(_capi.cameras_bytes(cams), np.uint8).copy()))
    _capi.pulsar_fwd_batched_devcam(scenes, d_cams, d["pos"], d["rad"], d["opa"], d["pay"],
                                    d["bg"], ps, image, aux, ws)
    code, _ = _capi.pulsar_query_status(ws)
    assert code == _capi.PULSAR_OK
