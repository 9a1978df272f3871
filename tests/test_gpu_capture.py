"""Lazy pair-capacity checks of the autograd front end, and a Renderer step
(forward and backward) captured in a HIP graph and replayed."""
import sys

import numpy as np
import pytest

from paper_2004_07484_amd import _capi
from paper_2004_07484_amd import scenegen as sg

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _tensors(wl, grad=True):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    leaves = [t(wl.scene.pos), t(wl.scene.payload), t(wl.scene.radius), t(wl.scene.opacity)]
    if grad:
        for x in leaves:
            x.requires_grad_(True)
    return leaves


def test_lazy_check_reports_an_overflow_on_the_next_call():
    """With a pair capacity far below the scene's, the first call overflows
    without waiting; the next call reads that status, warns and renders with a
    larger capacity, which then equals a render with ample capacity."""
    import torch
    from paper_2004_07484_amd.renderer import Renderer
    wl = sg.config1()
    _say("[capture] lazy overflow check")
    pos, pay, rad, opa = _tensors(wl, grad=False)
    r = Renderer(64, 64, wl.scene.n, n_channels=3, K=5, max_pairs=100)
    r(pos, pay, rad, wl.camera, opacity=opa)
    torch.cuda.synchronize()
    with pytest.warns(RuntimeWarning, match="tile pairs"):
        img = r(pos, pay, rad, wl.camera, opacity=opa)
    assert r.max_pairs > 100
    ok = Renderer(64, 64, wl.scene.n, n_channels=3, K=5, check_capacity="sync")
    ref_img = ok(pos, pay, rad, wl.camera, opacity=opa)
    torch.cuda.synchronize()
    r.check_status(wait=True)  # the second call fitted
    assert torch.equal(img, ref_img)


def test_lazy_check_stops_the_backward_of_an_overflowed_forward():
    import torch
    from paper_2004_07484_amd.renderer import Renderer
    wl = sg.config1()
    _say("[capture] backward after an overflow")
    pos, pay, rad, opa = _tensors(wl)
    r = Renderer(64, 64, wl.scene.n, n_channels=3, K=5, max_pairs=100)
    img = r(pos, pay, rad, wl.camera, opacity=opa)
    torch.cuda.synchronize()  # the status has landed
    with pytest.raises(_capi.PulsarError):
        img.backward(torch.ones_like(img))


def test_renderer_step_in_a_graph():
    """Forward and backward of a Renderer captured once; each replay, after new
    inputs are copied into the captured tensors and some eager work with a
    synchronisation, equals an eager step on the same inputs bitwise."""
    import torch
    from paper_2004_07484_amd.renderer import Renderer
    wl = sg.config1()
    _say("[capture] renderer step in a graph")
    r = Renderer(64, 64, wl.scene.n, n_channels=3, K=5)
    pos, pay, rad, opa = _tensors(wl)
    G = torch.from_numpy(sg.upstream_grad(55, 64, 64, 3)).cuda()
    leaves = (pos, pay, rad, opa)

    def step():
        img = r(pos, pay, rad, wl.camera, opacity=opa)
        img.backward(G)
        return img

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            for x in leaves:
                x.grad = None
            step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for x in leaves:
        x.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        img_g = step()
    grads_g = [x.grad for x in leaves]

    rng = np.random.default_rng(3)
    for k in range(4):
        with torch.no_grad():
            pos.copy_(torch.from_numpy(wl.scene.pos + rng.normal(0, 0.01, wl.scene.pos.shape)
                                       .astype(np.float32)).cuda())
            pay.copy_(torch.from_numpy(rng.uniform(0, 1, wl.scene.payload.shape)
                                       .astype(np.float32)).cuda())
        graph.replay()
        torch.cuda.synchronize()
        got = [img_g.detach().clone()] + [g.detach().clone() for g in grads_g]
        # eager work between replays: an eager step on the same inputs
        saved = [x.grad for x in leaves]
        for x in leaves:
            x.grad = None
        img_e = step()
        torch.cuda.synchronize()
        want = [img_e.detach()] + [x.grad.detach() for x in leaves]
        for x, sv in zip(leaves, saved):
            x.grad = sv
        for name, a, b in zip(["image", "pos", "payload", "radius", "opacity"], got, want):
            assert torch.equal(a, b), f"replay {k}: {name} differs from the eager step"
