"""The forward + backward captured in a HIP graph replays like eager launches."""
import numpy as np
import pytest

from paper_2004_07484_amd import _capi
from paper_2004_07484_amd import scenegen as sg
from tests.gpu_helpers import assert_close, cam_struct, to_dev

pytestmark = pytest.mark.gpu


def test_graph_replay_matches_eager():
    import torch
    wl = sg.config2()
    sc, cam, par = wl.scene, wl.camera, wl.params
    n, C = sc.payload.shape
    H, W = cam.height, cam.width
    cs = cam_struct(cam)
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    pos, rad, opa, pay, bg = (to_dev(a) for a in (sc.pos, sc.radius, sc.opacity, sc.payload,
                                                  sc.bg))
    G = to_dev(sg.upstream_grad(11, H, W, C))
    ws = torch.empty(_capi.pulsar_workspace_size(n, W, H, C, ps), dtype=torch.uint8,
                     device="cuda:0")
    img = torch.empty((H, W, C), device="cuda:0")
    aux = torch.empty((H, W), device="cuda:0")
    outs = [torch.empty((n, 3), device="cuda:0"), torch.empty(n, device="cuda:0"),
            torch.empty(n, device="cuda:0"), torch.empty((n, C), device="cuda:0"),
            torch.empty(C, device="cuda:0")]

    def step(stream):
        _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, img, aux, ws, stream)
        _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, ps, img, aux, G, *outs, ws, stream)

    def snapshot():
        torch.cuda.synchronize()
        return [img.cpu().numpy().copy(), aux.cpu().numpy().copy()] + \
            [o.cpu().numpy().copy() for o in outs]

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
        # eager work between replays
        step(torch.cuda.current_stream())
        torch.cuda.synchronize()
    # the graph reads its inputs from device memory: new opacities show up
    opa.mul_(0.5)
    step(torch.cuda.current_stream())
    eager_half = snapshot()
    graph.replay()
    got = snapshot()
    assert np.array_equal(got[0], eager_half[0])
    assert not np.array_equal(got[0], eager[0])
    code, _ = _capi.pulsar_query_status(ws)
    assert code == _capi.PULSAR_OK
