"""pulsar_fwd_noalloc (the forward on the library's static scratch buffer,
for callers that cannot allocate) against pulsar_fwd with a caller
workspace, through the C ABI: two calls in a row, the second with a smaller
scene and image, so the second runs on what the first left in the buffer."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2004_07484_amd import _capi
from paper_2004_07484_amd import scenegen as sg
from tests.gpu_helpers import cam_struct, to_dev

pytestmark = pytest.mark.gpu


def _forward(wl, noalloc):
    import torch
    sc, cam, par = wl.scene, wl.camera, wl.params
    cs = cam_struct(cam)
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    n, C = sc.payload.shape
    pos, rad, opa, pay, bg = (to_dev(x) for x in (sc.pos, sc.radius, sc.opacity, sc.payload,
                                                  sc.bg))
    image = torch.full((cam.height, cam.width, C), float("nan"), device="cuda:0")
    aux = torch.full((cam.height, cam.width), float("nan"), device="cuda:0")
    if noalloc:
        assert _capi.pulsar_workspace_size(n, cam.width, cam.height, C, ps) <= \
            _capi.PULSAR_NOALLOC_SCRATCH_BYTES
        _capi.pulsar_fwd_noalloc(pos, rad, opa, pay, bg, cs, ps, image, aux)
    else:
        ws = torch.empty(_capi.pulsar_workspace_size(n, cam.width, cam.height, C, ps),
                         dtype=torch.uint8, device="cuda:0")
        _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux, ws)
        code, _ = _capi.pulsar_query_status(ws)
        assert code == _capi.PULSAR_OK
    torch.cuda.synchronize()
    return image.cpu().numpy(), aux.cpu().numpy()


def test_noalloc_forward_equals_workspace_forward():
    for make in (sg.config2, sg.config1):  # 100k spheres at 512^2, then 1k at 64^2
        wl = make()
        print(f"[noalloc] {make.__name__}: {wl.scene.payload.shape[0]} spheres "
              f"{wl.camera.width}x{wl.camera.height}", flush=True)
        F0, L0 = _forward(wl, noalloc=True)
        F1, L1 = _forward(wl, noalloc=False)
        assert np.isfinite(F0).all() and np.isfinite(L0).all()
        # the same kernels and launch shape on the same inputs: bitwise equal,
        # which is inside the parity tolerance (1e-4 relative for images)
        assert np.array_equal(F0, F1)
        assert np.array_equal(L0, L1)
