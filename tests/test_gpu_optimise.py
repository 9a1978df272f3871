"""The optimisation workload: 3,000,000 spheres on 20 blobs at 1920x1080, a
16-channel N(0,1) payload, K = 8 (seed 5). Checked at full size in two ways:
parity with the oracle on two seeded rows of the central band (forward and
all gradients, G zero elsewhere), and 100 Adam steps through the autograd
Function against a target rendered from a copy of the scene whose positions
carry N(0, 0.01^2) noise (seed 6), with an L1 image loss.
"""
import time

import numpy as np
import pytest

from oracle import reference as ref
from paper_2004_07484_amd import _capi
from paper_2004_07484_amd import scenegen as sg
from tests.gpu_helpers import GRAD_REL, IMAGE_REL, assert_close, compare_grads, gpu_render, \
    masked_G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg5():
    return sg.config5()


def test_config5_full_size_row_subset(cfg5):
    wl = cfg5
    sc, cam, par = wl.scene, wl.camera, wl.params
    # rows of the central band, where the blobs are (others have no hits)
    rows = sorted((380 + np.random.default_rng(79).choice(320, 2, replace=False)).tolist())
    print(f"[parity] 3M blobs 1920x1080 C=16 rows={rows}", flush=True)
    fwd = ref.forward(sc, cam, par, rows=rows)
    assert fwd["nhits"][rows].max() > par.K
    G = sg.upstream_grad(wl.seed + 1000, cam.height, cam.width, sc.C)
    Gm = masked_G(G, rows, fwd["ambiguous"])
    out = gpu_render(sc, cam, par, Gm)
    assert out["status"] == _capi.PULSAR_OK
    assert_close(out["F"][rows], fwd["F"][rows], IMAGE_REL, "3M image")
    assert_close(out["L"][rows], fwd["L"][rows], IMAGE_REL, "3M log-normaliser")
    assert np.isfinite(out["F"]).all()
    g = ref.backward(sc, cam, par, Gm, fwd, rows=rows)
    compare_grads(out, g, "3M")


def test_config5_optimisation_loop(cfg5):
    """100 Adam steps (lr 1e-3 for positions, opacities and payloads; 1e-5
    for radii, whose values are of order 1e-3) on an L1 loss. Radii and
    opacities are kept in their domains (r > 0, 0 <= o <= 1) after each step.
    The loss must fall, every step must stay finite."""
    import torch
    from paper_2004_07484_amd.renderer import Renderer
    wl = cfg5
    sc, cam, par = wl.scene, wl.camera, wl.params
    dev = "cuda:0"
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    r = Renderer(cam.width, cam.height, sc.n, n_channels=sc.C, K=par.K)
    noisy = (sc.pos.astype(np.float64) +
             0.01 * np.random.default_rng(6).standard_normal(sc.pos.shape)).astype(np.float32)
    with torch.no_grad():
        target = r(t(noisy), t(sc.payload), t(sc.radius), cam, opacity=t(sc.opacity),
                   gamma=par.gamma)
    pos, rad, opa, pay = (t(a).requires_grad_(True)
                          for a in (sc.pos, sc.radius, sc.opacity, sc.payload))
    opt = torch.optim.Adam([{"params": [pos, opa, pay], "lr": 1e-3},
                            {"params": [rad], "lr": 1e-5}])
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(100):
        opt.zero_grad(set_to_none=True)
        img = r(pos, pay, rad, cam, opacity=opa, gamma=par.gamma)
        loss = (img - target).abs().mean()
        loss.backward()
        opt.step()
        with torch.no_grad():
            rad.clamp_(min=1e-5)
            opa.clamp_(0.0, 1.0)
        losses.append(loss.detach())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 100
    losses = torch.stack(losses).cpu().numpy()
    print(f"[optimise] 3M spheres 1920x1080 C=16: {ms:.2f} ms per step (render, loss, "
          f"Adam); L1 {losses[0]:.5f} -> {losses[-1]:.5f}", flush=True)
    assert np.isfinite(losses).all()
    for a in (pos, rad, opa, pay):
        assert torch.isfinite(a).all()
    assert losses[-1] < 0.9 * losses[0]
