"""Benchmark: forward + backward of the sphere renderer at 1M spheres, 1024x1024, FP32.

One step = pulsar_fwd + pulsar_bwd on the blob workload (1,000,000 spheres on
20 Gaussian blobs, 8-channel N(0,1) payload, K = 8, gamma = 0.1) with every
input already resident in HBM. Prints one JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# unpacked FP32 VALU: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def io_bytes(n: int, H: int, W: int, C: int):
    """Compulsory bytes: read pos, radius, opacity, payload; write F and L
    (forward); re-read the scene, read G, F and L, write every gradient
    (backward)."""
    fwd = n * (20 + 4 * C) + H * W * (4 * C + 4)
    bwd = n * (20 + 4 * C) + H * W * (8 * C + 4) + n * 4 * (C + 5) + 4 * C
    return fwd, bwd


COMMON_SOURCES = ["paper_2004_07484_amd/csrc/hit_geometry.h",
                  "paper_2004_07484_amd/csrc/device_common.h",
                  "paper_2004_07484_amd/csrc/pulsar_internal.h"]
_BIN = ["paper_2004_07484_amd/csrc/binning.hip"] + COMMON_SOURCES
TRAFFIC_SOURCES = {
    "k_project": ["paper_2004_07484_amd/csrc/project.hip"] + COMMON_SOURCES,
    "k_emit": _BIN, "k_sort_hist": _BIN, "k_sort_scatter": _BIN, "k_ranges": _BIN,
    "k_plan": _BIN,
    "k_fwd_chunks": ["paper_2004_07484_amd/csrc/raster_fwd.hip"] + COMMON_SOURCES,
    "k_fwd_merge": ["paper_2004_07484_amd/csrc/raster_fwd.hip"] + COMMON_SOURCES,
    "k_bwd_items": ["paper_2004_07484_amd/csrc/raster_bwd.hip"] + COMMON_SOURCES,
    "k_bwd_spheres": ["paper_2004_07484_amd/csrc/raster_bwd.hip"] + COMMON_SOURCES,
    "k_finalize": ["paper_2004_07484_amd/csrc/raster_bwd.hip"] + COMMON_SOURCES,
}


def sources_hash(kernel: str) -> str:
    import hashlib
    return hashlib.sha256(b"".join(open(os.path.join(ROOT, p), "rb").read()
                                   for p in TRAFFIC_SOURCES[kernel])).hexdigest()[:16]


def measured_record(kernel: str, workload: str):
    """The kernel's record in the committed rocprofv3 summary (HBM bytes per
    dispatch from FETCH_SIZE and WRITE_SIZE scaled by the copy calibration,
    and its VALU-active share of wave cycles), or None when the summary is
    missing or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{workload}.md")
    if kernel not in TRAFFIC_SOURCES or not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.strip().startswith("TRAFFIC "):
            r = json.loads(line.strip()[len("TRAFFIC "):])
            if r.get("kernel") == kernel:
                rec = r
    if rec is None or sources_hash(kernel) != rec.get("sources_sha256_16"):
        return None
    return rec


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per dispatch from the committed rocprofv3 summary, or None."""
    rec = measured_record(kernel, workload)
    return None if rec is None else int(rec["bytes"])


def binning_launches(T: int) -> dict:
    """Launches of each binning kernel for T tiles: the emission, then LSD
    passes of at most 8-bit digits (a histogram before every pass but the
    first), the tile ranges and the work items."""
    bits = max(0, (T - 1).bit_length())
    passes = (bits + 7) // 8
    return {"k_emit": 1, "k_sort_scatter": passes, "k_sort_hist": max(0, passes - 1),
            "k_ranges": 1, "k_plan": 1}


def cpu_baseline(wl, G, rows_n: int):
    """FP64 brute-force oracle on a seeded row subset of the same workload,
    extrapolated linearly to the full frame. Also returns what the parity
    check needs: the rows, the oracle's forward and gradients, and the
    upstream gradient they were taken for (G on those rows, zero elsewhere
    and on pixels whose K nearest hits are rounding-sensitive)."""
    from oracle import reference as ref
    H = wl.camera.height
    rows = sorted(np.random.default_rng(12345).choice(H, rows_n, replace=False).tolist())
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    if os.environ.get("OMP_NUM_THREADS"):
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    t0 = time.perf_counter()
    fwd = ref.forward(wl.scene, wl.camera, wl.params, rows=rows, n_threads=threads)
    t1 = time.perf_counter()
    Gm = np.zeros_like(G)
    Gm[rows] = G[rows]
    Gm[fwd["ambiguous"]] = 0.0
    grads = ref.backward(wl.scene, wl.camera, wl.params, Gm, fwd, rows=rows)
    t2 = time.perf_counter()
    scale = H / rows_n
    total_ms = (t2 - t0) * 1e3 * scale
    base = {"value": round(total_ms, 1), "unit": "ms/frame (extrapolated)", "cores": threads,
            "kind": "oracle",
            "sample": f"{rows_n} of {H} seeded rows of the same workload (fwd {t1 - t0:.1f} s, "
                      f"bwd {t2 - t1:.1f} s), scaled by {scale:.0f}",
            "fwd_ms": round((t1 - t0) * 1e3 * scale, 1),
            "bwd_ms": round((t2 - t1) * 1e3 * scale, 1)}
    return base, dict(rows=rows, fwd=fwd, grads=grads, G=Gm)


def at_knobs(p) -> dict:
    from paper_2004_07484_amd import autotune as at
    return at.knobs_of(p)


def cpu_one_thread(wl, rows_n: int = 2) -> dict:
    """The oracle on one thread, on a few seeded rows of the same workload,
    extrapolated to the full frame (the per-core cost of the baseline)."""
    from oracle import reference as ref
    H, W, C = wl.camera.height, wl.camera.width, wl.scene.C
    rows = sorted(np.random.default_rng(54321).choice(H, rows_n, replace=False).tolist())
    t0 = time.perf_counter()
    fwd = ref.forward(wl.scene, wl.camera, wl.params, rows=rows, n_threads=1)
    G = np.zeros((H, W, C), np.float32)
    G[rows] = 1.0
    G[fwd["ambiguous"]] = 0.0
    ref.backward(wl.scene, wl.camera, wl.params, G, fwd, rows=rows)
    dt = time.perf_counter() - t0
    return {"value": round(dt * 1e3 * H / rows_n, 1), "unit": "ms/frame (extrapolated)",
            "cores": 1, "sample": f"{rows_n} of {H} seeded rows, {dt:.1f} s"}


def graph_time(fn, steps: int, warmup: int, stream) -> float:
    """Median ms of fn(s) captured once in a HIP graph (s: the capturing
    stream) and replayed on `stream`."""
    import torch
    fn(stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn(torch.cuda.current_stream())
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for e0, e1 in evs:
        e0.record(stream)
        graph.replay()
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def bench_small(args, dev, wl) -> dict:
    """One fwd + bwd of a small workload: microseconds per frame, eager and
    graph-replayed (launch latency dominates at these sizes)."""
    import torch

    from paper_2004_07484_amd import _capi
    sc, cam, par = wl.scene, wl.camera, wl.params
    n, C = sc.payload.shape
    H, W = cam.height, cam.width
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pos, rad, opa, pay, bg = t(sc.pos), t(sc.radius), t(sc.opacity), t(sc.payload), t(sc.bg)
    G = t(np.random.default_rng(wl.seed + 1000).standard_normal((H, W, C)).astype(np.float32))
    cs = _capi.make_camera(cam.R, cam.t, cam.focal, cam.sensor_width, cam.znear, cam.zfar, W, H)
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    ws = torch.empty(_capi.pulsar_workspace_size(n, W, H, C, ps), dtype=torch.uint8, device=dev)
    image, aux = torch.empty((H, W, C), device=dev), torch.empty((H, W), device=dev)
    gp, gr, go = torch.empty((n, 3), device=dev), torch.empty(n, device=dev), \
        torch.empty(n, device=dev)
    gf, gb = torch.empty((n, C), device=dev), torch.empty(C, device=dev)
    stream = torch.cuda.current_stream()

    def step(s=stream):
        _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux, ws, s)
        _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, ps, image, aux, G, gp, gr, go, gf, gb, ws, s)

    step()
    code, pairs = _capi.pulsar_query_status(ws, stream)
    assert code == _capi.PULSAR_OK
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    eager = float(np.median([a.elapsed_time(b) for a, b in evs]))
    graph = graph_time(step, args.steps, args.warmup, stream)
    code, _ = _capi.pulsar_query_status(ws, stream)
    assert code == _capi.PULSAR_OK
    fb, bb = io_bytes(n, H, W, C)
    return {"workload": wl.name, "spheres": int(n), "width": W, "height": H, "channels": int(C),
            "K": int(par.K), "tile_pairs": int(pairs), "eager_us": round(eager * 1e3, 1),
            "graph_us": round(graph * 1e3, 1),
            "io_roofline_frac": round((fb + bb) / (graph * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}


def bench_optimise(args, dev, steps: int = 100) -> dict:
    """The optimisation workload (3M spheres on blobs, 1920x1080, C = 16,
    K = 8): the renderer's fwd + bwd alone (C ABI, eager, HIP events), and
    `steps` Adam steps (torch's fused Adam) through the autograd Renderer
    against a target from a copy of the scene with N(0, 0.01^2) position
    noise (L1 loss), with the loss curve. A whole step (render, loss,
    backward, Adam, clamps) is timed over the steps after the first
    `cold` ones, which also allocate the optimiser state and the autograd
    buffers (reported apart)."""
    import torch

    from paper_2004_07484_amd import _capi
    from paper_2004_07484_amd import scenegen as sg
    from paper_2004_07484_amd.renderer import Renderer
    wl = sg.config5()
    sc, cam, par = wl.scene, wl.camera, wl.params
    n, C = sc.payload.shape
    H, W = cam.height, cam.width
    log(f"[optimise] {n} spheres {W}x{H} C={C}")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    stream = torch.cuda.current_stream()
    # renderer alone
    pos, rad, opa, pay, bg = t(sc.pos), t(sc.radius), t(sc.opacity), t(sc.payload), t(sc.bg)
    G = t(sg.upstream_grad(wl.seed + 1000, H, W, C))
    cs = _capi.make_camera(cam.R, cam.t, cam.focal, cam.sensor_width, cam.znear, cam.zfar, W, H)
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    ws = torch.empty(_capi.pulsar_workspace_size(n, W, H, C, ps), dtype=torch.uint8, device=dev)
    image, aux = torch.empty((H, W, C), device=dev), torch.empty((H, W), device=dev)
    gp, gr, go = torch.empty((n, 3), device=dev), torch.empty(n, device=dev), \
        torch.empty(n, device=dev)
    gf, gb = torch.empty((n, C), device=dev), torch.empty(C, device=dev)

    def step():
        _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux, ws, stream)
        _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, ps, image, aux, G, gp, gr, go, gf, gb, ws,
                         stream)

    step()
    code, pairs = _capi.pulsar_query_status(ws, stream)
    assert code == _capi.PULSAR_OK
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    render_ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
    del ws, gp, gr, go, gf, gb
    # the optimisation loop
    r = Renderer(W, H, n, n_channels=C, K=par.K)
    noisy = (sc.pos.astype(np.float64) +
             0.01 * np.random.default_rng(6).standard_normal(sc.pos.shape)).astype(np.float32)
    with torch.no_grad():
        target = r(t(noisy), pay, rad, cam, opacity=opa, gamma=par.gamma)
    vp, vr, vo, vf = (x.clone().requires_grad_(True) for x in (pos, rad, opa, pay))
    opt = torch.optim.Adam([{"params": [vp, vo, vf], "lr": 1e-3}, {"params": [vr], "lr": 1e-5}],
                           fused=True)
    losses = []
    cold = 10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_cold = t0
    for k in range(steps):
        if k == cold:
            torch.cuda.synchronize()
            t_cold = time.perf_counter()
        opt.zero_grad(set_to_none=True)
        img = r(vp, vf, vr, cam, opacity=vo, gamma=par.gamma)
        loss = (img - target).abs().mean()
        loss.backward()
        opt.step()
        with torch.no_grad():
            vr.clamp_(min=1e-5)
            vo.clamp_(0.0, 1.0)
        losses.append(loss.detach())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = (t1 - t_cold) * 1e3 / (steps - cold)
    cold_ms = (t_cold - t0) * 1e3 / cold
    r.check_status(wait=True)
    curve = torch.stack(losses).cpu().numpy()
    log(f"[optimise] renderer {render_ms:.3f} ms, whole step {step_ms:.3f} ms, L1 "
        f"{curve[0]:.5f} -> {curve[-1]:.5f}")
    fb, bb = io_bytes(n, H, W, C)
    return {"workload": wl.name, "spheres": int(n), "width": W, "height": H, "channels": int(C),
            "K": int(par.K), "tile_pairs": int(pairs), "renderer_ms_per_step": round(render_ms, 4),
            "renderer_io_roofline_frac": round((fb + bb) / (render_ms * 1e-3) /
                                               (HBM_PEAK_GBS * 1e9), 4),
            "whole_step_ms": round(step_ms, 4), "first_steps_ms": round(cold_ms, 4),
            "timed_steps": f"{cold}..{steps - 1}", "optimizer": "torch.optim.Adam(fused=True)",
            "adam_steps": steps,
            "loss_curve": {str(k): round(float(curve[k]), 6)
                           for k in list(range(0, steps, 10)) + [steps - 1]}}


def max_rel(got, want, floor=1e-2) -> float:
    """Largest |got - want| / max(|want|, floor max|want|) (the parity scale)."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    if want.size == 0:
        return 0.0
    scale = np.maximum(np.abs(want), floor * np.abs(want).max())
    return float((np.abs(got - want) / np.maximum(scale, 1e-300)).max())


def stage_kernels(by_sphere: bool = True) -> dict:
    """The kernel that does each stage's work (the backward in sphere order
    writes the sphere gradients itself; the tile-order one leaves them to
    k_finalize)."""
    return {"project": "k_project", "binning": "binning (several kernels)",
            "raster_fwd": "k_fwd_chunks", "merge": "k_fwd_merge",
            "raster_bwd": "k_bwd_spheres" if by_sphere else "k_bwd_items",
            "finalize": "k_finalize"}


def stage_bytes(n: int, H: int, W: int, C: int, pairs: int, by_sphere: bool = True) -> dict:
    """Algorithmic bytes each stage must move whatever the implementation:
    the compulsory I/O of the frame that falls to it, and for binning the tile
    lists it must produce.
      project     read pos, radius, opacity: n (12 + 4 + 4)
      binning     write the tile lists: one sphere index per (tile, sphere)
                  pair (4 B) and the tile ranges (4 B per tile)
      raster_fwd  read the payload rows, write F and L: n 4C + HW (4C + 4)
                  (split tiles' pixels are written by the merge, counted here)
      merge       none beyond the forward's (intermediate partial blends)
      raster_bwd  read G, F and L and the payload rows: HW (8C + 4) + n 4C;
                  in sphere order it also re-reads the scene for the chain
                  rule, n 20, and writes every sphere gradient, n 4 (C + 5)
      finalize    the background gradient 4C, and in tile order the scene
                  re-read and every sphere gradient, n 20 + n 4 (C + 5)
    The stages add up to io_bytes() plus the tile lists."""
    T = ((W + 7) // 8) * ((H + 7) // 8)
    grads = 20 * n + 4 * (C + 5) * n  # the scene re-read and every gradient
    return {"project": 20 * n, "binning": 4 * pairs + 4 * (T + 1),
            "raster_fwd": 4 * C * n + H * W * (4 * C + 4), "merge": 0,
            "raster_bwd": H * W * (8 * C + 4) + 4 * C * n + (grads if by_sphere else 0),
            "finalize": 4 * C + (0 if by_sphere else grads)}


def stage_roofline(stage_avg: dict, n, H, W, C, pairs, workload, by_sphere: bool = True):
    """roofline object for the stage that takes longest (its algorithmic bytes
    over its average duration against the HBM peak), and the same figures
    for every stage."""
    sb = stage_bytes(n, H, W, C, pairs, by_sphere)
    names = stage_kernels(by_sphere)
    T = ((W + 7) // 8) * ((H + 7) // 8)
    kernels = {}
    for st, nbytes in sb.items():
        ms = stage_avg.get(st, 0.0)
        kernels[st] = {"kernel": names[st], "avg_ms": round(ms, 4),
                       "bytes_per_launch": nbytes,
                       "achieved_GBs": round(nbytes / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
                       "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                       if ms > 0 else None}
        # counter traffic (over the compulsory bytes) and VALU-active share
        # from the committed profile of this workload, while it is current
        if st == "binning":
            recs = [(measured_record(k, workload), c) for k, c in binning_launches(T).items()]
            traffic = (sum(int(r["bytes"]) * c for r, c in recs)
                       if all(r is not None for r, _ in recs) else None)
            valu = None
        else:
            rec = measured_record(names[st], workload)
            traffic = None if rec is None else int(rec["bytes"])
            valu = None if rec is None else rec.get("valu_active")
        kernels[st]["traffic"] = traffic
        kernels[st]["traffic_ratio"] = (round(traffic / nbytes, 3)
                                        if traffic is not None and nbytes > 0 else None)
        kernels[st]["valu_active"] = valu
    # the dominant kernel: the longest stage that is a single kernel, so its
    # average duration can be checked against the rocprofv3 kernel trace
    # (binning is six kernels; its own figures are in `kernels` and in
    # `longest_stage` when it takes longest)
    single = [k for k in sb if k != "binning"]
    dom = max(single, key=lambda k: stage_avg.get(k, 0.0))
    ms = stage_avg[dom]
    achieved = sb[dom] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    kname = names[dom]
    roofline = {"kernel": kname, "stage": dom, "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kname, workload), "avg_ms": round(ms, 4),
                "bytes_per_launch": sb[dom]}
    longest = max(sb, key=lambda k: stage_avg.get(k, 0.0))
    roofline["longest_stage"] = {"stage": longest, "kernel": names[longest],
                                 "avg_ms": round(stage_avg.get(longest, 0.0), 4),
                                 "frac": kernels[longest]["frac"]}
    return roofline, kernels


def bench_batch(args, dev) -> dict:
    """Uneven batch of 32 scenes (1k-500k spheres, 256^2-1024^2, random
    cameras; C = 3, K = 5): one batched fwd+bwd per step against a loop of
    single-scene fwd+bwd calls on the same stream, both eager and replayed
    from a HIP graph."""
    import torch

    from paper_2004_07484_amd import _capi
    from paper_2004_07484_amd import scenegen as sg

    wls = sg.config4_scenes()
    par = wls[0].params
    C = wls[0].scene.C
    B = len(wls)
    cams = [_capi.make_camera(w.camera.R, w.camera.t, w.camera.focal, w.camera.sensor_width,
                              w.camera.znear, w.camera.zfar, w.camera.width, w.camera.height)
            for w in wls]
    counts = [w.scene.n for w in wls]
    scenes = _capi.make_scenes(cams, counts)
    N, P = _capi.batch_sizes(scenes)
    log(f"[batch] {B} scenes, {N} spheres, {P} pixels")

    def t(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)

    pos = t(np.concatenate([w.scene.pos for w in wls]))
    rad = t(np.concatenate([w.scene.radius for w in wls]))
    opa = t(np.concatenate([w.scene.opacity for w in wls]))
    pay = t(np.concatenate([w.scene.payload for w in wls]))
    bg = t(np.stack([w.scene.bg for w in wls]))
    G = t(np.concatenate([sg.upstream_grad(w.seed + 1000 + b, w.camera.height, w.camera.width, C)
                          .reshape(-1, C) for b, w in enumerate(wls)]))
    image = torch.empty((P, C), device=dev)
    aux = torch.empty((P,), device=dev)
    gp, gr, go = torch.empty((N, 3), device=dev), torch.empty(N, device=dev), \
        torch.empty(N, device=dev)
    gf, gb = torch.empty((N, C), device=dev), torch.empty((B, C), device=dev)
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    ws = torch.empty(_capi.pulsar_batch_workspace_size(scenes, C, ps), dtype=torch.uint8,
                     device=dev)
    stream = torch.cuda.current_stream()

    def batched(s):
        _capi.pulsar_fwd_batched(scenes, pos, rad, opa, pay, bg, ps, image, aux, ws, s)
        _capi.pulsar_bwd_batched(scenes, pos, rad, opa, pay, bg, ps, image, aux, G, gp, gr, go,
                                 gf, gb, ws, s)

    # per-scene views into the same packed buffers; one workspace serves every
    # scene because the calls run one after another on one stream
    views, n0, p0 = [], 0, 0
    for b, (w, c) in enumerate(zip(wls, cams)):
        n, hw = w.scene.n, w.camera.height * w.camera.width
        H, W = w.camera.height, w.camera.width
        views.append((c, pos[n0:n0 + n], rad[n0:n0 + n], opa[n0:n0 + n], pay[n0:n0 + n], bg[b],
                      image[p0:p0 + hw].view(H, W, C), aux[p0:p0 + hw].view(H, W),
                      G[p0:p0 + hw].view(H, W, C), gp[n0:n0 + n], gr[n0:n0 + n], go[n0:n0 + n],
                      gf[n0:n0 + n], gb[b]))
        n0 += n
        p0 += hw
    ws1 = torch.empty(max(_capi.pulsar_workspace_size(w.scene.n, w.camera.width,
                                                      w.camera.height, C, ps) for w in wls),
                      dtype=torch.uint8, device=dev)

    def looped(s):
        for (c, p_, r_, o_, f_, b_, im, ax, g_, gp_, gr_, go_, gf_, gb_) in views:
            _capi.pulsar_fwd(p_, r_, o_, f_, b_, c, ps, im, ax, ws1, s)
            _capi.pulsar_bwd(p_, r_, o_, f_, b_, c, ps, im, ax, g_, gp_, gr_, go_, gf_, gb_, ws1, s)

    # K steps back to back, bracketed by synchronisations (frames/s is a rate)
    def time_eager(fn):
        for _ in range(args.warmup):
            fn(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    def time_graph(fn):
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fn(torch.cuda.current_stream())
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    batched(stream)
    code, pairs = _capi.pulsar_query_status(ws, stream)
    assert code == _capi.PULSAR_OK, "batched tile-pair capacity"
    knobs = None
    if args.batch_knobs:
        from paper_2004_07484_amd import autotune as at
        for k, v in parse_knobs(args.batch_knobs):
            at.set_knob(ps, k, v)
        ws = torch.empty(_capi.pulsar_batch_workspace_size(scenes, C, ps), dtype=torch.uint8,
                         device=dev)
        knobs = at.knobs_of(ps)
        log(f"[batch] fixed knobs {knobs}")
        ws1 = torch.empty(max(_capi.pulsar_workspace_size(w.scene.n, w.camera.width,
                                                          w.camera.height, C, ps) for w in wls),
                          dtype=torch.uint8, device=dev)
        batched(stream)
    elif not args.no_tune:
        from paper_2004_07484_amd import autotune as at
        wss = {}

        def run(p):
            key = (p.chunk, p.raster_blocks, p.flags)
            if key not in wss:
                wss[key] = torch.empty(_capi.pulsar_batch_workspace_size(scenes, C, p),
                                       dtype=torch.uint8, device=dev)
            w = wss[key]
            _capi.pulsar_fwd_batched(scenes, pos, rad, opa, pay, bg, p, image, aux, w, stream)
            _capi.pulsar_bwd_batched(scenes, pos, rad, opa, pay, bg, p, image, aux, G, gp, gr, go,
                                     gf, gb, w, stream)

        tuned, info = at.tune(run, ps, reps=5, warmup=2)
        ps.chunk, ps.raster_blocks, ps.flags = tuned.chunk, tuned.raster_blocks, tuned.flags
        ws = wss[(ps.chunk, ps.raster_blocks, ps.flags)]
        wss.clear()
        knobs = info["knobs"]
        log(f"[batch] tuned knobs {knobs}")
        # the looped calls use the same knobs; their workspace may grow with them
        ws1 = torch.empty(max(_capi.pulsar_workspace_size(w.scene.n, w.camera.width,
                                                          w.camera.height, C, ps) for w in wls),
                          dtype=torch.uint8, device=dev)
    looped(stream)
    torch.cuda.synchronize()
    res = {"batched_eager_ms": time_eager(batched), "looped_eager_ms": time_eager(looped)}
    if not args.no_graph:
        res["batched_graph_ms"] = time_graph(batched)
        res["looped_graph_ms"] = time_graph(looped)
    code, _ = _capi.pulsar_query_status(ws, stream)
    assert code == _capi.PULSAR_OK
    # each side at its faster way of running (launched directly or replayed)
    bt = min(res.get("batched_graph_ms", np.inf), res["batched_eager_ms"])
    lt = min(res.get("looped_graph_ms", np.inf), res["looped_eager_ms"])
    log(f"[batch] batched {bt:.3f} ms, looped {lt:.3f} ms per batch of {B}")
    io = sum(sum(io_bytes(w.scene.n, w.camera.height, w.camera.width, C)) for w in wls)
    out = {"workload": "uneven32_c3_k5", "scenes": B, "spheres": int(N), "pixels": int(P),
           "tile_pairs": int(pairs), "io_bytes": int(io),
           "io_roofline_frac": round(io / (bt * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
           "batched_frames_per_s": round(B / (bt * 1e-3), 1),
           "looped_frames_per_s": round(B / (lt * 1e-3), 1),
           "speedup": round(lt / bt, 3), "tuned_knobs": knobs}
    out.update({k: round(v, 4) for k, v in res.items()})
    return out


KNOB_NAMES = ("raster_blocks", "chunk", "store_hits", "bwd_tiles")


def parse_knobs(text: str):
    """[(knob, value)] from "k=v,k=v" (launch knobs only)."""
    out = []
    for kv in text.split(","):
        k, v = kv.split("=")
        if k not in KNOB_NAMES:
            raise SystemExit(f"unknown knob {k}")
        out.append((k, int(v)))
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=64)
    ap.add_argument("--spheres", type=int, default=1_000_000)
    ap.add_argument("--no-graph", action="store_true", help="time eager launches only")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-vs-looped measurement of 32 uneven scenes")
    ap.add_argument("--no-camera", action="store_true",
                    help="skip timing the backward that also returns camera gradients")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the latency of the 1k and 100k sphere workloads")
    ap.add_argument("--no-optimise", action="store_true",
                    help="skip the 3M-sphere optimisation workload")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the default launch knobs instead of autotuning them first")
    ap.add_argument("--knobs", default="", metavar="K=V,...",
                    help="fixed launch knobs for the single-scene workload, e.g. "
                         "raster_blocks=4096,chunk=128 (implies no tuning)")
    ap.add_argument("--batch-knobs", default="", metavar="K=V,...",
                    help="fixed launch knobs for the 32-scene batch (implies no tuning there)")
    ap.add_argument("--only-batch", action="store_true",
                    help="only run the batched-vs-looped measurement and print its JSON object "
                         "(for profiling the batch on its own; not the bench line)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (5 times) and exit; "
                         "calibrates the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe * (1 << 20) // 4, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "launches": 5}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build "
              "(the renderer runs on a single MI355X).", file=sys.stderr)
        return 2

    import torch

    from paper_2004_07484_amd import _capi
    from paper_2004_07484_amd import scenegen as sg

    _capi.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    if args.only_batch:
        print(json.dumps(bench_batch(args, dev)), flush=True)
        return 0
    log(f"[bench] generating workload ({args.spheres} spheres)")
    wl = sg.config3(args.spheres)
    sc, cam, par = wl.scene, wl.camera, wl.params
    n, C = sc.payload.shape
    H, W = cam.height, cam.width
    G_np = sg.upstream_grad(wl.seed + 1000, H, W, C)

    def t(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    pos, rad, opa, pay, bg, G = t(sc.pos), t(sc.radius), t(sc.opacity), t(sc.payload), \
        t(sc.bg), t(G_np)
    cs = _capi.make_camera(cam.R, cam.t, cam.focal, cam.sensor_width, cam.znear, cam.zfar, W, H)
    ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K)
    ws = torch.empty(_capi.pulsar_workspace_size(n, W, H, C, ps), dtype=torch.uint8, device=dev)
    image = torch.empty((H, W, C), device=dev)
    aux = torch.empty((H, W), device=dev)
    gp, gr, go = torch.empty((n, 3), device=dev), torch.empty(n, device=dev), \
        torch.empty(n, device=dev)
    gf, gb = torch.empty((n, C), device=dev), torch.empty(C, device=dev)
    stream = torch.cuda.current_stream()

    def step(s=None):
        s = stream if s is None else s
        _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux, ws, s)
        _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, ps, image, aux, G, gp, gr, go, gf, gb, ws, s)

    log("[bench] first step")
    step()
    code, pairs = _capi.pulsar_query_status(ws, stream)
    if code != _capi.PULSAR_OK:
        ps = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K,
                               max_pairs=int(pairs * 1.25) + 1024)
        ws = torch.empty(_capi.pulsar_workspace_size(n, W, H, C, ps), dtype=torch.uint8,
                         device=dev)
        step()
        code, pairs = _capi.pulsar_query_status(ws, stream)
        assert code == _capi.PULSAR_OK
    tune_info = None
    if args.knobs:
        from paper_2004_07484_amd import autotune as at
        for k, v in parse_knobs(args.knobs):
            at.set_knob(ps, k, v)
        ws = torch.empty(_capi.pulsar_workspace_size(n, W, H, C, ps), dtype=torch.uint8,
                         device=dev)
        step()
        from paper_2004_07484_amd import autotune as at
        tune_info = {"knobs": at.knobs_of(ps)}
        log(f"[bench] fixed knobs {tune_info['knobs']}")
    elif not args.no_tune:
        from paper_2004_07484_amd import autotune as at
        wss, graphs = {}, {}

        def run(p):
            # each setting is timed as the step below is: replayed from a HIP
            # graph, captured after one eager step (which also rejects the
            # settings the library refuses)
            key = (p.chunk, p.raster_blocks, p.flags)
            if key not in wss:
                wss[key] = torch.empty(_capi.pulsar_workspace_size(n, W, H, C, p),
                                       dtype=torch.uint8, device=dev)
            w = wss[key]
            if key not in graphs:
                _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, p, image, aux, w, stream)
                _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, p, image, aux, G, gp, gr, go, gf, gb,
                                 w, stream)
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    s = torch.cuda.current_stream()
                    _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, p, image, aux, w, s)
                    _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, p, image, aux, G, gp, gr, go, gf,
                                     gb, w, s)
                graphs[key] = g
            graphs[key].replay()

        ps, tune_info = at.tune(run, ps, reps=5, warmup=2)
        torch.cuda.synchronize()
        ws = wss[(ps.chunk, ps.raster_blocks, ps.flags)]
        graphs.clear()
        wss.clear()
        log(f"[bench] tuned knobs {tune_info['knobs']} ({tune_info['ms']:.3f} ms per replayed "
            f"step)")
    log(f"[bench] {pairs} tile pairs; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # K steps back to back, bracketed by synchronisations (the step's rate
    # as a caller sees it; nothing is recorded between the launches)
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # the same K steps again with HIP events around each call and each stage
    # (the per-stage durations and the roofline; the events add some time)
    _capi.pulsar_timing_enable(True)
    _capi.pulsar_timing_read()  # drop anything recorded before
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(stream)
        _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux, ws, stream)
        e1.record(stream)
        _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, ps, image, aux, G, gp, gr, go, gf, gb, ws,
                         stream)
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = _capi.pulsar_timing_read()
    _capi.pulsar_timing_enable(False)
    code, _ = _capi.pulsar_query_status(ws, stream)
    assert code == _capi.PULSAR_OK
    fwd_ms = float(np.median([a.elapsed_time(b) for a, b, _ in ev]))
    bwd_ms = float(np.median([b.elapsed_time(c) for _, b, c in ev]))
    timed_ms = float(np.median([a.elapsed_time(c) for a, _, c in ev]))
    wall_ms = wall * 1e3 / args.steps
    log(f"[bench] eager: {eager_ms:.3f} ms per step; with events per call and stage: median fwd "
        f"{fwd_ms:.3f} ms, bwd {bwd_ms:.3f} ms, step {timed_ms:.3f} ms, wall/step {wall_ms:.3f} ms")

    # the same step captured once in a HIP graph: K replays back to back,
    # bracketed by synchronisations (`value`), then K replays with HIP events
    # around each (the per-replay median, for reference)
    graph_ms = graph_event_ms = None
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step(torch.cuda.current_stream())
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        for e0, e1 in gev:
            e0.record(stream)
            graph.replay()
            e1.record(stream)
        torch.cuda.synchronize()
        code, _ = _capi.pulsar_query_status(ws, stream)
        assert code == _capi.PULSAR_OK
        graph_event_ms = float(np.median([a.elapsed_time(b) for a, b in gev]))
        log(f"[bench] graph replay: {graph_ms:.3f} ms per step ({args.steps} back to back), "
            f"median replay {graph_event_ms:.3f} ms")
    # value: the faster way of running the step, launched directly or replayed
    # from the graph (both timed the same way, K steps between synchronisations)
    value_mode = "graph" if graph_ms is not None and graph_ms < eager_ms else "eager"
    step_ms = graph_ms if value_mode == "graph" else eager_ms

    fwd_b, bwd_b = io_bytes(n, H, W, C)
    stage_avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    by_sphere = not (int(ps.flags) & (_capi.PULSAR_BWD_TILES | _capi.PULSAR_STORE_HITS))
    roofline, kernels = stage_roofline(stage_avg, n, H, W, C, int(pairs), wl.name, by_sphere)
    io_frac = (fwd_b + bwd_b) / (step_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)

    # the backward with camera gradients against the plain one, each timed
    # after a forward of its own, like the step above
    camera = None
    if not args.no_camera:
        gcam = torch.empty(14, device=dev)

        def bwd_plain():
            _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, ps, image, aux, G, gp, gr, go, gf, gb,
                             ws, stream)

        def bwd_cam():
            _capi.pulsar_bwd_camera(pos, rad, opa, pay, bg, cs, ps, image, aux, G, gp, gr, go, gf,
                                    gb, gcam, ws, stream)

        cms = {}
        for name, fn in (("plain", bwd_plain), ("camera", bwd_cam)):
            cev = []
            for k in range(args.warmup + args.steps):
                _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux, ws, stream)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                if k >= args.warmup:
                    cev.append((e0, e1))
            torch.cuda.synchronize()
            cms[name] = float(np.median([a.elapsed_time(b) for a, b in cev]))
        assert bool(torch.isfinite(gcam).all())
        camera = {"bwd_with_camera_ms": round(cms["camera"], 4), "bwd_ms": round(cms["plain"], 4),
                  "extra_ms": round(cms["camera"] - cms["plain"], 4)}
        log(f"[bench] backward with camera gradients: {cms['camera']:.3f} ms (without: "
            f"{cms['plain']:.3f})")
        # the flag variants on the same workload: top-K-only blend (forward)
        # and the paper's gradient normalisation (backward)
        p_topk = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K, ps.max_pairs,
                                   ps.depth_bits, ps.chunk, ps.raster_blocks,
                                   _capi.PULSAR_BLEND_TOPK)
        p_norm = _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K, ps.max_pairs,
                                   ps.depth_bits, ps.chunk, ps.raster_blocks,
                                   _capi.PULSAR_GRAD_PAPER_NORM)

        def timed(fn, before=None):
            evs = []
            for k in range(args.warmup + args.steps):
                if before is not None:
                    before()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                if k >= args.warmup:
                    evs.append((e0, e1))
            torch.cuda.synchronize()
            return float(np.median([a.elapsed_time(b) for a, b in evs]))

        fwd_plain = timed(lambda: _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux,
                                                   ws, stream))
        fwd_topk = timed(lambda: _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, p_topk, image, aux,
                                                  ws, stream))
        fwd_again = lambda: _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux, ws,
                                             stream)
        bwd_norm = timed(lambda: _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, p_norm, image, aux,
                                                  G, gp, gr, go, gf, gb, ws, stream), fwd_again)
        camera["variants_ms"] = {"fwd": round(fwd_plain, 4), "fwd_topk_blend": round(fwd_topk, 4),
                                 "bwd": round(cms["plain"], 4),
                                 "bwd_paper_norm": round(bwd_norm, 4)}
        log(f"[bench] forward {fwd_plain:.3f} ms, top-K blend {fwd_topk:.3f} ms; backward with "
            f"the paper's normalisation {bwd_norm:.3f} ms")
        # early ray termination at a 1 % share, the stored-hits backward and
        # the backward in tile order, each on a workspace of its own
        for name, pv in (("early_stop_1pct",
                          _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K,
                                            ps.max_pairs, 0, 0, ps.raster_blocks, 0, 0.01)),
                         ("store_hits",
                          _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K,
                                            ps.max_pairs, 0, ps.chunk, ps.raster_blocks,
                                            _capi.PULSAR_STORE_HITS)),
                         ("bwd_tiles",
                          _capi.make_params(par.gamma, par.eps, par.min_radius_px, par.K,
                                            ps.max_pairs, 0, ps.chunk, ps.raster_blocks,
                                            _capi.PULSAR_BWD_TILES))):
            wv = torch.empty(_capi.pulsar_workspace_size(n, W, H, C, pv), dtype=torch.uint8,
                             device=dev)
            fv = lambda pv=pv, wv=wv: _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, pv, image,
                                                       aux, wv, stream)
            t_f = timed(fv)
            t_b = timed(lambda pv=pv, wv=wv: _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, pv,
                                                              image, aux, G, gp, gr, go, gf, gb,
                                                              wv, stream), fv)
            code, _ = _capi.pulsar_query_status(wv, stream)
            assert code == _capi.PULSAR_OK, name
            camera["variants_ms"][f"fwd_{name}"] = round(t_f, 4)
            camera["variants_ms"][f"bwd_{name}"] = round(t_b, 4)
            log(f"[bench] {name}: forward {t_f:.3f} ms, backward {t_b:.3f} ms")
            del wv

    batch = None
    if not args.no_batch:
        batch = bench_batch(args, dev)

    small = None
    if not args.no_small:
        small = {}
        for make in (sg.config1, sg.config2):
            w = make()
            log(f"[small] {w.name}")
            small[w.name] = bench_small(args, dev, w)
            log(f"[small] {w.name}: graph {small[w.name]['graph_us']} us, eager "
                f"{small[w.name]['eager_us']} us per fwd+bwd")

    optimise = None
    if not args.no_optimise:
        optimise = bench_optimise(args, dev)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline on {args.cpu_rows} rows")
        cpu, orc = cpu_baseline(wl, G_np, args.cpu_rows)
        log(f"[bench] oracle {cpu['value']} ms/frame on {cpu['cores']} threads")
        cpu["one_thread"] = cpu_one_thread(wl)
        log(f"[bench] oracle on one thread {cpu['one_thread']['value']} ms/frame")
        # parity of the timed configuration: one more fwd + bwd with the same
        # launch knobs and workspace, G restricted to the oracle's rows
        Gd = t(orc["G"].astype(np.float32))
        step_g = lambda: (
            _capi.pulsar_fwd(pos, rad, opa, pay, bg, cs, ps, image, aux, ws, stream),
            _capi.pulsar_bwd(pos, rad, opa, pay, bg, cs, ps, image, aux, Gd, gp, gr, go, gf, gb,
                             ws, stream))
        step_g()
        code, _ = _capi.pulsar_query_status(ws, stream)
        assert code == _capi.PULSAR_OK
        rows = orc["rows"]
        F, L = image.cpu().numpy(), aux.cpu().numpy()
        rel_img = max(max_rel(F[rows], orc["fwd"]["F"][rows]),
                      max_rel(L[rows], orc["fwd"]["L"][rows]))
        got = {"grad_pos": gp, "grad_radius": gr, "grad_opacity": go, "grad_payload": gf,
               "grad_bg": gb}
        rel_grad = {k: max_rel(v.cpu().numpy(), orc["grads"][k]) for k, v in got.items()}
        parity = {"rows": len(rows), "pixels": len(rows) * W,
                  "masked_pixels": int(orc["fwd"]["ambiguous"][rows].sum()),
                  "max_rel_image": rel_img, "max_rel_grad": max(rel_grad.values()),
                  "max_rel_grad_by_tensor": rel_grad, "tolerance": {"image": 1e-4, "grad": 1e-3},
                  "knobs": at_knobs(ps)}
        parity["pass"] = bool(rel_img <= 1e-4 and parity["max_rel_grad"] <= 1e-3)
        log(f"[bench] parity on {len(rows)} oracle rows: image {rel_img:.2e}, gradients "
            f"{parity['max_rel_grad']:.2e} ({'pass' if parity['pass'] else 'FAIL'})")

    out = {
        "metric": "fwd+bwd ms/frame at 1M spheres 1024^2 FP32; batched vs looped frames/s",
        "value": round(step_ms, 4),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "spheres": int(n), "width": W, "height": H,
                   "channels": int(C), "K": int(par.K), "gamma": par.gamma,
                   "tile_pairs": int(pairs)},
        "value_mode": value_mode,
        "eager_ms_per_step": round(eager_ms, 4),
        "graph_ms_per_step": None if graph_ms is None else round(graph_ms, 4),
        "graph_replay_median_ms": None if graph_event_ms is None else round(graph_event_ms, 4),
        "fwd_ms": round(fwd_ms, 4),
        "bwd_ms": round(bwd_ms, 4),
        "timed_step_median_ms": round(timed_ms, 4),
        "frames_per_s": round(1e3 / step_ms, 2),
        "wall_ms_per_step": round(wall_ms, 4),
        "io_bytes": {"fwd": fwd_b, "bwd": bwd_b},
        "io_roofline_frac": round(io_frac, 4),
        "stages_ms": {k: round(v, 4) for k, v in stage_avg.items()},
        "roofline": roofline,
        "kernels": kernels,
        "tuned_knobs": None if tune_info is None else tune_info["knobs"],
        "tune_trials": None if tune_info is None else tune_info.get("trials"),
        "camera_gradients_and_variants": camera,
        "batched": batch,
        "small_workloads": small,
        "optimisation": optimise,
        "cpu_baseline": cpu,
        "parity": parity,
        "paper_context": "RTX 2080, 1M spheres at 1000^2: fwd 19 ms, bwd 4.7 ms (CUDA only)",
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
