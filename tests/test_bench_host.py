"""Host-side checks of bench.py's accounting: the compulsory bytes of each
stage, the roofline object built from stage times, the lookup of counter
traffic in a profile summary (only while the kernel's sources are unchanged),
and the refusal of more than one GPU. None of these touches a GPU."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stage_bytes_of_the_1m_sphere_frame():
    n, H, W, C, pairs = 1_000_000, 1024, 1024, 8, 508_606
    sb = bench.stage_bytes(n, H, W, C, pairs)
    T = (W // 8) * (H // 8)
    assert sb["project"] == 20 * n  # pos, radius, opacity
    assert sb["binning"] == 4 * pairs + 4 * (T + 1)
    assert sb["raster_fwd"] == 4 * C * n + H * W * (4 * C + 4)  # payload in, F and L out
    # G, F, L, the payload and the scene (chain rule) in, every sphere
    # gradient out
    assert sb["raster_bwd"] == H * W * (8 * C + 4) + 4 * C * n + 20 * n + 4 * (C + 5) * n
    assert sb["finalize"] == 4 * C
    # in tile order the gradients are written by the finalize instead
    tiles = bench.stage_bytes(n, H, W, C, pairs, by_sphere=False)
    assert tiles["raster_bwd"] + tiles["finalize"] == sb["raster_bwd"] + sb["finalize"]
    # the whole frame's compulsory I/O equals io_bytes()
    fb, bb = bench.io_bytes(n, H, W, C)
    assert sum(v for k, v in sb.items() if k != "binning") == fb + bb


def test_roofline_takes_the_longest_single_kernel_stage():
    n, H, W, C, pairs = 1_000_000, 1024, 1024, 8, 508_606
    avg = {"project": 0.025, "binning": 0.052, "raster_fwd": 0.045, "merge": 0.011,
           "raster_bwd": 0.048, "finalize": 0.004, "raster_bwd_tiles": 0.006, "zero": 0.0}
    roof, kernels = bench.stage_roofline(avg, n, H, W, C, pairs, "no_such_workload")
    sb = bench.stage_bytes(n, H, W, C, pairs)
    assert roof["stage"] == "raster_bwd" and roof["kernel"] == "k_bwd_spheres"
    assert roof["bound"] == "hbm" and roof["peak"] == bench.HBM_PEAK_GBS
    achieved = sb["raster_bwd"] / 0.048e-3 / 1e9
    assert roof["achieved"] == pytest.approx(achieved, abs=0.1)
    assert roof["frac"] == pytest.approx(achieved / bench.HBM_PEAK_GBS, abs=1e-4)
    assert roof["traffic"] is None  # no summary for that workload
    # binning is reported as the longest stage, not as the dominant kernel
    assert roof["longest_stage"]["stage"] == "binning"
    assert set(kernels) == set(sb)


def _fake_profile(tmp_path, monkeypatch, kernel, nbytes, digest):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for rel in bench.TRAFFIC_SOURCES[kernel]:
        p = tmp_path / rel
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_text(f"source of {rel}\n")
    (tmp_path / "profiles").mkdir()
    rec = {"kernel": kernel, "bytes": nbytes, "sources_sha256_16": digest or bench.sources_hash(kernel),
           "valu_active": 0.25}
    (tmp_path / "profiles" / "wl.md").write_text("# summary\n\n    TRAFFIC " + json.dumps(rec) + "\n")


def test_traffic_is_reported_while_the_sources_match(tmp_path, monkeypatch):
    _fake_profile(tmp_path, monkeypatch, "k_bwd_spheres", 123456, None)
    assert bench.measured_traffic("k_bwd_spheres", "wl") == 123456
    assert bench.measured_record("k_bwd_spheres", "wl")["valu_active"] == 0.25
    # the stage of that kernel carries the traffic, its ratio to the
    # compulsory bytes and the VALU share
    n, H, W, C = 1000, 64, 64, 3
    avg = {"project": 0.01, "binning": 0.01, "raster_fwd": 0.01, "merge": 0.01,
           "raster_bwd": 0.02, "finalize": 0.01}
    _, kernels = bench.stage_roofline(avg, n, H, W, C, 500, "wl")
    k = kernels["raster_bwd"]
    assert k["traffic"] == 123456 and k["valu_active"] == 0.25
    assert k["traffic_ratio"] == pytest.approx(123456 / k["bytes_per_launch"], rel=1e-3)
    assert kernels["raster_fwd"]["traffic"] is None  # no record for it
    assert kernels["binning"]["traffic"] is None  # its kernels have none
    assert bench.measured_traffic("k_fwd_chunks", "wl") is None  # no record for it
    assert bench.measured_traffic("k_bwd_spheres", "other") is None  # no summary
    assert bench.measured_traffic("no_such_kernel", "wl") is None
    # a changed source makes the counters stale
    first = bench.TRAFFIC_SOURCES["k_bwd_spheres"][0]
    (tmp_path / first).write_text("changed\n")
    assert bench.measured_traffic("k_bwd_spheres", "wl") is None


def test_binning_launch_counts_follow_the_tile_bits():
    # a single tile: nothing to sort; 2^14 tiles: two 7-bit passes; the
    # 32-scene batch's 258,048 tiles: three 6-bit passes
    assert bench.binning_launches(1)["k_sort_scatter"] == 0
    one = bench.binning_launches(256)
    assert (one["k_sort_scatter"], one["k_sort_hist"]) == (1, 0)
    two = bench.binning_launches(16384)
    assert (two["k_sort_scatter"], two["k_sort_hist"]) == (2, 1)
    assert bench.binning_launches(258048)["k_sort_scatter"] == 3
    assert all(two[k] == 1 for k in ("k_emit", "k_ranges", "k_plan"))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
