"""Autotuner for the renderer's result-neutral launch knobs.

The paper picked its tile and block sizes empirically for its GPU (App. B,
Step 1 and Step 2). Here the knobs that can change without changing what is
computed are measured on the device instead:

  raster_blocks  size of the persistent raster grid (never changes the image)
  chunk          sphere records per raster work item (changes only the
                 summation order of the blend)
  store_hits     keep each pixel's K nearest hits for the backward
                 (PULSAR_STORE_HITS, the paper's choice) or recompute them
                 (changes only the summation order of the gradients)
  bwd_tiles      recompute them walking the tile lists (PULSAR_BWD_TILES)
                 or walking the spheres (the default; changes only the
                 summation order of the gradients)

The 8x8 tile is not a knob: one wave64 owns one tile, lane = pixel, which the
kernels rely on for their LDS layouts and ballots.

A search times one forward + backward per candidate with HIP events on the
caller's stream (median of `reps` after `warmup` runs), one knob at a time in
the order above, each starting from the best values found so far. The choice
is cached in a JSON file keyed by (GPU architecture, sphere-count bucket,
pixel-count bucket, C, K, scene-count bucket); the file is read once per
process and written atomically.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
import threading
from typing import Callable, Dict, Iterable, List, Optional, Tuple

from . import _capi

KNOBS: Tuple[Tuple[str, Tuple[int, ...]], ...] = (
    ("raster_blocks", (1024, 2048, 4096, 8192, 16384)),
    ("chunk", (64, 128, 192, 256, 320, 512)),
    ("store_hits", (0, 1)),
    ("bwd_tiles", (0, 1)),
)
# knobs that are bits of params.flags rather than fields of their own
FLAG_KNOBS = {"store_hits": _capi.PULSAR_STORE_HITS, "bwd_tiles": _capi.PULSAR_BWD_TILES}


def get_knob(params, name: str) -> int:
    if name in FLAG_KNOBS:
        return int(bool(int(params.flags) & FLAG_KNOBS[name]))
    return int(getattr(params, name))


def set_knob(params, name: str, value: int) -> None:
    if name in FLAG_KNOBS:
        bit = FLAG_KNOBS[name]
        params.flags = (int(params.flags) | bit) if int(value) else (int(params.flags) & ~bit)
    else:
        setattr(params, name, int(value))

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pulsar_amd_autotune.json")


def _bucket(x: int) -> int:
    """Power-of-two bucket: ceil(log2(max(x, 1)))."""
    return int(math.ceil(math.log2(max(int(x), 1))))


def cache_key(arch: str, n: int, pixels: int, C: int, K: int, B: int = 1) -> str:
    return f"{arch}|n2^{_bucket(n)}|px2^{_bucket(pixels)}|C{int(C)}|K{int(K)}|B2^{_bucket(B)}"


def knobs_of(params) -> Dict[str, int]:
    return {name: get_knob(params, name) for name, _ in KNOBS}


def with_knobs(params, knobs: Dict[str, int]):
    """A copy of a pulsar_params_t with the given knob values."""
    p = _capi.pulsar_params_t()
    ctypes_copy(p, params)
    for k, v in knobs.items():
        set_knob(p, k, v)
    return p


def ctypes_copy(dst, src) -> None:
    for name, _ in src._fields_:
        setattr(dst, name, getattr(src, name))


class TuneCache:
    """JSON cache of tuned knobs, loaded once, safe to share between threads."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or os.environ.get("PULSAR_AUTOTUNE_CACHE", DEFAULT_CACHE)
        self._lock = threading.Lock()
        self._data: Optional[dict] = None

    def _load(self) -> dict:
        if self._data is None:
            try:
                with open(self.path) as f:
                    data = json.load(f)
                self._data = data if isinstance(data, dict) else {}
            except (OSError, ValueError):
                self._data = {}
        return self._data

    def get(self, key: str) -> Optional[Dict[str, int]]:
        with self._lock:
            entry = self._load().get(key)
            if not isinstance(entry, dict) or "knobs" not in entry:
                return None
            return {k: int(v) for k, v in entry["knobs"].items() if k in dict(KNOBS)}

    def put(self, key: str, knobs: Dict[str, int], ms: float) -> None:
        with self._lock:
            data = self._load()
            data[key] = {"knobs": {k: int(v) for k, v in knobs.items()}, "ms": float(ms)}
            d = os.path.dirname(self.path) or "."
            os.makedirs(d, exist_ok=True)
            fd, tmp = tempfile.mkstemp(dir=d, prefix=".pulsar_tune_")
            with os.fdopen(fd, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def search(measure: Callable[[Dict[str, int]], Optional[float]], start: Dict[str, int],
           knobs: Iterable[Tuple[str, Iterable[int]]] = KNOBS) -> Tuple[Dict[str, int], float,
                                                                          List[tuple]]:
    """Coordinate search: for each knob in turn, try every value with the
    others at their best so far. `measure` returns milliseconds, or None for a
    candidate the library rejects. Returns (best knobs, best ms, all trials)."""
    best = dict(start)
    best_ms = measure(best)
    if best_ms is None:
        raise ValueError(f"the starting knobs {best} are not valid for this workload")
    trials = [(dict(best), best_ms)]
    for name, values in knobs:
        for v in values:
            if v == best.get(name):
                continue
            cand = dict(best)
            cand[name] = int(v)
            ms = measure(cand)
            trials.append((dict(cand), ms))
            if ms is not None and ms < best_ms:
                best, best_ms = cand, ms
    return best, best_ms, trials


def event_timer(run: Callable[[object], None], reps: int = 5, warmup: int = 2):
    """measure(params) for `search`: median HIP-event time of run(params) on the
    current stream, None when the library rejects the parameters."""
    import torch

    def measure_params(params) -> Optional[float]:
        stream = torch.cuda.current_stream()
        try:
            for _ in range(warmup):
                run(params)
        except _capi.PulsarError as e:
            if e.code in (_capi.PULSAR_ERR_UNSUPPORTED, _capi.PULSAR_ERR_INVALID_ARGUMENT,
                          _capi.PULSAR_ERR_WORKSPACE):
                return None
            raise
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run(params)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        times.sort()
        return float(times[len(times) // 2])

    return measure_params


def arch_name() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return str(getattr(props, "gcnArchName", props.name)).split(":")[0]


def tune(run: Callable[[object], None], base_params, key: Optional[str] = None,
         cache: Optional[TuneCache] = None, reps: int = 5, warmup: int = 2,
         force: bool = False):
    """Tuned copy of base_params for the workload `run(params)` enqueues (one
    forward + backward). Uses the cache entry for `key` unless force is set;
    stores a fresh result under `key` when a cache is given. Returns
    (params, info dict)."""
    if cache is not None and key is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            return with_knobs(base_params, hit), {"cached": True, "knobs": hit}
    measure_params = event_timer(run, reps, warmup)
    best, best_ms, trials = search(lambda k: measure_params(with_knobs(base_params, k)),
                                   knobs_of(base_params))
    if cache is not None and key is not None:
        cache.put(key, best, best_ms)
    return with_knobs(base_params, best), {"cached": False, "knobs": best, "ms": best_ms,
                                           "trials": [(k, None if m is None else round(m, 4))
                                                      for k, m in trials]}
