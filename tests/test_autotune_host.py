"""Host-side checks of the autotuner: cache keys, the JSON cache and the
coordinate search (driven by a synthetic cost, no GPU)."""
import json

from paper_2004_07484_amd import _capi
from paper_2004_07484_amd import autotune as at


def test_cache_key_buckets():
    k1 = at.cache_key("gfx950", 1_000_000, 1024 * 1024, 8, 8)
    k2 = at.cache_key("gfx950", 600_000, 1000 * 1000, 8, 8)
    k3 = at.cache_key("gfx950", 1_100_000, 1024 * 1024, 8, 8)
    assert k1 == k2  # same power-of-two buckets
    assert k1 != k3
    assert at.cache_key("gfx950", 10, 64, 3, 5, B=32) != at.cache_key("gfx950", 10, 64, 3, 5)
    assert at.cache_key("gfx950", 0, 1, 1, 1).startswith("gfx950|n2^0|px2^0")


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = at.TuneCache(path)
    assert c.get("x") is None
    c.put("x", {"raster_blocks": 2048, "chunk": 256}, 0.5)
    again = at.TuneCache(path)
    assert again.get("x") == {"raster_blocks": 2048, "chunk": 256}
    data = json.load(open(path))
    assert data["x"]["ms"] == 0.5
    # a corrupt file reads as empty instead of failing
    open(path, "w").write("{not json")
    assert at.TuneCache(path).get("x") is None


def test_with_knobs_keeps_other_fields():
    p = _capi.make_params(gamma=0.3, eps=2e-5, K=7, max_pairs=1234)
    q = at.with_knobs(p, {"chunk": 256, "raster_blocks": 8192})
    assert (q.gamma, q.eps, q.K, q.max_pairs) == (p.gamma, p.eps, p.K, p.max_pairs)
    assert (q.chunk, q.raster_blocks, p.chunk, p.raster_blocks) == (256, 8192, 0, 0)
    assert at.knobs_of(q) == {"raster_blocks": 8192, "chunk": 256, "store_hits": 0,
                             "bwd_tiles": 0}
    r = at.with_knobs(p, {"store_hits": 1})
    assert r.flags & _capi.PULSAR_STORE_HITS and at.knobs_of(r)["store_hits"] == 1
    assert at.with_knobs(r, {"store_hits": 0}).flags == p.flags


def test_coordinate_search_finds_separable_optimum():
    calls = []

    def cost(k):
        calls.append(dict(k))
        if k["chunk"] == 1024:
            return None  # rejected by the library for this workload
        return abs(k["raster_blocks"] - 8192) / 1000 + abs(k["chunk"] - 256) / 100 + 1.0

    knobs = (("raster_blocks", (1024, 4096, 8192)), ("chunk", (64, 256, 1024)))
    best, ms, trials = at.search(cost, {"raster_blocks": 0, "chunk": 0}, knobs)
    assert best == {"raster_blocks": 8192, "chunk": 256}
    assert ms == 1.0
    assert len(trials) == len(calls)
    assert any(m is None for _, m in trials)


def test_search_rejects_invalid_start():
    import pytest
    with pytest.raises(ValueError):
        at.search(lambda k: None, {"raster_blocks": 0, "chunk": 0})
