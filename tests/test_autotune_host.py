"""Host-side behaviour of the GEMM autotuner's settings (no GPU): the cache
round trip and the scoped application of a workload's settings."""
import json

from paper_2508_07610_amd import autotune as AT
from paper_2508_07610_amd import mpdo as M


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "cache.json")
    assert AT.load(path, "k") is None
    s = {"q2_gram_C": {"tile": 32, "form": 3, "split_scale": 2.0, "ms": 1.0, "default_ms": 2.0}}
    AT.save(path, "k", s)
    AT.save(path, "other", {})
    assert AT.load(path, "k") == s
    assert set(json.load(open(path))) == {"k", "other"}


def test_applied_scopes_the_settings():
    AT.reset()
    gc = AT.SITE_INDEX["q2_gram_C"]
    w1 = AT.SITE_INDEX["q3_W1"]
    M.tune_set(w1, 64, 4, 0.0)
    before = AT.snapshot()
    with AT.applied({"q2_gram_C": {"tile": 32, "form": 3, "split_scale": 2.0}}):
        assert M.tune_get(gc) == (32, 3, 2.0)
        assert M.tune_get(w1) == (0, 0, 0.0)      # everything else at the built-in choice
    assert AT.snapshot() == before
    with AT.applied(None):
        assert all(t == (0, 0, 0.0) for t in AT.snapshot())
    assert AT.snapshot() == before
    AT.reset()


def test_committed_cache_names_known_sites():
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2508_07610_amd",
                        "autotune_cache.json")
    data = json.load(open(path))
    assert data
    for key, settings in data.items():
        for site, s in settings.items():
            assert site in AT.SITE_INDEX, (key, site)
            assert s["tile"] in (0, 32, 64) and s["form"] in (0, 3, 4) and s["split_scale"] >= 0
