"""Autotuner logic on the CPU (timings faked; no device work)."""
import json

from paper_1911_08275_amd import autotune


def test_signature_buckets():
    a = autotune.signature("xi", 10**6, 0, 420.0 ** 3, 25.0, 0.0, "fp32", True, True)
    b = autotune.signature("xi", 10**6 + 10, 0, 420.0 ** 3, 25.0, 0.0, "fp32", True, True)
    c = autotune.signature("wp", 10**6, 0, 420.0 ** 3, 25.0, 40.0, "fp32", True, True)
    d = autotune.signature("xi", 10**6, 0, 420.0 ** 3, 25.0, 0.0, "fp64", True, True)
    assert a == b and a != c and a != d and c.startswith("wp/")


def test_tune_picks_fastest_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("CP_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    calls = []

    def run(r):
        calls.append(r)
        return {(2, 2, 2): 1.0, (3, 3, 3): 0.5}.get(r, 2.0)

    best = autotune.tune(run, "sig", candidates=[(2, 2, 1), (2, 2, 2), (3, 3, 3)], reps=2)
    assert best == (3, 3, 3)
    assert len(calls) == 6
    stored = json.load(open(tmp_path / "cache.json"))
    assert stored["sig"]["refine"] == [3, 3, 3]
    # cached: no further runs
    assert autotune.tune(run, "sig", candidates=[(2, 2, 1)]) == (3, 3, 3)
    assert len(calls) == 6
    assert autotune.lookup("other") is None
