"""Host-side parts of the autotuner: the library's knob registry (no kernel
launches) and the JSON cache of tuned settings."""
import pytest

pytest.importorskip("torch")


def test_knob_registry_ranges_and_errors():
    from paper_2209_04579_amd import TqpError, tune_knobs, tune_set
    knobs = tune_knobs()
    assert set(knobs) == {"filter.per_cu", "sort.per_cu", "rle.per_cu", "match.per_cu",
                          "gbscan.per_cu", "part.ovf_cap", "sort.mode", "semijoin.per_cu",
                          "semijoin.wg"}
    for name, (value, lo, hi) in knobs.items():
        assert 0 <= lo <= value <= hi
    name, (value, lo, hi) = "filter.per_cu", knobs["filter.per_cu"]
    try:
        tune_set(name, hi)
        assert tune_knobs()[name][0] == hi
        with pytest.raises(TqpError):
            tune_set(name, hi + 1)
        with pytest.raises(TqpError):
            tune_set(name, lo - 1)
        with pytest.raises(TqpError):
            tune_set("no.such.knob", 1)
        assert tune_knobs()[name][0] == hi
    finally:
        tune_set(name, value)


def test_cache_roundtrip(tmp_path):
    from paper_2209_04579_amd import autotune
    path = str(tmp_path / "tune.json")
    key = autotune.cache_key("star_q2", 60_000_000, "zipf1", "int32")
    assert "log2n=25" in key and "star_q2" in key and "int32" in key and "zipf1" in key
    assert autotune.load(path, key) is None
    autotune.save(path, key, {"filter.per_cu": 3})
    autotune.save(path, "other", {"sort.per_cu": 1})
    assert autotune.load(path, key) == {"filter.per_cu": 3}
    assert autotune.load(path, "other") == {"sort.per_cu": 1}


class _FakePlan:
    """A plan whose time is a function of its setting (no GPU): time_plan is
    replaced by a lookup so the descent itself is tested on the host."""
    def __init__(self, t):
        self.t = t


def test_tune_params_descends_to_the_best_setting(monkeypatch):
    from paper_2209_04579_amd import autotune
    cost = lambda t: (t["bits"] - 17) ** 2 + abs(t["leaves"] - 1704) / 100 + 1.0
    monkeypatch.setattr(autotune, "time_plan", lambda plan, reps=3: cost(plan.t))
    best, ms, timings = autotune.tune_params(
        _FakePlan, {"bits": [15, 16, 17, 18], "leaves": [852, 1704, 3408]},
        {"bits": 15, "leaves": 852})
    assert best == {"bits": 17, "leaves": 1704} and ms == 1.0
    assert len(timings) <= 4 + 3 + 4 + 3


def test_tune_cached_tunes_once(tmp_path, monkeypatch):
    from paper_2209_04579_amd import autotune
    path = str(tmp_path / "sub" / "tune.json")
    calls = []

    def tuner():
        calls.append(1)
        return {"bits": 16}, 2.5, {}
    s1, ms1, hit1 = autotune.tune_cached(path, "k", tuner)
    s2, ms2, hit2 = autotune.tune_cached(path, "k", tuner)
    assert (s1, ms1, hit1) == ({"bits": 16}, 2.5, False)
    assert (s2, ms2, hit2) == ({"bits": 16}, 2.5, True)
    assert len(calls) == 1
