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
    key = autotune.cache_key("star_q2", 60_000_000, "zipf1")
    assert "log2n=25" in key and "star_q2" in key
    assert autotune.load(path, key) is None
    autotune.save(path, key, {"filter.per_cu": 3})
    autotune.save(path, "other", {"sort.per_cu": 1})
    assert autotune.load(path, key) == {"filter.per_cu": 3}
    assert autotune.load(path, "other") == {"sort.per_cu": 1}
