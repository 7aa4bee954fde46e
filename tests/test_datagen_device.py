"""The torch generators draw the same integers as the numpy ones (checked on
the CPU device)."""
import numpy as np
import pytest

import tqp_datagen as dg

torch = pytest.importorskip("torch")
from tqp_datagen import device as dd  # noqa: E402


def test_raw_and_uniform_match_host():
    for seed, stream, lo, hi in ((0, 1, 0, 10_000), (7, 3, 1, 5001), (3, 9, -5, 2 ** 31),
                                 (1, 2, 0, 1 << 32), (2, 4, -(2 ** 31), 2 ** 31 - 1)):
        h = dg.uniform_int(seed, stream, 50_000, lo, hi, np.int64, start=123)
        d = dd.uniform_int(seed, stream, 50_000, lo, hi, "cpu", start=123).numpy()
        assert np.array_equal(h, d), (seed, stream, lo, hi)
    assert np.array_equal(dg.raw_u64(5, 6, 1000).view(np.int64),
                          dd.raw_u64(5, 6, 1000, "cpu").numpy())


def test_permutation_and_zipf_match_host():
    assert np.array_equal(dg.permutation(4, 4, 20_000), dd.permutation(4, 4, 20_000, "cpu").numpy())
    h = dg.zipf_ranks(1, 1, 100_000, 50_000, 1.0)
    d = dd.zipf_ranks(1, 1, 100_000, 50_000, 1.0, "cpu").numpy()
    assert np.mean(h == d) > 0.9999


def test_config5_instance_matches_host():
    h = dg.config5(0, instances=3, fact_hi=50_000)
    d = dd.config5(0, instances=3, fact_hi=50_000, device="cpu")
    for a, b in zip(h, d):
        for t in ("fact", "dim"):
            for k in a[t]:
                if k == "fk":
                    assert np.mean(a[t][k] == b[t][k].numpy()) > 0.9999
                else:
                    assert np.array_equal(a[t][k], b[t][k].numpy()), (t, k)


def test_config3_matches_host():
    h = dg.config3(2, n_fact=30_000, dims=(5000, 700, 25))
    d = dd.config3(2, n_fact=30_000, dims=(5000, 700, 25), device="cpu")
    assert h["attr_cut"] == d["attr_cut"]
    for t in ("fact", "d1", "d2", "d3"):
        assert set(h[t]) == set(d[t])
        for k in h[t]:
            assert h[t][k].dtype == d[t][k].numpy().dtype, (t, k)
            assert np.array_equal(h[t][k], d[t][k].numpy()), (t, k)
