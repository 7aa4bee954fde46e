"""The seeded generators: determinism, counter-based slicing, ranges and
distribution shape of the synthetic star-schema tables."""
import numpy as np

import tqp_datagen as dg


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 0: the first outputs of the generator whose state
    # advances by the golden-ratio increment (Steele, Lea, Flood 2014).
    x = np.array([0, 0x9E3779B97F4A7C15, (2 * 0x9E3779B97F4A7C15) % 2 ** 64], np.uint64)
    out = dg.splitmix64(x)
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4
    assert int(out[2]) == 0x06C45D188009454F


def test_counter_based_slices_agree():
    a = dg.uniform_int(7, 3, 10_000, 0, 2557)
    b = dg.uniform_int(7, 3, 4_000, 0, 2557, start=6_000)
    assert np.array_equal(a[6_000:], b)
    assert np.array_equal(a, dg.uniform_int(7, 3, 10_000, 0, 2557))
    assert not np.array_equal(a, dg.uniform_int(8, 3, 10_000, 0, 2557))


def test_uniform_ranges_and_mean():
    v = dg.uniform_int(0, 1, 1_000_000, 1, 5001)
    assert v.min() == 1 and v.max() == 5000
    assert abs(v.mean() - 2500.5) < 10


def test_config1_shape():
    c = dg.config1(0)
    f, d = c["fact"], c["dim"]
    assert f["fk"].dtype == np.int32 and f["qty"].dtype == np.int64
    assert len(f["fk"]) == 1_000_000 and len(d["pk"]) == 10_000
    assert np.array_equal(np.sort(d["pk"]), np.arange(10_000))
    assert f["day"].min() >= 0 and f["day"].max() < dg.DAY_DOMAIN
    assert d["cat"].min() == 0 and d["cat"].max() == 24


def test_zipf_top_share():
    N = 200_000
    r = dg.zipf_ranks(0, 1, 2_000_000, N, 1.0)
    H = np.sum(1.0 / np.arange(1, N + 1))
    share = np.mean(r == 1)
    assert abs(share - 1.0 / H) < 0.003
    assert r.min() == 1 and r.max() <= N
    u = dg.zipf_ranks(0, 1, 200_000, 100, 0.0)      # s = 0 is uniform
    assert abs(np.mean(u == 1) - 0.01) < 0.002


def test_config5_params():
    p = dg.config5_params(0)
    assert len(p) == 256
    assert all(10_000 <= q["n_fact"] <= 20_000_000 for q in p)
    assert all(q["n_dim"] == max(1, q["n_fact"] // 20) for q in p)
    assert all(1 <= q["groups"] <= q["n_dim"] for q in p)
