"""GPU parity of whole queries: filter -> sort -> merge join -> group-by on the
star-schema workloads, at the small size and at the full benchmark size,
bit-exact against the CPU oracle's whole-query statement."""
import numpy as np
import pytest

import oracle
import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def to_dev(tbl):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in tbl.items()}


def check_q1(cfg):
    from paper_2209_04579_amd.pipeline import StarQuery
    q = StarQuery(to_dev(cfg["fact"]), to_dev(cfg["dim"]), cfg["day_cut"], mode="q1")
    q.run()
    got = q.result()
    want = oracle.q1(cfg["fact"], cfg["dim"], cfg["day_cut"])
    assert not want["overflow"]
    for k in ("key", "sum_qty", "count"):
        assert np.array_equal(got[k], want[k]), k
    keep = int(np.sum(cfg["fact"]["day"] < cfg["day_cut"]))
    assert got["rows_filtered"] == keep
    return q


@pytest.mark.parametrize("seed", [0, 1])
def test_q1_small_config(seed):
    check_q1(dg.config1(seed))


def test_q1_degenerate_tables():
    c = dg.config1(2, n_fact=5, n_dim=3)
    check_q1(c)
    c = dg.config1(3, n_fact=50_000, n_dim=1)
    check_q1(c)
    c = dg.config1(4, n_fact=20_000, n_dim=500)
    c["day_cut"] = 0                                       # nothing passes
    check_q1(c)


def test_q1_replay_is_identical():
    q = check_q1(dg.config1(0))
    first = q.result()
    for _ in range(3):
        q.run()
        again = q.result()
        for k in ("key", "sum_qty", "count"):
            assert np.array_equal(again[k], first[k])


def check_q2(cfg, overlap=False, fused=True):
    from paper_2209_04579_amd.pipeline import StarQuery
    q = StarQuery(to_dev(cfg["fact"]), to_dev(cfg["dim"]), cfg["day_cut"], mode="q2",
                  overlap=overlap, fused=fused)
    q.run()
    got = q.result()
    want = oracle.q2(cfg["fact"], cfg["dim"], cfg["day_cut"])
    assert not want["overflow"]
    for k in ("a_key", "a_qty", "a_price", "a_count", "b_key", "b_qty", "b_count"):
        assert np.array_equal(got[k], want[k]), k
    return got


def test_q2_reduced_size():
    check_q2(dg.config2(0, n_fact=3_000_000, n_dim=100_000))


def test_q2_with_the_dimension_sort_on_a_second_stream():
    cfg = dg.config2(5, n_fact=3_000_000, n_dim=200_000)
    assert check_q2(cfg, overlap=True)["pairs"] > 0


def test_q2_with_a_separate_filter_and_sort():
    """The unfused plan (the filter writes the kept rows, the sort reads them)."""
    cfg = dg.config2(6, n_fact=2_000_000, n_dim=150_000)
    assert check_q2(cfg, fused=False)["pairs"] > 0
    assert check_q2(cfg, overlap=True, fused=False)["pairs"] > 0


def test_q2_full_size():
    got = check_q2(dg.config2(0))
    assert got["rows_filtered"] > 29_000_000
    assert got["pairs"] == got["rows_filtered"]


PLANS3 = ["semijoin", "sort"]


def run_q3(cfg, dev_cfg=None, plan="semijoin"):
    from paper_2209_04579_amd.pipeline import StarQuery3
    d = dev_cfg or {t: to_dev(cfg[t]) for t in ("fact", "d1", "d2", "d3")}
    q = StarQuery3(d["fact"], d["d1"], d["d2"], d["d3"], cfg["attr_cut"], plan=plan)
    q.run()
    return q, q.result()


def check_q3(cfg, dev_cfg=None, plan="semijoin", want=None):
    q, got = run_q3(cfg, dev_cfg, plan)
    want = want or oracle.q3(cfg)
    assert not want["overflow"]
    for k in ("key", "sum_qp", "count"):
        assert np.array_equal(got[k], want[k]), k
    # COUNT conserves the last join's pairs
    assert int(got["count"].sum()) == got["pairs"][2]
    if plan == "semijoin":
        # pk is unique in every dimension, so every reduced row joins once
        assert got["pairs"] == [got["reduced"]] * 3
    return q, got


@pytest.mark.parametrize("plan", PLANS3)
def test_q3_reduced_size(plan):
    cfg = dg.config3(0, n_fact=3_000_000, dims=(100_000, 10_000, 25))
    _, got = check_q3(cfg, plan=plan)
    assert got["pairs"][0] > 0 and got["pairs"][2] > 0


@pytest.mark.parametrize("plan", PLANS3)
def test_q3_degenerate(plan):
    # one-row dims, and dims whose filter keeps nothing
    c = dg.config3(1, n_fact=20_000, dims=(1, 1, 1))
    check_q3(c, plan=plan)
    c = dg.config3(2, n_fact=50_000, dims=(3000, 500, 25))
    c["attr_cut"] = 0
    _, got = check_q3(c, plan=plan)
    assert got["pairs"] == [0, 0, 0] and len(got["key"]) == 0
    c = dg.config3(3, n_fact=7, dims=(50, 20, 25))
    check_q3(c, plan=plan)


def test_q3_fact_keys_outside_the_dimensions():
    # foreign keys below and above every dimension key, and dims whose keys
    # do not start at 0: the key sets must reject them, not wrap
    c = dg.config3(5, n_fact=200_003, dims=(5000, 700, 25))
    for t, off in (("d1", 1000), ("d2", -300), ("d3", 7)):
        c[t]["pk"] = (c[t]["pk"] + off).astype(np.int32)
    f = c["fact"]
    f["fk1"] = (f["fk1"] + 990).astype(np.int32)
    f["fk2"] = (f["fk2"] - 310).astype(np.int32)
    f["fk3"] = (f["fk3"] + 5).astype(np.int32)
    f["fk1"][::101] = np.iinfo(np.int32).min
    f["fk2"][::103] = np.iinfo(np.int32).max
    want = oracle.q3(c)
    for plan in PLANS3:
        check_q3(c, plan=plan, want=want)


@pytest.mark.parametrize("plan", PLANS3)
def test_q3_replay_is_identical(plan):
    cfg = dg.config3(4, n_fact=1_000_000, dims=(50_000, 5_000, 25))
    q, first = check_q3(cfg, plan=plan)
    for _ in range(2):
        q.run()
        again = q.result()
        for k in ("key", "sum_qp", "count"):
            assert np.array_equal(again[k], first[k])


@pytest.mark.parametrize("plan", PLANS3)
def test_q3_graph_replays_match_eager(plan):
    """The whole star query captured through the library into one HIP graph:
    every replay gives the eager run's (and the oracle's) groups, with eager
    work and synchronizations between the replays and the outputs cleared
    first, so each replay recomputes them."""
    import paper_2209_04579_amd as tqp
    cfg = dg.config3(6, n_fact=1_500_000, dims=(60_000, 6_000, 25))
    q, first = check_q3(cfg, plan=plan)
    g = tqp.batch_capture(q.run)
    for i in range(3):
        for t in q.g_out:
            t.zero_()
        g.run()
        again = q.result()
        for k in ("key", "sum_qp", "count"):
            assert np.array_equal(again[k], first[k]), (i, k)
        q.run()                                  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.timeout(400)
def test_q3_full_size():
    """The 600M-row three-dimension star at full size, both plans: tables
    drawn on the GPU (bit-identical to the host generator), the oracle run on
    host copies."""
    from tqp_datagen import device as dgd
    dcfg = dgd.config3(0, device="cuda")
    cfg = {t: {k: v.cpu().numpy() for k, v in dcfg[t].items()} for t in ("fact", "d1", "d2", "d3")}
    cfg["attr_cut"] = dcfg["attr_cut"]
    want = oracle.q3(cfg)
    for plan in PLANS3:
        q, got = check_q3(cfg, dcfg, plan=plan, want=want)
        assert len(got["key"]) == 125
        del q
        torch.cuda.empty_cache()
    assert 4_000_000 < got["pairs"][2] < 5_600_000
