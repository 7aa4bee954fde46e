"""The GPU pipelines against the stored expected results under
tests/golden/ (the oracle's answers, written by make_golden.py), without
calling the oracle: a small seeded instance of every workload."""
import json
import os

import numpy as np
import pytest

import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        return json.load(fh)


def dev(d):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in d.items()}


def test_golden_star_queries():
    from paper_2209_04579_amd.pipeline import StarQuery
    g = golden("q1_small_star")
    c = dg.config1(0, 200_000, 2_000)
    q = StarQuery(dev(c["fact"]), dev(c["dim"]), c["day_cut"], mode="q1")
    q.run()
    r = q.result()
    assert (r["key"].tolist(), r["sum_qty"].tolist(), r["count"].tolist()) == \
        (g["key"], g["sum_qty"], g["count"])
    g = golden("q2_skewed_star")
    c = dg.config2(0, 200_000, 20_000)
    q = StarQuery(dev(c["fact"]), dev(c["dim"]), c["day_cut"], mode="q2")
    q.run()
    r = q.result()
    for k in ("a_key", "a_qty", "a_price", "a_count"):
        assert r[k].tolist() == g[k], k
    assert len(r["b_key"]) == g["b_groups"]
    assert int(r["b_qty"].sum()) == g["b_qty_total"] and int(r["b_count"].sum()) == g["b_count_total"]


def test_golden_q6_q14_predict():
    from paper_2209_04579_amd.pipeline import PredictQuery, Q14Query, Q6Scan
    g = golden("q6_scan")
    c = dg.config_q6(0, 500_000)
    q = Q6Scan(dev(c["items"]), c)
    q.run()
    assert q.result() == {"sum": g["sum"], "count": g["count"]}
    g = golden("q14_join")
    c = dg.config_q14(0, 500_000, 20_000)
    q = Q14Query(dev(c["items"]), dev(c["part"]), c["prefix"], c["ship_lo"], c["ship_hi"])
    q.run()
    r = q.result()
    assert (r["promo_rev"], r["total_rev"], r["count"], r["promo_count"]) == \
        (g["promo_rev"], g["total_rev"], g["count"], g["promo_count"])
    g = golden("predict_query")
    c = dg.config_predict(0, 200_000)
    q = PredictQuery(dev(c["reviews"]), c["model"], c["nfeat"], c["hidden"], c["classes"],
                     c["year_min"], c["nratings"])
    q.run()
    r = q.result()
    assert r["positive"].tolist() == g["positive"] and r["count"].tolist() == g["count"]
