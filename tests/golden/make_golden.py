"""Writes the stored expected results under tests/golden/ from the CPU oracle.

The paper prints no result values (its evaluation reports speed-ups only,
Section 2.3), so no fixture holds a value of the paper's; each one is the
oracle's answer, written by this script (which calls only ``oracle`` and the
seeded generators), for a small seeded instance of one workload.  The tests
recompute every fixture with the oracle (a change to the oracle's arithmetic
must then be deliberate) and compare the GPU pipelines against the stored
values.  Run from the repository root: ``python tests/golden/make_golden.py``.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                     # noqa: E402
import tqp_datagen as dg          # noqa: E402


def ints(a):
    return [int(x) for x in a]


def fixtures():
    """name -> (description, generator call, oracle result as plain ints)."""
    out = {}
    c1 = dg.config1(0, 200_000, 2_000)
    r = oracle.q1(c1["fact"], c1["dim"], c1["day_cut"])
    out["q1_small_star"] = {
        "query": "star query: WHERE day < 1278, JOIN fk = pk, GROUP BY cat: SUM(qty), COUNT",
        "generator": "config1(seed=0, n_fact=200000, n_dim=2000)",
        "key": ints(r["key"]), "sum_qty": ints(r["sum_qty"]), "count": ints(r["count"])}
    c2 = dg.config2(0, 200_000, 20_000)
    r = oracle.q2(c2["fact"], c2["dim"], c2["day_cut"])
    out["q2_skewed_star"] = {
        "query": "skewed star: (a) GROUP BY flag*2 + cat mod 2: SUM(qty), SUM(price), COUNT; "
                 "(b) GROUP BY fk: SUM(qty), COUNT",
        "generator": "config2(seed=0, n_fact=200000, n_dim=20000)",
        "a_key": ints(r["a_key"]), "a_qty": ints(r["a_qty"]), "a_price": ints(r["a_price"]),
        "a_count": ints(r["a_count"]), "b_groups": len(r["b_key"]),
        "b_qty_total": int(sum(int(x) for x in r["b_qty"])),
        "b_count_total": int(sum(int(x) for x in r["b_count"]))}
    c6 = dg.config_q6(0, 500_000)
    r = oracle.q6(c6)
    out["q6_scan"] = {"query": "Q6 shape: SUM(price * discount), COUNT over one year of ship dates, "
                               "discount in [5, 7], quantity < 24",
                      "generator": "config_q6(seed=0, n=500000)", "sum": r["sum"], "count": r["count"]}
    c14 = dg.config_q14(0, 500_000, 20_000)
    r = oracle.q14(c14)
    out["q14_join"] = {"query": "Q14 shape: promo and total revenue over one month, JOIN partkey = pk, "
                                "type LIKE prefix%",
                       "generator": "config_q14(seed=0, n_items=500000, n_part=20000)",
                       "promo_rev": r["promo_rev"], "total_rev": r["total_rev"], "count": r["count"],
                       "promo_count": r["promo_count"]}
    cp = dg.config_predict(0, 200_000)
    r = oracle.q_predict(cp)
    out["predict_query"] = {"query": "WHERE year >= 2016, PREDICT (fp32 8 -> 16 -> 2 MLP), "
                                     "GROUP BY rating: SUM(CASE class = 1), COUNT",
                            "generator": "config_predict(seed=0, n=200000)",
                            "positive": ints(r["positive"]), "count": ints(r["count"])}
    return out


if __name__ == "__main__":
    for name, fx in fixtures().items():
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(fx, fh, indent=1)
        print("wrote", name)
