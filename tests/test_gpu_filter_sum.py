"""GPU parity for the fused WHERE + aggregate (tqp_filter_sum, the shape of
TPC-H Q6 in Section 2.3): SUM(a * b) and COUNT over the kept rows, against
the CPU oracle, bit for bit (int64 modulo 2^64), on seeded tables spanning
several tiles and ragged tails, every column dtype, wrap-around sums, no /
all rows kept, and the 60M-row Q6-shaped table."""
import numpy as np
import pytest

import oracle
import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = [0, 1, 15, 16, 17, 4095, 4096, 4097, 65_537, 1_000_003]
I64 = np.iinfo(np.int64)
DTS = [np.int8, np.int32, np.int64]


@pytest.fixture(scope="module")
def tqp():
    import paper_2209_04579_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(tqp, cols, preds, a=None, b=None):
    s = torch.empty(1, dtype=torch.int64, device="cuda")
    c = torch.empty(1, dtype=torch.int64, device="cuda")
    tqp.filter_sum_into([dev(x) for x in cols], preds, s, c,
                        None if a is None else dev(a), None if b is None else dev(b))
    torch.cuda.synchronize()
    return int(s.item()), int(c.item())


@pytest.mark.parametrize("n", SIZES)
def test_filter_sum_matches_oracle(tqp, n):
    cols = [dg.uniform_int(n, 1, n, -100, 100, np.int8),
            dg.uniform_int(n, 2, n, -1000, 1000, np.int32),
            dg.uniform_int(n, 3, n, -10 ** 6, 10 ** 6, np.int64)]
    a = dg.uniform_int(n, 4, n, -(1 << 31), 1 << 31, np.int64) * 3
    b = dg.uniform_int(n, 5, n, -50, 50, np.int32)
    for preds in ([(0, ">=", -30), (1, "<", 500), (2, "!=", 7)],
                  [(2, ">", 0), (2, "<=", 500_000)],
                  [(0, "==", 3)],
                  []):
        want = oracle.filter_sum(cols, preds, a, b)
        assert run(tqp, cols, preds, a, b) == want[:2], preds
        assert run(tqp, cols, preds, a) == oracle.filter_sum(cols, preds, a)[:2], preds
        assert run(tqp, cols, preds) == (0, want[1]), preds


@pytest.mark.parametrize("adt", DTS)
@pytest.mark.parametrize("bdt", DTS)
def test_filter_sum_value_dtypes(tqp, adt, bdt):
    n = 50_001
    info_a, info_b = np.iinfo(adt), np.iinfo(bdt)
    a = dg.uniform_int(7, 1, n, max(info_a.min, -(1 << 31)), min(info_a.max, (1 << 31) - 1), adt)
    b = dg.uniform_int(7, 2, n, max(info_b.min, -(1 << 31)), min(info_b.max, (1 << 31) - 1), bdt)
    key = dg.uniform_int(7, 3, n, 0, 10, np.int8)
    preds = [(0, "<", 7)]
    assert run(tqp, [key], preds, a, b) == oracle.filter_sum([key], preds, a, b)[:2]


def test_filter_sum_wraps_modulo_2_64(tqp):
    n = 9_000
    a = np.full(n, I64.max // 3, np.int64)
    b = np.full(n, 5, np.int8)
    key = np.arange(n, dtype=np.int32)
    s, c, exact = oracle.filter_sum([key], [(0, "<", 8_000)], a, b)
    assert not exact
    assert run(tqp, [key], [(0, "<", 8_000)], a, b) == (s, c)


def test_filter_sum_none_all_and_outside_literals(tqp):
    n = 20_000
    c8 = dg.uniform_int(1, 1, n, -128, 128, np.int8)
    a = dg.uniform_int(1, 2, n, 0, 1000, np.int64)
    assert run(tqp, [c8], [(0, ">=", 200)], a) == (0, 0)
    assert run(tqp, [c8], [(0, ">", -1000)], a) == (int(a.sum()), n)
    assert run(tqp, [c8], [], a, c8) == oracle.filter_sum([c8], [], a, c8)[:2]


@pytest.mark.parametrize("ncols", [2, 3, 4, 5])
def test_filter_sum_columns_loaded_together(tqp, ncols):
    """Predicates interleaved over up to five columns of mixed dtypes (up to
    four are loaded together per tile, five take the per-column path), with
    the value operands among the predicate columns, outside them, or both."""
    n = 300_007
    dts = [np.int64, np.int8, np.int32, np.int64, np.int32]
    spans = [(-10 ** 6, 10 ** 6), (-100, 100), (-1000, 1000), (0, 50), (-7, 7)]
    cols = [dg.uniform_int(ncols, 30 + c, n, lo, hi, dts[c]) for c, (lo, hi) in
            enumerate(spans[:ncols])]
    cuts = [(">=", -600_000), ("<", 90), (">", -900), ("!=", 13), ("<=", 5)]
    preds = []
    for rep in range(2):          # each column's predicates far apart in the list
        for c in range(ncols):
            op, lit = cuts[c]
            if len(preds) < 8:        # the most a call takes
                preds.append((c, op, lit + rep * (1 if op in ("<", "<=") else -1)))
    price = dg.uniform_int(ncols, 40, n, -(1 << 31), 1 << 31, np.int64)
    for a, b in ((price, cols[1]), (cols[0], cols[ncols - 1]), (price, None), (cols[2 % ncols], None),
                 (cols[1], cols[1])):
        want = oracle.filter_sum(cols, preds, a, b)[:2]
        assert run(tqp, cols, preds, a, b) == want
    # the same predicate columns through their own device tensors as a and b
    dcols = [dev(x) for x in cols]
    s_ = torch.empty(1, dtype=torch.int64, device="cuda")
    c_ = torch.empty(1, dtype=torch.int64, device="cuda")
    old = tqp.tune_knobs()["filter.per_cu"][0]
    try:
        for per_cu in (1, old, 8):
            tqp.tune_set("filter.per_cu", per_cu)
            tqp.filter_sum_into(dcols, preds, s_, c_, dcols[0], dcols[ncols - 1])
            torch.cuda.synchronize()
            assert (int(s_.item()), int(c_.item())) == oracle.filter_sum(cols, preds, cols[0],
                                                                         cols[ncols - 1])[:2]
    finally:
        tqp.tune_set("filter.per_cu", old)


def test_filter_sum_repeatable_and_knob_independent(tqp):
    cfg = dg.config_q6(5, 3_000_000)
    t = cfg["items"]
    want = oracle.q6(cfg)
    cols = [dev(t["ship"]), dev(t["discount"]), dev(t["quantity"])]
    preds = [(0, ">=", cfg["ship_lo"]), (0, "<", cfg["ship_hi"]), (1, ">=", cfg["disc_lo"]),
             (1, "<=", cfg["disc_hi"]), (2, "<", cfg["qty_cut"])]
    price = dev(t["price"])
    s = torch.empty(1, dtype=torch.int64, device="cuda")
    c = torch.empty(1, dtype=torch.int64, device="cuda")
    old = tqp.tune_knobs()["filter.per_cu"][0]
    try:
        for per_cu in (1, 2, 4, old):
            tqp.tune_set("filter.per_cu", per_cu)
            for _ in range(3):
                tqp.filter_sum_into(cols, preds, s, c, price, cols[1])
                torch.cuda.synchronize()
                assert (int(s.item()), int(c.item())) == (want["sum"], want["count"])
    finally:
        tqp.tune_set("filter.per_cu", old)


def test_q6_full_size(tqp):
    """60M rows, drawn on the GPU; the oracle reads the same table."""
    from tqp_datagen import device as dgd
    from paper_2209_04579_amd.pipeline import Q6Scan
    d = dgd.config_q6(0, device="cuda")
    q = Q6Scan(d["items"], d)
    q.run()
    got = q.result()
    host = {"items": {k: v.cpu().numpy() for k, v in d["items"].items()},
            **{k: d[k] for k in ("ship_lo", "ship_hi", "disc_lo", "disc_hi", "qty_cut")}}
    want = oracle.q6(host)
    assert want["exact"]
    assert (got["sum"], got["count"]) == (want["sum"], want["count"])
