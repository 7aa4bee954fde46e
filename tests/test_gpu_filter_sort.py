"""GPU parity of the fused WHERE + stable sort (tqp_filter_sort) against the
CPU oracle: the oracle filters (row ids ascending), then stable-sorts the
kept keys; the fused operator must give the same keys, row ids and payload
bytes, and the same kept count."""
import numpy as np
import pytest

import oracle
import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def keys_of(kind, n, dtype, seed=0):
    if kind == "dup":
        return dg.uniform_int(seed, 1, n, -3, 4, dtype)
    if kind == "full":
        u = dg.raw_u64(seed, 1, n).view(np.int64)
        return (u if dtype == np.int64 else (u >> 32)).astype(dtype)
    if kind == "zipf":
        return (dg.zipf_ranks(seed, 1, n, 2_000_000, 1.0) - 1).astype(dtype)
    return np.full(n, 7, dtype)


def expected(cols, preds, keys, payload):
    rows = oracle.filter_rows(cols, preds)
    ok, perm = oracle.sort(keys[rows])
    r = rows[perm]
    return ok, r, [p[r] for p in payload]


def run(tqp, cols, preds, keys, payload, key_bits=0, key_min=0, want_rows=True):
    n = len(keys)
    dk = dev(keys)
    out_key = torch.empty_like(dk)
    out_rows = torch.full((n,), -1, dtype=torch.int32, device="cuda") if want_rows else None
    pin = [dev(p) for p in payload]
    pout = [torch.empty_like(p) for p in pin]
    cnt = torch.full((1,), -5, dtype=torch.int64, device="cuda")
    pay_bytes = sum(p.element_size() for p in pin)
    ws = tqp.workspace(tqp.sort_workspace_bytes(n, dk.dtype, pay_bytes), dk.device)
    tqp.filter_sort_into([dev(c) for c in cols], preds, dk, out_key, out_rows, cnt, ws,
                         key_bits=key_bits, key_min=key_min, pay_in=pin, pay_out=pout)
    k = int(cnt.item())
    return (k, host(out_key)[:k], None if out_rows is None else host(out_rows)[:k],
            [host(p)[:k] for p in pout])


@pytest.fixture
def tqp():
    import paper_2209_04579_amd as m
    return m


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("kind", ["dup", "full", "zipf", "const"])
@pytest.mark.parametrize("n", [0, 1, 65, 4096, 4097, 100_003, 1_000_003])
def test_filter_sort_matches_oracle(tqp, dtype, kind, n):
    keys = keys_of(kind, n, dtype)
    day = dg.uniform_int(n + 1, 2, n, 0, 2557, np.int32)
    cols, preds = [day], [(0, "<", 1278)]
    want_k, want_r, _ = expected(cols, preds, keys, [])
    k, got_k, got_r, _ = run(tqp, cols, preds, keys, [])
    assert k == len(want_k)
    assert np.array_equal(got_k, want_k)
    assert np.array_equal(got_r, want_r)


@pytest.mark.parametrize("cut", [-1, 0, 25, 2557, 9999])
def test_filter_sort_selectivity_extremes(tqp, cut):
    """Nothing kept, 1% kept, everything kept, and the boundaries."""
    n = 200_003
    keys = keys_of("zipf", n, np.int32, seed=3)
    day = dg.uniform_int(7, 2, n, 0, 2557, np.int32)
    cols, preds = [day], [(0, "<", cut)]
    want_k, want_r, _ = expected(cols, preds, keys, [])
    k, got_k, got_r, _ = run(tqp, cols, preds, keys, [])
    assert k == len(want_k)
    assert np.array_equal(got_k, want_k)
    assert np.array_equal(got_r, want_r)


def test_filter_sort_payload_predicates_and_key_bits(tqp):
    """Four predicates over int8 / int32 / int64 columns, three payload
    columns of every dtype, a caller-given key range (three passes), and the
    same without row ids."""
    n = 700_001
    keys = dg.uniform_int(11, 1, n, -1_000_000, 1_000_000, np.int64)
    c8 = dg.uniform_int(11, 2, n, -128, 128, np.int8)
    c32 = dg.uniform_int(11, 3, n, 0, 100, np.int32)
    c64 = dg.raw_u64(11, 4, n).view(np.int64)
    cols = [c8, c32, c64]
    preds = [(0, ">=", -100), (1, "!=", 42), (2, "<", 1 << 61), (1, "<=", 90)]
    payload = [dg.uniform_int(11, 5, n, -128, 128, np.int8),
               dg.uniform_int(11, 6, n, -(1 << 31), 1 << 31, np.int32),
               dg.raw_u64(11, 7, n).view(np.int64)]
    want_k, want_r, want_p = expected(cols, preds, keys, payload)
    assert 0 < len(want_k) < n
    for key_bits, key_min in ((0, 0), (21, -1_000_000), (64, int(np.iinfo(np.int64).min))):
        k, got_k, got_r, got_p = run(tqp, cols, preds, keys, payload, key_bits, key_min)
        assert k == len(want_k)
        assert np.array_equal(got_k, want_k)
        assert np.array_equal(got_r, want_r)
        for g, w in zip(got_p, want_p):
            assert np.array_equal(g, w)
    k, got_k, got_r, got_p = run(tqp, cols, preds, keys, payload, 21, -1_000_000, want_rows=False)
    assert got_r is None and k == len(want_k)
    assert np.array_equal(got_k, want_k)
    for g, w in zip(got_p, want_p):
        assert np.array_equal(g, w)


def test_filter_sort_with_tile_count_mode(tqp):
    """sort.mode = 1: the filtered first pass still takes its offsets by
    look-back, the later passes by tile counts; the results are the same."""
    old = tqp.tune_knobs()["sort.mode"][0]
    n = 500_009
    keys = keys_of("zipf", n, np.int32, seed=5)
    day = dg.uniform_int(5, 2, n, 0, 2557, np.int32)
    cols, preds = [day], [(0, "<", 1278)]
    want_k, want_r, _ = expected(cols, preds, keys, [])
    tqp.tune_set("sort.mode", 1)
    try:
        k, got_k, got_r, _ = run(tqp, cols, preds, keys, [])
    finally:
        tqp.tune_set("sort.mode", old)
    assert k == len(want_k)
    assert np.array_equal(got_k, want_k)
    assert np.array_equal(got_r, want_r)


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_filter_sort_four_payload_columns_and_rows(tqp, dtype):
    """The widest pass: four payload columns and the row ids (five moved
    columns), keys spanning four 8-bit digits, an equality predicate on an
    int8 column."""
    n = 333_337
    keys = dg.uniform_int(21, 1, n, -(1 << 31), 1 << 31, dtype)
    flag = dg.uniform_int(21, 2, n, 0, 3, np.int8)
    cols, preds = [flag], [(0, "==", 1)]
    payload = [dg.uniform_int(21, 3 + c, n, -100, 100, t)
               for c, t in enumerate((np.int64, np.int8, np.int32, np.int64))]
    want_k, want_r, want_p = expected(cols, preds, keys, payload)
    k, got_k, got_r, got_p = run(tqp, cols, preds, keys, payload)
    assert k == len(want_k) and 0 < k < n
    assert np.array_equal(got_k, want_k)
    assert np.array_equal(got_r, want_r)
    for g, w in zip(got_p, want_p):
        assert np.array_equal(g, w)
