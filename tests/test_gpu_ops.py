"""GPU parity: every operator through the C ABI against the CPU oracle, bit
for bit, on seeded inputs spanning several tiles, ragged tails and the edge
cases of each operator (empty input, one row, all / no rows kept, one key,
all keys distinct, extreme values, skew)."""
import numpy as np
import pytest

import oracle
import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = [0, 1, 63, 64, 65, 4095, 4096, 4097, 12_289, 100_003]
I32 = np.iinfo(np.int32)
I64 = np.iinfo(np.int64)


@pytest.fixture(scope="module")
def tqp():
    import paper_2209_04579_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


# ----------------------------------------------------------------- filter ----

@pytest.mark.parametrize("n", SIZES)
def test_filter_single_predicate(tqp, n):
    day = dg.uniform_int(n, 3, n, 0, dg.DAY_DOMAIN, np.int32)
    qty = dg.uniform_int(n, 2, n, 1, 5001, np.int64)
    rows, (q,) = tqp.filter([dev(day)], [(0, "<", 1278)], payload=[dev(qty)])
    want = oracle.filter_rows([day], [(0, "<", 1278)])
    assert np.array_equal(host(rows), want)
    assert np.array_equal(host(q), oracle.gather(qty, want))


@pytest.mark.parametrize("seed", range(4))
def test_filter_conjunction_mixed_dtypes(tqp, seed):
    n = 50_000 + 777 * seed
    cols = [dg.uniform_int(seed, 1, n, -100, 100, np.int8),
            dg.uniform_int(seed, 2, n, -1000, 1000, np.int32),
            dg.uniform_int(seed, 3, n, -10 ** 6, 10 ** 6, np.int64)]
    preds = [(0, ">=", -50 + seed), (1, "<", 500), (2, "!=", int(cols[2][7])), (0, "<=", 90),
             (1, ">", -900 + seed)]
    rows, pay = tqp.filter([dev(c) for c in cols], preds, payload=[dev(c) for c in cols])
    want = oracle.filter_rows(cols, preds)
    assert np.array_equal(host(rows), want)
    for c, p in zip(cols, pay):
        assert np.array_equal(host(p), oracle.gather(c, want))


def test_filter_all_none_and_extremes(tqp):
    x = np.array([I32.min, -1, 0, 1, I32.max] * 1000, np.int32)
    for preds in ([(0, ">=", I32.min)], [(0, "<", I32.min)], [(0, ">", 2 ** 40)],
                  [(0, "==", I32.max)], [(0, "<=", -(2 ** 40))]):
        rows, _ = tqp.filter([dev(x)], preds)
        assert np.array_equal(host(rows), oracle.filter_rows([x], preds)), preds
    y = np.array([I64.min, I64.max, 0] * 3000, np.int64)
    rows, _ = tqp.filter([dev(y)], [(0, "<", I64.max)])
    assert np.array_equal(host(rows), oracle.filter_rows([y], [(0, "<", I64.max)]))


@pytest.mark.parametrize("seed,offset", [(0, 0), (1, 0), (2, 1)])
def test_filter_runs_of_mixed_density_with_payload(tqp, seed, offset):
    """Runs of rows whose kept share swings between none, a few and all, at
    run lengths aligned with nothing, so sparse and dense stretches follow
    each other in every pattern; payload columns of every dtype, 16-byte
    aligned or not (offset 1 starts each column one element in)."""
    n = 1_500_000 + 9_871 * seed
    lens = dg.uniform_int(seed, 1, 4000, 1, 20_000, np.int64)
    ends = np.minimum(np.cumsum(lens), n)
    share = np.array([0, 1, 20, 250, 600, 999, 1000], np.int64)
    pick = dg.uniform_int(seed, 2, len(ends), 0, len(share), np.int64)
    per_row = share[pick][np.searchsorted(ends, np.arange(n), side="right").clip(0, len(ends) - 1)]
    u = dg.uniform_int(seed, 3, n, 0, 1000, np.int64)
    flag = (u >= per_row).astype(np.int8)          # 0 where the row is kept
    pays = [dg.uniform_int(seed, 4, n + offset, -128, 128, np.int8),
            dg.uniform_int(seed, 5, n + offset, I32.min, I32.max, np.int32),
            (dg.uniform_int(seed, 6, n + offset, -2 ** 31, 2 ** 31, np.int64) << 32)
            + dg.uniform_int(seed, 7, n + offset, 0, 2 ** 32, np.int64)]
    dpays = [dev(p)[offset:] for p in pays]
    rows, got = tqp.filter([dev(flag)], [(0, "==", 0)], payload=dpays)
    want = oracle.filter_rows([flag], [(0, "==", 0)])
    assert np.array_equal(host(rows), want)
    for p, g in zip(pays, got):
        assert np.array_equal(host(g), oracle.gather(p[offset:], want))


def test_filter_is_deterministic_across_runs(tqp):
    n = 3_000_000
    day = dev(dg.uniform_int(11, 3, n, 0, dg.DAY_DOMAIN, np.int32))
    a, _ = tqp.filter([day], [(0, "<", 1278)])
    b, _ = tqp.filter([day], [(0, "<", 1278)])
    assert torch.equal(a, b)
    assert np.array_equal(host(a), np.nonzero(host(day) < 1278)[0].astype(np.int32))


# ----------------------------------------------------------------- gather ----

@pytest.mark.parametrize("dtype", [np.int8, np.int32, np.int64])
def test_gather(tqp, dtype):
    src = dg.uniform_int(1, 1, 70_001, -100, 100, dtype)
    idx = dg.uniform_int(1, 2, 33_333, 0, 70_001, np.int32)
    assert np.array_equal(host(tqp.gather(dev(src), dev(idx))), oracle.gather(src, idx))


def test_pack_key(tqp):
    n = 10_007
    flag = dg.uniform_int(2, 1, n, 0, 3, np.int8)
    cat = dg.uniform_int(2, 2, 5000, -30, 30, np.int32)
    rows = dg.uniform_int(2, 3, n, 0, 5000, np.int32)
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    tqp.pack_key_into([(dev(flag), None, 0, 2), (dev(cat), dev(rows), 2, 1)], n, out)
    want = flag.astype(np.int64) * 2 + np.mod(cat[rows], 2)
    assert np.array_equal(host(out), want)


# ------------------------------------------------------------------- sort ----

def sort_case(n, dtype, kind, seed=0):
    if kind == "dup":
        return dg.uniform_int(seed, 1, n, -3, 4, dtype)
    if kind == "dom":
        return dg.uniform_int(seed, 1, n, 0, 10_000, dtype)
    if kind == "neg":
        return dg.uniform_int(seed, 1, n, -(2 ** 31), 2 ** 31 - 1, np.int64).astype(dtype)
    if kind == "full":
        u = dg.raw_u64(seed, 1, n).view(np.int64)
        k = u if dtype == np.int64 else (u >> 32).astype(np.int32)
        k = k.astype(dtype)
        info = np.iinfo(dtype)
        k[: min(n, 4)] = [info.min, info.max, 0, -1][: min(n, 4)]
        return k
    if kind == "zipf":
        return (dg.zipf_ranks(seed, 1, n, 2_000_000, 1.0) - 1).astype(dtype)
    if kind == "const":
        return np.full(n, 42, dtype)
    raise ValueError(kind)


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("kind", ["dup", "dom", "neg", "full", "zipf", "const"])
@pytest.mark.parametrize("n", [0, 1, 65, 4096, 4097, 100_003])
def test_sort_matches_oracle(tqp, dtype, kind, n):
    keys = sort_case(n, dtype, kind)
    sk, perm = tqp.sort(dev(keys))
    ok, operm = oracle.sort(keys)
    assert np.array_equal(host(perm), operm)
    assert np.array_equal(host(sk), ok)


def test_sort_carries_rows_and_explicit_bits(tqp):
    n = 1_000_003
    keys = dg.uniform_int(5, 1, n, 1000, 1000 + 2 ** 21, np.int32)
    rows = dg.uniform_int(5, 2, n, 0, 2 ** 31 - 1, np.int32)
    sk, r = tqp.sort(dev(keys), in_rows=dev(rows), key_bits=21, key_min=1000)
    ok, perm = oracle.sort(keys)
    assert np.array_equal(host(sk), ok)
    assert np.array_equal(host(r), rows[perm])


@pytest.mark.parametrize("n", [1, 4097, 300_007])
def test_sort_carries_payload_columns(tqp, n):
    keys = dg.uniform_int(n, 1, n, -500, 500, np.int64)
    p8 = dg.uniform_int(n, 2, n, -128, 128, np.int8)
    p32 = dg.uniform_int(n, 3, n, -(2 ** 31), 2 ** 31 - 1, np.int64).astype(np.int32)
    p64 = dg.raw_u64(n, 4, n).view(np.int64)
    sk, rows, (q8, q32, q64) = tqp.sort(dev(keys), payload=[dev(p8), dev(p32), dev(p64)])
    ok, perm = oracle.sort(keys)
    assert np.array_equal(host(sk), ok) and np.array_equal(host(rows), perm)
    assert np.array_equal(host(q8), p8[perm])
    assert np.array_equal(host(q32), p32[perm])
    assert np.array_equal(host(q64), p64[perm])
    sk2, none, (q64b,) = tqp.sort(dev(keys), payload=[dev(p64)], want_rows=False,
                                  key_bits=10, key_min=-500)
    assert none is None
    assert np.array_equal(host(sk2), ok) and np.array_equal(host(q64b), p64[perm])


def test_sort_large_zipf_is_deterministic(tqp):
    n = 30_000_000
    keys = dev(sort_case(n, np.int32, "zipf", seed=3))
    a = tqp.sort(keys, key_bits=21, key_min=0)
    b = tqp.sort(keys, key_bits=21, key_min=0)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    want = np.argsort(host(keys), kind="stable").astype(np.int32)
    assert np.array_equal(host(a[1]), want)


# ------------------------------------------------------------------- join ----

@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("nl,nr,dom", [(0, 10, 5), (10, 0, 5), (1, 1, 1), (5000, 3000, 1),
                                       (5000, 3000, 7), (20_000, 7_000, 5000),
                                       (100_003, 4097, 10 ** 6), (4096, 4096, 4096)])
def test_join_pairs_match_oracle(tqp, dtype, nl, nr, dom):
    lk = dg.uniform_int(nl + 1, 1, nl, -dom // 2, dom - dom // 2, dtype) if nl else np.zeros(0, dtype)
    rk = dg.uniform_int(nr + 2, 2, nr, -dom // 2, dom - dom // 2, dtype) if nr else np.zeros(0, dtype)
    cnt, ol, orr = oracle.join(lk, rk)
    if cnt > 30_000_000:
        pytest.skip("pair count too large for this test")
    gl, gr, gk = tqp.join(dev(lk), dev(rk), cap=cnt, with_key=True)
    assert gl.numel() == cnt
    assert np.array_equal(host(gl), ol)
    assert np.array_equal(host(gr), orr)
    assert np.array_equal(host(gk), lk[ol])


def test_join_extreme_and_disjoint_keys(tqp):
    e = np.array([I64.min, I64.max, 0, I64.min, -1], np.int64)
    cnt, ol, orr = oracle.join(e, e)
    gl, gr = tqp.join(dev(e), dev(e))
    assert np.array_equal(host(gl), ol) and np.array_equal(host(gr), orr)
    a = np.arange(0, 10_000, 2, dtype=np.int32)
    b = np.arange(1, 10_001, 2, dtype=np.int32)
    gl, gr = tqp.join(dev(a), dev(b))
    assert gl.numel() == 0


def test_join_capacity_overflow_reports_count(tqp):
    k = np.zeros(300, np.int32)
    gl, gr = tqp.join(dev(k), dev(k), cap=1000)          # 90_000 pairs: retried
    assert gl.numel() == 90_000
    assert np.array_equal(host(gl), np.repeat(np.arange(300, dtype=np.int32), 300))


def test_join_sorted_inputs_with_row_maps(tqp):
    lk = dg.uniform_int(8, 1, 50_000, 0, 3000, np.int32)
    rk = dg.uniform_int(8, 2, 9_000, 0, 3000, np.int32)
    sl, pl = oracle.sort(lk)
    sr, pr = oracle.sort(rk)
    cnt, ol, orr = oracle.join(lk, rk)
    gl, gr = tqp.join(dev(sl), dev(sr), lrows=dev(pl), rrows=dev(pr), sorted_inputs=True, cap=cnt)
    assert np.array_equal(host(gl), ol) and np.array_equal(host(gr), orr)


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_join_ranges_match_oracle(tqp, dtype):
    lk = np.sort(dg.uniform_int(4, 1, 200_000, -5000, 5000, dtype))
    rk = np.sort(dg.uniform_int(4, 2, 30_000, -2000, 9000, dtype))
    want = oracle.join_ranges(lk, rk)
    got = tqp.join_ranges(dev(lk), dev(rk))
    for k in ("key", "lstart", "lcnt", "rstart", "rcnt"):
        assert np.array_equal(host(got[k]), want[k]), k
    assert got["total"] == want["total"]


# --------------------------------------------------------------- group-by ----

AGGS = [("sum", 0), ("count",), ("sum_product", 0, 1), ("sum", 1)]


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("n", [0, 1, 4095, 4097, 100_003])
@pytest.mark.parametrize("dom", [1, 6, 5000, 10 ** 7])
def test_groupby_sort_path(tqp, dtype, n, dom):
    keys = dg.uniform_int(n + dom, 1, n, -dom // 3, dom - dom // 3, dtype)
    a = dg.uniform_int(n, 2, n, 1, 5001, np.int64)
    b = dg.uniform_int(n, 3, n, -10 ** 7, 10 ** 7, np.int32)
    uk, aggs = tqp.groupby_agg(dev(keys), [dev(a), dev(b)], AGGS)
    wk, wa, _ = oracle.groupby(keys, [a, b], AGGS)
    assert np.array_equal(host(uk).astype(np.int64), wk)
    for g, w in zip(aggs, wa):
        assert np.array_equal(host(g), w)


@pytest.mark.parametrize("n", [0, 1, 100_003, 2_000_000])
@pytest.mark.parametrize("span", [1, 6, 25, 125, 1024])
def test_groupby_dense_path(tqp, n, span):
    lo = -7
    keys = dg.uniform_int(n + span, 1, n, lo, lo + span, np.int64)
    a = dg.uniform_int(n, 2, n, 1, 5001, np.int64)
    b = dg.uniform_int(n, 3, n, 100, 10 ** 7, np.int64)
    uk, aggs = tqp.groupby_agg(dev(keys), [dev(a), dev(b)], AGGS[:3], flags=tqp.GB_DENSE,
                               key_lo=lo, key_span=span)
    wk, wa, _ = oracle.groupby(keys, [a, b], AGGS[:3])
    assert np.array_equal(host(uk), wk)
    for g, w in zip(aggs, wa):
        assert np.array_equal(host(g), w)


def test_groupby_sorted_flag_and_val_rows(tqp):
    n = 300_000
    keys = np.sort(dg.zipf_ranks(9, 1, n, 50_000, 1.0).astype(np.int32))
    vals = dg.uniform_int(9, 2, 1_000_000, 1, 5001, np.int64)
    rows = dg.uniform_int(9, 3, n, 0, 1_000_000, np.int32)
    uk, (s, c) = tqp.groupby_agg(dev(keys), [dev(vals)], [("sum", 0), ("count",)],
                                 flags=tqp.GB_SORTED, val_rows=dev(rows))
    wk, (ws, wc), _ = oracle.groupby(keys, [vals[rows]], [("sum", 0), ("count",)])
    assert np.array_equal(host(uk), wk) and np.array_equal(host(s), ws)
    assert np.array_equal(host(c), wc)


def test_groupby_wraps_modulo_2_64(tqp):
    keys = np.zeros(10_000, np.int64)
    vals = np.full(10_000, I64.max, np.int64)
    uk, (s,) = tqp.groupby_agg(dev(keys), [dev(vals)], [("sum", 0)])
    wk, (w,), ovf = oracle.groupby(keys, [vals], [("sum", 0)])
    assert ovf and np.array_equal(host(s), w)


def packed_key_host(terms_np, n):
    """The packed key on the host: sum of mul * f(col[rows]) (numpy int64)."""
    key = np.zeros(n, np.int64)
    for col, rows, mod, mul in terms_np:
        if col is None:
            key += mul
            continue
        v = (col[rows] if rows is not None else col[:n]).astype(np.int64)
        if mod > 0:
            v = np.mod(v, mod)
        key += mul * v
    return key


@pytest.mark.parametrize("n", [0, 1, 4097, 1_000_003])
@pytest.mark.parametrize("out_dtype", [np.int32, np.int64])
def test_groupby_agg_terms_matches_oracle(tqp, n, out_dtype):
    """Dense group-by over a packed key computed in the kernel: the same groups
    as the oracle over the key packed on the host."""
    m = 50_000
    flag = dg.uniform_int(n + 1, 1, m, 0, 3, np.int8)
    cat = dg.uniform_int(n + 1, 2, m, -9, 25, np.int32)
    lrow = dg.uniform_int(n + 1, 3, n, 0, m, np.int32)
    rrow = dg.uniform_int(n + 1, 4, n, 0, m, np.int32)
    qty = dg.uniform_int(n + 1, 5, m, 1, 5001, np.int64)
    price = dg.uniform_int(n + 1, 6, m, 100, 10 ** 7, np.int64)
    # key = 2 * flag + (cat mod 4) + 10, in [10, 20)
    terms_np = [(flag, lrow, 0, 2), (cat, rrow, 4, 1), (None, None, 0, 10)]
    terms = [(dev(flag), dev(lrow), 0, 2), (dev(cat), dev(rrow), 4, 1), (None, None, 0, 10)]
    aggs = [("sum", 0), ("sum_product", 0, 1), ("count",)]
    span, lo = 10, 10
    out_key = torch.empty(span, dtype=torch.int32 if out_dtype == np.int32 else torch.int64,
                          device="cuda")
    outs = [torch.empty(span, dtype=torch.int64, device="cuda") for _ in aggs]
    ng = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = tqp.workspace(tqp.groupby_terms_workspace_bytes(len(aggs), span))
    tqp.groupby_agg_terms_into(terms, n, [dev(qty), dev(price)], aggs, out_key, outs, ng, ws,
                               lo, span, val_rows=dev(lrow))
    g = int(ng.item())
    key = packed_key_host(terms_np, n)
    wk, wa, _ = oracle.groupby(key, [qty[lrow], price[lrow]], aggs)
    assert np.array_equal(host(out_key[:g]).astype(np.int64), wk)
    for o, w in zip(outs, wa):
        assert np.array_equal(host(o[:g]), w)


def test_groupby_agg_terms_device_count_and_limits(tqp):
    n = 200_000
    cat = dg.uniform_int(3, 1, n, 0, 6, np.int32)
    qty = dg.uniform_int(3, 2, n, 1, 5001, np.int64)
    d_n = torch.tensor([123_457], dtype=torch.int64, device="cuda")
    out_key = torch.empty(6, dtype=torch.int64, device="cuda")
    outs = [torch.empty(6, dtype=torch.int64, device="cuda") for _ in range(2)]
    ng = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = tqp.workspace(tqp.groupby_terms_workspace_bytes(2, 6))
    tqp.groupby_agg_terms_into([(dev(cat), None, 0, 1)], n, [dev(qty)], [("sum", 0), ("count",)],
                               out_key, outs, ng, ws, 0, 6, d_n=d_n)
    g = int(ng.item())
    wk, wa, _ = oracle.groupby(cat[:123_457].astype(np.int64), [qty[:123_457]],
                               [("sum", 0), ("count",)])
    assert np.array_equal(host(out_key[:g]), wk)
    for o, w in zip(outs, wa):
        assert np.array_equal(host(o[:g]), w)
    with pytest.raises(tqp.TqpError):          # accumulators beyond the LDS budget
        tqp.groupby_agg_terms_into([(dev(cat), None, 0, 1)], n, [dev(qty)],
                                   [("sum", 0), ("count",)], out_key, outs, ng, ws, 0, 4000)


DIFF_AGGS = [("sum_diff_product", 0, 1, 100), ("count",), ("sum_diff_product", 1, 0, -7),
             ("sum", 0)]


@pytest.mark.parametrize("path", ["sort", "sorted", "dense", "terms_tiny", "terms_dense"])
@pytest.mark.parametrize("n", [0, 1, 4097, 300_001])
def test_groupby_sum_diff_product_every_path(tqp, path, n):
    """SUM(a * (c - b)) (Q14's revenue shape) through each group-by kernel,
    against the oracle, including a negative constant and int8 b."""
    span = 2 if path == "terms_tiny" else 125
    keys = dg.uniform_int(n + 5, 1, n, 0, span, np.int32)
    if path == "sorted":
        keys = np.sort(keys)
    a = dg.uniform_int(n + 5, 2, n, 90_000, 10_494_951, np.int64)
    b = dg.uniform_int(n + 5, 3, n, 0, 11, np.int8)
    wk, wa, ovf = oracle.groupby(keys, [a, b], DIFF_AGGS)
    assert not ovf
    if path in ("sort", "sorted", "dense"):
        flags = {"sort": 0, "sorted": tqp.GB_SORTED, "dense": tqp.GB_DENSE}[path]
        uk, aggs = tqp.groupby_agg(dev(keys), [dev(a), dev(b)], DIFF_AGGS, flags=flags,
                                   key_lo=0, key_span=span if path == "dense" else 0)
    else:
        out_key = torch.empty(span, dtype=torch.int32, device="cuda")
        aggs = [torch.empty(span, dtype=torch.int64, device="cuda") for _ in DIFF_AGGS]
        ng = torch.zeros(1, dtype=torch.int64, device="cuda")
        ws = tqp.workspace(tqp.groupby_terms_workspace_bytes(len(DIFF_AGGS), span))
        tqp.groupby_agg_terms_into([(dev(keys), None, 0, 1)], n, [dev(a), dev(b)], DIFF_AGGS,
                                   out_key, aggs, ng, ws, 0, span)
        g = int(ng.item())
        uk, aggs = out_key[:g], [t[:g] for t in aggs]
    assert np.array_equal(host(uk).astype(np.int64), wk)
    for got, w in zip(aggs, wa):
        assert np.array_equal(host(got), w)
