"""Pins for the CPU oracle: each check compares it with something other than
itself -- brute-force loops over tiny tables, numpy library routines with the
same definition, closed forms and invariants.

The paper prints no result values (its figures carry only speed-ups,
Section 2.3), so the pins are the SQL definitions of the operators (Sections
2.2-2.3) evaluated independently, plus the invariants the method must keep:
join cardinality equals the sum over keys of count_L * count_R, and group
sums conserve the filtered total.
"""
import itertools

import numpy as np
import pytest

import oracle
import tqp_datagen as dg

I32_MIN, I32_MAX = -(2 ** 31), 2 ** 31 - 1
I64_MIN, I64_MAX = -(2 ** 63), 2 ** 63 - 1
OPS = {"<": lambda a, b: a < b, "<=": lambda a, b: a <= b, ">": lambda a, b: a > b,
       ">=": lambda a, b: a >= b, "==": lambda a, b: a == b, "!=": lambda a, b: a != b}


def rng_cols(seed, n, dom=50):
    return [
        dg.uniform_int(seed, 1, n, -dom, dom, np.int8),
        dg.uniform_int(seed, 2, n, -dom, dom, np.int32),
        dg.uniform_int(seed, 3, n, -dom, dom, np.int64),
    ]


# ----------------------------------------------------------------- filter ----

@pytest.mark.parametrize("seed", range(6))
def test_filter_brute_force(seed):
    n = 300 + 37 * seed
    cols = rng_cols(seed, n, dom=20)
    opnames = list(OPS)
    for trial in range(12):
        k = 1 + trial % 4
        preds = []
        for q in range(k):
            c = (trial + q) % 3
            op = opnames[(trial * 7 + q * 3 + seed) % 6]
            lit = int(cols[c][(trial * 13 + q) % n])      # literal on a data value
            preds.append((c, op, lit))
        got = oracle.filter_rows(cols, preds)
        want = [i for i in range(n)
                if all(OPS[op](int(cols[c][i]), lit) for c, op, lit in preds)]
        assert got.tolist() == want, preds


@pytest.mark.parametrize("seed", range(5))
def test_semijoin_brute_force(seed):
    """Semi-join over one to three right sides: a Python set per side and a
    row loop, on tiny tables with duplicates, misses, negative keys and mixed
    dtypes."""
    n = 200 + 41 * seed
    left = rng_cols(seed, n, dom=30)
    for trial in range(8):
        k = 1 + trial % 3
        cols = [(trial + q) % 3 for q in range(k)]
        keys = [left[c] for c in cols]
        sets = []
        for q in range(k):
            m = (trial * 5 + q * 11 + seed) % 40
            dt = (np.int8, np.int32, np.int64)[(trial + q + seed) % 3]
            sets.append(dg.uniform_int(seed + 100 * trial, 20 + q, m, -30, 30, dt))
        got = oracle.semijoin_rows(keys, sets)
        py = [set(int(v) for v in t) for t in sets]
        want = [i for i in range(n) if all(int(keys[q][i]) in py[q] for q in range(k))]
        assert got.tolist() == want, (trial, [len(t) for t in sets])


def test_semijoin_matches_numpy_isin_and_edge_cases():
    rng = np.random.default_rng(7)
    n = 50_000
    k1 = rng.integers(-(2 ** 40), 2 ** 40, n, dtype=np.int64)
    k2 = rng.integers(0, 1000, n, dtype=np.int64).astype(np.int32)
    s1 = np.concatenate([k1[rng.integers(0, n, 3000)], rng.integers(0, 2 ** 40, 500)])
    s2 = rng.integers(0, 1000, 300).astype(np.int32)
    want = np.nonzero(np.isin(k1, s1) & np.isin(k2, s2))[0].astype(np.int32)
    assert np.array_equal(oracle.semijoin_rows([k1, k2], [s1, s2]), want)
    # an empty right side keeps nothing; the full domain keeps everything
    assert len(oracle.semijoin_rows([k2], [np.zeros(0, np.int32)])) == 0
    assert np.array_equal(oracle.semijoin_rows([k2], [np.arange(1000, dtype=np.int32)]),
                          np.arange(n, dtype=np.int32))
    # empty left side; int64 extremes compare exactly (no wrap, no truncation)
    assert len(oracle.semijoin_rows([k1[:0]], [s1])) == 0
    ext = np.array([I64_MIN, -1, 0, I64_MAX, I32_MAX + 1], np.int64)
    assert oracle.semijoin_rows([ext], [np.array([I64_MAX, I32_MAX], np.int64)]).tolist() == [3]
    assert oracle.semijoin_rows([ext], [np.array([I32_MAX], np.int32)]).tolist() == []
    assert oracle.semijoin_rows([ext], [np.array([-1], np.int8)]).tolist() == [1]


def test_filter_literal_outside_column_range():
    c8 = np.array([-128, -1, 0, 1, 127], np.int8)
    # mathematical comparison: nothing in int8 is >= 200, everything is > -1000
    assert oracle.filter_rows([c8], [(0, ">=", 200)]).tolist() == []
    assert oracle.filter_rows([c8], [(0, ">", -1000)]).tolist() == [0, 1, 2, 3, 4]
    c32 = np.array([I32_MIN, 0, I32_MAX], np.int32)
    assert oracle.filter_rows([c32], [(0, "<", I32_MAX)]).tolist() == [0, 1]
    c64 = np.array([I64_MIN, 0, I64_MAX], np.int64)
    assert oracle.filter_rows([c64], [(0, "<=", I64_MIN)]).tolist() == [0]
    assert oracle.filter_rows([c64], [(0, ">=", I64_MAX)]).tolist() == [2]


def test_filter_matches_numpy_mask_and_complement():
    day = dg.uniform_int(0, 3, 200_000, 0, dg.DAY_DOMAIN, np.int32)
    lt = oracle.filter_rows([day], [(0, "<", 1278)])
    ge = oracle.filter_rows([day], [(0, ">=", 1278)])
    assert np.array_equal(lt, np.nonzero(day < 1278)[0].astype(np.int32))
    assert len(lt) + len(ge) == len(day)
    assert np.array_equal(np.sort(np.concatenate([lt, ge])), np.arange(len(day)))
    assert np.all(np.diff(lt) > 0)


def test_filter_empty_and_all():
    x = np.arange(10, dtype=np.int32)
    assert oracle.filter_rows([x], [(0, "<", 0)]).tolist() == []
    assert oracle.filter_rows([x], [(0, ">=", 0)]).tolist() == list(range(10))
    assert oracle.filter_rows([x[:0]], [(0, "<", 5)]).tolist() == []


# ------------------------------------------------------------------- sort ----

@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("dom", [3, 1000, None])
def test_sort_matches_numpy_stable_argsort(dtype, dom):
    n = 5000
    if dom is None:
        info = np.iinfo(dtype)
        keys = dg.raw_u64(9, 1, n).view(np.int64)
        keys = keys.astype(dtype) if dtype == np.int64 else (keys >> 32).astype(np.int32)
        keys[:4] = [info.min, info.max, 0, -1]
    else:
        keys = dg.uniform_int(1, 1, n, -dom, dom, dtype)
    sk, perm = oracle.sort(keys)
    want = np.argsort(keys, kind="stable")
    assert np.array_equal(perm, want.astype(np.int32))
    assert np.array_equal(sk, keys[want])


def test_sort_brute_force_tiny():
    keys = np.array([3, -1, 3, 0, -1, 7, 3, -5], np.int64)
    # stable order by (key, position), written out by hand
    want = [7, 1, 4, 3, 0, 2, 6, 5]
    sk, perm = oracle.sort(keys)
    assert perm.tolist() == want
    assert sk.tolist() == [-5, -1, -1, 0, 3, 3, 3, 7]
    for n in range(0, 7):
        for ks in itertools.product([-1, 0, 2], repeat=n):
            a = np.array(ks, np.int32)
            _, p = oracle.sort(a)
            brute = sorted(range(n), key=lambda i: (ks[i], i))
            assert p.tolist() == brute


# ------------------------------------------------------------------- join ----

def brute_join(lk, rk):
    pairs = [(int(lk[i]), i, j) for i in range(len(lk)) for j in range(len(rk))
             if lk[i] == rk[j]]
    pairs.sort()
    return [(i, j) for _, i, j in pairs]


@pytest.mark.parametrize("seed", range(8))
def test_join_brute_force(seed):
    nl, nr = 150 + 31 * seed, 90 + 17 * seed
    dom = [1, 3, 20, 200][seed % 4]
    dt = np.int32 if seed % 2 else np.int64
    lk = dg.uniform_int(seed, 1, nl, -dom, dom, dt)
    rk = dg.uniform_int(seed, 2, nr, -dom, dom, dt)
    cnt, ol, orr = oracle.join(lk, rk)
    want = brute_join(lk, rk)
    assert cnt == len(want)
    assert list(zip(ol.tolist(), orr.tolist())) == want


def test_join_cardinality_and_checksum_closed_form():
    lk = dg.uniform_int(3, 1, 40_000, 0, 3000, np.int32)
    rk = dg.uniform_int(3, 2, 9_000, 0, 3000, np.int32)
    cnt, ol, orr = oracle.join(lk, rk)
    ul, cl = np.unique(lk, return_counts=True)
    ur, cr = np.unique(rk, return_counts=True)
    common, il, ir = np.intersect1d(ul, ur, return_indices=True)
    assert cnt == int(np.sum(cl[il].astype(np.int64) * cr[ir]))
    # checksum: sum over pairs of (A*i + B*j) = sum over keys (A*cR*sum_i + B*cL*sum_j)
    A, B = 3, 7
    suml = np.bincount(lk, weights=np.arange(len(lk), dtype=np.float64), minlength=3000)
    sumr = np.bincount(rk, weights=np.arange(len(rk), dtype=np.float64), minlength=3000)
    cntl = np.bincount(lk, minlength=3000).astype(np.int64)
    cntr = np.bincount(rk, minlength=3000).astype(np.int64)
    closed = int(np.sum(A * cntr * suml.astype(np.int64) + B * cntl * sumr.astype(np.int64)))
    assert int(np.sum(A * ol.astype(np.int64) + B * orr.astype(np.int64))) == closed
    assert np.all(lk[ol] == rk[orr])


def test_join_edge_cases():
    e32 = np.zeros(0, np.int32)
    assert oracle.join(e32, np.arange(5, dtype=np.int32))[0] == 0
    assert oracle.join(np.arange(5, dtype=np.int32), e32)[0] == 0
    assert oracle.join(np.arange(5, dtype=np.int32), np.arange(5, 10, dtype=np.int32))[0] == 0
    k = np.full(50, 7, np.int64)
    cnt, ol, orr = oracle.join(k, k[:30])
    assert cnt == 1500
    assert ol.tolist() == [i for i in range(50) for _ in range(30)]
    assert orr.tolist() == list(range(30)) * 50
    ext = np.array([I64_MIN, I64_MAX, 0, I64_MIN], np.int64)
    assert oracle.join(ext, ext)[0] == 6


def test_join_ranges_definition():
    lk = dg.uniform_int(5, 1, 3000, -40, 40, np.int64)
    rk = dg.uniform_int(5, 2, 800, -60, 20, np.int64)
    r = oracle.join_ranges(lk, rk)
    sl, sr = np.sort(lk, kind="stable"), np.sort(rk, kind="stable")
    keys = sorted(set(lk.tolist()) & set(rk.tolist()))
    assert r["key"].tolist() == keys
    for q, k in enumerate(keys):
        assert r["lstart"][q] == int(np.sum(lk < k))
        assert r["lcnt"][q] == int(np.sum(lk == k))
        assert r["rstart"][q] == int(np.sum(rk < k))
        assert r["rcnt"][q] == int(np.sum(rk == k))
        assert np.all(sl[r["lstart"][q]:r["lstart"][q] + r["lcnt"][q]] == k)
        assert np.all(sr[r["rstart"][q]:r["rstart"][q] + r["rcnt"][q]] == k)
    assert r["total"] == oracle.join(lk, rk)[0]


# ---------------------------------------------------------------- group-by ---

@pytest.mark.parametrize("seed", range(5))
def test_groupby_matches_numpy_unique_add_at(seed):
    n = 20_000
    dom = [1, 6, 125, 5000, 10 ** 6][seed]
    keys = dg.uniform_int(seed, 1, n, -dom // 2 - 1, dom // 2 + 1, np.int32)
    a = dg.uniform_int(seed, 2, n, 1, 5001, np.int64)
    b = dg.uniform_int(seed, 3, n, 100, 10_000_001, np.int64)
    uk, (s, c, sp), ovf = oracle.groupby(keys, [a, b], [("sum", 0), ("count",), ("sum_product", 0, 1)])
    nk, inv = np.unique(keys, return_inverse=True)
    ws = np.zeros(len(nk), np.int64)
    np.add.at(ws, inv, a)
    wc = np.bincount(inv, minlength=len(nk)).astype(np.int64)
    wp = np.zeros(len(nk), np.int64)
    np.add.at(wp, inv, a * b)
    assert not ovf
    assert np.array_equal(uk, nk.astype(np.int64))
    assert np.array_equal(s, ws)
    assert np.array_equal(c, wc)
    assert np.array_equal(sp, wp)
    assert int(s.sum()) == int(a.sum())          # conservation
    assert int(c.sum()) == n


def test_groupby_brute_force_tiny():
    keys = np.array([5, -2, 5, 0, -2, 5], np.int64)
    vals = np.array([1, 10, 100, 1000, 10000, 100000], np.int64)
    uk, (s, c), _ = oracle.groupby(keys, [vals], [("sum", 0), ("count",)])
    assert uk.tolist() == [-2, 0, 5]
    assert s.tolist() == [10010, 1000, 100101]
    assert c.tolist() == [2, 1, 3]


def test_groupby_sum_diff_product_brute_force():
    # SUM(a * (c - b)): Python integers row by row, and the identity
    # c * SUM(a) - SUM(a * b) (exact, no wrap at these sizes)
    keys = np.array([3, 1, 3, 3, 1, -4, 1], np.int32)
    a = np.array([900, 15, -7, 10 ** 7, 3, 0, 2 ** 40], np.int64)
    b = np.array([5, 100, 11, 7, -3, 9, 99], np.int8)
    c = 100
    uk, (sdp, sa, sab, cnt), ovf = oracle.groupby(
        keys, [a, b], [("sum_diff_product", 0, 1, c), ("sum", 0), ("sum_product", 0, 1),
                       ("count",)])
    assert not ovf
    want = {}
    for k, x, y in zip(keys.tolist(), a.tolist(), b.tolist()):
        want[k] = want.get(k, 0) + x * (c - y)
    assert uk.tolist() == sorted(want)
    assert sdp.tolist() == [want[k] for k in sorted(want)]
    assert (c * sa - sab).tolist() == sdp.tolist()
    # the constant enters as given: a negative one, and c = 0 gives -SUM(a * b)
    _, (neg,), _ = oracle.groupby(keys, [a, b], [("sum_diff_product", 0, 1, -3)])
    assert neg.tolist() == [sum(x * (-3 - y) for kk, x, y in zip(keys.tolist(), a.tolist(),
                                                                  b.tolist()) if kk == k)
                            for k in sorted(want)]
    _, (zero, sab2), _ = oracle.groupby(keys, [a, b], [("sum_diff_product", 0, 1, 0),
                                                       ("sum_product", 0, 1)])
    assert (zero == -sab2).all()


def test_groupby_wraps_mod_2_64_and_flags_overflow():
    keys = np.zeros(3, np.int32)
    vals = np.array([I64_MAX, I64_MAX, 5], np.int64)
    uk, (s,), ovf = oracle.groupby(keys, [vals], [("sum", 0)])
    assert ovf
    exact = I64_MAX * 2 + 5
    assert int(s[0]) == (exact + 2 ** 63) % 2 ** 64 - 2 ** 63
    assert oracle.groupby(np.zeros(0, np.int32), [np.zeros(0, np.int64)], [("sum", 0)])[0].size == 0


# ------------------------------------------------------------ whole query ----

def composed_q1(fact, dim, cut):
    """Q1 from the operator oracles: filter -> join -> gather -> group-by."""
    rows = oracle.filter_rows([fact["day"]], [(0, "<", cut)])
    fk = oracle.gather(fact["fk"], rows)
    cnt, li, ri = oracle.join(fk, dim["pk"])
    cat = oracle.gather(dim["cat"], ri)
    qty = oracle.gather(oracle.gather(fact["qty"], rows), li)
    uk, (s, c), _ = oracle.groupby(cat, [qty], [("sum", 0), ("count",)])
    return uk, s, c


@pytest.mark.parametrize("seed", [0, 1])
def test_q1_whole_query_equals_composed_and_invariants(seed):
    c = dg.config1(seed, n_fact=200_000, n_dim=2_000)
    r = oracle.q1(c["fact"], c["dim"], c["day_cut"])
    uk, s, cnt = composed_q1(c["fact"], c["dim"], c["day_cut"])
    assert np.array_equal(r["key"], uk)
    assert np.array_equal(r["sum_qty"], s)
    assert np.array_equal(r["count"], cnt)
    keep = c["fact"]["day"] < c["day_cut"]
    # pk is a permutation covering every fk, so the join keeps every filtered row
    assert int(r["count"].sum()) == int(keep.sum())
    assert int(r["sum_qty"].sum()) == int(c["fact"]["qty"][keep].sum())
    # independent numpy statement: cat of each kept row via an inverse permutation
    inv = np.empty(len(c["dim"]["pk"]), np.int64)
    inv[c["dim"]["pk"]] = np.arange(len(c["dim"]["pk"]))
    cats = c["dim"]["cat"][inv[c["fact"]["fk"][keep]]]
    w = np.bincount(cats, weights=None, minlength=25)
    assert np.array_equal(r["count"], w[w > 0])


def brute_q1(fact, dim, cut):
    g = {}
    for i in range(len(fact["fk"])):
        if fact["day"][i] < cut:
            for j in range(len(dim["pk"])):
                if dim["pk"][j] == fact["fk"][i]:
                    k = int(dim["cat"][j])
                    s, c = g.get(k, (0, 0))
                    g[k] = (s + int(fact["qty"][i]), c + 1)
    ks = sorted(g)
    return ks, [g[k][0] for k in ks], [g[k][1] for k in ks]


def test_q1_brute_force_with_duplicate_dim_keys():
    fact = {"fk": dg.uniform_int(4, 1, 400, 0, 30, np.int32),
            "qty": dg.uniform_int(4, 2, 400, 1, 5001, np.int64),
            "day": dg.uniform_int(4, 3, 400, 0, 10, np.int32)}
    dim = {"pk": dg.uniform_int(4, 4, 40, 0, 35, np.int32),   # duplicates + misses
           "cat": dg.uniform_int(4, 5, 40, 0, 7, np.int32)}
    r = oracle.q1(fact, dim, 5)
    ks, s, c = brute_q1(fact, dim, 5)
    assert r["key"].tolist() == ks and r["sum_qty"].tolist() == s and r["count"].tolist() == c
    uk, s2, c2 = composed_q1(fact, dim, 5)
    assert uk.tolist() == ks and s2.tolist() == s and c2.tolist() == c


def test_q2_matches_composed_operators():
    c = dg.config2(0, n_fact=300_000, n_dim=20_000)
    f, d = c["fact"], c["dim"]
    r = oracle.q2(f, d, c["day_cut"])
    rows = oracle.filter_rows([f["day"]], [(0, "<", c["day_cut"])])
    fk = oracle.gather(f["fk"], rows)
    cnt, li, ri = oracle.join(fk, d["pk"])
    frow = rows[li]
    key = f["flag"][frow].astype(np.int64) * 2 + (d["cat"][ri] % 2)
    uk, (sq, sp, sc), _ = oracle.groupby(key, [f["qty"][frow], f["price"][frow]],
                                         [("sum", 0), ("sum", 1), ("count",)])
    assert np.array_equal(r["a_key"], uk)
    assert np.array_equal(r["a_qty"], sq) and np.array_equal(r["a_price"], sp)
    assert np.array_equal(r["a_count"], sc)
    ub, (bq, bc), _ = oracle.groupby(f["fk"][frow], [f["qty"][frow]], [("sum", 0), ("count",)])
    assert np.array_equal(r["b_key"], ub)
    assert np.array_equal(r["b_qty"], bq) and np.array_equal(r["b_count"], bc)
    assert int(r["a_count"].sum()) == cnt == len(rows)
    assert int(r["b_qty"].sum()) == int(f["qty"][rows].sum())
    assert len(r["b_key"]) == len(np.unique(f["fk"][rows]))


def test_q3_matches_numpy_statement():
    c = dg.config3(0, n_fact=200_000, dims=(5_000, 800, 25))
    r = oracle.q3(c)
    f = c["fact"]
    cut = c["attr_cut"]
    inv = []
    for d in (c["d1"], c["d2"], c["d3"]):
        x = np.empty(len(d["pk"]), np.int64)
        x[d["pk"]] = np.arange(len(d["pk"]))
        inv.append(x)
    j1, j2, j3 = inv[0][f["fk1"]], inv[1][f["fk2"]], inv[2][f["fk3"]]
    keep = ((c["d1"]["attr"][j1] < cut) & (c["d2"]["attr"][j2] < cut)
            & (c["d3"]["attr"][j3] < cut))
    key = c["d1"]["cat"][j1[keep]].astype(np.int64) * 5 + c["d2"]["cat"][j2[keep]]
    nk, ix = np.unique(key, return_inverse=True)
    sp = np.zeros(len(nk), np.int64)
    np.add.at(sp, ix, f["qty"][keep] * f["price"][keep])
    assert np.array_equal(r["key"], nk)
    assert np.array_equal(r["sum_qp"], sp)
    assert np.array_equal(r["count"], np.bincount(ix).astype(np.int64))


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_multithreaded_whole_queries_equal_the_single_thread_oracle(threads):
    """The multi-core timing leg (per-thread group accumulators merged at the
    end) returns the single-thread oracle's bytes, including with duplicate
    dimension keys, misses and an empty fact table."""
    c1 = dg.config1(3, n_fact=50_000, n_dim=700)
    c1["dim"]["pk"][::7] = 5                      # duplicate keys and misses
    for fact, dim in ((c1["fact"], c1["dim"]),
                      ({k: v[:0] for k, v in c1["fact"].items()}, c1["dim"])):
        a = oracle.q1(fact, dim, c1["day_cut"])
        b = oracle.q1(fact, dim, c1["day_cut"], threads=threads)
        assert all(np.array_equal(a[k], b[k]) for k in a)
    c2 = dg.config2(1, n_fact=120_000, n_dim=9_000)
    a = oracle.q2(c2["fact"], c2["dim"], c2["day_cut"])
    b = oracle.q2(c2["fact"], c2["dim"], c2["day_cut"], threads=threads)
    assert all(np.array_equal(a[k], b[k]) for k in a)
    c3 = dg.config3(2, n_fact=150_000, dims=(4_000, 600, 25))
    a = oracle.q3(c3)
    b = oracle.q3(c3, threads=threads)
    assert all(np.array_equal(a[k], b[k]) for k in a)


# -------------------------------------------- filter + aggregate (Q6 shape) ----

def wrap64(x: int) -> int:
    return (x + 2 ** 63) % 2 ** 64 - 2 ** 63


@pytest.mark.parametrize("seed", range(4))
def test_filter_sum_brute_force(seed):
    """Python integers over every kept row: the product, the wrap, the count."""
    n = 257 + 61 * seed
    cols = rng_cols(seed, n, dom=20)
    a = dg.uniform_int(seed, 7, n, -2 ** 31, 2 ** 31, np.int64) * 4_000_000_007
    b = dg.uniform_int(seed, 8, n, -128, 128, np.int8)
    preds = [((seed + q) % 3, list(OPS)[(seed * 5 + q) % 6], int(cols[(seed + q) % 3][q * 7 % n]))
             for q in range(1 + seed % 3)]
    keep = [i for i in range(n) if all(OPS[op](int(cols[c][i]), lit) for c, op, lit in preds)]
    exact = sum(int(a[i]) * int(b[i]) for i in keep)
    s, c, ex = oracle.filter_sum(cols, preds, a, b)
    assert c == len(keep) and s == wrap64(exact) and ex == (I64_MIN <= exact <= I64_MAX)
    s1, c1, _ = oracle.filter_sum(cols, preds, a)
    assert c1 == len(keep) and s1 == wrap64(sum(int(a[i]) for i in keep))
    assert oracle.filter_sum(cols, preds) == (0, len(keep), True)


def test_filter_sum_matches_numpy_and_edge_cases():
    n = 5000
    cols = rng_cols(11, n, dom=100)
    a = dg.uniform_int(11, 9, n, 0, 1 << 30, np.int64)
    b = dg.uniform_int(11, 10, n, -5, 6, np.int32)
    preds = [(0, ">=", -40), (1, "<", 60), (2, "!=", 3)]
    m = (cols[0] >= -40) & (cols[1] < 60) & (cols[2] != 3)
    s, c, ex = oracle.filter_sum(cols, preds, a, b)
    assert c == int(m.sum()) and s == int(np.sum(a[m] * b[m])) and ex
    # no predicate keeps every row; an impossible one keeps none
    assert oracle.filter_sum(cols, [], a, b)[:2] == (int(np.sum(a * b)), n)
    assert oracle.filter_sum(cols, [(0, ">", 1000)], a, b) == (0, 0, True)
    e = [np.zeros(0, np.int32)]
    assert oracle.filter_sum(e, [(0, "<", 5)], np.zeros(0, np.int64)) == (0, 0, True)
    # the sum leaves int64: wrapped mod 2**64 and flagged
    big = np.full(4, I64_MAX // 2 + 7, np.int64)
    s, c, ex = oracle.filter_sum([np.arange(4, dtype=np.int32)], [], big, np.full(4, 3, np.int8))
    assert c == 4 and not ex and s == wrap64(4 * 3 * (I64_MAX // 2 + 7))


@pytest.mark.parametrize("n", [0, 1, 999, 20_000])
def test_q6_whole_query_equals_generic_filter_sum(n):
    """The directly written Q6 loop against the generic conjunction (the same
    five comparisons as predicates) and a numpy statement of the query."""
    cfg = dg.config_q6(3, n)
    t = cfg["items"]
    got = oracle.q6(cfg)
    preds = [(0, ">=", cfg["ship_lo"]), (0, "<", cfg["ship_hi"]), (1, ">=", cfg["disc_lo"]),
             (1, "<=", cfg["disc_hi"]), (2, "<", cfg["qty_cut"])]
    s, c, ex = oracle.filter_sum([t["ship"], t["discount"], t["quantity"]], preds, t["price"],
                                 t["discount"])
    assert (got["sum"], got["count"], got["exact"]) == (s, c, ex) and ex
    m = ((t["ship"] >= cfg["ship_lo"]) & (t["ship"] < cfg["ship_hi"]) & (t["discount"] >= 5)
         & (t["discount"] <= 7) & (t["quantity"] < 24))
    assert c == int(m.sum())
    assert s == int(np.sum(t["price"][m] * t["discount"][m].astype(np.int64)))


def test_q6_table_shape():
    """Timestamps are whole seconds inside the seven-year window; the kept
    fraction is near the product of the three selectivities."""
    cfg = dg.config_q6(0, 200_000)
    t = cfg["items"]
    ns_day = 86_400 * 10 ** 9
    assert t["ship"].dtype == np.int64 and (t["ship"] % 10 ** 9 == 0).all()
    assert t["ship"].min() >= 8035 * ns_day and t["ship"].max() < (8035 + 2557) * ns_day
    assert t["discount"].min() == 0 and t["discount"].max() == 10
    frac = oracle.q6(cfg)["count"] / 200_000
    expect = 365 / 2557 * 3 / 11 * 23 / 50
    assert abs(frac - expect) < 0.1 * expect


# ------------------------------------------ strings and the Q14 shape ----

def test_str_match_brute_force():
    """Python bytes comparisons row by row, patterns of every length."""
    n, m = 700, 12
    lens = dg.uniform_int(4, 1, n, 0, m + 1, np.int64)
    chars = np.zeros((n, m), np.uint8)
    letters = dg.uniform_int(4, 2, n * m, 65, 69, np.uint8).reshape(n, m)   # 'A'..'D'
    for i in range(n):
        chars[i, :lens[i]] = letters[i, :lens[i]]
    rows = [bytes(chars[i]) for i in range(n)]
    for pat in [b"", b"A", b"AB", b"ABC", b"DDDD", bytes(chars[3][:lens[3]]), b"A" * m, b"A" * (m + 1)]:
        pre = oracle.str_match(chars, pat, "prefix")
        eq = oracle.str_match(chars, pat, "equal")
        assert pre.tolist() == [int(len(pat) <= m and r[:len(pat)] == pat) for r in rows], pat
        assert eq.tolist() == [int(len(pat) <= m and r == pat + bytes(m - len(pat))) for r in rows], pat
    assert oracle.str_match(np.zeros((0, 5), np.uint8), b"A").size == 0


def composed_q14(cfg):
    """Q14 from the operator oracles: filter -> gather -> join -> string match."""
    t, p = cfg["items"], cfg["part"]
    rows = oracle.filter_rows([t["ship"]], [(0, ">=", cfg["ship_lo"]), (0, "<", cfg["ship_hi"])])
    cnt, li, ri = oracle.join(oracle.gather(t["partkey"], rows), p["pk"])
    flag = oracle.str_match(p["type"], cfg["prefix"])[ri]
    price = oracle.gather(oracle.gather(t["price"], rows), li).astype(object)
    disc = oracle.gather(oracle.gather(t["discount"], rows), li).astype(object)
    rev = price * (100 - disc)
    return int(sum(rev[flag == 1])), int(sum(rev)), int(cnt), int((flag == 1).sum())


@pytest.mark.parametrize("seed,ni,npart", [(0, 30_000, 2_000), (1, 5_000, 37), (2, 0, 10)])
def test_q14_whole_query_equals_composed_and_numpy(seed, ni, npart):
    cfg = dg.config_q14(seed, ni, npart)
    got = oracle.q14(cfg)
    promo, total, cnt, pcnt = composed_q14(cfg)
    assert (got["promo_rev"], got["total_rev"], got["count"], got["promo_count"]) == \
        (promo, total, cnt, pcnt) and got["exact"]
    # numpy statement: pk is a permutation, so the part row of key k is inv[k]
    t, p = cfg["items"], cfg["part"]
    inv = np.empty(npart, np.int64)
    inv[p["pk"]] = np.arange(npart)
    m = (t["ship"] >= cfg["ship_lo"]) & (t["ship"] < cfg["ship_hi"])
    row = inv[t["partkey"][m]]
    pl = len(cfg["prefix"])
    promo_row = (p["type"][:, :pl] == np.frombuffer(cfg["prefix"], np.uint8)).all(axis=1)[row]
    rev = t["price"][m] * (100 - t["discount"][m].astype(np.int64))
    assert got["total_rev"] == int(rev.sum()) and got["promo_rev"] == int(rev[promo_row].sum())


def test_q14_empty_prefix_selects_every_type():
    cfg = dg.config_q14(3, 20_000, 300)
    cfg = dict(cfg, prefix=b"")
    got = oracle.q14(cfg)
    assert got["promo_rev"] == got["total_rev"] and got["promo_count"] == got["count"] > 0


def test_type_vocabulary_shape():
    table, prefix = dg.type_vocabulary(0)
    names = {bytes(r).rstrip(b"\0") for r in table}
    assert table.shape[0] == 150 and len(names) == 150
    # a sixth of the types start with the prefix word (followed by its space)
    assert sum(nm.startswith(prefix) for nm in names) == 25
    assert all(nm.count(b" ") == 2 for nm in names)


# --------------------------------------------- PREDICT inside a query ----

def int_mlp_class(model, F, H, C, x):
    """Exact integer forward pass (every value below is a small integer, so
    the fp32 fused multiply-adds of the oracle are exact too)."""
    w1 = model[:H * F].reshape(H, F)
    b1 = model[H * F:H * F + H]
    w2 = model[H * F + H:H * F + H + C * H].reshape(C, H)
    b2 = model[H * F + H + C * H:]
    h = [max(int(b1[j]) + sum(int(w1[j, k]) * int(x[k]) for k in range(F)), 0) for j in range(H)]
    z = [int(b2[c]) + sum(int(w2[c, j]) * h[j] for j in range(H)) for c in range(C)]
    return z.index(max(z))            # the first of the largest


@pytest.mark.parametrize("seed", range(3))
def test_mlp_predict_exact_on_integer_models(seed):
    F, H, C, n = 5, 7, 3, 400
    model = dg.uniform_int(seed, 30, H * F + H + C * H + C, -4, 5, np.int64).astype(np.float32)
    feats = [dg.uniform_int(seed, 40 + k, n, -6, 7, np.int32) for k in range(F)]
    got = oracle.mlp_predict(feats, model, H, C)
    want = [int_mlp_class(model, F, H, C, [f[i] for f in feats]) for i in range(n)]
    assert got.tolist() == want


def test_mlp_predict_agrees_with_float64_away_from_ties():
    cfg = dg.config_predict(1, 50_000)
    t, model, F, H = cfg["reviews"], cfg["model"].astype(np.float64), cfg["nfeat"], cfg["hidden"]
    X = np.stack([t[f"f{k}"] for k in range(F)], axis=1).astype(np.float64)
    w1, b1 = model[:H * F].reshape(H, F), model[H * F:H * F + H]
    w2, b2 = model[H * F + H:H * F + H + 2 * H].reshape(2, H), model[H * F + H + 2 * H:]
    z = np.maximum(X @ w1.T + b1, 0) @ w2.T + b2
    got = oracle.mlp_predict([t[f"f{k}"] for k in range(F)], cfg["model"], H, 2)
    clear = np.abs(z[:, 1] - z[:, 0]) > 1e-3
    assert clear.mean() > 0.99
    assert np.array_equal(got[clear], np.argmax(z[clear], axis=1).astype(np.int8))


def test_mlp_predict_ties_rows_and_empty():
    F, H, C = 3, 4, 3
    zero = np.zeros(H * F + H + C * H + C, np.float32)
    feats = [np.arange(10, dtype=np.int32)] * F
    assert oracle.mlp_predict(feats, zero, H, C).tolist() == [0] * 10      # all tied: first
    m = zero.copy()
    m[-1] = 1.0                                                            # b2 = (0, 0, 1)
    assert oracle.mlp_predict(feats, m, H, C).tolist() == [2] * 10
    cfg = dg.config_predict(2, 3_000)
    fs = [cfg["reviews"][f"f{k}"] for k in range(cfg["nfeat"])]
    rows = np.array([5, 0, 2999, 5, 17], np.int32)
    full = oracle.mlp_predict(fs, cfg["model"], cfg["hidden"], 2)
    assert np.array_equal(oracle.mlp_predict(fs, cfg["model"], cfg["hidden"], 2, rows), full[rows])
    assert oracle.mlp_predict(fs, cfg["model"], cfg["hidden"], 2, rows[:0]).size == 0


@pytest.mark.parametrize("n", [0, 1, 20_000])
def test_q_predict_equals_composed(n):
    cfg = dg.config_predict(3, n)
    t = cfg["reviews"]
    got = oracle.q_predict(cfg)
    rows = oracle.filter_rows([t["year"]], [(0, ">=", cfg["year_min"])])
    cls = oracle.mlp_predict([t[f"f{k}"] for k in range(cfg["nfeat"])], cfg["model"],
                             cfg["hidden"], cfg["classes"], rows)
    r = t["rating"][rows].astype(np.int64)
    assert np.array_equal(got["count"], np.bincount(r, minlength=cfg["nratings"]))
    assert np.array_equal(got["positive"], np.bincount(r[cls == 1], minlength=cfg["nratings"]))
