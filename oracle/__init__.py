"""CPU oracle for the relational hot path -- TEST INFRASTRUCTURE ONLY.

Plain definitions of filter, stable sort, equi-join, join ranges, group-by
aggregation and whole queries, in C (``tqp_oracle.c``, built with gcc) behind
ctypes.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark import this package; the GPU library never does, and the two share
no code.  All inputs are numpy arrays; all outputs are numpy arrays.

Conventions (the paper states SQL semantics only, Sections 2.2-2.3):
  * filter keeps rows in ascending row-id order;
  * sort is stable and ascending on the signed value;
  * join returns every (i, j) with L[i] == R[j], ordered by (key, i, j);
  * group-by emits the groups that occur, ascending by key, SUM mod 2**64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tqp_oracle.c")
_LIB = os.path.join(_HERE, "libtqp_oracle.so")

DT = {np.dtype(np.int8): 1, np.dtype(np.int32): 2, np.dtype(np.int64): 3}
OPS = {"<": 0, "<=": 1, ">": 2, ">=": 3, "==": 4, "!=": 5}
AGG_SUM, AGG_COUNT, AGG_SUM_PRODUCT, AGG_SUM_DIFF_PRODUCT = 0, 1, 2, 3

_lib = None


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc into ``oracle/libtqp_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        # no contraction: every fused multiply-add in the source is an explicit fmaf
        # -fopenmp: only the *_mt whole-query functions (the multi-core timing
        # leg) use threads; everything else is single-threaded
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fopenmp", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        _lib.orc_filter.restype = i64
        _lib.orc_filter.argtypes = [i64, vp, vp, i32, vp, vp, vp, vp]
        _lib.orc_semijoin.restype = i64
        _lib.orc_semijoin.argtypes = [i64, i32, vp, vp, vp, vp, vp, vp]
        _lib.orc_gather.restype = None
        _lib.orc_gather.argtypes = [i64, vp, i32, vp, vp]
        _lib.orc_sort.restype = i32
        _lib.orc_sort.argtypes = [i64, vp, i32, vp, vp]
        _lib.orc_join.restype = i64
        _lib.orc_join.argtypes = [i64, vp, i64, vp, i32, i64, vp, vp]
        _lib.orc_join_ranges.restype = i64
        _lib.orc_join_ranges.argtypes = [i64, vp, i64, vp, i32, i64, vp, vp, vp,
                                         vp, vp, vp, vp]
        _lib.orc_groupby.restype = i64
        _lib.orc_groupby.argtypes = [i64, vp, i32, vp, vp, i32, vp, vp, vp, vp, i64,
                                     vp, vp, vp]
        _lib.orc_q1.restype = i64
        _lib.orc_q1.argtypes = [i64, vp, vp, vp, i64, i64, vp, vp, i64, vp, vp,
                                vp, vp]
        _lib.orc_q2.restype = i32
        _lib.orc_q2.argtypes = [i64, vp, vp, vp, vp, vp, i64, i64, vp, vp,
                                i64, vp, vp, vp, vp, vp,
                                i64, vp, vp, vp, vp, vp]
        _lib.orc_filter_sum.restype = None
        _lib.orc_filter_sum.argtypes = [i64, vp, vp, i32, vp, vp, vp, vp, i32, vp, i32, vp, vp,
                                        vp]
        _lib.orc_q6.restype = None
        _lib.orc_q6.argtypes = [i64, vp, vp, vp, vp, i64, i64, i64, i64, i64, vp, vp, vp]
        _lib.orc_str_match.restype = None
        _lib.orc_str_match.argtypes = [i64, i32, vp, vp, i32, i32, vp]
        _lib.orc_q14.restype = None
        _lib.orc_q14.argtypes = [i64, vp, vp, vp, vp, i64, i64, i64, vp, i32, vp, vp, i32,
                                 vp, vp, vp, vp, vp]
        _lib.orc_mlp_predict.restype = None
        _lib.orc_mlp_predict.argtypes = [i64, vp, vp, i32, vp, vp, i32, i32, vp]
        _lib.orc_q_predict.restype = None
        _lib.orc_q_predict.argtypes = [i64, vp, vp, i64, vp, i32, vp, i32, i32, i32, vp, vp]
        _lib.orc_max_threads.restype = i32
        _lib.orc_max_threads.argtypes = []
        _lib.orc_q1_mt.restype = i64
        _lib.orc_q1_mt.argtypes = [i32] + list(_lib.orc_q1.argtypes)
        _lib.orc_q2_mt.restype = i32
        _lib.orc_q2_mt.argtypes = [i32] + list(_lib.orc_q2.argtypes)
        _lib.orc_q3_mt.restype = i64
        _lib.orc_q3_mt.argtypes = [i32, i64, vp, vp, vp, vp, vp,
                                   i64, vp, vp, vp, i64, vp, vp, vp, i64, vp, vp,
                                   i64, i64, vp, vp, vp, vp]
        _lib.orc_q3.restype = i64
        _lib.orc_q3.argtypes = [i64, vp, vp, vp, vp, vp,
                                i64, vp, vp, vp, i64, vp, vp, vp, i64, vp, vp,
                                i64, i64, vp, vp, vp, vp]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype=dtype))
    return a


def _ptr_array(arrs):
    return (ctypes.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])


def filter_rows(cols, preds) -> np.ndarray:
    """Row ids (int32, ascending) where every predicate holds.

    cols: list of 1-D int8/int32/int64 arrays of equal length.
    preds: list of (col_index, op_string, literal).
    """
    cols = [_c(c) for c in cols]
    n = len(cols[0]) if cols else 0
    dts = np.array([DT[c.dtype] for c in cols], dtype=np.int32)
    pc = np.array([p[0] for p in preds], dtype=np.int32)
    po = np.array([OPS[p[1]] for p in preds], dtype=np.int32)
    pl = np.array([int(p[2]) for p in preds], dtype=np.int64)
    out = np.empty(max(n, 1), dtype=np.int32)
    ptrs = _ptr_array(cols)
    cnt = lib().orc_filter(n, ptrs, _p(dts), len(preds), _p(pc), _p(po), _p(pl), _p(out))
    return out[:cnt].copy()


def filter_sum(cols, preds, a=None, b=None):
    """WHERE + aggregate over the kept rows, nothing materialised.

    cols/preds as in filter_rows; a, b: value arrays (or None).  Returns
    (SUM(a*b) or SUM(a) mod 2**64 as int, COUNT, exact) where exact says the
    true sum stayed inside int64.
    """
    cols = [_c(c) for c in cols]
    n = len(cols[0]) if cols else (len(a) if a is not None else 0)
    dts = np.array([DT[c.dtype] for c in cols] or [0], dtype=np.int32)
    pc = np.array([p[0] for p in preds] or [0], dtype=np.int32)
    po = np.array([OPS[p[1]] for p in preds] or [0], dtype=np.int32)
    pl = np.array([int(p[2]) for p in preds] or [0], dtype=np.int64)
    a = None if a is None else _c(a)
    b = None if b is None else _c(b)
    s, c, ex = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int(0)
    lib().orc_filter_sum(n, _ptr_array(cols), _p(dts), len(preds), _p(pc), _p(po), _p(pl),
                         None if a is None else _p(a), 0 if a is None else DT[a.dtype],
                         None if b is None else _p(b), 0 if b is None else DT[b.dtype],
                         ctypes.byref(s), ctypes.byref(c), ctypes.byref(ex))
    return int(s.value), int(c.value), bool(ex.value)


def q6(cfg: dict):
    """Q6-shaped scan: SUM(price * discount), COUNT(*) under the date,
    discount and quantity conjunction (see orc_q6)."""
    t = cfg["items"]
    ship, disc = _c(t["ship"], np.int64), _c(t["discount"], np.int8)
    qty, price = _c(t["quantity"], np.int32), _c(t["price"], np.int64)
    s, c, ex = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int(0)
    lib().orc_q6(len(ship), _p(ship), _p(disc), _p(qty), _p(price), cfg["ship_lo"],
                 cfg["ship_hi"], cfg["disc_lo"], cfg["disc_hi"], cfg["qty_cut"],
                 ctypes.byref(s), ctypes.byref(c), ctypes.byref(ex))
    return {"sum": int(s.value), "count": int(c.value), "exact": bool(ex.value)}


def str_match(chars: np.ndarray, pattern: bytes, mode: str = "prefix") -> np.ndarray:
    """LIKE 'pattern%' (mode "prefix") or = 'pattern' (mode "equal") over an
    (n, m) uint8 matrix of zero-padded strings; int8 0/1 per row."""
    chars = _c(chars, np.uint8)
    n, m = chars.shape
    pat = np.frombuffer(bytes(pattern), np.uint8).copy() if pattern else np.zeros(1, np.uint8)
    out = np.empty(max(n, 1), np.int8)
    lib().orc_str_match(n, m, _p(chars), _p(pat), len(pattern), {"prefix": 0, "equal": 1}[mode],
                        _p(out))
    return out[:n].copy()


def q14(cfg: dict):
    """Q14-shaped join: promo and total revenue, row counts (see orc_q14)."""
    t, p = cfg["items"], cfg["part"]
    ship, pkey = _c(t["ship"], np.int64), _c(t["partkey"], np.int32)
    price, disc = _c(t["price"], np.int64), _c(t["discount"], np.int8)
    pk, types = _c(p["pk"], np.int32), _c(p["type"], np.uint8)
    pre = np.frombuffer(bytes(cfg["prefix"]), np.uint8).copy()
    out = [ctypes.c_int64(0) for _ in range(4)]
    ex = ctypes.c_int(0)
    lib().orc_q14(len(ship), _p(ship), _p(pkey), _p(price), _p(disc), cfg["ship_lo"],
                  cfg["ship_hi"], len(pk), _p(pk), types.shape[1], _p(types), _p(pre), len(pre),
                  *[ctypes.byref(o) for o in out], ctypes.byref(ex))
    return {"promo_rev": out[0].value, "total_rev": out[1].value, "count": out[2].value,
            "promo_count": out[3].value, "exact": bool(ex.value)}


def mlp_predict(feats, model: np.ndarray, hidden: int, classes: int, rows=None) -> np.ndarray:
    """Class (int8) of each row under the fp32 one-hidden-layer MLP (see
    orc_mlp_predict); feats: list of F integer columns; rows: optional row
    ids (int32) selecting the rows scored."""
    feats = [_c(f) for f in feats]
    model = _c(model, np.float32)
    rows = None if rows is None else _c(rows, np.int32)
    n = len(rows) if rows is not None else (len(feats[0]) if feats else 0)
    dts = np.array([DT[f.dtype] for f in feats], np.int32)
    out = np.empty(max(n, 1), np.int8)
    lib().orc_mlp_predict(n, _ptr_array(feats), _p(dts), len(feats),
                          None if rows is None else _p(rows), _p(model), hidden, classes, _p(out))
    return out[:n].copy()


def q_predict(cfg: dict):
    """Per rating: predicted-positive count and row count (see orc_q_predict)."""
    t = cfg["reviews"]
    feats = [_c(t[f"f{k}"], np.int32) for k in range(cfg["nfeat"])]
    nr = cfg["nratings"]
    pos, cnt = np.zeros(nr, np.int64), np.zeros(nr, np.int64)
    lib().orc_q_predict(len(t["rating"]), _p(_c(t["rating"], np.int8)), _p(_c(t["year"], np.int32)),
                        cfg["year_min"], _ptr_array(feats), len(feats),
                        _p(_c(cfg["model"], np.float32)), cfg["hidden"], cfg["classes"], nr,
                        _p(pos), _p(cnt))
    return {"positive": pos, "count": cnt}


def semijoin_rows(keys, sets) -> np.ndarray:
    """Row ids (int32, ascending) of the left table whose key keys[s][i]
    occurs among sets[s] (the other side's keys) for every s.

    keys: list of equal-length 1-D int8/int32/int64 arrays (the left side's
    key columns); sets: list of 1-D integer arrays, one per key column.
    """
    keys = [_c(k) for k in keys]
    sets = [_c(t) for t in sets]
    n = len(keys[0]) if keys else 0
    dts = np.array([DT[k.dtype] for k in keys] or [0], dtype=np.int32)
    sdt = np.array([DT[t.dtype] for t in sets] or [0], dtype=np.int32)
    sn = np.array([len(t) for t in sets] or [0], dtype=np.int64)
    out = np.empty(max(n, 1), dtype=np.int32)
    cnt = lib().orc_semijoin(n, len(keys), _ptr_array(keys), _p(dts), _ptr_array(sets), _p(sdt),
                             _p(sn), _p(out))
    return out[:cnt].copy()


def gather(src: np.ndarray, idx: np.ndarray) -> np.ndarray:
    src = _c(src)
    idx = _c(idx, np.int32)
    out = np.empty(len(idx), dtype=src.dtype)
    lib().orc_gather(len(idx), _p(src), DT[src.dtype], _p(idx), _p(out))
    return out


def sort(keys: np.ndarray):
    """Stable ascending sort. Returns (sorted_keys, perm int32)."""
    keys = _c(keys)
    n = len(keys)
    ok = np.empty(max(n, 1), dtype=keys.dtype)
    perm = np.empty(max(n, 1), dtype=np.int32)
    rc = lib().orc_sort(n, _p(keys), DT[keys.dtype], _p(ok), _p(perm))
    assert rc == 0
    return ok[:n].copy(), perm[:n].copy()


def join(lk: np.ndarray, rk: np.ndarray, cap: int | None = None):
    """Inner equi-join pairs (L row, R row) in (key, i, j) order.

    Returns (count, out_l, out_r); the arrays are empty if count > cap.
    """
    lk = _c(lk)
    rk = _c(rk)
    assert lk.dtype == rk.dtype
    if cap is None:
        cnt = lib().orc_join(len(lk), _p(lk), len(rk), _p(rk), DT[lk.dtype], 0,
                             None, None)
        cap = cnt
    ol = np.empty(max(cap, 1), dtype=np.int32)
    orr = np.empty(max(cap, 1), dtype=np.int32)
    cnt = lib().orc_join(len(lk), _p(lk), len(rk), _p(rk), DT[lk.dtype], cap,
                         _p(ol), _p(orr))
    if cnt > cap:
        return cnt, np.empty(0, np.int32), np.empty(0, np.int32)
    return cnt, ol[:cnt].copy(), orr[:cnt].copy()


def join_ranges(lk: np.ndarray, rk: np.ndarray):
    """Per matched key: key, lstart, lcnt, rstart, rcnt (int64) and the total."""
    lk = _c(lk)
    rk = _c(rk)
    cap = min(len(lk), len(rk))
    bufs = [np.empty(max(cap, 1), dtype=np.int64) for _ in range(5)]
    total = ctypes.c_int64(0)
    ovf = ctypes.c_int(0)
    m = lib().orc_join_ranges(len(lk), _p(lk), len(rk), _p(rk), DT[lk.dtype], cap,
                              *[_p(b) for b in bufs], ctypes.byref(total),
                              ctypes.byref(ovf))
    out = {k: b[:m].copy() for k, b in zip(("key", "lstart", "lcnt", "rstart", "rcnt"), bufs)}
    out["total"] = total.value
    out["total_overflow"] = bool(ovf.value)
    return out


def groupby(keys: np.ndarray, vals, aggs):
    """GROUP BY keys.  aggs: list of ("sum", a) | ("count",) | ("sum_product", a, b)
    | ("sum_diff_product", a, b, c): SUM(vals[a] * (c - vals[b])).

    Returns (unique_keys int64, [agg arrays int64], overflow flag).
    """
    keys = _c(keys)
    vals = [_c(v) for v in vals]
    n = len(keys)
    op = np.array([{"sum": AGG_SUM, "count": AGG_COUNT, "sum_product": AGG_SUM_PRODUCT,
                    "sum_diff_product": AGG_SUM_DIFF_PRODUCT}[a[0]]
                   for a in aggs], dtype=np.int32)
    aa = np.array([a[1] if len(a) > 1 else 0 for a in aggs], dtype=np.int32)
    ab = np.array([a[2] if len(a) > 2 else 0 for a in aggs], dtype=np.int32)
    ac = np.array([a[3] if len(a) > 3 else 0 for a in aggs], dtype=np.int64)
    vdt = np.array([DT[v.dtype] for v in vals] or [3], dtype=np.int32)
    ok = np.empty(max(n, 1), dtype=np.int64)
    outs = [np.empty(max(n, 1), dtype=np.int64) for _ in aggs]
    ovf = ctypes.c_int(0)
    ng = lib().orc_groupby(n, _p(keys), DT[keys.dtype], _ptr_array(vals), _p(vdt),
                           len(aggs), _p(op), _p(aa), _p(ab), _p(ac), n, _p(ok),
                           _ptr_array(outs), ctypes.byref(ovf))
    return ok[:ng].copy(), [o[:ng].copy() for o in outs], bool(ovf.value)


def max_threads() -> int:
    """Threads the multi-core whole-query functions use by default."""
    return int(lib().orc_max_threads())


def _mt(fn_1, fn_mt, threads):
    """The single-thread function (threads 0: the parity checker) or its
    multi-threaded twin bound to a thread count."""
    if not threads:
        return fn_1
    return lambda *a: fn_mt(int(threads), *a)


def q1(fact: dict, dim: dict, day_cut: int, threads: int = 0):
    """SELECT cat, SUM(qty), COUNT(*) ... WHERE day < day_cut GROUP BY cat.
    threads > 0 runs the multi-threaded twin (same result)."""
    fk, qty, day = _c(fact["fk"], np.int32), _c(fact["qty"], np.int64), _c(fact["day"], np.int32)
    pk, cat = _c(dim["pk"], np.int32), _c(dim["cat"], np.int32)
    cap = max(len(pk), 1)
    k, s, c = (np.empty(cap, np.int64) for _ in range(3))
    ovf = ctypes.c_int(0)
    ng = _mt(lib().orc_q1, lib().orc_q1_mt, threads)(
        len(fk), _p(fk), _p(qty), _p(day), day_cut, len(pk), _p(pk),
                      _p(cat), cap, _p(k), _p(s), _p(c), ctypes.byref(ovf))
    return {"key": k[:ng].copy(), "sum_qty": s[:ng].copy(), "count": c[:ng].copy(),
            "overflow": bool(ovf.value)}


def q2(fact: dict, dim: dict, day_cut: int, threads: int = 0):
    """Skewed star query: low-cardinality and per-fk group-bys after the join.
    threads > 0 runs the multi-threaded twin (same result)."""
    fk = _c(fact["fk"], np.int32)
    qty = _c(fact["qty"], np.int64)
    price = _c(fact["price"], np.int64)
    flag = _c(fact["flag"], np.int8)
    day = _c(fact["day"], np.int32)
    pk, cat = _c(dim["pk"], np.int32), _c(dim["cat"], np.int32)
    capa = 1024
    capb = max(len(pk), 1)
    a = [np.empty(capa, np.int64) for _ in range(4)]
    b = [np.empty(capb, np.int64) for _ in range(3)]
    nga, ngb = ctypes.c_int64(0), ctypes.c_int64(0)
    ovf = ctypes.c_int(0)
    _mt(lib().orc_q2, lib().orc_q2_mt, threads)(
        len(fk), _p(fk), _p(qty), _p(price), _p(flag), _p(day), day_cut,
                 len(pk), _p(pk), _p(cat), capa, *[_p(x) for x in a], ctypes.byref(nga),
                 capb, *[_p(x) for x in b], ctypes.byref(ngb), ctypes.byref(ovf))
    na, nb = nga.value, ngb.value
    return {"a_key": a[0][:na].copy(), "a_qty": a[1][:na].copy(),
            "a_price": a[2][:na].copy(), "a_count": a[3][:na].copy(),
            "b_key": b[0][:nb].copy(), "b_qty": b[1][:nb].copy(),
            "b_count": b[2][:nb].copy(), "overflow": bool(ovf.value)}


def q3(cfg: dict, threads: int = 0):
    """Star join over three filtered dims, GROUP BY d1.cat * 5 + d2.cat.
    threads > 0 runs the multi-threaded twin (same result)."""
    f, d1, d2, d3 = cfg["fact"], cfg["d1"], cfg["d2"], cfg["d3"]
    fk1, fk2, fk3 = (_c(f[k], np.int32) for k in ("fk1", "fk2", "fk3"))
    qty, price = _c(f["qty"], np.int64), _c(f["price"], np.int64)
    a1 = [_c(d1[k], np.int32) for k in ("pk", "cat", "attr")]
    a2 = [_c(d2[k], np.int32) for k in ("pk", "cat", "attr")]
    a3 = [_c(d3[k], np.int32) for k in ("pk", "attr")]
    cap = 1 << 16
    k, s, c = (np.empty(cap, np.int64) for _ in range(3))
    ovf = ctypes.c_int(0)
    ng = _mt(lib().orc_q3, lib().orc_q3_mt, threads)(
        len(fk1), _p(fk1), _p(fk2), _p(fk3), _p(qty), _p(price),
                      len(a1[0]), *[_p(x) for x in a1], len(a2[0]), *[_p(x) for x in a2],
                      len(a3[0]), *[_p(x) for x in a3], cfg["attr_cut"], cap,
                      _p(k), _p(s), _p(c), ctypes.byref(ovf))
    return {"key": k[:ng].copy(), "sum_qp": s[:ng].copy(), "count": c[:ng].copy(),
            "overflow": bool(ovf.value)}
