"""Filter -> sort -> sort-merge join -> group-by pipelines over device columns.

A plan allocates every buffer once for given table sizes; ``run()`` only
enqueues libtqp calls on the current stream (no host synchronization, counts
stay on the device), so the same plan can be timed or replayed; ``result()``
synchronizes and returns host arrays.

Key ranges come from catalog statistics (per-column min / max taken when a
table is loaded, outside any query), the way a database planner knows them:
they fix the radix pass count and the dense group-by domain, so no operator
has to read a range back from the device in the middle of a query.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (GB_DENSE, GB_SORTED, JOIN_SORTED, filter_into, filter_sum_into,
               filter_workspace_bytes, keyset_build_into, keyset_words, minmax,
               semijoin_into, semijoin_workspace_bytes,
               gather_into, groupby_agg_into, groupby_agg_terms_into,
               groupby_terms_workspace_bytes, groupby_workspace_bytes, join_into, join_workspace_bytes,
               mlp_predict_into,
               filter_sort_into, pack_key_into, pay_bytes_of, sort_into, sort_workspace_bytes,
               str_match_into,
               tune_set, workspace)


def col_stats(col: torch.Tensor):
    """Catalog statistics of an integer column: (min, max), or None when it
    is empty (libtqp's min / max reduction, read back once at plan time)."""
    return minmax(col) if col.numel() else None


def key_range(col: torch.Tensor):
    """Catalog statistics of an integer column: (min, bits of max - min)."""
    st = col_stats(col)
    if st is None:
        return 0, 0
    lo, hi = st
    return lo, int(hi - lo).bit_length()


def col_max(col: torch.Tensor, empty: int = 0) -> int:
    st = col_stats(col)
    return empty if st is None else st[1]


def _i64(n, dev):
    return torch.empty(max(int(n), 1), dtype=torch.int64, device=dev)


def _i32(n, dev):
    return torch.empty(max(int(n), 1), dtype=torch.int32, device=dev)


class StarQuery:
    """WHERE day < cut, JOIN fact.fk = dim.pk, then group-bys.

    mode "q1": GROUP BY dim.cat: SUM(qty), COUNT(*)
    mode "q2": (a) GROUP BY flag * 2 + (cat mod 2): SUM(qty), SUM(price), COUNT(*)
               (b) GROUP BY fk: SUM(qty), COUNT(*)
    """

    def __init__(self, fact: dict, dim: dict, day_cut: int, mode: str = "q1",
                 tuning: dict | None = None, overlap: bool = False, fused: bool = True):
        self.mode = mode
        # fused: WHERE and the fact side's sort are one operator
        # (filter_sort_into), so the filtered table is never written; else a
        # filter writes it and the sort reads it back
        self.fused = fused
        # library knobs (see tune_knobs()) applied before each run; the
        # "gb.dense_max" entry is the largest key domain aggregated directly
        self.tuning = dict(tuning or {})
        self.dense_max = int(self.tuning.pop("gb.dense_max", 1024))
        self.f = fact
        self.d = dim
        self.cut = int(day_cut)
        dev = fact["fk"].device
        self.dev = dev
        n, nd = fact["fk"].numel(), dim["pk"].numel()
        self.n, self.nd = n, nd
        # catalog statistics (taken once, outside the query)
        self.fk_min, self.fk_bits = key_range(fact["fk"])
        self.pk_min, self.pk_bits = key_range(dim["pk"])
        self.cat_min, cat_bits = key_range(dim["cat"])
        self.cat_span = col_max(dim["cat"]) - self.cat_min + 1 if nd else 1
        if mode == "q2":
            self.flag_min, _ = key_range(fact["flag"])
            self.flag_span = col_max(fact["flag"]) - self.flag_min + 1 if n else 1
        # join key range covering both sides
        lo = min(self.fk_min, self.pk_min)
        hi = max(self.fk_min + (1 << self.fk_bits) - 1, self.pk_min + (1 << self.pk_bits) - 1)
        self.jk_min, self.jk_bits = lo, int(hi - lo).bit_length()

        pay = ["fk", "qty"] + (["price", "flag"] if mode == "q2" else [])
        self.pay_names = pay
        self.pay_in = [fact[k] for k in pay]
        self.cnt = _i64(1, dev)
        if not fused:
            self.pay_out = [torch.empty(max(n, 1), dtype=fact[k].dtype, device=dev) for k in pay]
            self.ws_f = workspace(filter_workspace_bytes(n), dev)
        # sorts: the fact side carries its payload, the dim side its category
        self.fk_s = torch.empty(max(n, 1), dtype=fact["fk"].dtype, device=dev)
        self.fpay_s = [torch.empty(max(n, 1), dtype=t.dtype, device=dev) for t in self.pay_in[1:]]
        self.pk_s = torch.empty(max(nd, 1), dtype=dim["pk"].dtype, device=dev)
        self.cat_s = torch.empty(max(nd, 1), dtype=dim["cat"].dtype, device=dev)
        self.ws_s = workspace(max(sort_workspace_bytes(n, fact["fk"].dtype,
                                                       pay_bytes_of(self.fpay_s)),
                                  sort_workspace_bytes(nd, dim["pk"].dtype, 4)), dev)
        # overlap (opt-in): the dimension side's sort runs on a second stream
        # (default priority) beside the fact side's filter and sort, with its
        # own workspace; the join waits for both.  Off by default: the overlap
        # saves about 1% of the query but makes the dimension side's kernels
        # share the GPU with the filter, which inflates their measured times.
        self.side = torch.cuda.Stream(device=dev) if overlap else None
        self.ws_sd = (workspace(sort_workspace_bytes(nd, dim["pk"].dtype, 4), dev) if overlap
                      else self.ws_s)
        # join: pk is unique for these schemas, so pairs <= |filtered fact|;
        # the pair count is checked after the run.  Pairs are positions in
        # the sorted sides, so later reads of the sorted payload are sequential.
        self.cap = max(n, 1)
        self.out_l = _i32(self.cap, dev)
        self.out_r = _i32(self.cap, dev)
        self.out_k = torch.empty(self.cap, dtype=fact["fk"].dtype, device=dev)
        self.npairs = _i64(1, dev)
        self.ws_j = workspace(join_workspace_bytes(n, nd, fact["fk"].dtype, JOIN_SORTED,
                                                   self.cap), dev)
        # group-bys; the packed key is int32 when its catalog range fits
        if mode == "q1":
            self.ga_span = self.cat_span
            self.ga_lo = self.cat_min
            self.ga_aggs = [("sum", 0), ("count",)]
        else:
            self.ga_span = self.flag_span * 2
            self.ga_lo = self.flag_min * 2
            self.ga_aggs = [("sum", 0), ("sum", 1), ("count",)]
        fits32 = -(1 << 31) <= self.ga_lo and self.ga_lo + self.ga_span <= (1 << 31)
        kdt = torch.int32 if fits32 else torch.int64
        dense = 0 < self.ga_span <= min(self.dense_max, 1024)
        self.gkey = None if dense else torch.empty(self.cap, dtype=kdt, device=dev)
        self.ga_dense = dense
        self.ga_flags = GB_DENSE if dense else 0
        self.ga_key = torch.empty(max(self.ga_span, 1) if dense else self.cap, dtype=kdt,
                                  device=dev)
        self.ga_out = [_i64(self.ga_key.numel(), dev) for _ in self.ga_aggs]
        self.ga_ng = _i64(1, dev)
        # a dense domain aggregates over the packed key directly (never
        # written); otherwise the key is packed, then sorted by the group-by
        self.ws_ga = workspace(
            groupby_terms_workspace_bytes(len(self.ga_aggs), self.ga_span) if dense else
            groupby_workspace_bytes(self.cap, kdt, len(self.ga_aggs), self.ga_flags,
                                    self.ga_span), dev)
        if mode == "q2":
            self.gb_key = torch.empty(self.cap, dtype=fact["fk"].dtype, device=dev)
            self.gb_out = [_i64(self.cap, dev) for _ in range(2)]
            self.gb_ng = _i64(1, dev)
            self.ws_gb = workspace(groupby_workspace_bytes(self.cap, fact["fk"].dtype, 2,
                                                           GB_SORTED), dev)

    def run(self):
        for name, value in self.tuning.items():
            tune_set(name, value)
        f, d = self.f, self.d
        main = torch.cuda.current_stream(self.dev)

        def dim_sort():
            sort_into(d["pk"], None, self.nd, self.pk_s, None, self.ws_sd, key_bits=self.jk_bits,
                      key_min=self.jk_min, pay_in=[d["cat"]], pay_out=[self.cat_s])
        if self.side is not None:
            self.side.wait_stream(main)
            with torch.cuda.stream(self.side):
                dim_sort()
        # 1. WHERE day < cut, and 2. sort both join sides (stable), payload
        # moving with the keys
        if self.fused:
            filter_sort_into([f["day"]], [(0, "<", self.cut)], f["fk"], self.fk_s, None,
                             self.cnt, self.ws_s, key_bits=self.jk_bits, key_min=self.jk_min,
                             pay_in=self.pay_in[1:], pay_out=self.fpay_s)
        else:
            filter_into([f["day"]], [(0, "<", self.cut)], self.pay_in, self.pay_out, None,
                        self.cnt, self.ws_f)
            sort_into(self.pay_out[0], None, self.n, self.fk_s, None, self.ws_s, d_n=self.cnt,
                      key_bits=self.jk_bits, key_min=self.jk_min, pay_in=self.pay_out[1:],
                      pay_out=self.fpay_s)
        if self.side is not None:
            main.wait_stream(self.side)
        else:
            dim_sort()
        # 3. merge join of the sorted sides -> (left position, right position, key)
        join_into(self.fk_s, self.pk_s, JOIN_SORTED, self.out_l, self.out_r, self.out_k,
                  self.cap, self.npairs, self.ws_j, d_nl=self.cnt)
        # 4. group-bys over the joined rows
        qty_s = self.fpay_s[0]
        if self.mode == "q1":
            terms = [(self.cat_s, self.out_r, 0, 1)]
            vals = [qty_s]
        else:
            price_s, flag_s = self.fpay_s[1], self.fpay_s[2]
            terms = [(flag_s, self.out_l, 0, 2), (self.cat_s, self.out_r, 2, 1)]
            vals = [qty_s, price_s]
        if self.ga_dense:
            groupby_agg_terms_into(terms, self.cap, vals, self.ga_aggs, self.ga_key, self.ga_out,
                                   self.ga_ng, self.ws_ga, self.ga_lo, self.ga_span,
                                   val_rows=self.out_l, d_n=self.npairs)
        else:
            pack_key_into(terms, self.cap, self.gkey, d_n=self.npairs)
            groupby_agg_into(self.gkey[:self.cap], vals, self.ga_aggs, self.ga_key, self.ga_out,
                             self.ga_ng, self.ws_ga, flags=self.ga_flags, key_lo=self.ga_lo,
                             key_span=self.ga_span, val_rows=self.out_l, d_n=self.npairs)
        if self.mode == "q2":
            groupby_agg_into(self.out_k[:self.cap], [qty_s], [("sum", 0), ("count",)],
                             self.gb_key, self.gb_out, self.gb_ng, self.ws_gb, flags=GB_SORTED,
                             val_rows=self.out_l, d_n=self.npairs)

    def result(self) -> dict:
        torch.cuda.synchronize()
        npairs = int(self.npairs.item())
        if npairs > self.cap:
            raise RuntimeError(f"join produced {npairs} pairs, more than the {self.cap} planned")
        g = int(self.ga_ng.item())
        out = {"rows_filtered": int(self.cnt.item()), "pairs": npairs}
        key = self.ga_key[:g].cpu().numpy().astype(np.int64)
        if self.mode == "q1":
            out.update(key=key, sum_qty=self.ga_out[0][:g].cpu().numpy(),
                       count=self.ga_out[1][:g].cpu().numpy())
        else:
            out.update(a_key=key, a_qty=self.ga_out[0][:g].cpu().numpy(),
                       a_price=self.ga_out[1][:g].cpu().numpy(),
                       a_count=self.ga_out[2][:g].cpu().numpy())
            gb = int(self.gb_ng.item())
            out.update(b_key=self.gb_key[:gb].cpu().numpy().astype(np.int64),
                       b_qty=self.gb_out[0][:gb].cpu().numpy(),
                       b_count=self.gb_out[1][:gb].cpu().numpy())
        return out


class StarQuery3:
    """Star join over three filtered dimensions:

        WHERE d1.attr < cut AND d2.attr < cut AND d3.attr < cut
        JOIN fact.fk3 = d3.pk, fact.fk2 = d2.pk, fact.fk1 = d1.pk
        GROUP BY d1.cat * 5 + d2.cat: SUM(qty * price), COUNT(*)

    plan "semijoin" (default): each filtered dimension's keys become a key
    set (a bitmap over the dimension's key range), and one scan of the three
    foreign-key columns keeps the fact rows whose keys are in all three sets
    (the semi-join reduction: rows outside cannot join, so the inner joins'
    result is unchanged), carrying their keys.  The sort-merge joins then
    run on those rows only (about 0.8% of the fact table at 20% per
    dimension), in the order fk3 -> fk2 -> fk1, each sort carrying the row
    ids and the keys still to be joined; qty and price are read once, by the
    group-by, for the final rows.

    plan "sort": no reduction; all fact rows are sorted on the narrowest key
    fk3 (one radix pass, row ids out) and merged with d3, then the survivors'
    fk2 and fk1 are gathered from the fact table and sorted in turn.

    Dimension keys are unique (primary keys), so every join's pair count is
    at most its left side.
    """

    def __init__(self, fact: dict, d1: dict, d2: dict, d3: dict, attr_cut: int,
                 plan: str = "semijoin"):
        if plan not in ("semijoin", "sort"):
            raise ValueError("plan is 'semijoin' or 'sort'")
        self.plan = plan
        self.f, self.d1, self.d2, self.d3 = fact, d1, d2, d3
        self.cut = int(attr_cut)
        dev = fact["fk1"].device
        n = fact["fk1"].numel()
        self.n = n
        self.nd = [d1["pk"].numel(), d2["pk"].numel(), d3["pk"].numel()]
        dims = (d1, d2, d3)
        # catalog statistics: a join key range covering both sides of each
        # join, and each dimension's own key range (its key set's range)
        self.jk, self.pk_rng = [], []
        for fk, d in zip(("fk1", "fk2", "fk3"), dims):
            flo, fbits = key_range(fact[fk])
            plo, pbits = key_range(d["pk"])
            lo = min(flo, plo)
            hi = max(flo + (1 << fbits) - 1, plo + (1 << pbits) - 1)
            self.jk.append((lo, int(hi - lo).bit_length()))
            st = col_stats(d["pk"])
            self.pk_rng.append((0, 0) if st is None else (st[0], st[1] - st[0] + 1))
        self.cat_lo = [key_range(d1["cat"])[0], key_range(d2["cat"])[0]]
        c1_hi = col_max(d1["cat"])
        c2_hi = col_max(d2["cat"])
        if self.nd[0] and self.nd[1] and (self.cat_lo[0] < 0 or self.cat_lo[1] < 0 or c2_hi >= 5):
            raise ValueError("expects d1.cat >= 0 and d2.cat in [0, 5)")
        self.g_span = max(c1_hi * 5 + c2_hi + 1, 1)
        self.g_dense = self.g_span <= 1024

        # filtered, pk-sorted dimensions (category carried)
        self.dcnt = [_i64(1, dev) for _ in range(3)]
        self.dpk = [_i32(m, dev) for m in self.nd]
        self.dcat = [_i32(self.nd[0], dev), _i32(self.nd[1], dev)]
        self.dpk_s = [_i32(m, dev) for m in self.nd]
        self.dcat_s = [_i32(self.nd[0], dev), _i32(self.nd[1], dev)]
        self.ws_f = workspace(filter_workspace_bytes(max(self.nd + [1])), dev)
        ws_sort = max(sort_workspace_bytes(max(m, 1), torch.int32, 4) for m in self.nd)
        # fact side, every buffer at the fact table's size (the plan makes no
        # assumption about selectivity)
        self.fk_s = _i32(n, dev)
        self.rows_s = _i32(n, dev)
        ws_sort = max(ws_sort, sort_workspace_bytes(max(n, 1), torch.int32, 8))
        self.ws_s = workspace(ws_sort, dev)
        self.cnt = [_i64(1, dev) for _ in range(3)]        # pairs after each join
        self.r = [_i32(n, dev) for _ in range(3)]          # fact row ids after each join
        self.rpos = _i32(n, dev)                           # dim positions of the last join
        self.jpos = _i32(n, dev)
        self.key_g = _i32(n, dev)                          # next join key of the survivors
        self.c2 = _i32(n, dev)                             # d2.cat per survivor
        self.c2_s = _i32(n, dev)
        if plan == "semijoin":
            self.bits = [torch.empty(max(keyset_words(nb), 1), dtype=torch.int32, device=dev)
                         for _, nb in self.pk_rng]
            self.sj_cnt = _i64(1, dev)
            self.sj_rows = _i32(n, dev)
            self.sj_keys = [_i32(n, dev) for _ in range(3)]   # fk1, fk2, fk3 of kept rows
            self.ws_sj = workspace(semijoin_workspace_bytes(n, torch.int32), dev)
            self.k_s = [_i32(n, dev) for _ in range(2)]      # keys carried by the sorts
            self.k_g = _i32(n, dev)
        ws_j = max(join_workspace_bytes(n, max(m, 1), torch.int32, JOIN_SORTED, max(n, 1))
                   for m in self.nd)
        self.ws_j = workspace(ws_j, dev)
        self.aggs = [("sum_product", 0, 1), ("count",)]
        gflags = GB_DENSE if self.g_dense else 0
        self.g_flags = gflags
        self.gkey = None if self.g_dense else _i64(n, dev)
        self.g_key = _i64(self.g_span if self.g_dense else n, dev)
        self.g_out = [_i64(self.g_key.numel(), dev) for _ in self.aggs]
        self.g_ng = _i64(1, dev)
        self.ws_g = workspace(groupby_terms_workspace_bytes(2, self.g_span) if self.g_dense else
                              groupby_workspace_bytes(max(n, 1), torch.int64, 2, gflags,
                                                      self.g_span), dev)

    def _dims(self):
        """Filter each dimension, sort it by pk carrying its category; with
        the semi-join plan, also its key set."""
        for i, d in enumerate((self.d1, self.d2, self.d3)):
            pay_in = [d["pk"]] + ([d["cat"]] if i < 2 else [])
            pay_out = [self.dpk[i]] + ([self.dcat[i]] if i < 2 else [])
            filter_into([d["attr"]], [(0, "<", self.cut)], pay_in, pay_out, None, self.dcnt[i],
                        self.ws_f)
            lo, bits = self.jk[i]
            sort_into(self.dpk[i], None, self.nd[i], self.dpk_s[i], None, self.ws_s,
                      d_n=self.dcnt[i], key_bits=bits, key_min=lo,
                      pay_in=pay_out[1:], pay_out=[self.dcat_s[i]] if i < 2 else [])
            if self.plan == "semijoin":
                plo, pn = self.pk_rng[i]
                keyset_build_into(self.dpk[i], plo, pn, self.bits[i], d_n=self.dcnt[i])

    def _group(self, n):
        # GROUP BY d1.cat * 5 + d2.cat: SUM(qty * price), COUNT(*); the final
        # fact rows are r[2], their d1 positions rpos, their d2.cat c2_s[jpos]
        f = self.f
        terms = [(self.dcat_s[0], self.rpos, 0, 5), (self.c2_s, self.jpos, 0, 1)]
        if self.g_dense:
            groupby_agg_terms_into(terms, n, [f["qty"], f["price"]], self.aggs, self.g_key,
                                   self.g_out, self.g_ng, self.ws_g, 0, self.g_span,
                                   val_rows=self.r[2], d_n=self.cnt[2])
        else:
            pack_key_into(terms, n, self.gkey, d_n=self.cnt[2])
            groupby_agg_into(self.gkey[:n], [f["qty"], f["price"]], self.aggs, self.g_key,
                             self.g_out, self.g_ng, self.ws_g, flags=self.g_flags, key_lo=0,
                             key_span=self.g_span, val_rows=self.r[2], d_n=self.cnt[2])

    def run(self):
        self._dims()
        if self.plan == "semijoin":
            self._run_semijoin()
        else:
            self._run_sort()

    def _run_semijoin(self):
        f, n = self.f, self.n
        # 1. semi-join reduction: rows whose fk1, fk2, fk3 are all in the
        # filtered dimensions, with their three keys
        semijoin_into([f["fk1"], f["fk2"], f["fk3"]],
                      [(b, lo, nb) for b, (lo, nb) in zip(self.bits, self.pk_rng)],
                      self.sj_rows, self.sj_cnt, self.ws_sj, keys_out=self.sj_keys)
        k1, k2, k3 = self.sj_keys
        # 2. fk3: sort carrying row ids, fk2 and fk1; merge with d3
        lo, bits = self.jk[2]
        sort_into(k3, self.sj_rows, n, self.fk_s, self.rows_s, self.ws_s, d_n=self.sj_cnt,
                  key_bits=bits, key_min=lo, pay_in=[k2, k1], pay_out=self.k_s)
        join_into(self.fk_s, self.dpk_s[2], JOIN_SORTED, self.jpos, None, None, n, self.cnt[0],
                  self.ws_j, d_nl=self.sj_cnt, d_nr=self.dcnt[2])
        gather_into(self.rows_s, self.jpos, n, self.r[0], d_n=self.cnt[0])
        gather_into(self.k_s[0], self.jpos, n, self.key_g, d_n=self.cnt[0])
        gather_into(self.k_s[1], self.jpos, n, self.k_g, d_n=self.cnt[0])
        # 3. fk2: sort carrying row ids and fk1; merge with d2 (d2.cat out)
        lo, bits = self.jk[1]
        sort_into(self.key_g, self.r[0], n, self.fk_s, self.rows_s, self.ws_s, d_n=self.cnt[0],
                  key_bits=bits, key_min=lo, pay_in=[self.k_g], pay_out=[self.k_s[0]])
        join_into(self.fk_s, self.dpk_s[1], JOIN_SORTED, self.jpos, self.rpos, None, n,
                  self.cnt[1], self.ws_j, d_nl=self.cnt[0], d_nr=self.dcnt[1])
        gather_into(self.dcat_s[1], self.rpos, n, self.c2, d_n=self.cnt[1])
        gather_into(self.rows_s, self.jpos, n, self.r[1], d_n=self.cnt[1])
        gather_into(self.k_s[0], self.jpos, n, self.key_g, d_n=self.cnt[1])
        # 4. fk1: sort carrying row ids and d2.cat; merge with d1
        lo, bits = self.jk[0]
        sort_into(self.key_g, self.r[1], n, self.fk_s, self.rows_s, self.ws_s, d_n=self.cnt[1],
                  key_bits=bits, key_min=lo, pay_in=[self.c2], pay_out=[self.c2_s])
        join_into(self.fk_s, self.dpk_s[0], JOIN_SORTED, self.jpos, self.rpos, None, n,
                  self.cnt[2], self.ws_j, d_nl=self.cnt[1], d_nr=self.dcnt[0])
        gather_into(self.rows_s, self.jpos, n, self.r[2], d_n=self.cnt[2])
        self._group(n)

    def _run_sort(self):
        f, n = self.f, self.n
        # 2. fk3: sort all fact rows (row ids out), merge with d3 -> fact rows r0
        lo, bits = self.jk[2]
        sort_into(f["fk3"], None, n, self.fk_s, self.rows_s, self.ws_s, key_bits=bits,
                  key_min=lo)
        join_into(self.fk_s, self.dpk_s[2], JOIN_SORTED, self.r[0], None, None, n, self.cnt[0],
                  self.ws_j, lrows=self.rows_s, d_nr=self.dcnt[2])
        # 3. fk2 of the survivors: sort carrying their row ids, merge with d2
        gather_into(f["fk2"], self.r[0], n, self.key_g, d_n=self.cnt[0])
        lo, bits = self.jk[1]
        sort_into(self.key_g, self.r[0], n, self.fk_s, self.rows_s, self.ws_s, d_n=self.cnt[0],
                  key_bits=bits, key_min=lo)
        join_into(self.fk_s, self.dpk_s[1], JOIN_SORTED, self.r[1], self.rpos, None, n,
                  self.cnt[1], self.ws_j, lrows=self.rows_s, d_nl=self.cnt[0],
                  d_nr=self.dcnt[1])
        gather_into(self.dcat_s[1], self.rpos, n, self.c2, d_n=self.cnt[1])
        # 4. fk1 of the survivors: sort carrying row ids and d2.cat, merge with d1
        gather_into(f["fk1"], self.r[1], n, self.key_g, d_n=self.cnt[1])
        lo, bits = self.jk[0]
        sort_into(self.key_g, self.r[1], n, self.fk_s, self.rows_s, self.ws_s, d_n=self.cnt[1],
                  key_bits=bits, key_min=lo, pay_in=[self.c2], pay_out=[self.c2_s])
        join_into(self.fk_s, self.dpk_s[0], JOIN_SORTED, self.jpos, self.rpos, None, n,
                  self.cnt[2], self.ws_j, d_nl=self.cnt[1], d_nr=self.dcnt[0])
        gather_into(self.rows_s, self.jpos, n, self.r[2], d_n=self.cnt[2])
        self._group(n)

    def result(self) -> dict:
        torch.cuda.synchronize()
        pairs = [int(c.item()) for c in self.cnt]
        if max(pairs) > self.n:
            raise RuntimeError(f"join produced {max(pairs)} pairs, more than the {self.n} planned")
        g = int(self.g_ng.item())
        out = {"dims_kept": [int(c.item()) for c in self.dcnt], "pairs": pairs,
               "key": self.g_key[:g].cpu().numpy().astype(np.int64),
               "sum_qp": self.g_out[0][:g].cpu().numpy(),
               "count": self.g_out[1][:g].cpu().numpy()}
        if self.plan == "semijoin":
            out["reduced"] = int(self.sj_cnt.item())
        return out


class Q6Scan:
    """The Q6-shaped scan (Section 2.3: filters over columns of different
    types feeding one aggregate):

        SELECT SUM(price * discount), COUNT(*) FROM items
        WHERE ship >= ship_lo AND ship < ship_hi
          AND discount >= disc_lo AND discount <= disc_hi AND quantity < qty_cut

    ship is int64 epoch nanoseconds, discount int8 hundredths, quantity int32,
    price int64 cents.  One fused launch; nothing is compacted.
    """

    def __init__(self, items: dict, bounds: dict):
        self.cols = [items["ship"], items["discount"], items["quantity"]]
        self.price = items["price"]
        self.n = items["ship"].numel()
        self.preds = [(0, ">=", bounds["ship_lo"]), (0, "<", bounds["ship_hi"]),
                      (1, ">=", bounds["disc_lo"]), (1, "<=", bounds["disc_hi"]),
                      (2, "<", bounds["qty_cut"])]
        dev = self.price.device
        self.d_sum = torch.empty(1, dtype=torch.int64, device=dev)
        self.d_count = torch.empty(1, dtype=torch.int64, device=dev)

    def run(self):
        filter_sum_into(self.cols, self.preds, self.d_sum, self.d_count, self.price, self.cols[1])

    def result(self) -> dict:
        torch.cuda.synchronize()
        return {"sum": int(self.d_sum.item()), "count": int(self.d_count.item())}


class Q14Query:
    """Q14-shaped join with a string predicate (Section 2.3: Q14 joins the
    items with the parts and aggregates a CASE over a LIKE on a string):

        SELECT SUM(CASE WHEN type LIKE 'prefix%' THEN price * (100 - discount)
                   ELSE 0 END), SUM(price * (100 - discount)), COUNT(*)
        FROM items JOIN part ON partkey = pk
        WHERE ship >= ship_lo AND ship < ship_hi

    Plan: filter the month carrying partkey, price and discount; the LIKE over
    the part types (an (n, m) byte matrix) gives a 0/1 flag column; sort both
    join sides (the part side carrying the flag); merge join; then two
    aggregations of price * (100 - discount) and COUNT over the joined rows,
    one grouped by the flag (the CASE: the group of flag 1) and one over all
    rows (a single group), both exact in int64 on the device.
    """

    AGGS = [("sum_diff_product", 0, 1, 100), ("count",)]

    def __init__(self, items: dict, part: dict, prefix: bytes, ship_lo: int, ship_hi: int):
        self.items, self.part = items, part
        self.prefix = bytes(prefix)
        self.preds = [(0, ">=", int(ship_lo)), (0, "<", int(ship_hi))]
        dev = items["ship"].device
        n, npart = items["ship"].numel(), part["pk"].numel()
        self.n, self.npart = n, npart
        # catalog statistics of the join key (taken once, outside the query)
        st = [col_stats(items["partkey"]) or (0, 0), col_stats(part["pk"]) or (0, 0)]
        lo, hi = min(st[0][0], st[1][0]), max(st[0][1], st[1][1])
        self.jk_min, self.jk_bits = lo, int(hi - lo).bit_length()
        self.pay_in = [items["partkey"], items["price"], items["discount"]]
        self.pay_out = [torch.empty(max(n, 1), dtype=t.dtype, device=dev) for t in self.pay_in]
        self.cnt = _i64(1, dev)
        self.ws_f = workspace(filter_workspace_bytes(n), dev)
        self.flag = torch.empty(max(npart, 1), dtype=torch.int8, device=dev)
        self.fk_s = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        self.fpay_s = [torch.empty(max(n, 1), dtype=t.dtype, device=dev) for t in self.pay_out[1:]]
        self.pk_s = torch.empty(max(npart, 1), dtype=torch.int32, device=dev)
        self.flag_s = torch.empty(max(npart, 1), dtype=torch.int8, device=dev)
        self.ws_s = workspace(sort_workspace_bytes(n, torch.int32, pay_bytes_of(self.fpay_s)), dev)
        # the part side (string match and its sort) runs on a second stream
        # beside the items' filter and sort; the join waits for both
        self.side = torch.cuda.Stream(device=dev)
        self.ws_sp = workspace(sort_workspace_bytes(npart, torch.int32, 1), dev)
        self.cap = max(n, 1)
        self.out_l = _i32(self.cap, dev)
        self.out_r = _i32(self.cap, dev)
        self.out_k = torch.empty(self.cap, dtype=torch.int32, device=dev)
        self.npairs = _i64(1, dev)
        self.ws_j = workspace(join_workspace_bytes(n, npart, torch.int32, JOIN_SORTED, self.cap), dev)
        # by flag (2 groups) and over all rows (1 group)
        self.g_key = torch.empty(2, dtype=torch.int32, device=dev)
        self.g_out = [_i64(2, dev) for _ in self.AGGS]
        self.g_ng = _i64(1, dev)
        self.t_key = torch.empty(1, dtype=torch.int32, device=dev)
        self.t_out = [_i64(1, dev) for _ in self.AGGS]
        self.t_ng = _i64(1, dev)
        self.ws_g = workspace(groupby_terms_workspace_bytes(len(self.AGGS), 2), dev)

    def run(self):
        it, pt = self.items, self.part
        main = torch.cuda.current_stream(self.items["ship"].device)
        self.side.wait_stream(main)
        with torch.cuda.stream(self.side):
            str_match_into(pt["type"], self.prefix, self.flag)
            sort_into(pt["pk"], None, self.npart, self.pk_s, None, self.ws_sp,
                      key_bits=self.jk_bits, key_min=self.jk_min, pay_in=[self.flag],
                      pay_out=[self.flag_s])
        filter_into([it["ship"]], self.preds, self.pay_in, self.pay_out, None, self.cnt, self.ws_f)
        sort_into(self.pay_out[0], None, self.n, self.fk_s, None, self.ws_s, d_n=self.cnt,
                  key_bits=self.jk_bits, key_min=self.jk_min, pay_in=self.pay_out[1:],
                  pay_out=self.fpay_s)
        main.wait_stream(self.side)
        join_into(self.fk_s, self.pk_s, JOIN_SORTED, self.out_l, self.out_r, self.out_k,
                  self.cap, self.npairs, self.ws_j, d_nl=self.cnt)
        groupby_agg_terms_into([(self.flag_s, self.out_r, 0, 1)], self.cap, self.fpay_s,
                               self.AGGS, self.g_key, self.g_out, self.g_ng, self.ws_g, 0, 2,
                               val_rows=self.out_l, d_n=self.npairs)
        groupby_agg_terms_into([(None, None, 0, 0)], self.cap, self.fpay_s, self.AGGS,
                               self.t_key, self.t_out, self.t_ng, self.ws_g, 0, 1,
                               val_rows=self.out_l, d_n=self.npairs)

    def result(self) -> dict:
        torch.cuda.synchronize()
        npairs = int(self.npairs.item())
        if npairs > self.cap:
            raise RuntimeError(f"join produced {npairs} pairs, more than the {self.cap} planned")
        g = int(self.g_ng.item())
        keys = self.g_key[:g].cpu().tolist()
        rev, cnt = (o[:g].cpu().tolist() for o in self.g_out)
        promo = keys.index(1) if 1 in keys else None
        t = int(self.t_ng.item())
        return {"rows_filtered": int(self.cnt.item()), "pairs": npairs,
                "promo_rev": rev[promo] if promo is not None else 0,
                "total_rev": int(self.t_out[0][0].item()) if t else 0,
                "count": int(self.t_out[1][0].item()) if t else 0,
                "promo_count": cnt[promo] if promo is not None else 0}


class PredictQuery:
    """PREDICT inside a query (Section 3.3's prediction query):

        SELECT rating, SUM(CASE WHEN PREDICT(model, f0..) = 1 THEN 1 ELSE 0 END), COUNT(*)
        FROM reviews WHERE year >= year_min GROUP BY rating

    Plan: filter the years carrying the rating and the kept row ids; score
    the kept rows (features read through the row ids) with a two-class
    model, whose class is 0 or 1, so the CASE is the class itself; group by
    rating (a dense domain) with SUM(class) and COUNT.
    """

    def __init__(self, reviews: dict, model, nfeat: int, hidden: int, classes: int,
                 year_min: int, nratings: int):
        if classes != 2:
            raise ValueError("the prediction query's CASE over the class needs a two-class model")
        dev = reviews["rating"].device
        n = reviews["rating"].numel()
        self.n, self.hidden, self.classes, self.nratings = n, hidden, classes, nratings
        self.year, self.rating = reviews["year"], reviews["rating"]
        self.feats = [reviews[f"f{k}"] for k in range(nfeat)]
        self.model = torch.as_tensor(model, dtype=torch.float32).to(dev).contiguous()
        self.preds = [(0, ">=", int(year_min))]
        self.rows = _i32(n, dev)
        self.rating_f = torch.empty(max(n, 1), dtype=torch.int8, device=dev)
        self.cnt = _i64(1, dev)
        self.ws_f = workspace(filter_workspace_bytes(n), dev)
        self.cls = torch.empty(max(n, 1), dtype=torch.int8, device=dev)
        self.span = nratings
        self.g_key = torch.empty(self.span, dtype=torch.int32, device=dev)
        self.g_out = [_i64(self.span, dev) for _ in range(2)]
        self.g_ng = _i64(1, dev)
        self.ws_g = workspace(groupby_terms_workspace_bytes(2, self.span), dev)

    def run(self):
        filter_into([self.year], self.preds, [self.rating], [self.rating_f], self.rows, self.cnt,
                    self.ws_f)
        mlp_predict_into(self.feats, self.model, self.hidden, self.classes, self.cls, n=self.n,
                         rows=self.rows, d_n=self.cnt)
        groupby_agg_terms_into([(self.rating_f, None, 0, 1)], self.n, [self.cls],
                               [("sum", 0), ("count",)], self.g_key, self.g_out, self.g_ng,
                               self.ws_g, 0, self.span, d_n=self.cnt)

    def result(self) -> dict:
        torch.cuda.synchronize()
        g = int(self.g_ng.item())
        pos = np.zeros(self.nratings, np.int64)
        cnt = np.zeros(self.nratings, np.int64)
        keys = self.g_key[:g].cpu().numpy()
        pos[keys] = self.g_out[0][:g].cpu().numpy()
        cnt[keys] = self.g_out[1][:g].cpu().numpy()
        return {"rows_filtered": int(self.cnt.item()), "positive": pos, "count": cnt}
