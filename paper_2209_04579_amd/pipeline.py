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

from . import (GB_DENSE, GB_SORTED, JOIN_SORTED, filter_into, filter_workspace_bytes,
               groupby_agg_into, groupby_workspace_bytes, join_into, join_workspace_bytes,
               pack_key_into, pay_bytes_of, sort_into, sort_workspace_bytes, tune_set,
               workspace)


def key_range(col: torch.Tensor):
    """Catalog statistics of an integer column: (min, bits of max - min)."""
    if col.numel() == 0:
        return 0, 0
    lo, hi = int(col.min().item()), int(col.max().item())
    return lo, int(hi - lo).bit_length()


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
                 tuning: dict | None = None):
        self.mode = mode
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
        self.cat_span = int(dim["cat"].max().item()) - self.cat_min + 1 if nd else 1
        if mode == "q2":
            self.flag_min, _ = key_range(fact["flag"])
            self.flag_span = int(fact["flag"].max().item()) - self.flag_min + 1 if n else 1
        # join key range covering both sides
        lo = min(self.fk_min, self.pk_min)
        hi = max(self.fk_min + (1 << self.fk_bits) - 1, self.pk_min + (1 << self.pk_bits) - 1)
        self.jk_min, self.jk_bits = lo, int(hi - lo).bit_length()

        pay = ["fk", "qty"] + (["price", "flag"] if mode == "q2" else [])
        self.pay_names = pay
        self.pay_in = [fact[k] for k in pay]
        self.pay_out = [torch.empty(max(n, 1), dtype=fact[k].dtype, device=dev) for k in pay]
        self.cnt = _i64(1, dev)
        self.ws_f = workspace(filter_workspace_bytes(n), dev)
        # sorts: the fact side carries its payload, the dim side its category
        self.fk_s = torch.empty(max(n, 1), dtype=fact["fk"].dtype, device=dev)
        self.fpay_s = [torch.empty(max(n, 1), dtype=t.dtype, device=dev) for t in self.pay_out[1:]]
        self.pk_s = torch.empty(max(nd, 1), dtype=dim["pk"].dtype, device=dev)
        self.cat_s = torch.empty(max(nd, 1), dtype=dim["cat"].dtype, device=dev)
        self.ws_s = workspace(max(sort_workspace_bytes(n, fact["fk"].dtype,
                                                       pay_bytes_of(self.fpay_s)),
                                  sort_workspace_bytes(nd, dim["pk"].dtype, 4)), dev)
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
        # group-bys
        self.gkey = _i64(self.cap, dev)
        if mode == "q1":
            self.ga_span = self.cat_span
            self.ga_lo = self.cat_min
            self.ga_aggs = [("sum", 0), ("count",)]
        else:
            self.ga_span = self.flag_span * 2
            self.ga_lo = self.flag_min * 2
            self.ga_aggs = [("sum", 0), ("sum", 1), ("count",)]
        dense = 0 < self.ga_span <= min(self.dense_max, 1024)
        self.ga_flags = GB_DENSE if dense else 0
        self.ga_key = _i64(max(self.ga_span, 1) if dense else self.cap, dev)
        self.ga_out = [_i64(self.ga_key.numel(), dev) for _ in self.ga_aggs]
        self.ga_ng = _i64(1, dev)
        self.ws_ga = workspace(groupby_workspace_bytes(self.cap, torch.int64, len(self.ga_aggs),
                                                       self.ga_flags, self.ga_span), dev)
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
        # 1. WHERE day < cut, carrying the payload columns
        filter_into([f["day"]], [(0, "<", self.cut)], self.pay_in, self.pay_out, None,
                    self.cnt, self.ws_f)
        # 2. sort both join sides (stable), payload moving with the keys
        sort_into(self.pay_out[0], None, self.n, self.fk_s, None, self.ws_s, d_n=self.cnt,
                  key_bits=self.jk_bits, key_min=self.jk_min, pay_in=self.pay_out[1:],
                  pay_out=self.fpay_s)
        sort_into(d["pk"], None, self.nd, self.pk_s, None, self.ws_s, key_bits=self.jk_bits,
                  key_min=self.jk_min, pay_in=[d["cat"]], pay_out=[self.cat_s])
        # 3. merge join of the sorted sides -> (left position, right position, key)
        join_into(self.fk_s, self.pk_s, JOIN_SORTED, self.out_l, self.out_r, self.out_k,
                  self.cap, self.npairs, self.ws_j, d_nl=self.cnt)
        # 4. group-bys over the joined rows
        qty_s = self.fpay_s[0]
        if self.mode == "q1":
            pack_key_into([(self.cat_s, self.out_r, 0, 1)], self.cap, self.gkey, d_n=self.npairs)
            vals = [qty_s]
        else:
            price_s, flag_s = self.fpay_s[1], self.fpay_s[2]
            pack_key_into([(flag_s, self.out_l, 0, 2), (self.cat_s, self.out_r, 2, 1)],
                          self.cap, self.gkey, d_n=self.npairs)
            vals = [qty_s, price_s]
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
