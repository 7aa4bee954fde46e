"""Many independent star queries of uneven sizes as one batched execution.

Layout.  The instances' tables are stored as one columnar arena: instance k's
fact rows follow instance k-1's, every join key carries its instance number in
its high bits (fk' = k << FB | fk, pk' = k << FB | pk), and every category is
offset past the categories of the instances before it (cat' = G_0 + ... +
G_{k-1} + cat, G_j = instance j's category count from catalog statistics).
Keys of different instances never compare equal, and keys of instance k sort
before those of k+1, so one filter -> sort -> merge join -> group-by over the
arena computes every instance's result at once, in instance order; the dense
category offsets keep the group key's range, and so its sort, small.  Each
operator is then a single persistent launch over all instances -- small
instances no longer pay a dozen launches each, and large ones no longer run
alone -- and the whole query is captured in one HIP graph and replayed with a
single launch.

(A single kernel walking (instance, phase, tile) items with per-instance
phase counters would need an agent-scope release/acquire -- an L2 write-back
and invalidate on the XCD -- at every phase hand-off; kernel boundaries give
that visibility once per phase instead.)
"""
from __future__ import annotations

import numpy as np
import torch

from . import pack_key_into
from .pipeline import StarQuery


def _bits(v: int) -> int:
    return max(1, int(v).bit_length())


class BatchStarQuery:
    """Q1 (WHERE day < cut, JOIN fk = pk, GROUP BY cat: SUM(qty), COUNT) over
    many instances.  instances: list of {"fact": {fk, qty, day}, "dim": {pk, cat}}
    with device tensors; all share day_cut."""

    def __init__(self, instances: list, day_cut: int, tuning: dict | None = None):
        self.k = len(instances)
        dev = instances[0]["fact"]["fk"].device
        self.dev = dev
        # catalog statistics: keys and categories must be non-negative, and
        # the prefix goes above the largest of them over all instances
        def cmax(t):
            if t.numel() == 0:
                return 0
            if int(t.min().item()) < 0:
                raise ValueError("batched keys and categories must be non-negative")
            return int(t.max().item())
        max_key = max(max(cmax(i["fact"]["fk"]), cmax(i["dim"]["pk"])) for i in instances)
        ncat = [cmax(i["dim"]["cat"]) + 1 for i in instances]
        self.fb = _bits(max_key)                       # bits of a join key
        self.cat_off = np.concatenate([[0], np.cumsum(ncat)]).astype(np.int64)
        if self.fb + _bits(self.k - 1) > 31 or int(self.cat_off[-1]) >= (1 << 31):
            raise ValueError("instance-prefixed keys do not fit int32")
        nf = [int(i["fact"]["fk"].numel()) for i in instances]
        nd = [int(i["dim"]["pk"].numel()) for i in instances]
        self.fact_off = np.concatenate([[0], np.cumsum(nf)]).astype(np.int64)
        self.dim_off = np.concatenate([[0], np.cumsum(nd)]).astype(np.int64)
        NF, ND = int(self.fact_off[-1]), int(self.dim_off[-1])
        fact = {"fk": torch.empty(NF, dtype=torch.int32, device=dev),
                "qty": torch.empty(NF, dtype=torch.int64, device=dev),
                "day": torch.empty(NF, dtype=torch.int32, device=dev)}
        dim = {"pk": torch.empty(ND, dtype=torch.int32, device=dev),
               "cat": torch.empty(ND, dtype=torch.int32, device=dev)}
        # ingestion into the arena: plain columns are copied, keys get their prefix
        for k, inst in enumerate(instances):
            f0, f1 = int(self.fact_off[k]), int(self.fact_off[k + 1])
            d0, d1 = int(self.dim_off[k]), int(self.dim_off[k + 1])
            fact["qty"][f0:f1].copy_(inst["fact"]["qty"])
            fact["day"][f0:f1].copy_(inst["fact"]["day"])
            if f1 > f0:
                pack_key_into([(inst["fact"]["fk"], None, 0, 1), (None, None, 0, k << self.fb)],
                              f1 - f0, fact["fk"][f0:f1])
            if d1 > d0:
                pack_key_into([(inst["dim"]["pk"], None, 0, 1), (None, None, 0, k << self.fb)],
                              d1 - d0, dim["pk"][d0:d1])
                pack_key_into([(inst["dim"]["cat"], None, 0, 1),
                               (None, None, 0, int(self.cat_off[k]))], d1 - d0, dim["cat"][d0:d1])
        self.fact, self.dim = fact, dim
        self.q = StarQuery(fact, dim, day_cut, mode="q1", tuning=tuning)
        self.graph = None

    def run(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self.q.run()

    def capture(self):
        """Captures the whole batched query into one HIP graph."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.q.run()                                # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.q.run()
        self.graph = g
        return g

    def results(self) -> list:
        """Per-instance {key, sum_qty, count} (host arrays), instance order."""
        r = self.q.result()
        out = []
        bounds = np.searchsorted(r["key"], self.cat_off)
        for k in range(self.k):
            a, b = bounds[k], bounds[k + 1]
            out.append({"key": r["key"][a:b] - self.cat_off[k], "sum_qty": r["sum_qty"][a:b],
                        "count": r["count"][a:b]})
        return out


class SequentialStarQueries:
    """The same instances as independent queries, launched one after another."""

    def __init__(self, instances: list, day_cut: int, tuning: dict | None = None):
        self.qs = [StarQuery(i["fact"], i["dim"], day_cut, mode="q1", tuning=tuning)
                   for i in instances]

    def run(self):
        for q in self.qs:
            q.run()

    def results(self) -> list:
        out = []
        for q in self.qs:
            r = q.result()
            out.append({"key": r["key"], "sum_qty": r["sum_qty"], "count": r["count"]})
        return out
