"""Many independent star queries of uneven sizes as one batched execution.

Layout (libtqp's tqp_batch_plan).  The instances' tables are stored as one
columnar arena: instance k's fact rows follow instance k-1's, every join key
carries its instance number in its high bits (fk' = k << FB | fk,
pk' = k << FB | pk) and every category likewise (cat' = k << CB | cat).  Keys
of different instances never compare equal, and keys of instance k sort
before those of k+1, so one filter -> sort -> merge join -> group-by over the
arena computes every instance's result at once, in instance order.  Each
operator is then a single persistent launch over all instances -- small
instances no longer pay a dozen launches each, and large ones no longer run
alone -- and the whole query is captured in one HIP graph (tqp_batch_capture)
and replayed with a single launch (tqp_batch_run).  The result is split back
on the device: tqp_lower_bound finds where each instance's groups start and
the category is the group key modulo 2^CB.

(This is one launch per operator over all instances, inside one graph, not
one kernel for the whole query: a single kernel walking (instance, phase,
tile) items would need an agent-scope release/acquire -- an L2 write-back and
invalidate on the XCD -- at every phase hand-off, which kernel boundaries
give once per phase.)
"""
from __future__ import annotations

import numpy as np
import torch

from . import batch_capture, batch_plan, lower_bound_into, minmax, pack_key_into
from .pipeline import StarQuery


class BatchStarQuery:
    """Q1 (WHERE day < cut, JOIN fk = pk, GROUP BY cat: SUM(qty), COUNT) over
    many instances.  instances: list of {"fact": {fk, qty, day}, "dim": {pk, cat}}
    with device tensors; all share day_cut."""

    def __init__(self, instances: list, day_cut: int, tuning: dict | None = None):
        self.k = len(instances)
        dev = instances[0]["fact"]["fk"].device
        self.dev = dev
        # catalog statistics: keys and categories must be non-negative (the
        # plan checks), the prefix goes above the largest of them
        def stats(t):
            st = minmax(t) if t.numel() else None
            return (0, 0) if st is None else st
        keys = [stats(i["fact"]["fk"]) for i in instances] + \
               [stats(i["dim"]["pk"]) for i in instances]
        cats = [stats(i["dim"]["cat"]) for i in instances]
        if min(k[0] for k in keys + cats) < 0:
            raise ValueError("batched keys and categories must be non-negative")
        lay = batch_plan([int(i["fact"]["fk"].numel()) for i in instances],
                         [int(i["dim"]["pk"].numel()) for i in instances],
                         max(k[1] for k in keys), max(c[1] for c in cats))
        self.layout = lay
        fo, do = lay["fact_off"], lay["dim_off"]
        NF, ND = lay["fact_rows"], lay["dim_rows"]
        fb, cb = lay["key_shift"], lay["cat_shift"]
        fact = {"fk": torch.empty(NF, dtype=torch.int32, device=dev),
                "qty": torch.empty(NF, dtype=torch.int64, device=dev),
                "day": torch.empty(NF, dtype=torch.int32, device=dev)}
        dim = {"pk": torch.empty(ND, dtype=torch.int32, device=dev),
               "cat": torch.empty(ND, dtype=torch.int32, device=dev)}
        # ingestion into the arena: plain columns are copied, keys get their prefix
        for k, inst in enumerate(instances):
            f0, f1, d0, d1 = fo[k], fo[k + 1], do[k], do[k + 1]
            fact["qty"][f0:f1].copy_(inst["fact"]["qty"])
            fact["day"][f0:f1].copy_(inst["fact"]["day"])
            if f1 > f0:
                pack_key_into([(inst["fact"]["fk"], None, 0, 1), (None, None, 0, k << fb)],
                              f1 - f0, fact["fk"][f0:f1])
            if d1 > d0:
                pack_key_into([(inst["dim"]["pk"], None, 0, 1), (None, None, 0, k << fb)],
                              d1 - d0, dim["pk"][d0:d1])
                pack_key_into([(inst["dim"]["cat"], None, 0, 1), (None, None, 0, k << cb)],
                              d1 - d0, dim["cat"][d0:d1])
        self.fact, self.dim = fact, dim
        self.q = StarQuery(fact, dim, day_cut, mode="q1", tuning=tuning)
        self.graph = None
        # where each instance's groups start: the first group key >= k << CB
        self.bound_q = torch.tensor([k << cb for k in range(self.k + 1)], dtype=torch.int64,
                                    device=dev)
        self.bounds = torch.empty(self.k + 1, dtype=torch.int64, device=dev)
        self.local_key = torch.empty(self.q.ga_key.numel(), dtype=torch.int64, device=dev)

    def run(self):
        if self.graph is not None:
            self.graph.run()
        else:
            self.q.run()

    def capture(self):
        """Captures the whole batched query into one graph (libtqp)."""
        self.q.run()                       # warm-up (and tuning knobs applied) outside the capture
        torch.cuda.synchronize()
        self.graph = batch_capture(self.q.run)
        return self.graph

    def results(self) -> list:
        """Per-instance {key, sum_qty, count} (host arrays), instance order."""
        q = self.q
        lower_bound_into(q.ga_key, self.bound_q, self.bounds, d_n=q.ga_ng)
        pack_key_into([(q.ga_key, None, 1 << self.layout["cat_shift"], 1)], q.ga_key.numel(),
                      self.local_key, d_n=q.ga_ng)
        r = q.result()
        g = len(r["key"])
        bounds = self.bounds.cpu().tolist()
        key = self.local_key[:g].cpu().numpy()
        return [{"key": key[a:b], "sum_qty": r["sum_qty"][a:b], "count": r["count"][a:b]}
                for a, b in zip(bounds[:-1], bounds[1:])]


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
