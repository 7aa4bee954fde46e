#!/usr/bin/env python3
"""Benchmark: rows/s of the filter -> sort -> join -> group-by pipeline on the
skewed star-schema workload, with the dominant kernel's HBM roofline and the
CPU oracle timed beside it.

Workload (one step = one whole query over one batch of resident input):
  fact 60M rows {fk int32 Zipf s=1 over 2M keys, qty int64 [1,5000] cents,
  price int64 [100,1e7] cents, flag int8 [0,3), day int32 [0,2557)},
  dim 2M rows {pk = permutation, cat int32 [0,25)};
  WHERE day < 1278, JOIN fk = pk,
  GROUP BY (flag, cat mod 2): SUM(qty), SUM(price), COUNT;  GROUP BY fk: SUM(qty), COUNT.

Prints one JSON line.  Only one GPU is used.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
METRIC = "rows/s filter→join→group-by, % peak HBM GB/s; learned vs radix partition"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n-fact", type=int, default=60_000_000)
    ap.add_argument("--n-dim", type=int, default=2_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the steps without per-kernel events")
    return ap.parse_args()


def kernel_bytes(name: str, launches: int, st: dict) -> float | None:
    """Algorithmic HBM bytes of all launches of one kernel in one step.

    Each kernel's bytes are its per-element figure times the elements its
    launches process (the figures are stated in the design notes)."""
    n, kept, nd, pairs = st["n"], st["kept"], st["nd"], st["pairs"]
    ul, ur, gb = st["uniq_l"], st["uniq_r"], st["groups_b"]
    if name == "filter":
        return n * (4 + 4 + 8 + 8 + 1) + kept * (4 + 8 + 8 + 1)
    if name == "radix_hist":
        return 4.0 * (kept + nd)
    if name == "onesweep":
        # every pass reads and writes each element once: the fact side moves
        # fk (4) + qty (8) + price (8) + flag (1), the dim side pk (4) + cat (4)
        p = st["passes"]
        return p * (kept * 2.0 * 21 + nd * 2.0 * 8)
    if name == "rle":
        return 4.0 * (kept + nd) + 8.0 * (ul + ur)
    if name == "join_match":
        return ul * (4 + 4 + 4 + 4 + 6 * 8)
    if name == "join_expand":
        return pairs * (4 + 4 + 4) + ul * 6 * 8
    if name == "pack_key":
        return pairs * (4 + 4 + 1 + 4 + 8)
    if name in ("gb_dense", "gb_tiny"):
        return pairs * (8 + 4 + 8 + 8)
    if name == "gb_scan":
        return pairs * (4 + 4 + 8) + gb * (4 + 16)
    if name == "gb_diff":
        return gb * 32.0
    return None


def source_sha(kernel_file: str) -> str:
    h = hashlib.sha256()
    for f in (kernel_file, "tqp_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2209_04579_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_FILE = {"filter": "filter.hip", "onesweep": "sort.hip", "radix_hist": "sort.hip",
               "rle": "join.hip", "join_match": "join.hip", "join_expand": "join.hip",
               "pack_key": "gather.hip", "gb_dense": "groupby.hip", "gb_scan": "groupby.hip",
               "gb_tiny": "groupby.hip",
               "gb_diff": "groupby.hip"}


def traffic_for(kernel: str):
    """Counter-measured HBM bytes per launch, if a profile of the current source exists."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_star60m_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha") != source_sha(KERNEL_FILE[kernel]):
        return None
    return t.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import tqp_datagen as dg
    import paper_2209_04579_amd as tqp
    from paper_2209_04579_amd.pipeline import StarQuery

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tqp.lib()
    t0 = time.time()
    cfg = dg.config2(args.seed, n_fact=args.n_fact, n_dim=args.n_dim)
    print(f"[bench] generated {args.n_fact} fact rows in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    fact = {k: torch.from_numpy(v).cuda() for k, v in cfg["fact"].items()}
    dim = {k: torch.from_numpy(v).cuda() for k, v in cfg["dim"].items()}
    q = StarQuery(fact, dim, cfg["day_cut"], mode="q2")
    stream = torch.cuda.current_stream()

    # plain-copy bandwidth on the same run (2 GiB), the scale for the HBM counters
    src = torch.empty(1 << 31, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    for _ in range(args.warmup):
        q.run()
    res = q.result()
    print(f"[bench] warmup done: {res['rows_filtered']} rows kept, {res['pairs']} pairs, "
          f"{len(res['b_key'])} fk groups", file=sys.stderr, flush=True)

    use_events = not args.no_kernel_events
    tqp.profile_reset()
    tqp.profile_enable(use_events)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        q.run()
    e1.record(stream)
    torch.cuda.synchronize()
    tqp.profile_enable(False)
    ms = e0.elapsed_time(e1) / args.steps
    prof = tqp.profile_collect() if use_events else {}
    tqp.profile_reset()

    st = {"n": args.n_fact, "nd": args.n_dim, "kept": res["rows_filtered"],
          "pairs": res["pairs"], "groups_b": len(res["b_key"]),
          "passes": (q.jk_bits + 7) // 8}
    # distinct keys on each join side (for the per-kernel byte figures)
    st["uniq_l"] = len(res["b_key"])
    st["uniq_r"] = args.n_dim
    kernels = {}
    for name, (cnt, tot_ms) in prof.items():
        per_step = cnt / args.steps
        avg_ms = tot_ms / cnt
        b = kernel_bytes(name, per_step, st)
        kernels[name] = {"launches_per_step": per_step, "avg_ms": round(avg_ms, 5),
                         "ms_per_step": round(tot_ms / args.steps, 5)}
        if b is not None:
            kernels[name]["algo_GBps"] = round(b / (tot_ms / args.steps * 1e-3) / 1e9, 1)
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
        d = kernels[dom]
        b_step = kernel_bytes(dom, d["launches_per_step"], st)
        per_launch = b_step / d["launches_per_step"]
        achieved = per_launch / (d["avg_ms"] * 1e-3) / 1e9
        roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic_for(dom),
                    "algo_bytes_per_launch": int(per_launch),
                    "avg_launch_ms": d["avg_ms"]}

    # algorithmic bytes of the whole step, from the per-kernel figures
    step_bytes = sum(kernel_bytes(k, kernels[k]["launches_per_step"], st) or 0 for k in kernels)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.lib()
        t0 = time.perf_counter()
        want = oracle.q2(cfg["fact"], cfg["dim"], cfg["day_cut"])
        dt = time.perf_counter() - t0
        ok = all(np.array_equal(res[k], want[k]) for k in
                 ("a_key", "a_qty", "a_price", "a_count", "b_key", "b_qty", "b_count"))
        cpu = {"value": round(args.n_fact / dt, 1), "unit": "rows/s", "cores": 1,
               "kind": "oracle", "seconds": round(dt, 3), "matches_gpu": bool(ok),
               "sample": f"the whole workload ({args.n_fact} fact rows), one run, "
                         "single-threaded C oracle (hash join + hash group-by)"}

    out = {
        "metric": METRIC,
        "value": round(args.n_fact / (ms * 1e-3), 1),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "skewed star query: fact 60M rows (fk Zipf s=1 over 2M keys), "
                               "dim 2M; day<1278; join fk=pk; group by (flag, cat mod 2) "
                               "and by fk",
                   "fact_rows": args.n_fact, "dim_rows": args.n_dim, "seed": args.seed,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "pipeline_hbm": {"algo_bytes_per_step": int(step_bytes),
                         "GBps": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                         "frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "stream_copy_GBps": round(copy_gbs, 1),
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
