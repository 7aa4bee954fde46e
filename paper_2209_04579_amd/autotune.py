"""Autotuner for the library's launch knobs and a plan's own parameters.

A plan (anything with ``run()`` that enqueues one whole query on the current
stream) is timed with HIP events while one knob at a time sweeps its range,
the others held at their best value so far (coordinate descent).  The best
setting is cached as JSON under a key of (GPU architecture, operation, key
dtype, log2 of the row count, skew class), so a later plan of the same class
starts from it without re-tuning (``tune_cached``).

Knobs: every library knob from ``tune_knobs()`` (persistent-grid workgroups
per CU of the filter, radix passes, run-length encoding, join match and
sorted group-by; the radix pass mode; the semi-join's workgroup size, which
is its tile size) and ``gb.dense_max``, the largest group-key domain the
star query aggregates directly instead of by sort.  ``tune_params`` sweeps a
plan's own discrete parameters the same way: for the learned partition sort,
the bucket count (2^bits), the model's leaf count and its training steps.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import tune_knobs

DENSE_MAX_CHOICES = (0, 64, 1024)


def cache_key(op: str, rows: int, skew: str = "", dtype: str = "") -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    return f"{arch}/{op}/{dtype}/log2n={int(math.log2(max(rows, 1)))}/{skew}"


def load(path: str, key: str) -> dict | None:
    if not path or not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh).get(key)


def save(path: str, key: str, value: dict):
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[key] = value
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_plan(plan, reps: int = 5) -> float:
    """Median milliseconds of plan.run() over reps runs (after one warm-up)."""
    stream = torch.cuda.current_stream()
    plan.run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.run()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(make_plan, reps: int = 5, rounds: int = 2, include_dense: bool = True,
         log=None, only=None) -> tuple[dict, float, dict]:
    """Coordinate descent over the knobs.

    make_plan(tuning) -> plan.  Returns (best tuning, best ms, all timings).
    Knobs with at most 16 settings are swept (grid sizes, the radix pass
    mode, workgroup sizes), not capacity limits; ``only`` limits the sweep to
    the knobs of the kernels the plan runs."""
    knobs = {k: v for k, v in tune_knobs().items()
             if v[2] - v[1] <= 16 and (only is None or k in only)}
    best = {k: v[0] for k, v in knobs.items()}
    if include_dense:
        best["gb.dense_max"] = 1024
    timings = {}

    def measure(t):
        key = json.dumps(t, sort_keys=True)
        if key not in timings:
            timings[key] = time_plan(make_plan(dict(t)), reps)
            if log:
                log(f"[tune] {t} -> {timings[key]:.3f} ms")
        return timings[key]

    best_ms = measure(best)
    for _ in range(rounds):
        improved = False
        for name, (_, lo, hi) in knobs.items():
            for v in range(lo, hi + 1):
                t = dict(best, **{name: v})
                ms = measure(t)
                if ms < best_ms * 0.995:
                    best, best_ms, improved = t, ms, True
        if include_dense:
            for v in DENSE_MAX_CHOICES:
                t = dict(best, **{"gb.dense_max": v})
                ms = measure(t)
                if ms < best_ms * 0.995:
                    best, best_ms, improved = t, ms, True
        if not improved:
            break
    return best, best_ms, timings


def tune_params(make_plan, space: dict, start: dict, reps: int = 3, rounds: int = 2,
                log=None) -> tuple[dict, float, dict]:
    """Coordinate descent over a plan's own discrete parameters.

    space: name -> list of choices; start: the first setting (one choice per
    name).  make_plan(setting) -> plan.  Returns (best, best ms, timings)."""
    best = dict(start)
    timings = {}

    def measure(t):
        key = json.dumps(t, sort_keys=True)
        if key not in timings:
            timings[key] = time_plan(make_plan(dict(t)), reps)
            if log:
                log(f"[tune] {t} -> {timings[key]:.3f} ms")
        return timings[key]

    best_ms = measure(best)
    for _ in range(rounds):
        improved = False
        for name, choices in space.items():
            for v in choices:
                t = dict(best, **{name: v})
                ms = measure(t)
                if ms < best_ms * 0.995:
                    best, best_ms, improved = t, ms, True
        if not improved:
            break
    return best, best_ms, timings


def tune_cached(path: str, key: str, run_tuner) -> tuple[dict, float | None, bool]:
    """The cached setting for key if there is one, else run_tuner() ->
    (best, best ms, timings), saved under key.  Returns (setting, ms or
    None, whether it came from the cache)."""
    hit = load(path, key)
    if hit is not None:
        return hit["setting"], hit.get("ms"), True
    best, best_ms, _ = run_tuner()
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        save(path, key, {"setting": best, "ms": round(best_ms, 4)})
    return best, best_ms, False
