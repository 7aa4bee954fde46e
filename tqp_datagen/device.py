"""The same seeded generators written with torch tensor ops, so the large
workloads (600M-row star, 250M-key join, 673M-row batch) are drawn on the
GPU in seconds instead of minutes on the host.

Integer draws (SplitMix64 counters, uniform integers, permutations) are
bit-identical to the numpy versions in ``tqp_datagen``.  Float draws
(Zipf inverse CDF, lognormal) use the same formulas but the device's float64
math library, so a rare draw can land one step away from the host's; these
tables are used for timing, and the parity tests use the host generators.
Like the host module, this holds no relational arithmetic.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import (_C4_SCATTER, _DAY0, _MASK62, _NS_PER_DAY, DAY_DOMAIN, Q6_BOUNDS, _zipf_cdf,
                config5_params, mlp_model, type_vocabulary)

_G = np.uint64(0x9E3779B97F4A7C15).astype(np.int64).item()
_M1 = np.uint64(0xBF58476D1CE4E5B9).astype(np.int64).item()
_M2 = np.uint64(0x94D049BB133111EB).astype(np.int64).item()


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def splitmix64(x: torch.Tensor) -> torch.Tensor:
    z = x + _G
    z = (z ^ _srl(z, 30)) * _M1
    z = (z ^ _srl(z, 27)) * _M2
    return z ^ _srl(z, 31)


def _as_i64(v: int) -> int:
    v &= (1 << 64) - 1
    return v - (1 << 64) if v >= (1 << 63) else v


def raw_u64(seed, stream, n, device, start=0) -> torch.Tensor:
    base = _as_i64(seed ^ (stream << 40))
    ctr = torch.arange(start, start + n, dtype=torch.int64, device=device)
    return splitmix64(ctr ^ base)


def uniform_int(seed, stream, n, lo, hi, device, dtype=torch.int64, start=0):
    span = hi - lo
    assert 0 < span <= (1 << 32)
    u = _srl(raw_u64(seed, stream, n, device, start), 32)
    # int64 products wrap modulo 2^64 like the host's uint64 ones, so the high
    # word is the same bit pattern
    v = _srl(u * span, 32)
    return (v + lo).to(dtype)


def uniform_float(seed, stream, n, device, start=0):
    u = _srl(raw_u64(seed, stream, n, device, start), 11)
    return u.to(torch.float64) * (2.0 ** -53)


def zipf_ranks(seed, stream, n, N, s, device, start=0):
    cdf = torch.from_numpy(_zipf_cdf(N, s)).to(device)
    u = uniform_float(seed, stream, n, device, start)
    r = torch.searchsorted(cdf, u, right=True) + 1
    return torch.clamp(r, max=N)


def permutation(seed, stream, n, device):
    # flipping the top bit makes signed int64 order equal unsigned order
    return torch.argsort(raw_u64(seed, stream, n, device) ^ (-(1 << 63)), stable=True)


def _normal(seed, stream, n, device):
    u1 = 1.0 - uniform_float(seed, stream, n, device)
    u2 = uniform_float(seed, stream + 100, n, device)
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)


def _c4_side(seed, stream0, n, centres, device, chunk=1 << 25):
    out = torch.empty(n, dtype=torch.int64, device=device)
    for s0 in range(0, n, chunk):
        m = min(chunk, n - s0)
        comp = uniform_int(seed, stream0, m, 0, 3, device, start=s0)
        z = _normal_at(seed, stream0 + 1, m, device, s0)
        ln = torch.floor(torch.exp(30.0 + 2.0 * z)).clamp(0.0, float(2 ** 62 - 1024)).to(torch.int64)
        cj = uniform_int(seed, stream0 + 2, m, 0, len(centres), device, start=s0)
        off = uniform_int(seed, stream0 + 3, m, 0, 1 << 20, device, start=s0)
        cl = centres[cj] + off
        r = zipf_ranks(seed, stream0 + 4, m, 1_000_000, 1.2, device, start=s0)
        zs = (r * _as_i64(_C4_SCATTER)) & _MASK62
        out[s0:s0 + m] = torch.where(comp == 0, ln, torch.where(comp == 1, cl, zs))
    return out


def _normal_at(seed, stream, n, device, start):
    u1 = 1.0 - uniform_float(seed, stream, n, device, start)
    u2 = uniform_float(seed, stream + 100, n, device, start)
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)


def config4(seed=0, n_left=200_000_000, n_right=50_000_000, device="cuda"):
    lo = uniform_int(seed, 50, 64, 0, 1 << 31, "cpu")
    hi = uniform_int(seed, 51, 64, 0, 1 << 31, "cpu")
    centres = (((hi << 31) | lo) % ((1 << 62) - (1 << 20))).to(device)
    return {"left": _c4_side(seed, 60, n_left, centres, device),
            "right": _c4_side(seed, 70, n_right, centres, device)}


def config5(seed=0, instances=256, fact_lo=10_000, fact_hi=20_000_000, device="cuda"):
    out = []
    for k, p in enumerate(config5_params(seed, instances, fact_lo, fact_hi)):
        sk = seed * 1_000_003 + 7919 * (k + 1)
        nf, nd = p["n_fact"], p["n_dim"]
        fact = {
            "fk": (zipf_ranks(sk, 1, nf, nd, p["zipf_s"], device) - 1).to(torch.int32),
            "qty": uniform_int(sk, 2, nf, 1, 5001, device),
            "day": uniform_int(sk, 3, nf, 0, DAY_DOMAIN, device, torch.int32),
        }
        dim = {"pk": permutation(sk, 4, nd, device).to(torch.int32),
               "cat": uniform_int(sk, 5, nd, 0, p["groups"], device, torch.int32)}
        out.append({"fact": fact, "dim": dim, "day_cut": 1278, **p})
    return out


def config3(seed=0, n_fact=600_000_000, dims=(1_000_000, 100_000, 25), device="cuda"):
    """Three-dimension star (every draw is an integer draw, so the tables are
    bit-identical to the host generator's)."""
    n1, n2, n3 = dims
    fact = {
        "fk1": uniform_int(seed, 1, n_fact, 0, n1, device, torch.int32),
        "fk2": uniform_int(seed, 2, n_fact, 0, n2, device, torch.int32),
        "fk3": uniform_int(seed, 3, n_fact, 0, n3, device, torch.int32),
        "qty": uniform_int(seed, 4, n_fact, 1, 5001, device),
        "price": uniform_int(seed, 5, n_fact, 100, 10_000_001, device),
    }
    d1 = {"pk": permutation(seed, 6, n1, device).to(torch.int32),
          "cat": uniform_int(seed, 7, n1, 0, 25, device, torch.int32),
          "attr": uniform_int(seed, 8, n1, 0, 100, device, torch.int32)}
    d2 = {"pk": permutation(seed, 9, n2, device).to(torch.int32),
          "cat": uniform_int(seed, 10, n2, 0, 5, device, torch.int32),
          "attr": uniform_int(seed, 11, n2, 0, 100, device, torch.int32)}
    pk3 = torch.arange(n3, dtype=torch.int32, device=device)
    d3 = {"pk": pk3, "attr": 4 * pk3}
    return {"fact": fact, "d1": d1, "d2": d2, "d3": d3, "attr_cut": 20}


def config_q6(seed=0, n=60_000_000, device="cuda"):
    """Q6-shaped table, bit-identical to the host generator's."""
    day = uniform_int(seed, 1, n, 0, DAY_DOMAIN, device)
    sec = uniform_int(seed, 2, n, 0, 86_400, device)
    items = {
        "ship": ((day + _DAY0) * 86_400 + sec) * 1_000_000_000,
        "discount": uniform_int(seed, 3, n, 0, 11, device, torch.int8),
        "quantity": uniform_int(seed, 4, n, 1, 51, device, torch.int32),
        "price": uniform_int(seed, 5, n, 90_000, 10_494_951, device),
    }
    return {"items": items, **Q6_BOUNDS}


def config_q14(seed=0, n_items=60_000_000, n_part=2_000_000, device="cuda"):
    """Q14-shaped tables, bit-identical to the host generator's."""
    day = uniform_int(seed, 1, n_items, 0, DAY_DOMAIN, device)
    sec = uniform_int(seed, 2, n_items, 0, 86_400, device)
    items = {
        "ship": ((day + _DAY0) * 86_400 + sec) * 1_000_000_000,
        "partkey": uniform_int(seed, 3, n_items, 0, n_part, device, torch.int32),
        "price": uniform_int(seed, 4, n_items, 90_000, 10_494_951, device),
        "discount": uniform_int(seed, 5, n_items, 0, 11, device, torch.int8),
    }
    table, prefix = type_vocabulary(seed)
    tid = uniform_int(seed, 6, n_part, 0, table.shape[0], device)
    part = {"pk": permutation(seed, 7, n_part, device).to(torch.int32),
            "type": torch.from_numpy(table).to(device)[tid].contiguous()}
    return {"items": items, "part": part, "prefix": prefix,
            "ship_lo": 9374 * _NS_PER_DAY, "ship_hi": 9404 * _NS_PER_DAY}


def config_predict(seed=0, n=20_000_000, nfeat=8, hidden=16, device="cuda"):
    """Prediction-query table, bit-identical to the host generator's (the
    model is drawn on the host)."""
    rating = uniform_int(seed, 1, n, 1, 6, device, torch.int8)
    reviews = {"rating": rating, "year": uniform_int(seed, 2, n, 2010, 2024, device, torch.int32)}
    for k in range(nfeat):
        slope = (k % 4) - 1
        reviews[f"f{k}"] = ((rating.to(torch.int32) - 3) * (slope * 4)
                            + uniform_int(seed, 10 + k, n, -8, 9, device, torch.int32)).to(torch.int32)
    return {"reviews": reviews, "model": mlp_model(seed, nfeat, hidden, 2), "nfeat": nfeat,
            "hidden": hidden, "classes": 2, "year_min": 2016, "nratings": 6}
