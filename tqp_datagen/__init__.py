"""Seeded synthetic table generators shared by the oracle side and the HIP side.

This module only draws input columns.  It holds none of the relational
arithmetic (no predicate, sort, join or aggregation): both the CPU oracle and
the GPU path receive the arrays produced here and nothing else.

Random numbers come from a counter-based SplitMix64 generator (the
"SplitMix64" mixing function of Steele, Lea and Flood, OOPSLA 2014, as used by
Vigna's xorshift family): draw ``i`` of stream ``s`` under seed ``seed`` is
``mix(seed ^ (s << 40) ^ i)``.  Counter-based means any slice of a column can
be regenerated without generating what precedes it.

The tables stand in for the TPC-H data the paper measures on (Section 2.3:
Q6 and Q14 at scale factor 1), which is not available: a 2557-day date domain,
25-way categories like nations, money as int64 cents, star-schema foreign keys.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "splitmix64", "raw_u64", "uniform_int", "uniform_float", "zipf_ranks",
    "permutation", "config1", "config2", "config3", "config4", "config5",
    "small_table", "DAY_DOMAIN", "config_q6", "Q6_BOUNDS", "type_vocabulary", "config_q14",
    "mlp_model", "config_predict",
]

DAY_DOMAIN = 2557          # seven years of day numbers, [0, 2557)
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to a uint64 array."""
    z = x + _GOLDEN
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def raw_u64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Draws ``start .. start+n-1`` of ``stream`` as uint64."""
    base = np.uint64((seed ^ (stream << 40)) & 0xFFFFFFFFFFFFFFFF)
    ctr = np.arange(start, start + n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return splitmix64(ctr ^ base)


def uniform_int(seed: int, stream: int, n: int, lo: int, hi: int,
                dtype=np.int64, start: int = 0) -> np.ndarray:
    """Integers uniform on [lo, hi): lo + ((u >> 32) * (hi - lo) >> 32)."""
    span = hi - lo
    assert 0 < span <= (1 << 32)
    u = raw_u64(seed, stream, n, start) >> np.uint64(32)
    with np.errstate(over="ignore"):
        v = (u * np.uint64(span)) >> np.uint64(32)
    return (v.astype(np.int64) + lo).astype(dtype)


def uniform_float(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """float64 uniform on [0, 1) with 53 random bits."""
    u = raw_u64(seed, stream, n, start) >> np.uint64(11)
    return u.astype(np.float64) * (2.0 ** -53)


_zipf_cache: dict = {}


def _zipf_cdf(N: int, s: float) -> np.ndarray:
    key = (N, float(s))
    if key not in _zipf_cache:
        w = np.arange(1, N + 1, dtype=np.float64) ** (-float(s))
        c = np.cumsum(w)
        c /= c[-1]
        c[-1] = 1.0
        if len(_zipf_cache) > 8:
            _zipf_cache.clear()
        _zipf_cache[key] = c
    return _zipf_cache[key]


def zipf_ranks(seed: int, stream: int, n: int, N: int, s: float,
               start: int = 0) -> np.ndarray:
    """Bounded Zipf ranks r in [1, N] with P(r) proportional to r**-s.

    Inverse-CDF sampling: r = 1 + #{cdf entries <= u}.  s = 0 is uniform.
    """
    cdf = _zipf_cdf(N, s)
    u = uniform_float(seed, stream, n, start)
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, N).astype(np.int64)


def permutation(seed: int, stream: int, n: int) -> np.ndarray:
    """A seeded permutation of 0..n-1 (stable argsort of a SplitMix64 stream)."""
    return np.argsort(raw_u64(seed, stream, n), kind="stable").astype(np.int64)


# ----------------------------------------------------------------------------
# Workload configurations.  Every column is a 1-D contiguous array, the (n x 1)
# numeric column of the paper's Section 2.1.  Money is int64 cents.
# ----------------------------------------------------------------------------

def config1(seed: int = 0, n_fact: int = 1_000_000, n_dim: int = 10_000) -> dict:
    """Star query, small: fact {fk, qty, day}, dim {pk, cat}.

    Query: WHERE day < 1278, JOIN fk = pk, GROUP BY cat: SUM(qty), COUNT(*).
    """
    fact = {
        "fk": uniform_int(seed, 1, n_fact, 0, n_dim, np.int32),
        "qty": uniform_int(seed, 2, n_fact, 1, 5001, np.int64),
        "day": uniform_int(seed, 3, n_fact, 0, DAY_DOMAIN, np.int32),
    }
    dim = {
        "pk": permutation(seed, 4, n_dim).astype(np.int32),
        "cat": uniform_int(seed, 5, n_dim, 0, 25, np.int32),
    }
    return {"fact": fact, "dim": dim, "day_cut": 1278}


def config2(seed: int = 0, n_fact: int = 60_000_000, n_dim: int = 2_000_000,
            zipf_s: float = 1.0) -> dict:
    """Skewed star query: fk Zipf(s) over the dim keys (key = rank - 1).

    Query: WHERE day < 1278, JOIN fk = pk, then
      (a) GROUP BY (flag, cat mod 2): SUM(qty), SUM(price), COUNT(*)
      (b) GROUP BY fk: SUM(qty), COUNT(*).
    """
    fact = {
        "fk": (zipf_ranks(seed, 1, n_fact, n_dim, zipf_s) - 1).astype(np.int32),
        "qty": uniform_int(seed, 2, n_fact, 1, 5001, np.int64),
        "price": uniform_int(seed, 3, n_fact, 100, 10_000_001, np.int64),
        "flag": uniform_int(seed, 4, n_fact, 0, 3, np.int8),
        "day": uniform_int(seed, 5, n_fact, 0, DAY_DOMAIN, np.int32),
    }
    dim = {
        "pk": permutation(seed, 6, n_dim).astype(np.int32),
        "cat": uniform_int(seed, 7, n_dim, 0, 25, np.int32),
    }
    return {"fact": fact, "dim": dim, "day_cut": 1278}


def config3(seed: int = 0, n_fact: int = 600_000_000,
            dims=(1_000_000, 100_000, 25)) -> dict:
    """Star join over three dims.

    d1 {pk, cat25, attr}, d2 {pk, cat5, attr}, d3 {pk = 0..24, attr = 4 pk};
    each dim filtered by attr < 20.  GROUP BY (d1.cat25, d2.cat5):
    SUM(qty * price), COUNT(*).
    """
    n1, n2, n3 = dims
    fact = {
        "fk1": uniform_int(seed, 1, n_fact, 0, n1, np.int32),
        "fk2": uniform_int(seed, 2, n_fact, 0, n2, np.int32),
        "fk3": uniform_int(seed, 3, n_fact, 0, n3, np.int32),
        "qty": uniform_int(seed, 4, n_fact, 1, 5001, np.int64),
        "price": uniform_int(seed, 5, n_fact, 100, 10_000_001, np.int64),
    }
    d1 = {"pk": permutation(seed, 6, n1).astype(np.int32),
          "cat": uniform_int(seed, 7, n1, 0, 25, np.int32),
          "attr": uniform_int(seed, 8, n1, 0, 100, np.int32)}
    d2 = {"pk": permutation(seed, 9, n2).astype(np.int32),
          "cat": uniform_int(seed, 10, n2, 0, 5, np.int32),
          "attr": uniform_int(seed, 11, n2, 0, 100, np.int32)}
    pk3 = np.arange(n3, dtype=np.int32)
    d3 = {"pk": pk3, "attr": (4 * pk3).astype(np.int32)}
    return {"fact": fact, "d1": d1, "d2": d2, "d3": d3, "attr_cut": 20}


# Q6-shaped scan: ship timestamps as int64 epoch nanoseconds (the paper keeps
# dates as epoch-based integers, Section 2.1) over the same seven years
# (1992-01-01 is day 8035 after 1970-01-01), discount in hundredths (int8),
# quantity (int32), price in cents (int64).  The query keeps one year of
# ship dates, discounts 0.05..0.07 and quantities below 24.
_NS_PER_DAY = 86_400 * 1_000_000_000
_DAY0 = 8035
Q6_BOUNDS = {"ship_lo": 8766 * _NS_PER_DAY,      # 1994-01-01
             "ship_hi": 9131 * _NS_PER_DAY,      # 1995-01-01
             "disc_lo": 5, "disc_hi": 7, "qty_cut": 24}


def config_q6(seed: int = 0, n: int = 60_000_000) -> dict:
    """Q6-shaped table (TPC-H lineitem columns at scale factor 10 has 60M
    rows): SUM(price * discount), COUNT(*) WHERE ship in [1994, 1995) AND
    discount BETWEEN 5 AND 7 AND quantity < 24."""
    day = uniform_int(seed, 1, n, 0, DAY_DOMAIN, np.int64)
    sec = uniform_int(seed, 2, n, 0, 86_400, np.int64)
    items = {
        "ship": ((day + _DAY0) * 86_400 + sec) * 1_000_000_000,
        "discount": uniform_int(seed, 3, n, 0, 11, np.int8),
        "quantity": uniform_int(seed, 4, n, 1, 51, np.int32),
        "price": uniform_int(seed, 5, n, 90_000, 10_494_951, np.int64),
    }
    return {"items": items, **Q6_BOUNDS}


# Q14-shaped join with a string predicate.  Strings are the paper's (n x m)
# tensor of UTF-8 bytes, zero-padded to the longest (Section 2.1).  Part
# types are three words drawn from three seeded pools of synthetic upper-case
# words (6 x 5 x 5 = 150 types); the LIKE prefix is the first pool's first
# word, which no other word of that pool starts with, so a sixth of the types
# match.
def _word(seed: int, stream: int, k: int) -> bytes:
    ln = int(uniform_int(seed, stream, 1, 3, 10, start=k)[0])
    return bytes(int(c) for c in uniform_int(seed, stream + 1, ln, 65, 91, start=16 * k))


def type_vocabulary(seed: int = 0):
    """(table, prefix): table is (150, m) uint8, zero-padded; prefix bytes."""
    pools, k = [], 0
    for stream, size in ((60, 6), (62, 5), (64, 5)):
        pool = []
        while len(pool) < size:
            w = _word(seed, stream, k)
            k += 1
            if all(not (w.startswith(x) or x.startswith(w)) for x in pool):
                pool.append(w)
        pools.append(pool)
    names = [a + b" " + b + b" " + c for a in pools[0] for b in pools[1] for c in pools[2]]
    m = max(len(x) for x in names)
    table = np.zeros((len(names), m), np.uint8)
    for i, x in enumerate(names):
        table[i, :len(x)] = np.frombuffer(x, np.uint8)
    return table, pools[0][0]


def config_q14(seed: int = 0, n_items: int = 60_000_000, n_part: int = 2_000_000) -> dict:
    """Q14-shaped: items {ship int64 epoch-ns, partkey int32, price int64
    cents, discount int8 hundredths}; part {pk = a permutation, type as an
    (n_part, m) byte matrix}.  Query: ship in [1995-09-01, 1995-10-01), JOIN
    partkey = pk; revenue = price * (100 - discount); the promo share is
    SUM(revenue of types LIKE prefix%) over SUM(revenue)."""
    day = uniform_int(seed, 1, n_items, 0, DAY_DOMAIN, np.int64)
    sec = uniform_int(seed, 2, n_items, 0, 86_400, np.int64)
    items = {
        "ship": ((day + _DAY0) * 86_400 + sec) * 1_000_000_000,
        "partkey": uniform_int(seed, 3, n_items, 0, n_part, np.int32),
        "price": uniform_int(seed, 4, n_items, 90_000, 10_494_951, np.int64),
        "discount": uniform_int(seed, 5, n_items, 0, 11, np.int8),
    }
    table, prefix = type_vocabulary(seed)
    tid = uniform_int(seed, 6, n_part, 0, table.shape[0], np.int64)
    part = {"pk": permutation(seed, 7, n_part).astype(np.int32), "type": table[tid]}
    return {"items": items, "part": part, "prefix": prefix,
            "ship_lo": 9374 * _NS_PER_DAY, "ship_hi": 9404 * _NS_PER_DAY}


# Prediction query: reviews with a 1..5 rating, a year and eight small integer
# features that lean on the rating (feature k = (rating - 3) * 4 slope_k +
# noise in [-8, 8]), and
# a small fp32 model (8 -> 16 -> 2) with seeded weights: the paper's trained
# models and review data are not available, so the scores are synthetic.
def mlp_model(seed: int, nfeat: int, hidden: int, classes: int) -> np.ndarray:
    """[W1 (hidden x nfeat), b1, W2 (classes x hidden), b2] as float32, each
    weight uniform on [-1, 1) / sqrt(fan-in)."""
    parts = []
    for k, (rows, fan) in enumerate(((hidden * nfeat, nfeat), (hidden, nfeat),
                                     (classes * hidden, hidden), (classes, hidden))):
        u = uniform_float(seed, 80 + k, rows) * 2.0 - 1.0
        parts.append((u / np.sqrt(fan)).astype(np.float32))
    return np.concatenate(parts)


def config_predict(seed: int = 0, n: int = 20_000_000, nfeat: int = 8, hidden: int = 16) -> dict:
    """SELECT rating, SUM(CASE WHEN PREDICT(model, f0..f7) = 1 THEN 1 ELSE 0 END),
    COUNT(*) FROM reviews WHERE year >= 2016 GROUP BY rating."""
    rating = uniform_int(seed, 1, n, 1, 6, np.int8)
    reviews = {"rating": rating, "year": uniform_int(seed, 2, n, 2010, 2024, np.int32)}
    for k in range(nfeat):
        slope = (k % 4) - 1                       # -1, 0, 1, 2
        reviews[f"f{k}"] = ((rating.astype(np.int32) - 3) * slope * 4
                            + uniform_int(seed, 10 + k, n, -8, 9, np.int32)).astype(np.int32)
    return {"reviews": reviews, "model": mlp_model(seed, nfeat, hidden, 2), "nfeat": nfeat,
            "hidden": hidden, "classes": 2, "year_min": 2016, "nratings": 6}


_C4_SCATTER = 0x2545F4914F6CDD1D   # odd multiplier: a bijection modulo 2**62
_MASK62 = (1 << 62) - 1


def _c4_side(seed: int, stream0: int, n: int, centres: np.ndarray) -> np.ndarray:
    """int64 keys from an equal-weight mixture of three components."""
    comp = uniform_int(seed, stream0, n, 0, 3, np.int64)
    out = np.empty(n, dtype=np.int64)
    # lognormal(mean 30, sigma 2) clamped to [0, 2**62)
    z = _normal(seed, stream0 + 1, n)
    ln = np.floor(np.exp(30.0 + 2.0 * z))
    ln = np.clip(ln, 0.0, float(2 ** 62 - 1024)).astype(np.int64)
    # 64 dense clusters of width 2**20
    cj = uniform_int(seed, stream0 + 2, n, 0, len(centres), np.int64)
    off = uniform_int(seed, stream0 + 3, n, 0, 1 << 20, np.int64)
    cl = centres[cj] + off
    # Zipf s = 1.2 over 1e6 ranks, scattered by an odd-multiplier bijection
    r = zipf_ranks(seed, stream0 + 4, n, 1_000_000, 1.2).astype(np.uint64)
    with np.errstate(over="ignore"):
        zs = ((r * np.uint64(_C4_SCATTER)) & np.uint64(_MASK62)).astype(np.int64)
    out[:] = np.where(comp == 0, ln, np.where(comp == 1, cl, zs))
    return out


def _normal(seed: int, stream: int, n: int) -> np.ndarray:
    """Standard normal draws by Box-Muller on two uniform streams."""
    u1 = uniform_float(seed, stream, n)
    u2 = uniform_float(seed, stream + 100, n)
    u1 = 1.0 - u1                       # (0, 1]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def config4(seed: int = 0, n_left: int = 200_000_000,
            n_right: int = 50_000_000) -> dict:
    """Large-large int64 key join; keys from a lognormal / cluster / Zipf mix."""
    lo = uniform_int(seed, 50, 64, 0, 1 << 31, np.int64)
    hi = uniform_int(seed, 51, 64, 0, 1 << 31, np.int64)
    centres = ((hi << 31) | lo) % ((1 << 62) - (1 << 20))
    return {
        "left": _c4_side(seed, 60, n_left, centres),
        "right": _c4_side(seed, 70, n_right, centres),
    }


def config5_params(seed: int = 0, instances: int = 256,
                   fact_lo: int = 10_000, fact_hi: int = 20_000_000) -> list:
    """Per-instance sizes for the batched workload (log-uniform fact sizes)."""
    f = uniform_float(seed, 80, instances)
    fact = np.floor(np.exp(np.log(fact_lo) + f * (np.log(fact_hi) - np.log(fact_lo))))
    s = uniform_float(seed, 81, instances) * 1.5
    g = uniform_float(seed, 82, instances)
    groups = np.floor(np.exp(np.log(25) + g * (np.log(100_000) - np.log(25))))
    out = []
    for k in range(instances):
        nf = int(fact[k])
        nd = max(1, nf // 20)
        out.append({"n_fact": nf, "n_dim": nd, "zipf_s": float(s[k]),
                    "groups": int(min(groups[k], nd))})
    return out


def config5(seed: int = 0, instances: int = 256, fact_lo: int = 10_000,
            fact_hi: int = 20_000_000) -> list:
    """A batch of independent filter -> join -> group-by instances."""
    out = []
    for k, p in enumerate(config5_params(seed, instances, fact_lo, fact_hi)):
        sk = seed * 1_000_003 + 7919 * (k + 1)
        nf, nd = p["n_fact"], p["n_dim"]
        fact = {
            "fk": (zipf_ranks(sk, 1, nf, nd, p["zipf_s"]) - 1).astype(np.int32),
            "qty": uniform_int(sk, 2, nf, 1, 5001, np.int64),
            "day": uniform_int(sk, 3, nf, 0, DAY_DOMAIN, np.int32),
        }
        dim = {"pk": permutation(sk, 4, nd).astype(np.int32),
               "cat": uniform_int(sk, 5, nd, 0, p["groups"], np.int32)}
        out.append({"fact": fact, "dim": dim, "day_cut": 1278, **p})
    return out


def small_table(seed: int, n: int, lo: int, hi: int, dtype=np.int64,
                stream: int = 1) -> np.ndarray:
    """One uniform column, for edge-case tests (small domains force duplicates)."""
    return uniform_int(seed, stream, n, lo, hi, dtype)
