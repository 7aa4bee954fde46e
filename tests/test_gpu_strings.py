"""GPU parity for the string predicate (tqp_str_match over the paper's (n x m)
zero-padded byte matrices) and the Q14-shaped join built on it (Section 2.3),
against the CPU oracle: byte-exact flags for every pattern length and both
modes, and exact revenue sums and counts for the whole query."""
import numpy as np
import pytest

import oracle
import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tqp():
    import paper_2209_04579_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def strings(seed, n, m):
    """Rows of random length in [0, m] over a 4-letter alphabet (many shared
    prefixes), zero-padded."""
    lens = dg.uniform_int(seed, 1, n, 0, m + 1, np.int64)
    letters = dg.uniform_int(seed, 2, n * m, 65, 69, np.uint8).reshape(n, m)
    keep = np.arange(m)[None, :] < lens[:, None]
    return np.where(keep, letters, 0).astype(np.uint8)


@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 100_003])
@pytest.mark.parametrize("m", [1, 7, 24, 33])
def test_str_match_matches_oracle(tqp, n, m):
    chars = strings(n + m, n, m)
    d = torch.from_numpy(chars).cuda()
    out = torch.full((max(n, 1),), -1, dtype=torch.int8, device="cuda")
    pats = [b"", b"A", b"AB", b"DCBA", b"A" * m, b"A" * (m + 1)]
    if n:
        pats.append(bytes(chars[n // 2]).rstrip(b"\0"))
    for pat in pats:
        for mode in ("prefix", "equal"):
            tqp.str_match_into(d, pat, out, mode)
            torch.cuda.synchronize()
            assert np.array_equal(out[:n].cpu().numpy(), oracle.str_match(chars, pat, mode)), (pat, mode)


def run_q14(cfg, dev_cfg=None):
    from paper_2209_04579_amd.pipeline import Q14Query
    if dev_cfg is None:
        dev_cfg = {t: {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in cfg[t].items()}
                   for t in ("items", "part")}
    q = Q14Query(dev_cfg["items"], dev_cfg["part"], cfg["prefix"], cfg["ship_lo"], cfg["ship_hi"])
    q.run()
    return q, q.result()


def check_q14(cfg, dev_cfg=None):
    q, got = run_q14(cfg, dev_cfg)
    want = oracle.q14(cfg)
    assert want["exact"]
    for k in ("promo_rev", "total_rev", "count", "promo_count"):
        assert got[k] == want[k], (k, got[k], want[k])
    return q, got


@pytest.mark.parametrize("seed,ni,npart", [(0, 2_000_000, 100_000), (1, 50_000, 1), (2, 7, 5),
                                           (3, 300_000, 40_000)])
def test_q14_matches_oracle(tqp, seed, ni, npart):
    check_q14(dg.config_q14(seed, ni, npart))


def test_q14_prefix_all_and_none(tqp):
    cfg = dg.config_q14(4, 200_000, 20_000)
    _, got = check_q14(dict(cfg, prefix=b""))
    assert got["promo_rev"] == got["total_rev"] and got["count"] > 0
    _, got = check_q14(dict(cfg, prefix=b"QQQQQQQQQQQQQQQQQQQQQQQQQQQQQQ"))
    assert got["promo_rev"] == 0 and got["promo_count"] == 0


def test_q14_replay_is_identical(tqp):
    cfg = dg.config_q14(5, 1_000_000, 50_000)
    q, first = check_q14(cfg)
    for _ in range(3):
        q.run()
        assert q.result() == first


def test_q14_full_size(tqp):
    """60M items and 2M parts drawn on the GPU; the oracle reads host copies."""
    from tqp_datagen import device as dgd
    d = dgd.config_q14(0, device="cuda")
    host = {t: {k: v.cpu().numpy() for k, v in d[t].items()} for t in ("items", "part")}
    host.update({k: d[k] for k in ("prefix", "ship_lo", "ship_hi")})
    _, got = check_q14(host, d)
    assert got["pairs"] == got["rows_filtered"] > 0
