"""GPU parity of the semi-join reduction (tqp_keyset_build + tqp_semijoin)
against the oracle's semi-join (rows whose keys all occur on their right
sides), bit for bit: kept row ids, compacted key columns and payload, over
several tiles with ragged tails, int32 and int64 keys, one to four sets, sets
staged on chip and sets read from memory, keys below and above a set's range,
empty sets, empty and one-row tables."""
import numpy as np
import pytest

import oracle
import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = [0, 1, 15, 16, 17, 4095, 4096, 4097, 8191, 8193, 100_003]


@pytest.fixture(scope="module")
def tqp():
    import paper_2209_04579_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def run(tqp, keys, set_keys, ranges, payload=(), want_keys=True):
    """keys: host key columns; set_keys: host arrays given to the key-set
    build; ranges: (lo, nbits) per set.  Returns the device results on host."""
    n = len(keys[0])
    dk = [dev(k) for k in keys]
    sets = []
    for sk, (lo, nb) in zip(set_keys, ranges):
        bits = torch.empty(max(tqp.keyset_words(nb), 1), dtype=torch.int32, device="cuda")
        tqp.keyset_build_into(dev(sk), lo, nb, bits)
        sets.append((bits, lo, nb))
    rows = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    kout = [torch.empty(max(n, 1), dtype=k.dtype, device="cuda") for k in dk] if want_keys else None
    pin = [dev(p) for p in payload]
    pout = [torch.empty(max(n, 1), dtype=p.dtype, device="cuda") for p in pin]
    ws = torch.empty(tqp.semijoin_workspace_bytes(n, dk[0].dtype), dtype=torch.uint8,
                     device="cuda")
    tqp.semijoin_into(dk, sets, rows, cnt, ws, keys_out=kout, payload_in=pin, payload_out=pout)
    k = int(cnt.item())
    return (host(rows[:k]), [host(t[:k]) for t in kout] if kout else None,
            [host(t[:k]) for t in pout])


def in_range(sk, lo, nb):
    sk = np.asarray(sk, dtype=np.int64)
    return sk[(sk >= lo) & (sk < lo + nb)]


def check(tqp, keys, set_keys, ranges, payload=()):
    rows, kout, pout = run(tqp, keys, set_keys, ranges, payload)
    want = oracle.semijoin_rows(keys, [in_range(s, lo, nb) for s, (lo, nb) in zip(set_keys, ranges)])
    assert np.array_equal(rows, want)
    for k, got in zip(keys, kout):
        assert np.array_equal(got, oracle.gather(k, want))
    for p, got in zip(payload, pout):
        assert np.array_equal(got, oracle.gather(p, want))
    return want


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kdt", [np.int32, np.int64])
def test_semijoin_three_sets(tqp, n, kdt):
    # star-shaped: a small set (on chip), a mid one (on chip), a big one (memory)
    dims = [(25, 5), (3000, 600), (200_000, 40_000)]
    keys, set_keys, ranges = [], [], []
    for s, (dn, keep) in enumerate(dims):
        keys.append(dg.uniform_int(n + s, 1 + s, n, 0, dn, kdt))
        pk = dg.permutation(7 + s, 3, dn)
        set_keys.append(pk[:keep].astype(kdt))
        ranges.append((0, dn))
    qty = dg.uniform_int(n, 9, n, 1, 5001, np.int64)
    flag = dg.uniform_int(n, 10, n, -3, 3, np.int8)
    tag = dg.uniform_int(n, 11, n, -10 ** 6, 10 ** 6, np.int32)
    check(tqp, keys, set_keys, ranges, payload=[qty, flag, tag])


@pytest.mark.parametrize("nsets", [1, 2, 4])
def test_semijoin_set_counts(tqp, nsets):
    n = 50_001 + nsets
    keys = [dg.uniform_int(nsets, 20 + s, n, -50, 1000, np.int32) for s in range(nsets)]
    set_keys = [dg.uniform_int(nsets, 40 + s, 300, -80, 1200, np.int32) for s in range(nsets)]
    ranges = [(-60 + 5 * s, 1100 - 7 * s) for s in range(nsets)]
    check(tqp, keys, set_keys, ranges)


@pytest.mark.parametrize("kdt", [np.int32, np.int64])
@pytest.mark.parametrize("nb", [1, 31, 32, 33, 63, 64, 65])
def test_semijoin_tiny_sets(tqp, nb, kdt):
    """Sets of a few keys around one and two words, over ranges not starting
    at zero, with keys below, inside and beyond each range; beside a larger
    set so both kinds of test run in one scan."""
    n = 70_001
    lo = -17
    keys = [dg.uniform_int(nb, 60, n, lo - 5, lo + nb + 5, kdt),
            dg.uniform_int(nb, 61, n, 0, 5000, kdt)]
    set_keys = [dg.uniform_int(nb, 62, max(nb // 2, 1), lo - 3, lo + nb + 3, kdt),
                dg.permutation(nb, 63, 5000)[:1200].astype(kdt)]
    check(tqp, keys, set_keys, [(lo, nb), (0, 5000)])


def test_semijoin_keys_outside_every_range(tqp):
    n = 20_000
    k = dg.uniform_int(3, 1, n, -10 ** 9, 10 ** 9, np.int64)
    k[::7] = np.iinfo(np.int64).min
    k[3::7] = np.iinfo(np.int64).max
    sk = k[::13].copy()
    check(tqp, [k], [sk], [(-5 * 10 ** 8, 10 ** 9)])
    # a range far from every key keeps nothing
    want = check(tqp, [k], [sk], [(4 * 10 ** 9, 1000)])
    assert len(want) == 0


def test_semijoin_large_set_from_memory(tqp):
    # 2^22-key range: the set is read from memory for the rows that reach it
    n = 300_000
    k1 = dg.uniform_int(1, 1, n, 0, 4, np.int32)
    k2 = dg.uniform_int(1, 2, n, 0, 1 << 22, np.int32)
    s1 = np.array([1, 3], dtype=np.int32)
    s2 = dg.uniform_int(1, 3, 1 << 20, 0, 1 << 22, np.int32)
    check(tqp, [k1, k2], [s1, s2], [(0, 4), (0, 1 << 22)])


def test_semijoin_empty_set_and_all_kept(tqp):
    n = 9000
    k = dg.uniform_int(5, 1, n, 0, 100, np.int32)
    want = check(tqp, [k], [np.zeros(0, np.int32)], [(0, 0)])
    assert len(want) == 0
    want = check(tqp, [k], [np.arange(100, dtype=np.int32)], [(0, 100)])
    assert len(want) == n


def test_semijoin_unaligned_keys(tqp):
    # key columns that are views at odd offsets take the element-wise loads
    n = 10_001
    base = dg.uniform_int(6, 1, n + 1, 0, 500, np.int32)
    dk = dev(base)[1:]
    bits = torch.empty(16, dtype=torch.int32, device="cuda")
    sk = dg.uniform_int(6, 2, 100, 0, 500, np.int32)
    tqp.keyset_build_into(dev(sk), 0, 500, bits)
    rows = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(tqp.semijoin_workspace_bytes(n, torch.int32), dtype=torch.uint8, device="cuda")
    tqp.semijoin_into([dk], [(bits, 0, 500)], rows, cnt, ws)
    k = int(cnt.item())
    want = oracle.semijoin_rows([base[1:]], [sk])
    assert np.array_equal(host(rows[:k]), want)


@pytest.mark.timeout(300)
def test_semijoin_star_full_size(tqp):
    """The three-dimension star's reduction at full size (600M fact rows,
    drawn on the GPU), compared with the oracle on a sample of row blocks:
    each block's kept rows are a contiguous slice of the output, located by
    counting the kept rows before the block."""
    from tqp_datagen import device as dgd
    cfg = dgd.config3(0, device="cuda")
    f = cfg["fact"]
    n = f["fk1"].numel()
    sets, set_host = [], []
    for fk, d in (("fk1", cfg["d1"]), ("fk2", cfg["d2"]), ("fk3", cfg["d3"])):
        keep = d["pk"][d["attr"] < cfg["attr_cut"]]
        nb = d["pk"].numel()
        bits = torch.empty(tqp.keyset_words(nb), dtype=torch.int32, device="cuda")
        tqp.keyset_build_into(keep, 0, nb, bits)
        sets.append((bits, 0, nb))
        set_host.append(keep.cpu().numpy())
    keys = [f["fk1"], f["fk2"], f["fk3"]]
    rows = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    kout = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in keys]
    ws = torch.empty(tqp.semijoin_workspace_bytes(n, torch.int32), dtype=torch.uint8,
                     device="cuda")
    tqp.semijoin_into(keys, sets, rows, cnt, ws, keys_out=kout)
    k = int(cnt.item())
    assert 4_000_000 < k < 5_600_000
    got = host(rows[:k])
    assert np.all(np.diff(got) > 0)
    # sampled blocks, first and last included
    blk = 1 << 20
    starts = [0, n - blk] + [int(x) * blk for x in dg.uniform_int(0, 99, 6, 1, n // blk - 1, np.int64)]
    for st in starts:
        hk = [t[st:st + blk].cpu().numpy() for t in keys]
        want = oracle.semijoin_rows(hk, set_host) + st
        lo = int(np.searchsorted(got, st))
        assert np.array_equal(got[lo:lo + len(want)], want)
        for t, hkt in zip(kout, hk):
            assert np.array_equal(host(t[lo:lo + len(want)]), hkt[want - st])
    # everywhere: every kept row satisfies all three sets, and the kept count
    # is the number of rows that do (membership by table look-up, in chunks)
    member = [np.zeros(s[2], bool) for s in sets]
    for m, sh in zip(member, set_host):
        m[sh] = True
    kh = [host(t[:k]) for t in kout]
    for m, col in zip(member, kh):
        assert m[col].all()
    total = 0
    for st in range(0, n, 1 << 26):
        ok = np.ones(min(1 << 26, n - st), bool)
        for m, t in zip(member, keys):
            ok &= m[t[st:st + (1 << 26)].cpu().numpy()]
        total += int(ok.sum())
    assert total == k


@pytest.mark.parametrize("wg", [1, 2, 4])
@pytest.mark.parametrize("kdt", [np.int32, np.int64])
@pytest.mark.parametrize("nsets", [1, 3])
def test_semijoin_workgroup_sizes(tqp, wg, kdt, nsets):
    # every workgroup size (tile size) gives the same bytes; knobs restored after
    knobs = tqp.tune_knobs()
    try:
        tqp.tune_set("semijoin.wg", wg)
        n = 70_001 + 13 * wg
        dims = [(1 << 18, 1 << 14), (3000, 600), (25, 5)][:nsets]
        keys, set_keys, ranges = [], [], []
        for s, (dn, keep) in enumerate(dims):
            keys.append(dg.uniform_int(wg + s, 31 + s, n, 0, dn, kdt))
            set_keys.append(dg.permutation(17 + s, 3, dn)[:keep].astype(kdt))
            ranges.append((0, dn))
        check(tqp, keys, set_keys, ranges, payload=[dg.uniform_int(wg, 9, n, 1, 5001, np.int64)])
    finally:
        for name in ("semijoin.wg", "semijoin.per_cu"):
            tqp.tune_set(name, knobs[name][0])
