"""The allocation-free semi-join entry point (tqp_semijoin_noalloc) against
the workspace one (tqp_semijoin), through the C ABI: identical kept rows,
keys and payload on two calls in a row, the second with a smaller table (the
static scratch keeps the first call's contents and must be cleared), plus
its size limit and the rejection of oversized tables."""
import numpy as np
import pytest

import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tqp():
    import paper_2209_04579_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def tables(seed, n, kdt):
    dims = [(200_000, 40_000), (3000, 600), (25, 5)]
    keys, sets = [], []
    for s, (dn, keep) in enumerate(dims):
        keys.append(dev(dg.uniform_int(seed + s, 1 + s, n, 0, dn, kdt)))
        pk = dev(dg.permutation(seed + 7 + s, 3, dn)[:keep].astype(kdt))
        import paper_2209_04579_amd as m
        bits = torch.empty(max(m.keyset_words(dn), 1), dtype=torch.int32, device="cuda")
        m.keyset_build_into(pk, 0, dn, bits)
        sets.append((bits, 0, dn))
    pay = [dev(dg.uniform_int(seed, 9, n, 1, 5001, np.int64)),
           dev(dg.uniform_int(seed, 10, n, -3, 3, np.int8))]
    return keys, sets, pay


def both(tqp, keys, sets, pay):
    n = keys[0].numel()
    out = []
    for noalloc in (False, True):
        rows = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
        cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        kout = [torch.empty(max(n, 1), dtype=k.dtype, device="cuda") for k in keys]
        pout = [torch.empty(max(n, 1), dtype=p.dtype, device="cuda") for p in pay]
        if noalloc:
            tqp.semijoin_noalloc_into(keys, sets, rows, cnt, keys_out=kout, payload_in=pay,
                                      payload_out=pout)
        else:
            ws = torch.empty(tqp.semijoin_workspace_bytes(n, keys[0].dtype), dtype=torch.uint8,
                             device="cuda")
            tqp.semijoin_into(keys, sets, rows, cnt, ws, keys_out=kout, payload_in=pay,
                              payload_out=pout)
        k = int(cnt.item())
        out.append([rows[:k].cpu().numpy()] + [t[:k].cpu().numpy() for t in kout + pout])
    return out


@pytest.mark.parametrize("kdt", [np.int32, np.int64])
def test_noalloc_matches_the_workspace_entry_on_two_calls(tqp, kdt):
    for seed, n in ((1, 3_000_017), (2, 40_001)):       # second call smaller
        keys, sets, pay = tables(seed, n, kdt)
        got, want = both(tqp, keys, sets, pay)[::-1]
        assert len(want[0]) > 0
        for g, w in zip(got, want):
            assert np.array_equal(g, w)


def test_noalloc_empty_table_after_a_large_one(tqp):
    keys, sets, pay = tables(3, 1_000_003, np.int32)
    both(tqp, keys, sets, pay)
    keys0 = [k[:0] for k in keys]
    pay0 = [p[:0] for p in pay]
    got, want = both(tqp, keys0, sets, pay0)[::-1]
    assert len(got[0]) == 0 and len(want[0]) == 0


def test_noalloc_limit_and_rejection(tqp):
    lim32 = tqp.semijoin_noalloc_max_rows(torch.int32)
    lim64 = tqp.semijoin_noalloc_max_rows(torch.int64)
    assert lim32 == 2 ** 31 - 1
    assert 10 ** 9 < lim64 < 2 ** 31 - 1
    # a descriptor longer than the limit is rejected before anything runs
    # (the address is never dereferenced: validation fails first)
    L = tqp.lib()
    col = tqp.Col(0x10000, lim64 + 1, 3, 0)
    ks = tqp.KeySet(None, 0, 0)
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    rc = L.tqp_semijoin_noalloc(tqp.ctypes.byref(col), tqp.ctypes.byref(ks), 1, None, None, None,
                                0, None, cnt.data_ptr(), None)
    assert rc == tqp.TQP_ECAPACITY
    assert b"static scratch" in L.tqp_last_error()
