"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tqp.h")
LIB = os.path.join(ROOT, "paper_2209_04579_amd", "libtqp.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tqp_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_operator_set():
    names = declared()
    for fn in ("tqp_filter", "tqp_sort", "tqp_join", "tqp_groupby_agg", "tqp_gather",
               "tqp_last_error"):
        assert fn in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtqp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.tqp_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.tqp_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtqp.so not built")
def test_argument_errors_are_reported_without_a_gpu():
    import paper_2209_04579_amd as tqp
    L = tqp.lib()
    # null descriptors: rejected before anything touches a device
    assert L.tqp_filter(None, 0, None, 0, None, None, 0, None, None, None, 0, None) == tqp.TQP_EINVAL
    assert b"ncols" in L.tqp_last_error()
    assert L.tqp_sort(None, None, 0, None, 0, 0, None, None, None, None, 0, None, 0,
                      None) == tqp.TQP_EINVAL
    assert L.tqp_groupby_workspace_bytes(10, 9, 1, 0, 0) == 0       # bad dtype
    assert L.tqp_filter_workspace_bytes(1 << 20) > 0
    assert L.tqp_sort_workspace_bytes(1 << 20, 2, 0) > 8 * (1 << 20)
    assert L.tqp_sort_workspace_bytes(1 << 20, 2, 17) > L.tqp_sort_workspace_bytes(1 << 20, 2, 0)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtqp.so not built")
def test_unaligned_columns_are_rejected_without_a_gpu():
    """Columns of run-time dtype are read as aligned 8-byte words, so a column
    not aligned to its element size is an argument error (the fake addresses
    below are never dereferenced: validation fails first)."""
    import paper_2209_04579_amd as tqp
    L = tqp.lib()
    # dtype codes of the C header: int32 = 2, int64 = 3
    key = tqp.Col(0x10000, 10, 2, 0)
    out = tqp.Col(0x20000, 10, 2, 0)
    pin = (tqp.Col * 1)(tqp.Col(0x30004, 10, 3, 0))
    pout = (tqp.Col * 1)(tqp.Col(0x40000, 10, 3, 0))
    rc = L.tqp_sort(ctypes.byref(key), None, 10, None, 8, 0, ctypes.byref(out), None, pin, pout,
                    1, None, 0, None)
    assert rc == tqp.TQP_EINVAL and b"unaligned" in L.tqp_last_error()
    rc = L.tqp_sort(ctypes.byref(key), ctypes.c_void_p(0x50002), 10, None, 8, 0,
                    ctypes.byref(out), ctypes.c_void_p(0x60000), None, None, 0, None, 0, None)
    assert rc == tqp.TQP_EINVAL and b"aligned" in L.tqp_last_error()
    term = (tqp.KeyTerm * 1)(tqp.KeyTerm(tqp.Col(0x70002, 10, 2, 0), None, 0, 1))
    out64 = tqp.Col(0x80000, 10, 3, 0)
    rc = L.tqp_pack_key(term, 1, 10, None, ctypes.byref(out64), None)
    assert rc == tqp.TQP_EINVAL and b"unaligned" in L.tqp_last_error()
    src = tqp.Col(0x90004, 10, 3, 0)
    rc = L.tqp_gather(ctypes.byref(src), ctypes.c_void_p(0xA0000), 10, None,
                      ctypes.byref(out64), None)
    assert rc == tqp.TQP_EINVAL and b"aligned to their dtype" in L.tqp_last_error()
    # filter: a predicate column, then a payload column, off their element size
    col = (tqp.Col * 1)(tqp.Col(0xB0002, 10, 2, 0))
    pred = (tqp.Pred * 1)(tqp.Pred(0, 0, 5))
    cnt = ctypes.c_void_p(0xC0000)
    ws = ctypes.c_void_p(0xD0000)
    rc = L.tqp_filter(col, 1, pred, 1, None, None, 0, None, cnt, ws, 1 << 20, None)
    assert rc == tqp.TQP_EINVAL and b"unaligned" in L.tqp_last_error()
    col = (tqp.Col * 1)(tqp.Col(0xB0000, 10, 2, 0))
    pin = (tqp.Col * 1)(tqp.Col(0xE0004, 10, 3, 0))
    pout = (tqp.Col * 1)(tqp.Col(0xF0000, 10, 3, 0))
    rc = L.tqp_filter(col, 1, pred, 1, pin, pout, 1, None, cnt, ws, 1 << 20, None)
    assert rc == tqp.TQP_EINVAL and b"payload 0 is unaligned" in L.tqp_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtqp.so not built")
def test_string_match_argument_errors_without_a_gpu():
    import paper_2209_04579_amd as tqp
    L = tqp.lib()
    fake = ctypes.c_void_p(0x10000)
    assert L.tqp_str_match(fake, 10, 8, b"A" * 65, 65, 0, fake, None) == tqp.TQP_EINVAL
    assert b"pattern length" in L.tqp_last_error()
    assert L.tqp_str_match(fake, 10, 0, b"A", 1, 0, fake, None) == tqp.TQP_EINVAL
    assert L.tqp_str_match(fake, 10, 8, b"A", 1, 7, fake, None) == tqp.TQP_EINVAL
    assert L.tqp_str_match(None, 0, 8, b"A", 1, 0, None, None) == tqp.TQP_OK   # empty: no launch


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtqp.so not built")
def test_predict_argument_errors_without_a_gpu():
    import paper_2209_04579_amd as tqp
    L = tqp.lib()
    f = (tqp.Col * 1)(tqp.Col(0x10000, 10, 2, 0))
    fake = ctypes.c_void_p(0x20000)
    assert L.tqp_mlp_predict(f, 0, None, 10, None, fake, 4, 2, fake, None) == tqp.TQP_EINVAL
    assert L.tqp_mlp_predict(f, 1, None, 10, None, fake, 65, 2, fake, None) == tqp.TQP_EINVAL
    assert L.tqp_mlp_predict(f, 1, None, 10, None, fake, 4, 9, fake, None) == tqp.TQP_EINVAL
    assert L.tqp_mlp_predict(f, 1, None, 11, None, fake, 4, 2, fake, None) == tqp.TQP_EINVAL
    assert L.tqp_mlp_predict(f, 1, None, 0, None, fake, 4, 2, fake, None) == tqp.TQP_OK


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtqp.so not built")
def test_filter_sort_argument_errors_without_a_gpu():
    """Rejected before anything is enqueued (the fake addresses are never
    dereferenced)."""
    import paper_2209_04579_amd as tqp
    L = tqp.lib()
    cols = (tqp.Col * 1)(tqp.Col(0x10000, 10, 2, 0))
    pred = (tqp.Pred * 5)(*[tqp.Pred(0, 0, 5)] * 5)
    key = tqp.Col(0x20000, 10, 2, 0)
    out = tqp.Col(0x30000, 10, 2, 0)
    cnt, ws = ctypes.c_void_p(0x40000), ctypes.c_void_p(0x50000)
    big = 1 << 30

    def call(c=cols, nc=1, p=pred, np_=1, k=key, o=out, c_=cnt, wsb=big):
        return L.tqp_filter_sort(c, nc, p, np_, ctypes.byref(k), 0, 0, ctypes.byref(o), None,
                                 None, None, 0, c_, ws, wsb, None)
    assert call(np_=0) == tqp.TQP_EINVAL and b"npred" in L.tqp_last_error()
    assert call(np_=5) == tqp.TQP_EINVAL
    assert call(nc=0) == tqp.TQP_EINVAL and b"ncols" in L.tqp_last_error()
    assert call(c_=None) == tqp.TQP_EINVAL and b"d_count" in L.tqp_last_error()
    assert call(o=tqp.Col(0x30000, 10, 3, 0)) == tqp.TQP_EINVAL
    assert call(o=tqp.Col(0x30000, 9, 2, 0)) == tqp.TQP_ECAPACITY
    assert call(k=tqp.Col(0x20002, 10, 2, 0)) == tqp.TQP_EINVAL and b"unaligned" in L.tqp_last_error()
    bad_pred = (tqp.Pred * 1)(tqp.Pred(1, 0, 5))
    assert call(p=bad_pred) == tqp.TQP_EINVAL and b"predicate 0" in L.tqp_last_error()
    short = (tqp.Col * 1)(tqp.Col(0x10000, 9, 2, 0))
    assert call(c=short) == tqp.TQP_EINVAL and b"column 0" in L.tqp_last_error()
    assert call(wsb=16) == tqp.TQP_ECAPACITY and b"workspace" in L.tqp_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtqp.so not built")
def test_batch_plan_layout_and_limits_without_a_gpu():
    import paper_2209_04579_amd as tqp
    lay = tqp.batch_plan([10, 0, 25], [3, 1, 0], 999, 24)
    assert lay["fact_off"] == [0, 10, 10, 35] and lay["dim_off"] == [0, 3, 4, 4]
    assert lay["key_shift"] == 10 and lay["cat_shift"] == 5
    assert (lay["fact_rows"], lay["dim_rows"]) == (35, 4)
    # 256 instances need 8 prefix bits: 24-bit keys fit, 24-bit keys + 1 do not
    assert tqp.batch_plan([1] * 256, [1] * 256, (1 << 23) - 1, 1)["key_shift"] == 23
    with pytest.raises(tqp.TqpError):
        tqp.batch_plan([1] * 256, [1] * 256, 1 << 23, 1)
    with pytest.raises(tqp.TqpError):
        tqp.batch_plan([1], [1], -1, 0)
    L = tqp.lib()
    assert L.tqp_batch_capture_begin(None) == tqp.TQP_EINVAL
    assert L.tqp_batch_run(None, None) == tqp.TQP_EINVAL
    assert L.tqp_batch_destroy(None) == tqp.TQP_OK
