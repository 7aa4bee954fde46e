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
