"""Python binding of libtqp: the MI355X relational hot path.

Argument marshalling only: every operator runs in the HIP kernels of
``libtqp.so`` (built by ``paper_2209_04579_amd.build``).  Tensors are device
memory from PyTorch; the stream is PyTorch's current HIP stream.  Importing the
module does not need a GPU; calling an operator does, and fails loudly if the
library is missing.

Two layers:
  * ``*_into`` functions take preallocated outputs and workspace, enqueue the
    kernels and return immediately (counts stay on the device);
  * convenience functions allocate, run, read the counts back and return
    trimmed tensors (one synchronization).
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "TqpError", "lib", "library_path", "filter", "filter_into", "gather_into", "gather",
    "pack_key_into", "sort", "sort_into", "filter_sort_into", "join", "join_into", "join_ranges",
    "groupby_agg", "groupby_agg_into", "keyset_build_into", "semijoin_into", "minmax",
    "minmax_into", "lower_bound_into", "batch_plan", "batch_capture", "Graph", "OPS", "DTYPES",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtqp.so")

TQP_OK, TQP_EINVAL, TQP_ECAPACITY, TQP_EHIP = 0, 1, 2, 3
DTYPES = {torch.int8: 1, torch.int32: 2, torch.int64: 3}
OPS = {"<": 0, "<=": 1, ">": 2, ">=": 3, "==": 4, "!=": 5}
AGGS = {"sum": 0, "count": 1, "sum_product": 2, "sum_diff_product": 3}
JOIN_SORTED, JOIN_RANGES = 1, 2
GB_SORTED, GB_DENSE = 1, 2
GB_DENSE_MAX = 4096


class TqpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libtqp error {code}: {msg}")
        self.code = code


class Col(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("len", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Pred(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("op", ctypes.c_int32), ("literal", ctypes.c_int64)]


class Agg(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("c", ctypes.c_int32)]


class KeyTerm(ctypes.Structure):
    _fields_ = [("col", Col), ("rows", ctypes.c_void_p), ("mod", ctypes.c_int64),
                ("mul", ctypes.c_int64)]


class Ranges(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("lstart", ctypes.c_void_p),
                ("lcnt", ctypes.c_void_p), ("rstart", ctypes.c_void_p),
                ("rcnt", ctypes.c_void_p)]


class BatchLayout(ctypes.Structure):
    _fields_ = [("fact_off", ctypes.c_void_p), ("dim_off", ctypes.c_void_p),
                ("key_shift", ctypes.c_int32), ("cat_shift", ctypes.c_int32),
                ("fact_rows", ctypes.c_int64), ("dim_rows", ctypes.c_int64)]


class KeySet(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("lo", ctypes.c_int64), ("nbits", ctypes.c_int64)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Loads libtqp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: build it with paper_2209_04579_amd.build.build() "
                "(the operators have no other implementation)")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i64, i32, u32, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                 ctypes.c_uint32, ctypes.c_size_t)
        P = ctypes.POINTER
        L.tqp_last_error.restype = ctypes.c_char_p
        L.tqp_version.restype = ctypes.c_char_p
        L.tqp_filter_workspace_bytes.restype = sz
        L.tqp_filter_workspace_bytes.argtypes = [i64]
        L.tqp_mlp_predict.restype = i32
        L.tqp_mlp_predict.argtypes = [P(Col), i32, vp, i64, vp, vp, i32, i32, vp, vp]
        L.tqp_str_match.restype = i32
        L.tqp_str_match.argtypes = [vp, i64, i32, ctypes.c_char_p, i32, i32, vp, vp]
        L.tqp_filter_sum.restype = i32
        L.tqp_filter_sum.argtypes = [P(Col), i32, P(Pred), i32, P(Col), P(Col), vp, vp, vp]
        L.tqp_filter.restype = i32
        L.tqp_filter.argtypes = [P(Col), i32, P(Pred), i32, P(Col), P(Col), i32, vp, vp,
                                 vp, sz, vp]
        L.tqp_gather.restype = i32
        L.tqp_gather.argtypes = [P(Col), vp, i64, vp, P(Col), vp]
        L.tqp_pack_key.restype = i32
        L.tqp_pack_key.argtypes = [P(KeyTerm), i32, i64, vp, P(Col), vp]
        L.tqp_sort_workspace_bytes.restype = sz
        L.tqp_sort_workspace_bytes.argtypes = [i64, i32, i32]
        L.tqp_sort.restype = i32
        L.tqp_sort.argtypes = [P(Col), vp, i64, vp, i32, i64, P(Col), vp, P(Col), P(Col), i32,
                               vp, sz, vp]
        L.tqp_filter_sort.restype = i32
        L.tqp_filter_sort.argtypes = [P(Col), i32, P(Pred), i32, P(Col), i32, i64, P(Col), vp,
                                      P(Col), P(Col), i32, vp, vp, sz, vp]
        L.tqp_join_workspace_bytes.restype = sz
        L.tqp_join_workspace_bytes.argtypes = [i64, i64, i32, u32, i64]
        L.tqp_join.restype = i32
        L.tqp_join.argtypes = [P(Col), vp, vp, P(Col), vp, vp, u32, vp, vp, vp, i64, vp,
                               P(Ranges), i64, vp, vp, sz, vp]
        L.tqp_groupby_workspace_bytes.restype = sz
        L.tqp_groupby_workspace_bytes.argtypes = [i64, i32, i32, u32, i64]
        L.tqp_tune_set.restype = i32
        L.tqp_tune_set.argtypes = [ctypes.c_char_p, i32]
        L.tqp_tune_get.restype = i32
        L.tqp_tune_get.argtypes = [ctypes.c_char_p, P(ctypes.c_int), P(ctypes.c_int),
                                   P(ctypes.c_int)]
        L.tqp_tune_name.restype = ctypes.c_char_p
        L.tqp_tune_name.argtypes = [i32]
        L.tqp_profile_enable.restype = None
        L.tqp_profile_enable.argtypes = [i32]
        L.tqp_profile_collect.restype = i32
        L.tqp_profile_collect.argtypes = [ctypes.c_char_p, sz]
        L.tqp_profile_reset.restype = None
        L.tqp_profile_reset.argtypes = []
        L.tqp_groupby_agg.restype = i32
        L.tqp_groupby_agg.argtypes = [P(Col), vp, u32, i64, i64, P(Col), i32, vp, P(Agg), i32,
                                      P(Col), P(vp), vp, vp, sz, vp]
        L.tqp_groupby_terms_workspace_bytes.restype = sz
        L.tqp_groupby_terms_workspace_bytes.argtypes = [i32, i64]
        L.tqp_groupby_agg_terms.restype = i32
        L.tqp_groupby_agg_terms.argtypes = [P(KeyTerm), i32, i64, vp, i64, i64, P(Col), i32, vp,
                                            P(Agg), i32, P(Col), P(vp), vp, vp, sz, vp]
        L.tqp_lower_bound.restype = i32
        L.tqp_lower_bound.argtypes = [P(Col), vp, P(Col), vp, vp]
        L.tqp_batch_plan.restype = i32
        L.tqp_batch_plan.argtypes = [i32, vp, vp, i64, i64, P(BatchLayout)]
        L.tqp_batch_capture_begin.restype = i32
        L.tqp_batch_capture_begin.argtypes = [vp]
        L.tqp_batch_capture_end.restype = i32
        L.tqp_batch_capture_end.argtypes = [vp, P(vp)]
        L.tqp_batch_run.restype = i32
        L.tqp_batch_run.argtypes = [vp, vp]
        L.tqp_batch_destroy.restype = i32
        L.tqp_batch_destroy.argtypes = [vp]
        L.tqp_minmax.restype = i32
        L.tqp_minmax.argtypes = [P(Col), vp, vp, vp]
        L.tqp_keyset_build.restype = i32
        L.tqp_keyset_build.argtypes = [P(Col), vp, i64, i64, vp, vp]
        L.tqp_semijoin_workspace_bytes.restype = sz
        L.tqp_semijoin_workspace_bytes.argtypes = [i64, i32]
        L.tqp_semijoin_noalloc_max_rows.restype = i64
        L.tqp_semijoin_noalloc_max_rows.argtypes = [i32]
        L.tqp_semijoin_noalloc.restype = i32
        L.tqp_semijoin_noalloc.argtypes = [P(Col), P(KeySet), i32, P(Col), P(Col), P(Col), i32,
                                           vp, vp, vp]
        L.tqp_semijoin.restype = i32
        L.tqp_semijoin.argtypes = [P(Col), P(KeySet), i32, P(Col), P(Col), P(Col), i32, vp, vp,
                                   vp, sz, vp]
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers ----

def _check(rc: int):
    if rc != TQP_OK:
        raise TqpError(rc, lib().tqp_last_error().decode())


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _col(t: torch.Tensor) -> Col:
    if t.dtype not in DTYPES:
        raise TypeError(f"unsupported column dtype {t.dtype}")
    if not t.is_cuda or not t.is_contiguous() or t.dim() != 1:
        raise ValueError("columns must be contiguous 1-D device tensors")
    return Col(t.data_ptr(), t.numel(), DTYPES[t.dtype], 0)


def _cols(ts):
    arr = (Col * max(1, len(ts)))()
    for i, t in enumerate(ts):
        arr[i] = _col(t)
    return arr


def workspace(nbytes: int, device=None) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def _dev(t):
    return t.device


# ----------------------------------------------------------------- filter ----

def filter_into(cols, preds, payload_in, payload_out, out_rows, d_count, ws, stream=None):
    """Enqueues WHERE + compaction.  preds: [(col_index, op, literal)]."""
    pr = (Pred * len(preds))(*[Pred(c, OPS[op], int(lit)) for c, op, lit in preds])
    pin = _cols(payload_in)
    pout = _cols(payload_out)
    _check(lib().tqp_filter(_cols(cols), len(cols), pr, len(preds), pin, pout,
                            len(payload_in), _ptr(out_rows), _ptr(d_count), _ptr(ws),
                            ws.numel(), _stream(stream)))


def filter_workspace_bytes(n: int) -> int:
    return lib().tqp_filter_workspace_bytes(n)


def filter_sum_into(cols, preds, d_sum, d_count, a=None, b=None, stream=None):
    """Enqueues WHERE + SUM(a * b) (b None: SUM(a)) and COUNT(*) over the kept
    rows into the device int64 scalars d_sum and d_count; nothing is
    compacted.  preds: [(col_index, op, literal)], possibly empty."""
    pr = (Pred * max(len(preds), 1))(*[Pred(c, OPS[op], int(lit)) for c, op, lit in preds])
    _check(lib().tqp_filter_sum(_cols(cols), len(cols), pr, len(preds),
                                None if a is None else ctypes.byref(_col(a)),
                                None if b is None else ctypes.byref(_col(b)),
                                _ptr(d_sum), _ptr(d_count), _stream(stream)))


def mlp_predict_into(feats, model, hidden: int, classes: int, out, n=None, rows=None, d_n=None,
                     stream=None):
    """Enqueues PREDICT: out[i] = class of row rows[i] (or i) under the fp32
    one-hidden-layer MLP whose packed weights are the device float32 tensor
    model ([W1, b1, W2, b2])."""
    if model.dtype != torch.float32 or not model.is_cuda or not model.is_contiguous():
        raise ValueError("model must be a contiguous float32 device tensor")
    f = len(feats)
    if model.numel() != hidden * f + hidden + classes * hidden + classes:
        raise ValueError("model size does not match nfeat, hidden and classes")
    if n is None:
        n = rows.numel() if rows is not None else feats[0].numel()
    _check(lib().tqp_mlp_predict(_cols(feats), f, _ptr(rows), int(n), _ptr(d_n), _ptr(model),
                                 int(hidden), int(classes), _ptr(out), _stream(stream)))


STR_PREFIX, STR_EQUAL = 0, 1


def str_match_into(chars, pattern: bytes, out, mode: str = "prefix", stream=None):
    """Enqueues LIKE 'pattern%' (mode "prefix") or = 'pattern' ("equal") over
    the rows of an (n, m) uint8 device matrix; out: int8 device flags (n)."""
    if chars.dtype != torch.uint8 or chars.dim() != 2 or not chars.is_cuda or not chars.is_contiguous():
        raise ValueError("strings must be a contiguous (n, m) uint8 device tensor")
    if out.dtype != torch.int8 or out.numel() < chars.shape[0] or not out.is_cuda:
        raise ValueError("out must be an int8 device tensor with n entries")
    pattern = bytes(pattern)
    _check(lib().tqp_str_match(_ptr(chars), chars.shape[0], chars.shape[1], pattern, len(pattern),
                               {"prefix": STR_PREFIX, "equal": STR_EQUAL}[mode], _ptr(out),
                               _stream(stream)))


def filter(cols, preds, payload=(), want_rows=True):
    """Returns (row ids int32, [payload columns]) for rows where all preds hold."""
    n = cols[0].numel()
    dev = _dev(cols[0])
    rows = torch.empty(n, dtype=torch.int32, device=dev) if want_rows else None
    pout = [torch.empty(n, dtype=p.dtype, device=dev) for p in payload]
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    ws = workspace(filter_workspace_bytes(n), dev)
    filter_into(cols, preds, list(payload), pout, rows, cnt, ws)
    k = int(cnt.item())
    return (rows[:k] if rows is not None else None), [p[:k] for p in pout]


# ------------------------------------------------------------ statistics ----

def minmax_into(col, d_out, d_n=None, stream=None):
    """Enqueues d_out[0] = min, d_out[1] = max of the column (device int64 x 2)."""
    _check(lib().tqp_minmax(ctypes.byref(_col(col)), _ptr(d_n), _ptr(d_out), _stream(stream)))


def minmax(col):
    """(min, max) of a device column as Python ints, None when it is empty
    (reads the two values back: one synchronization)."""
    out = torch.empty(2, dtype=torch.int64, device=col.device)
    minmax_into(col, out)
    lo, hi = (int(v) for v in out.cpu().tolist())
    return None if lo > hi else (lo, hi)


# ------------------------------------------------------------------ batch ----

def lower_bound_into(sorted_keys, queries, out, d_n=None, stream=None):
    """Enqueues out[i] = number of the (first d_n) sorted keys below queries[i]."""
    _check(lib().tqp_lower_bound(ctypes.byref(_col(sorted_keys)), _ptr(d_n),
                                 ctypes.byref(_col(queries)), _ptr(out), _stream(stream)))


def batch_plan(fact_rows, dim_rows, max_key: int, max_cat: int) -> dict:
    """The arena layout of k instances (libtqp's tqp_batch_plan, host only)."""
    k = len(fact_rows)
    if len(dim_rows) != k:
        raise ValueError("one dimension size per instance")
    fo, do = (ctypes.c_int64 * (k + 1))(), (ctypes.c_int64 * (k + 1))()
    lay = BatchLayout(ctypes.cast(fo, ctypes.c_void_p), ctypes.cast(do, ctypes.c_void_p),
                      0, 0, 0, 0)
    fr = (ctypes.c_int64 * max(k, 1))(*[int(x) for x in fact_rows])
    dr = (ctypes.c_int64 * max(k, 1))(*[int(x) for x in dim_rows])
    _check(lib().tqp_batch_plan(k, fr, dr, int(max_key), int(max_cat), ctypes.byref(lay)))
    return {"fact_off": list(fo), "dim_off": list(do), "key_shift": lay.key_shift,
            "cat_shift": lay.cat_shift, "fact_rows": lay.fact_rows, "dim_rows": lay.dim_rows}


class Graph:
    """A captured plan (tqp_batch_capture_end's handle), replayed by run()."""

    def __init__(self, handle: int):
        self.handle = handle

    def run(self, stream=None):
        _check(lib().tqp_batch_run(self.handle, _stream(stream)))

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.tqp_batch_destroy(self.handle)
            self.handle = None


def batch_capture(fn, stream=None) -> Graph:
    """Records every library call fn() enqueues into one graph (on a side
    stream; fn must not allocate or synchronize) and returns it."""
    s = stream or torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        _check(lib().tqp_batch_capture_begin(s.cuda_stream))
        h = ctypes.c_void_p()
        try:
            fn()
        finally:
            rc = lib().tqp_batch_capture_end(s.cuda_stream, ctypes.byref(h))
        _check(rc)
    torch.cuda.current_stream().wait_stream(s)
    return Graph(h.value)


# -------------------------------------------------------------- semi-join ----

def keyset_words(nbits: int) -> int:
    """uint32 words of a key set over nbits keys."""
    return (int(nbits) + 31) // 32


def keyset_build_into(key, lo: int, nbits: int, bits, d_n=None, stream=None):
    """Enqueues the key set {key[i] : i < count} over [lo, lo + nbits) into the
    device int32 tensor bits (keyset_words(nbits) words); keys outside the
    range are ignored."""
    if nbits > 0 and (bits.dtype != torch.int32 or bits.numel() < keyset_words(nbits)
                      or not bits.is_cuda):
        raise ValueError("bits must be an int32 device tensor of keyset_words(nbits) words")
    _check(lib().tqp_keyset_build(ctypes.byref(_col(key)), _ptr(d_n), int(lo), int(nbits),
                                  _ptr(bits), _stream(stream)))


def semijoin_workspace_bytes(n: int, dtype) -> int:
    return lib().tqp_semijoin_workspace_bytes(int(n), DTYPES[dtype])


def semijoin_into(keys, sets, out_rows, d_count, ws, keys_out=None, payload_in=(),
                  payload_out=(), stream=None):
    """Enqueues the semi-join reduction: rows i where keys[s][i] is in sets[s]
    for every s, compacted in ascending order.  sets: [(bits, lo, nbits)];
    keys_out: optional list (entries may be None) of compacted key columns."""
    ns = len(keys)
    if len(sets) != ns:
        raise ValueError("one key set per key column")
    ks = (KeySet * ns)(*[KeySet(_ptr(b) if int(nb) > 0 else None, int(lo), int(nb))
                         for b, lo, nb in sets])
    ko = None
    if keys_out is not None:
        ko = (Col * ns)()
        for i, t in enumerate(keys_out):
            ko[i] = _col(t) if t is not None else Col(None, 0, 0, 0)
    _check(lib().tqp_semijoin(_cols(keys), ks, ns, ko, _cols(list(payload_in)),
                              _cols(list(payload_out)), len(payload_in), _ptr(out_rows),
                              _ptr(d_count), _ptr(ws), ws.numel(), _stream(stream)))


def semijoin_noalloc_max_rows(dtype) -> int:
    return lib().tqp_semijoin_noalloc_max_rows(DTYPES[dtype])


def semijoin_noalloc_into(keys, sets, out_rows, d_count, keys_out=None, payload_in=(),
                          payload_out=(), stream=None):
    """semijoin_into without a workspace: the library's static scratch is used
    (calls that overlap on one device race)."""
    ns = len(keys)
    if len(sets) != ns:
        raise ValueError("one key set per key column")
    ks = (KeySet * ns)(*[KeySet(_ptr(b) if int(nb) > 0 else None, int(lo), int(nb))
                         for b, lo, nb in sets])
    ko = None
    if keys_out is not None:
        ko = (Col * ns)()
        for i, t in enumerate(keys_out):
            ko[i] = _col(t) if t is not None else Col(None, 0, 0, 0)
    _check(lib().tqp_semijoin_noalloc(_cols(keys), ks, ns, ko, _cols(list(payload_in)),
                                      _cols(list(payload_out)), len(payload_in), _ptr(out_rows),
                                      _ptr(d_count), _stream(stream)))


# ----------------------------------------------------------------- gather ----

def gather_into(src, idx, n, dst, d_n=None, stream=None):
    _check(lib().tqp_gather(ctypes.byref(_col(src)), _ptr(idx), int(n), _ptr(d_n),
                            ctypes.byref(_col(dst)), _stream(stream)))


def gather(src, idx):
    out = torch.empty(idx.numel(), dtype=src.dtype, device=src.device)
    gather_into(src, idx, idx.numel(), out)
    return out


def pack_key_into(terms, n, out, d_n=None, stream=None):
    """terms: [(column or None, rows or None, mod, mul)] -> out[i] = sum mul * f(col[row]).

    A term with column None adds the constant mul.  out is int32 or int64."""
    _check(lib().tqp_pack_key(_terms(terms), len(terms), int(n), _ptr(d_n),
                              ctypes.byref(_col(out)), _stream(stream)))


# ------------------------------------------------------------------- sort ----

def sort_workspace_bytes(n: int, dtype, pay_bytes: int = 0) -> int:
    return lib().tqp_sort_workspace_bytes(n, DTYPES[dtype], int(pay_bytes))


def pay_bytes_of(cols) -> int:
    return sum(c.element_size() for c in cols)


def sort_into(key, in_rows, n, out_key, out_rows, ws, d_n=None, key_bits=0, key_min=0,
              pay_in=(), pay_out=(), stream=None):
    _check(lib().tqp_sort(ctypes.byref(_col(key)), _ptr(in_rows), int(n), _ptr(d_n),
                          int(key_bits), int(key_min), ctypes.byref(_col(out_key)),
                          _ptr(out_rows), _cols(list(pay_in)), _cols(list(pay_out)),
                          len(pay_in), _ptr(ws), ws.numel(), _stream(stream)))


def filter_sort_into(cols, preds, key, out_key, out_rows, d_count, ws, key_bits=0, key_min=0,
                     pay_in=(), pay_out=(), stream=None):
    """Enqueues WHERE then the stable sort by key of the kept rows, in one
    operator: out_key / out_rows / pay_out hold the kept rows sorted, d_count
    their number.  preds: [(col_index, op, literal)]; workspace as for the
    sort of key.numel() rows."""
    pr = (Pred * len(preds))(*[Pred(c, OPS[op], int(lit)) for c, op, lit in preds])
    _check(lib().tqp_filter_sort(_cols(cols), len(cols), pr, len(preds),
                                 ctypes.byref(_col(key)), int(key_bits), int(key_min),
                                 ctypes.byref(_col(out_key)), _ptr(out_rows),
                                 _cols(list(pay_in)), _cols(list(pay_out)), len(pay_in),
                                 _ptr(d_count), _ptr(ws), ws.numel(), _stream(stream)))


def sort(key, in_rows=None, key_bits=0, key_min=0, payload=(), want_rows=True):
    """Stable ascending sort: returns (sorted keys, carried row ids, [payloads])."""
    n = key.numel()
    ok = torch.empty_like(key)
    orows = torch.empty(n, dtype=torch.int32, device=key.device) if want_rows else None
    pout = [torch.empty_like(p[:n]) for p in payload]
    ws = workspace(sort_workspace_bytes(n, key.dtype, pay_bytes_of(payload)), key.device)
    sort_into(key, in_rows, n, ok, orows, ws, key_bits=key_bits, key_min=key_min,
              pay_in=payload, pay_out=pout)
    if payload:
        return ok, orows, pout
    return ok, orows


# ------------------------------------------------------------------- join ----

def join_workspace_bytes(nl, nr, dtype, flags, cap=0) -> int:
    return lib().tqp_join_workspace_bytes(nl, nr, DTYPES[dtype], flags, int(cap))


def join_into(lkey, rkey, flags, out_l, out_r, out_key, cap, d_count, ws, lrows=None,
              rrows=None, d_nl=None, d_nr=None, ranges=None, range_cap=0, d_nranges=None,
              stream=None):
    rg = None
    if ranges is not None:
        rg = Ranges(*[r.data_ptr() for r in ranges])
    _check(lib().tqp_join(ctypes.byref(_col(lkey)), _ptr(lrows), _ptr(d_nl),
                          ctypes.byref(_col(rkey)), _ptr(rrows), _ptr(d_nr), int(flags),
                          _ptr(out_l), _ptr(out_r), _ptr(out_key), int(cap), _ptr(d_count),
                          ctypes.byref(rg) if rg is not None else None, int(range_cap),
                          _ptr(d_nranges), _ptr(ws), ws.numel(), _stream(stream)))


def join(lkey, rkey, lrows=None, rrows=None, sorted_inputs=False, cap=None, with_key=False):
    """Pairs (L row, R row[, key]) of the inner equi-join, in (key, i, j) order.

    Re-runs once with the exact capacity when the first guess is too small.
    """
    dev = lkey.device
    flags = JOIN_SORTED if sorted_inputs else 0
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    cap = int(cap if cap is not None else max(lkey.numel(), rkey.numel(), 1))
    for _ in range(2):
        ws = workspace(join_workspace_bytes(lkey.numel(), rkey.numel(), lkey.dtype, flags, cap),
                       dev)
        ol = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        orr = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        ok = torch.empty(max(cap, 1), dtype=lkey.dtype, device=dev) if with_key else None
        join_into(lkey, rkey, flags, ol, orr, ok, cap, cnt, ws, lrows=lrows, rrows=rrows)
        total = int(cnt.item())
        if total <= cap:
            out = (ol[:total], orr[:total])
            return out + ((ok[:total],) if with_key else ())
        cap = total
    raise TqpError(TQP_ECAPACITY, "join output did not fit after a retry")


def join_ranges(lkey_sorted, rkey_sorted):
    """Ranges form over two ascending key columns: dict of int64 tensors + total."""
    dev = lkey_sorted.device
    flags = JOIN_SORTED | JOIN_RANGES
    cap = max(1, min(lkey_sorted.numel(), rkey_sorted.numel()))
    rng = [torch.empty(cap, dtype=torch.int64, device=dev) for _ in range(5)]
    nr = torch.empty(1, dtype=torch.int64, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    ws = workspace(join_workspace_bytes(lkey_sorted.numel(), rkey_sorted.numel(),
                                        lkey_sorted.dtype, flags), dev)
    join_into(lkey_sorted, rkey_sorted, flags, None, None, None, 0, cnt, ws, ranges=rng,
              range_cap=cap, d_nranges=nr)
    m = int(nr.item())
    out = {k: r[:m] for k, r in zip(("key", "lstart", "lcnt", "rstart", "rcnt"), rng)}
    out["total"] = int(cnt.item())
    return out


# --------------------------------------------------------------- group-by ----

def groupby_workspace_bytes(n, dtype, nagg, flags, key_span=0) -> int:
    return lib().tqp_groupby_workspace_bytes(n, DTYPES[dtype], nagg, flags, key_span)


def _aggs(aggs):
    arr = (Agg * len(aggs))()
    for i, a in enumerate(aggs):
        c = int(a[3]) if len(a) > 3 else 0
        if not -(1 << 31) <= c < (1 << 31):
            raise ValueError("the aggregate's constant must fit int32")
        arr[i] = Agg(AGGS[a[0]], a[1] if len(a) > 1 else 0, a[2] if len(a) > 2 else 0, c)
    return arr


def groupby_agg_into(key, vals, aggs, out_key, out_aggs, d_ngroups, ws, flags=0, key_lo=0,
                     key_span=0, val_rows=None, d_n=None, stream=None):
    outs = (ctypes.c_void_p * len(out_aggs))(*[o.data_ptr() for o in out_aggs])
    _check(lib().tqp_groupby_agg(ctypes.byref(_col(key)), _ptr(d_n), int(flags), int(key_lo),
                                 int(key_span), _cols(vals), len(vals), _ptr(val_rows),
                                 _aggs(aggs), len(aggs), ctypes.byref(_col(out_key)), outs,
                                 _ptr(d_ngroups), _ptr(ws), ws.numel(), _stream(stream)))


def _terms(terms):
    arr = (KeyTerm * len(terms))()
    for i, (c, rows, mod, mul) in enumerate(terms):
        col = _col(c) if c is not None else Col(None, 0, 3, 0)
        arr[i] = KeyTerm(col, _ptr(rows), int(mod), int(mul))
    return arr


def groupby_terms_workspace_bytes(nagg, key_span) -> int:
    return lib().tqp_groupby_terms_workspace_bytes(int(nagg), int(key_span))


def groupby_agg_terms_into(terms, n, vals, aggs, out_key, out_aggs, d_ngroups, ws, key_lo,
                           key_span, val_rows=None, d_n=None, stream=None):
    """Dense GROUP BY over the packed key of `terms` (as pack_key_into), not materialised."""
    outs = (ctypes.c_void_p * len(out_aggs))(*[o.data_ptr() for o in out_aggs])
    _check(lib().tqp_groupby_agg_terms(_terms(terms), len(terms), int(n), _ptr(d_n), int(key_lo),
                                       int(key_span), _cols(vals), len(vals), _ptr(val_rows),
                                       _aggs(aggs), len(aggs), ctypes.byref(_col(out_key)), outs,
                                       _ptr(d_ngroups), _ptr(ws), ws.numel(), _stream(stream)))


def groupby_agg(key, vals, aggs, flags=0, key_lo=0, key_span=0, val_rows=None, cap=None):
    """GROUP BY key: returns (unique keys, [int64 aggregate tensors])."""
    dev = key.device
    n = key.numel()
    cap = int(cap if cap is not None else max(n, 1))
    ok = torch.empty(cap, dtype=key.dtype, device=dev)
    outs = [torch.empty(cap, dtype=torch.int64, device=dev) for _ in aggs]
    ng = torch.empty(1, dtype=torch.int64, device=dev)
    ws = workspace(groupby_workspace_bytes(n, key.dtype, len(aggs), flags, key_span), dev)
    groupby_agg_into(key, list(vals), aggs, ok, outs, ng, ws, flags=flags, key_lo=key_lo,
                     key_span=key_span, val_rows=val_rows)
    g = int(ng.item())
    return ok[:g], [o[:g] for o in outs]


# ------------------------------------------------------------ tuning knobs ----

def tune_knobs() -> dict:
    """{knob name: (value, lo, hi)} for every library tuning knob."""
    L = lib()
    out = {}
    i = 0
    while True:
        name = L.tqp_tune_name(i)
        if not name:
            break
        v, lo, hi = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(L.tqp_tune_get(name, ctypes.byref(v), ctypes.byref(lo), ctypes.byref(hi)))
        out[name.decode()] = (v.value, lo.value, hi.value)
        i += 1
    return out


def tune_set(name: str, value: int):
    _check(lib().tqp_tune_set(name.encode(), int(value)))


# -------------------------------------------------------------- profiling ----

def profile_enable(on: bool = True):
    """Brackets every library kernel launch with HIP events (see tqp.h)."""
    lib().tqp_profile_enable(1 if on else 0)


def profile_reset():
    lib().tqp_profile_reset()


def profile_collect() -> dict:
    """{kernel name: (launches, total ms)} accumulated since the last reset."""
    L = lib()
    need = L.tqp_profile_collect(None, 0)
    buf = ctypes.create_string_buffer(need + 64)
    L.tqp_profile_collect(buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


# ------------------------------------------------------ learned partitioner ----

PART_LEARNED, PART_RADIX = 1, 2


def _bind_lcdf(L):
    vp, i64, i32, u32, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32,
                             ctypes.c_size_t)
    P = ctypes.POINTER
    L.tqp_lcdf_model_bytes.restype = sz
    L.tqp_lcdf_model_bytes.argtypes = [i32]
    L.tqp_lcdf_train_workspace_bytes.restype = sz
    L.tqp_lcdf_train_workspace_bytes.argtypes = [i64, i32]
    L.tqp_lcdf_train.restype = i32
    L.tqp_lcdf_train.argtypes = [P(Col), i32, i32, i32, i32, ctypes.c_float, vp, sz, vp, sz, vp]
    L.tqp_lcdf_buckets.restype = i32
    L.tqp_lcdf_buckets.argtypes = [vp, P(Col), i32, vp, vp]
    L.tqp_partition_sort_workspace_bytes.restype = sz
    L.tqp_partition_sort_workspace_bytes.argtypes = [i64, i32, i32]
    L.tqp_partition_sort.restype = i32
    L.tqp_partition_sort.argtypes = [P(Col), vp, u32, vp, i32, i32, i64, P(Col), vp, vp, vp, sz,
                                     vp]


def lcdf_train(cols, sample_stride=100, nleaf=1688, steps=50, lr=1e-2, stream=None):
    """Trains the learned CDF on the keys of cols (1 or 2 device columns).

    Returns the model as a device uint8 tensor."""
    L = lib()
    if not hasattr(L, "_lcdf_bound"):
        _bind_lcdf(L)
        L._lcdf_bound = True
    dev = cols[0].device
    model = torch.zeros(L.tqp_lcdf_model_bytes(nleaf), dtype=torch.uint8, device=dev)
    total = sum(c.numel() for c in cols)
    ws = workspace(L.tqp_lcdf_train_workspace_bytes(total, sample_stride), dev)
    _check(L.tqp_lcdf_train(_cols(cols), len(cols), sample_stride, nleaf, steps, float(lr),
                            model.data_ptr(), model.numel(), ws.data_ptr(), ws.numel(),
                            _stream(stream)))
    return model


def lcdf_model_info(model) -> dict:
    """Reads the training summary fields of a model (synchronizes)."""
    raw = model[:64].cpu().numpy()
    import numpy as np
    nleaf, steps = np.frombuffer(raw[16:24].tobytes(), dtype=np.int32)
    loss_first, loss_last, loss_best = np.frombuffer(raw[24:36].tobytes(), dtype=np.float32)
    return {"nleaf": int(nleaf), "steps": int(steps), "loss_first": float(loss_first),
            "loss_last": float(loss_last), "loss_best": float(loss_best)}


def lcdf_buckets(model, keys, bucket_bits, out=None, stream=None):
    L = lib()
    if not hasattr(L, "_lcdf_bound"):
        _bind_lcdf(L)
        L._lcdf_bound = True
    if out is None:
        out = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
    if out.dtype != torch.int32 or out.numel() < keys.numel() or not out.is_contiguous():
        raise ValueError("lcdf_buckets: out must be a contiguous int32 tensor of n entries")
    _check(L.tqp_lcdf_buckets(model.data_ptr(), ctypes.byref(_col(keys)), int(bucket_bits),
                              _ptr(out), _stream(stream)))
    return out


def partition_sort_into(key, in_rows, mode, model, bucket_bits, out_key, out_rows, ws,
                        key_bits=0, key_min=0, stream=None):
    """Stable sort by key-range buckets; returns the host stats dict (synchronizes)."""
    L = lib()
    if not hasattr(L, "_lcdf_bound"):
        _bind_lcdf(L)
        L._lcdf_bound = True
    st = (ctypes.c_int64 * 4)()
    _check(L.tqp_partition_sort(ctypes.byref(_col(key)), _ptr(in_rows), int(mode),
                                _ptr(model), int(bucket_bits), int(key_bits), int(key_min),
                                ctypes.byref(_col(out_key)), _ptr(out_rows), st, _ptr(ws),
                                ws.numel(), _stream(stream)))
    return {"max_bucket": st[0], "fallback_buckets": st[1], "fallback_keys": st[2],
            "single_valued_big": st[3]}


def partition_sort_workspace_bytes(n, dtype, bucket_bits):
    L = lib()
    if not hasattr(L, "_lcdf_bound"):
        _bind_lcdf(L)
        L._lcdf_bound = True
    return L.tqp_partition_sort_workspace_bytes(n, DTYPES[dtype], bucket_bits)


def partition_sort(key, mode=PART_LEARNED, model=None, bucket_bits=12, in_rows=None,
                   key_bits=0, key_min=0):
    """Returns (sorted keys, row ids, stats)."""
    n = key.numel()
    ok = torch.empty_like(key)
    rows = torch.empty(n, dtype=torch.int32, device=key.device)
    ws = workspace(partition_sort_workspace_bytes(n, key.dtype, bucket_bits), key.device)
    st = partition_sort_into(key, in_rows, mode, model, bucket_bits, ok, rows, ws,
                             key_bits=key_bits, key_min=key_min)
    return ok, rows, st
