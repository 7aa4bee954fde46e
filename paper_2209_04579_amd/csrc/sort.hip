// tqp_sort: stable ascending sort of signed int32 / int64 keys, the step under
// the sort-merge join and the sort-based group-by.  The keys are ranked on
// u = key - key_min (unsigned), which orders signed keys correctly and drops
// the bits that never vary; each 8-bit digit of u takes one stable pass of
// radix.hpp, least significant first.
#include "radix.hpp"

namespace tqp {

size_t sort_ws_bytes(int64_t n, int dtype, int key_bits, int pay_bytes) {
    Carver c(nullptr);
    c.take<int64_t>(2);                                   // key-range scratch
    c.take<char>(radix_ws_bytes(n, dtype_size(dtype), npass_for(key_bits), pay_bytes));
    return c.bytes();
}

size_t sort_ws_bytes(int64_t n, int dtype, int key_bits) { return sort_ws_bytes(n, dtype, key_bits, 0); }

static int sort_cols_impl(const void *key_in, int dtype, int64_t n, const int64_t *d_n, int key_bits,
                          int64_t key_min, void *key_out, const SortCols &sc, void *ws,
                          size_t ws_bytes, hipStream_t s, const PassPred *pred = nullptr,
                          int64_t *d_kept = nullptr) {
    const int width = dtype == TQP_INT32 ? 32 : 64;
    if (key_bits > width) key_bits = width;
    if (key_bits < 0) key_bits = 0;
    int pay_bytes = 0;
    for (int p = 0; p < sc.npay; p++) pay_bytes += dtype_size(sc.pdt[p]);
    const size_t need = sort_ws_bytes(n, dtype, key_bits, pay_bytes);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "sort: workspace needs %zu bytes", need);
    Carver cv(ws);
    cv.take<int64_t>(2);
    void *rws = cv.take<char>(radix_ws_bytes(n, dtype_size(dtype), npass_for(key_bits), pay_bytes));
    if (dtype == TQP_INT32)
        return run_radix<int32_t>(static_cast<const int32_t *>(key_in), n, d_n, key_bits,
                                  KeyOrd<int32_t>{int32_t(key_min)},
                                  static_cast<int32_t *>(key_out), sc, rws, s, pred, d_kept);
    return run_radix<int64_t>(static_cast<const int64_t *>(key_in), n, d_n, key_bits,
                              KeyOrd<int64_t>{key_min}, static_cast<int64_t *>(key_out), sc, rws, s,
                              pred, d_kept);
}

int sort_impl(const void *key_in, int dtype, const int32_t *rows_in, int64_t n, const int64_t *d_n,
              int key_bits, int64_t key_min, void *key_out, int32_t *rows_out, void *ws,
              size_t ws_bytes, hipStream_t s) {
    SortCols sc = {};
    sc.rows_in = rows_in;
    sc.rows_out = rows_out;
    return sort_cols_impl(key_in, dtype, n, d_n, key_bits, key_min, key_out, sc, ws, ws_bytes, s);
}

}  // namespace tqp

using namespace tqp;

TQP_API size_t tqp_sort_workspace_bytes(int64_t n, int dtype, int pay_bytes) {
    if (!dtype_ok(dtype) || n < 0 || pay_bytes < 0 || pay_bytes > 8 * kMaxSortPay) return 0;
    return sort_ws_bytes(n, dtype, dtype == TQP_INT32 ? 32 : 64, pay_bytes);
}

TQP_API int tqp_sort(const tqp_col *key, const int32_t *in_rows, int64_t n, const int64_t *d_n,
                     int key_bits, int64_t key_min, const tqp_col *out_key, int32_t *out_rows,
                     const tqp_col *pay_in, const tqp_col *pay_out, int npay, void *ws,
                     size_t ws_bytes, void *stream) {
    clear_error();
    if (!key || !out_key || (n > 0 && (!key->data || !out_key->data)))
        return set_error(TQP_EINVAL, "tqp_sort: null argument");
    if (key->dtype != TQP_INT32 && key->dtype != TQP_INT64)
        return set_error(TQP_EINVAL, "tqp_sort: keys must be int32 or int64");
    if (out_key->dtype != key->dtype)
        return set_error(TQP_EINVAL, "tqp_sort: out_key dtype differs from key dtype");
    if (n < 0 || n > (int64_t(1) << 30) - 1)
        return set_error(TQP_EINVAL, "tqp_sort: n must be in [0, 2^30 - 1]");
    if (key->len < n || out_key->len < n)
        return set_error(TQP_ECAPACITY, "tqp_sort: key or out_key shorter than n");
    if (key_bits < 0 || key_bits > 64)
        return set_error(TQP_EINVAL, "tqp_sort: key_bits must be in [0, 64]");
    if (npay < 0 || npay > kMaxSortPay || (npay > 0 && (!pay_in || !pay_out)))
        return set_error(TQP_EINVAL, "tqp_sort: npay must be in [0, %d] with both arrays", kMaxSortPay);
    if ((in_rows && !col_aligned(in_rows, TQP_INT32)) || (out_rows && !col_aligned(out_rows, TQP_INT32)))
        return set_error(TQP_EINVAL, "tqp_sort: row id arrays must be 4-byte aligned");
    SortCols sc = {};
    sc.rows_in = in_rows;
    sc.rows_out = out_rows;
    sc.npay = npay;
    int pay_bytes = 0;
    for (int p = 0; p < npay; p++) {
        if (!dtype_ok(pay_in[p].dtype) || pay_in[p].dtype != pay_out[p].dtype ||
            pay_in[p].len < n || pay_out[p].len < n ||
            (n > 0 && (!pay_in[p].data || !pay_out[p].data)) ||
            !col_aligned(pay_in[p].data, pay_in[p].dtype) || !col_aligned(pay_out[p].data, pay_out[p].dtype))
            return set_error(TQP_EINVAL, "tqp_sort: payload %d has a bad dtype, length or (unaligned) pointer", p);
        sc.pin[p] = pay_in[p].data;
        sc.pout[p] = pay_out[p].data;
        sc.pdt[p] = pay_in[p].dtype;
        pay_bytes += dtype_size(pay_in[p].dtype);
    }
    const size_t need = tqp_sort_workspace_bytes(n, key->dtype, pay_bytes);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "tqp_sort: workspace needs %zu bytes", need);
    if (n == 0) return TQP_OK;
    hipStream_t s = as_stream(stream);
    if (key_bits == 0) {
        int rc = derive_key_range(key->data, key->dtype, n, d_n, ws, s, &key_min, &key_bits);
        if (rc) return rc;
    }
    return sort_cols_impl(key->data, key->dtype, n, d_n, key_bits, key_min, out_key->data, sc, ws,
                          ws_bytes, s);
}

TQP_API int tqp_filter_sort(const tqp_col *cols, int ncols, const tqp_pred *preds, int npred,
                            const tqp_col *key, int key_bits, int64_t key_min,
                            const tqp_col *out_key, int32_t *out_rows, const tqp_col *pay_in,
                            const tqp_col *pay_out, int npay, int64_t *d_count, void *ws,
                            size_t ws_bytes, void *stream) {
    clear_error();
    if (!key || !out_key || !d_count)
        return set_error(TQP_EINVAL, "tqp_filter_sort: key, out_key and d_count are required");
    const int64_t n = key->len;
    if (key->dtype != TQP_INT32 && key->dtype != TQP_INT64)
        return set_error(TQP_EINVAL, "tqp_filter_sort: keys must be int32 or int64");
    if (out_key->dtype != key->dtype)
        return set_error(TQP_EINVAL, "tqp_filter_sort: out_key dtype differs from key dtype");
    if (n < 0 || n > (int64_t(1) << 30) - 1)
        return set_error(TQP_EINVAL, "tqp_filter_sort: key->len must be in [0, 2^30 - 1]");
    if (out_key->len < n || (n > 0 && (!key->data || !out_key->data)))
        return set_error(TQP_ECAPACITY, "tqp_filter_sort: out_key shorter than the table or null");
    if (!col_aligned(key->data, key->dtype) || !col_aligned(out_key->data, out_key->dtype) ||
        (out_rows && !col_aligned(out_rows, TQP_INT32)))
        return set_error(TQP_EINVAL, "tqp_filter_sort: key, out_key or out_rows unaligned");
    if (key_bits < 0 || key_bits > 64)
        return set_error(TQP_EINVAL, "tqp_filter_sort: key_bits must be in [0, 64]");
    if (!cols || ncols < 1 || ncols > 8)
        return set_error(TQP_EINVAL, "tqp_filter_sort: ncols must be in [1, 8]");
    if (!preds || npred < 1 || npred > kMaxSortPred)
        return set_error(TQP_EINVAL, "tqp_filter_sort: npred must be in [1, %d]", kMaxSortPred);
    for (int c = 0; c < ncols; c++)
        if (!dtype_ok(cols[c].dtype) || cols[c].len < n || (n > 0 && !cols[c].data) ||
            !col_aligned(cols[c].data, cols[c].dtype))
            return set_error(TQP_EINVAL, "tqp_filter_sort: column %d has a bad dtype, length or pointer", c);
    PassPred f = {};
    for (int q = 0; q < npred; q++) {
        if (preds[q].col < 0 || preds[q].col >= ncols || preds[q].op < TQP_LT || preds[q].op > TQP_NE)
            return set_error(TQP_EINVAL, "tqp_filter_sort: predicate %d is invalid", q);
        f.col[q] = cols[preds[q].col].data;
        f.dt[q] = cols[preds[q].col].dtype;
        f.op[q] = preds[q].op;
        f.lit[q] = preds[q].literal;
    }
    f.npred = npred;
    if (npay < 0 || npay > kMaxSortPay || (npay > 0 && (!pay_in || !pay_out)))
        return set_error(TQP_EINVAL, "tqp_filter_sort: npay must be in [0, %d] with both arrays",
                         kMaxSortPay);
    SortCols sc = {};
    sc.rows_out = out_rows;
    sc.npay = npay;
    int pay_bytes = 0;
    for (int p = 0; p < npay; p++) {
        if (!dtype_ok(pay_in[p].dtype) || pay_in[p].dtype != pay_out[p].dtype ||
            pay_in[p].len < n || pay_out[p].len < n ||
            (n > 0 && (!pay_in[p].data || !pay_out[p].data)) ||
            !col_aligned(pay_in[p].data, pay_in[p].dtype) || !col_aligned(pay_out[p].data, pay_out[p].dtype))
            return set_error(TQP_EINVAL, "tqp_filter_sort: payload %d has a bad dtype, length or (unaligned) pointer", p);
        sc.pin[p] = pay_in[p].data;
        sc.pout[p] = pay_out[p].data;
        sc.pdt[p] = pay_in[p].dtype;
        pay_bytes += dtype_size(pay_in[p].dtype);
    }
    const size_t need = tqp_sort_workspace_bytes(n, key->dtype, pay_bytes);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "tqp_filter_sort: workspace needs %zu bytes", need);
    hipStream_t s = as_stream(stream);
    if (n == 0) return fill_u64(d_count, 0, 1, s);
    if (key_bits == 0) {
        // the range of all n keys bounds the range of the kept ones
        int rc = derive_key_range(key->data, key->dtype, n, nullptr, ws, s, &key_min, &key_bits);
        if (rc) return rc;
    }
    if (key_bits < 1) key_bits = 1;       // the first pass also compacts, so one always runs
    return sort_cols_impl(key->data, key->dtype, n, nullptr, key_bits, key_min, out_key->data, sc,
                          ws, ws_bytes, s, &f, d_count);
}
