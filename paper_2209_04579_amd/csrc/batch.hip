// Batched execution of many independent queries: the arena layout
// (tqp_batch_plan), the split of a batched result back into its instances
// (tqp_lower_bound), and the capture of a whole batched plan into one HIP
// graph that is then replayed with a single launch (tqp_batch_capture_begin,
// tqp_batch_capture_end, tqp_batch_run, tqp_batch_destroy).
#include "tqp_internal.hpp"

namespace tqp {

// out[i] = the number of the first count sorted keys below queries[i]: one
// thread per query, a binary search over the keys.
template <class K>
__global__ __launch_bounds__(256) void k_lower_bound(const K *__restrict__ keys, int64_t n,
                                                     const int64_t *d_n, const void *queries,
                                                     int qdt, int64_t nq, int64_t *out) {
    const int64_t cnt = count_of(d_n, n);
    const int qlg = dtype_lg(qdt);
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nq;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t q = sext_of(load_word(queries, qlg, i), qdt);
        int64_t lo = 0, hi = cnt;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (int64_t(keys[mid]) < q) lo = mid + 1;
            else hi = mid;
        }
        out[i] = lo;
    }
}

static int bits_of(int64_t v) {
    int b = 0;
    while (b < 63 && (v >> b) != 0) b++;
    return b;
}

}  // namespace tqp

using namespace tqp;

TQP_API int tqp_lower_bound(const tqp_col *sorted, const int64_t *d_n, const tqp_col *queries,
                            int64_t *out, void *stream) {
    clear_error();
    if (!sorted || !queries || (sorted->dtype != TQP_INT32 && sorted->dtype != TQP_INT64) ||
        sorted->len < 0 || (sorted->len > 0 && !sorted->data) ||
        !col_aligned(sorted->data, sorted->dtype))
        return set_error(TQP_EINVAL, "tqp_lower_bound: sorted must be an int32 or int64 column");
    if (!dtype_ok(queries->dtype) || queries->len < 0 || (queries->len > 0 && !queries->data) ||
        !col_aligned(queries->data, queries->dtype))
        return set_error(TQP_EINVAL, "tqp_lower_bound: bad query column");
    if (queries->len > 0 && !out) return set_error(TQP_EINVAL, "tqp_lower_bound: out is required");
    if (queries->len == 0) return TQP_OK;
    hipStream_t s = as_stream(stream);
    int64_t blocks = ceil_div(queries->len, 256);
    if (blocks > 1024) blocks = 1024;
    if (sorted->dtype == TQP_INT32)
        TQP_LAUNCH("lower_bound", k_lower_bound<int32_t>, dim3(unsigned(blocks)), dim3(256), 0, s,
                   static_cast<const int32_t *>(sorted->data), sorted->len, d_n, queries->data,
                   queries->dtype, queries->len, out);
    else
        TQP_LAUNCH("lower_bound", k_lower_bound<int64_t>, dim3(unsigned(blocks)), dim3(256), 0, s,
                   static_cast<const int64_t *>(sorted->data), sorted->len, d_n, queries->data,
                   queries->dtype, queries->len, out);
    return check_launch("tqp_lower_bound");
}

TQP_API int tqp_batch_plan(int k, const int64_t *fact_rows, const int64_t *dim_rows,
                           int64_t max_key, int64_t max_cat, tqp_batch_layout *out) {
    clear_error();
    if (k < 1 || !fact_rows || !dim_rows || !out || !out->fact_off || !out->dim_off)
        return set_error(TQP_EINVAL, "tqp_batch_plan: k >= 1 instances and the offset arrays are required");
    if (max_key < 0 || max_cat < 0)
        return set_error(TQP_EINVAL, "tqp_batch_plan: keys and categories must be non-negative");
    int64_t f = 0, d = 0;
    out->fact_off[0] = 0;
    out->dim_off[0] = 0;
    for (int i = 0; i < k; i++) {
        if (fact_rows[i] < 0 || dim_rows[i] < 0)
            return set_error(TQP_EINVAL, "tqp_batch_plan: instance %d has a negative size", i);
        f += fact_rows[i];
        d += dim_rows[i];
        out->fact_off[i + 1] = f;
        out->dim_off[i + 1] = d;
    }
    const int kb = bits_of(int64_t(k - 1));
    const int key_bits = bits_of(max_key) > 0 ? bits_of(max_key) : 1;
    const int cat_bits = bits_of(max_cat) > 0 ? bits_of(max_cat) : 1;
    if (key_bits + kb > 31 || cat_bits + kb > 31)
        return set_error(TQP_EINVAL,
                         "tqp_batch_plan: %d instances with %d-bit keys / %d-bit categories do "
                         "not fit instance-prefixed int32 keys", k, key_bits, cat_bits);
    if (f > INT32_MAX || d > INT32_MAX)
        return set_error(TQP_EINVAL, "tqp_batch_plan: the arena exceeds 2^31 - 1 rows");
    out->key_shift = key_bits;
    out->cat_shift = cat_bits;
    out->fact_rows = f;
    out->dim_rows = d;
    return TQP_OK;
}

TQP_API int tqp_batch_capture_begin(void *stream) {
    clear_error();
    hipStream_t s = as_stream(stream);
    if (!s) return set_error(TQP_EINVAL, "tqp_batch_capture_begin: the null stream cannot be captured");
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return set_error(TQP_EHIP, "tqp_batch_capture_begin: %s", hipGetErrorString(e));
    return TQP_OK;
}

TQP_API int tqp_batch_capture_end(void *stream, void **graph) {
    clear_error();
    if (!graph) return set_error(TQP_EINVAL, "tqp_batch_capture_end: graph is required");
    *graph = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(as_stream(stream), &g);
    if (e != hipSuccess || !g)
        return set_error(TQP_EHIP, "tqp_batch_capture_end: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess)
        return set_error(TQP_EHIP, "tqp_batch_capture_end: instantiate: %s", hipGetErrorString(e));
    *graph = x;
    return TQP_OK;
}

TQP_API int tqp_batch_run(void *graph, void *stream) {
    clear_error();
    if (!graph) return set_error(TQP_EINVAL, "tqp_batch_run: graph is required");
    hipError_t e = hipGraphLaunch(static_cast<hipGraphExec_t>(graph), as_stream(stream));
    if (e != hipSuccess) return set_error(TQP_EHIP, "tqp_batch_run: %s", hipGetErrorString(e));
    return TQP_OK;
}

TQP_API int tqp_batch_destroy(void *graph) {
    clear_error();
    if (!graph) return TQP_OK;
    hipError_t e = hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph));
    if (e != hipSuccess) return set_error(TQP_EHIP, "tqp_batch_destroy: %s", hipGetErrorString(e));
    return TQP_OK;
}
