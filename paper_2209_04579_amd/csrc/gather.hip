// Gather (apply a row-id vector to a column) and packed-key projection.
// Both are one streaming pass over the index vector with one dependent read
// per element; indexes are read as 16-byte vectors, four per thread.
#include "tqp_internal.hpp"

namespace tqp {

constexpr int kGatherNT = 256;

template <class T>
__global__ __launch_bounds__(kGatherNT) void k_gather(const T *__restrict__ src, int64_t src_len,
                                                      const int32_t *__restrict__ idx, int64_t n,
                                                      const int64_t *d_n, T *__restrict__ dst) {
    const int64_t cnt = count_of(d_n, n);
    const int64_t nq = cnt / 4;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; q < nq; q += stride) {
        int4 ix = reinterpret_cast<const int4 *>(idx)[q];
        const int32_t r[4] = {ix.x, ix.y, ix.z, ix.w};
        T v[4];
#pragma unroll
        for (int k = 0; k < 4; k++)
            v[k] = (r[k] >= 0 && r[k] < src_len) ? src[r[k]] : T(0);
#pragma unroll
        for (int k = 0; k < 4; k++) dst[4 * q + k] = v[k];
    }
    const int64_t tail = nq * 4 + blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (tail < cnt) {
        const int32_t r = idx[tail];
        dst[tail] = (r >= 0 && r < src_len) ? src[r] : T(0);
    }
}

constexpr int kPackR = 4;

template <class O>
__global__ __launch_bounds__(kGatherNT) void k_pack_key(PackArgs a, int64_t n, const int64_t *d_n,
                                                        O *__restrict__ out) {
    constexpr int R = kPackR;
    const int64_t cnt = count_of(d_n, n);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x * R;
    for (int64_t base = blockIdx.x * int64_t(blockDim.x) * R; base < cnt; base += stride) {
        int64_t idx[R];
        uint64_t acc[R];
#pragma unroll
        for (int r = 0; r < R; r++) idx[r] = base + int64_t(r) * blockDim.x + threadIdx.x;
        pack_keys<R>(a, idx, cnt, acc);
#pragma unroll
        for (int r = 0; r < R; r++)
            if (idx[r] < cnt) out[idx[r]] = O(int64_t(acc[r]));
    }
}

static unsigned grid_for(int64_t work, int per_thread) {
    int64_t b = ceil_div(work > 0 ? work : 1, int64_t(kGatherNT) * per_thread);
    if (b > 16384) b = 16384;
    return unsigned(b);
}

int pack_args(const tqp_keyterm *terms, int nterms, int64_t n, PackArgs *a, const char *who) {
    *a = PackArgs{};
    for (int t = 0; t < nterms; t++) {
        const tqp_keyterm &k = terms[t];
        if (!k.col.data) {                          // constant term
            a->mul[t] = k.mul;
            continue;
        }
        if (!dtype_ok(k.col.dtype) || k.mod < 0 || !col_aligned(k.col.data, k.col.dtype) ||
            (k.rows && !col_aligned(k.rows, TQP_INT32)))
            return set_error(TQP_EINVAL, "%s: term %d is invalid or unaligned", who, t);
        if (!k.rows && k.col.len < n)
            return set_error(TQP_EINVAL, "%s: term %d column is shorter than n", who, t);
        a->col[t] = k.col.data;
        a->rows[t] = k.rows;
        a->len[t] = k.col.len;
        a->mod[t] = k.mod;
        a->mul[t] = k.mul;
        a->dt[t] = k.col.dtype;
    }
    a->nterms = nterms;
    return TQP_OK;
}

}  // namespace tqp

using namespace tqp;

TQP_API int tqp_gather(const tqp_col *src, const int32_t *idx, int64_t n, const int64_t *d_n,
                       const tqp_col *dst, void *stream) {
    clear_error();
    if (!src || !dst || n < 0 || (n > 0 && (!idx || !src->data || !dst->data)))
        return set_error(TQP_EINVAL, "tqp_gather: null argument or negative n");
    if (!dtype_ok(src->dtype) || src->dtype != dst->dtype)
        return set_error(TQP_EINVAL, "tqp_gather: src and dst need one valid dtype");
    if (dst->len < n) return set_error(TQP_ECAPACITY, "tqp_gather: dst holds %lld < %lld",
                                       (long long)dst->len, (long long)n);
    if (reinterpret_cast<uintptr_t>(idx) % 16 != 0)
        return set_error(TQP_EINVAL, "tqp_gather: idx must be 16-byte aligned");
    if (!col_aligned(src->data, src->dtype) || !col_aligned(dst->data, dst->dtype))
        return set_error(TQP_EINVAL, "tqp_gather: src and dst must be aligned to their dtype");
    if (n == 0) return TQP_OK;
    hipStream_t s = as_stream(stream);
    const unsigned g = grid_for(n, 4);
    switch (src->dtype) {
    case TQP_INT8:
        TQP_LAUNCH("gather", k_gather<int8_t>, dim3(g), dim3(kGatherNT), 0, s,
                           static_cast<const int8_t *>(src->data), src->len, idx, n, d_n,
                           static_cast<int8_t *>(dst->data));
        break;
    case TQP_INT32:
        TQP_LAUNCH("gather", k_gather<int32_t>, dim3(g), dim3(kGatherNT), 0, s,
                           static_cast<const int32_t *>(src->data), src->len, idx, n, d_n,
                           static_cast<int32_t *>(dst->data));
        break;
    default:
        TQP_LAUNCH("gather", k_gather<int64_t>, dim3(g), dim3(kGatherNT), 0, s,
                           static_cast<const int64_t *>(src->data), src->len, idx, n, d_n,
                           static_cast<int64_t *>(dst->data));
        break;
    }
    return check_launch("tqp_gather");
}

TQP_API int tqp_pack_key(const tqp_keyterm *terms, int nterms, int64_t n, const int64_t *d_n,
                         const tqp_col *out, void *stream) {
    clear_error();
    if (!terms || nterms < 1 || nterms > 4)
        return set_error(TQP_EINVAL, "tqp_pack_key: nterms must be in [1, 4]");
    if (n < 0 || !out || (out->dtype != TQP_INT32 && out->dtype != TQP_INT64) || out->len < n ||
        (n > 0 && !out->data))
        return set_error(TQP_EINVAL, "tqp_pack_key: bad output column");
    PackArgs a = {};
    const int rc = pack_args(terms, nterms, n, &a, "tqp_pack_key");
    if (rc) return rc;
    if (n == 0) return TQP_OK;
    hipStream_t s = as_stream(stream);
    if (out->dtype == TQP_INT32)
        TQP_LAUNCH("pack_key", k_pack_key<int32_t>, dim3(grid_for(n, 4 * kPackR)), dim3(kGatherNT), 0, s, a,
                   n, d_n, static_cast<int32_t *>(out->data));
    else
        TQP_LAUNCH("pack_key", k_pack_key<int64_t>, dim3(grid_for(n, 4 * kPackR)), dim3(kGatherNT), 0, s, a,
                   n, d_n, static_cast<int64_t *>(out->data));
    return check_launch("tqp_pack_key");
}
