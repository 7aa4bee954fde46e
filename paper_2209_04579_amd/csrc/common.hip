// Library-wide pieces: error text, fills, the key-range reduction.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "tqp_internal.hpp"

namespace tqp {

static thread_local char g_err[512];

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(TQP_EHIP, "%s: %s", what, hipGetErrorString(e));
    return TQP_OK;
}

int dtype_size(int dtype) {
    switch (dtype) {
    case TQP_INT8: return 1;
    case TQP_INT32: return 4;
    case TQP_INT64: return 8;
    default: return 0;
    }
}

bool dtype_ok(int dtype) { return dtype_size(dtype) != 0; }
bool col_aligned(const void *p, int dtype) {
    const int sz = dtype_size(dtype);
    return sz != 0 && reinterpret_cast<uintptr_t>(p) % uintptr_t(sz) == 0;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

int fill_u64(void *dst, uint64_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return TQP_OK;
    int64_t blocks = ceil_div(count, 256);
    if (blocks > 4096) blocks = 4096;
    TQP_LAUNCH("fill_u64", k_fill_u64, dim3(unsigned(blocks)), dim3(256), 0, s,
                       static_cast<uint64_t *>(dst), value, count);
    return check_launch("fill_u64");
}

int fill_u32(void *dst, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return TQP_OK;
    int64_t blocks = ceil_div(count, 256);
    if (blocks > 4096) blocks = 4096;
    TQP_LAUNCH("fill_u32", k_fill_u32, dim3(unsigned(blocks)), dim3(256), 0, s,
                       static_cast<uint32_t *>(dst), value, count);
    return check_launch("fill_u32");
}

// Clears the head words before p, then nsec sections of words: section k
// starts at p + k * stride and is cleared over its first ceil(count / per) *
// width words, count = min(*d_n, n).  Lets a call planned for capacity n
// clear only what its actual count will touch, together with the counters
// in front of the sections, in one launch.
__global__ void k_clear_sections(uint32_t *p, int64_t head, int nsec, int64_t stride,
                                 const int64_t *d_n, int64_t n, int64_t per, int64_t width) {
    const int64_t cnt = count_of(d_n, n);
    int64_t need = ceil_div(cnt > 0 ? cnt : 1, per) * width;
    if (need > stride) need = stride;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < head + need * nsec;
         i += int64_t(gridDim.x) * blockDim.x) {
        if (i < head) {
            p[i - head] = 0;
        } else {
            const int64_t j = i - head;
            p[(j / need) * stride + j % need] = 0;
        }
    }
}

int clear_sections(uint32_t *dst, int64_t head, int nsec, int64_t stride, const int64_t *d_n,
                   int64_t n, int64_t per, int64_t width, hipStream_t s) {
    if (head < 0) head = 0;
    if (nsec <= 0 || stride <= 0) return fill_u32(dst - head, 0, head, s);
    int64_t blocks = ceil_div(head + int64_t(nsec) * stride, 256);
    if (blocks > 2048) blocks = 2048;
    TQP_LAUNCH("clear_sections", k_clear_sections, dim3(unsigned(blocks)), dim3(256), 0, s, dst,
               head, nsec, stride, d_n, n, per, width);
    return check_launch("clear_sections");
}

// Min and max of the first count keys.  out[0], out[1] must hold INT64_MAX
// and INT64_MIN beforehand.
template <class K>
__global__ __launch_bounds__(256) void k_minmax(const K *key, int64_t n,
                                                const int64_t *d_n, int64_t *out) {
    const int64_t cnt = count_of(d_n, n);
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < cnt;
         i += int64_t(gridDim.x) * blockDim.x) {
        int64_t v = key[i];
        lo = v < lo ? v : lo;
        hi = v > hi ? v : hi;
    }
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        int64_t a = shfl_xor(lo, m), b = shfl_xor(hi, m);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    __shared__ int64_t slo[4], shi[4];
    if (lane_id() == 0) { slo[wave_id()] = lo; shi[wave_id()] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; w++) {
            lo = slo[w] < lo ? slo[w] : lo;
            hi = shi[w] > hi ? shi[w] : hi;
        }
        if (lo != INT64_MAX) atomicMin(reinterpret_cast<long long *>(&out[0]), (long long)lo);
        if (hi != INT64_MIN) atomicMax(reinterpret_cast<long long *>(&out[1]), (long long)hi);
    }
}

int launch_minmax(const void *key, int dtype, int64_t n, const int64_t *d_n,
                  int64_t *out, hipStream_t s) {
    int rc = fill_u64(out, uint64_t(INT64_MAX), 1, s);
    if (rc) return rc;
    rc = fill_u64(out + 1, uint64_t(INT64_MIN), 1, s);
    if (rc) return rc;
    if (n <= 0) return TQP_OK;
    int64_t blocks = ceil_div(n, 256 * 16);
    if (blocks > 2048) blocks = 2048;
    if (dtype == TQP_INT8)
        TQP_LAUNCH("minmax", k_minmax<int8_t>, dim3(unsigned(blocks)), dim3(256), 0, s,
                           static_cast<const int8_t *>(key), n, d_n, out);
    else if (dtype == TQP_INT32)
        TQP_LAUNCH("minmax", k_minmax<int32_t>, dim3(unsigned(blocks)), dim3(256), 0, s,
                           static_cast<const int32_t *>(key), n, d_n, out);
    else
        TQP_LAUNCH("minmax", k_minmax<int64_t>, dim3(unsigned(blocks)), dim3(256), 0, s,
                           static_cast<const int64_t *>(key), n, d_n, out);
    return check_launch("minmax");
}

int derive_key_range(const void *key, int dtype, int64_t n, const int64_t *d_n,
                     void *scratch16, hipStream_t s, int64_t *key_min, int *key_bits) {
    int64_t *dev = static_cast<int64_t *>(scratch16);
    int rc = launch_minmax(key, dtype, n, d_n, dev, s);
    if (rc) return rc;
    int64_t host[2];
    hipError_t e = hipMemcpyAsync(host, dev, sizeof host, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return set_error(TQP_EHIP, "key range read-back: %s", hipGetErrorString(e));
    if (host[0] > host[1]) {          // no keys
        *key_min = 0;
        *key_bits = 0;
        return TQP_OK;
    }
    uint64_t span = uint64_t(host[1]) - uint64_t(host[0]);
    int bits = 0;
    while (bits < 64 && (span >> bits) != 0) bits++;
    *key_min = host[0];
    *key_bits = bits;
    return TQP_OK;
}

}  // namespace tqp

namespace tqp {

struct KnobDef {
    const char *name;
    int def, lo, hi;
};
static const KnobDef kKnobs[kTuneCount] = {
    {"filter.per_cu", 4, 1, 8},
    {"sort.per_cu", 2, 1, 2},
    {"rle.per_cu", 1, 1, 2},
    {"match.per_cu", 4, 1, 8},
    {"gbscan.per_cu", 2, 1, 4},
    {"part.ovf_cap", 65536, 1, 65536},
    {"sort.mode", 0, 0, 1},
    {"semijoin.per_cu", 4, 1, 8},
    {"semijoin.wg", 4, 1, 4},
};
static int g_knob[kTuneCount] = {4, 2, 1, 4, 2, 65536, 0, 4, 4};

int tune(TuneKnob k) { return g_knob[k]; }

}  // namespace tqp

TQP_API const char *tqp_last_error(void) { return tqp::g_err; }

TQP_API int tqp_tune_set(const char *name, int value) {
    tqp::clear_error();
    for (int k = 0; k < tqp::kTuneCount; k++) {
        if (name && strcmp(name, tqp::kKnobs[k].name) == 0) {
            if (value < tqp::kKnobs[k].lo || value > tqp::kKnobs[k].hi)
                return tqp::set_error(TQP_EINVAL, "tqp_tune_set: %s must be in [%d, %d]", name,
                                      tqp::kKnobs[k].lo, tqp::kKnobs[k].hi);
            tqp::g_knob[k] = value;
            return TQP_OK;
        }
    }
    return tqp::set_error(TQP_EINVAL, "tqp_tune_set: unknown knob %s", name ? name : "(null)");
}

TQP_API int tqp_tune_get(const char *name, int *value, int *lo, int *hi) {
    for (int k = 0; k < tqp::kTuneCount; k++) {
        if (name && strcmp(name, tqp::kKnobs[k].name) == 0) {
            if (value) *value = tqp::g_knob[k];
            if (lo) *lo = tqp::kKnobs[k].lo;
            if (hi) *hi = tqp::kKnobs[k].hi;
            return TQP_OK;
        }
    }
    return tqp::set_error(TQP_EINVAL, "tqp_tune_get: unknown knob %s", name ? name : "(null)");
}

TQP_API const char *tqp_tune_name(int index) {
    return index >= 0 && index < tqp::kTuneCount ? tqp::kKnobs[index].name : nullptr;
}

TQP_API int tqp_minmax(const tqp_col *key, const int64_t *d_n, int64_t *d_out, void *stream) {
    tqp::clear_error();
    if (!key || !tqp::dtype_ok(key->dtype) || key->len < 0 || (key->len > 0 && !key->data) ||
        !tqp::col_aligned(key->data, key->dtype))
        return tqp::set_error(TQP_EINVAL, "tqp_minmax: bad key column");
    if (!d_out) return tqp::set_error(TQP_EINVAL, "tqp_minmax: d_out is required");
    return tqp::launch_minmax(key->data, key->dtype, key->len, d_n, d_out,
                              tqp::as_stream(stream));
}

TQP_API const char *tqp_version(void) { return "tqp-mi355x 0.1 (gfx950)"; }
