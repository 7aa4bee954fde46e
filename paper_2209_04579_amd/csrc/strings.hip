// String predicates over the paper's string column layout: an (n x m) tensor
// of UTF-8 bytes, one row per value, zero-padded to m.  One thread per row;
// the rows of a wave are 64 * m consecutive bytes, so the byte loads of a
// wave fall on a few cache lines and every line is fetched once.
#include "tqp_internal.hpp"

namespace tqp {

constexpr int kStrNT = 256;
constexpr int kMaxPattern = 64;

struct StrPattern {
    uint8_t b[kMaxPattern];
};

__global__ __launch_bounds__(kStrNT) void k_str_match(const uint8_t *__restrict__ chars, int64_t n,
                                                      int m, StrPattern pat, int plen, int mode,
                                                      int8_t *__restrict__ out) {
    const int64_t stride = int64_t(gridDim.x) * kStrNT;
    for (int64_t i = blockIdx.x * int64_t(kStrNT) + threadIdx.x; i < n; i += stride) {
        const uint8_t *row = chars + i * m;
        bool ok = plen <= m;
        for (int j = 0; ok && j < plen; j++) ok = row[j] == pat.b[j];
        if (mode == TQP_STR_EQUAL)
            for (int j = plen; ok && j < m; j++) ok = row[j] == 0;
        out[i] = ok ? 1 : 0;
    }
}

}  // namespace tqp

using namespace tqp;

TQP_API int tqp_str_match(const uint8_t *chars, int64_t n, int32_t m, const uint8_t *pattern,
                          int32_t plen, int32_t mode, int8_t *out, void *stream) {
    clear_error();
    if (n < 0 || m < 1 || (n > 0 && (!chars || !out)))
        return set_error(TQP_EINVAL, "tqp_str_match: need n >= 0, m >= 1 and device pointers");
    if (plen < 0 || plen > kMaxPattern || (plen > 0 && !pattern))
        return set_error(TQP_EINVAL, "tqp_str_match: pattern length must be in [0, %d]", kMaxPattern);
    if (mode != TQP_STR_PREFIX && mode != TQP_STR_EQUAL)
        return set_error(TQP_EINVAL, "tqp_str_match: unknown mode %d", mode);
    if (n == 0) return TQP_OK;
    StrPattern pat = {};
    for (int j = 0; j < plen; j++) pat.b[j] = pattern[j];
    int64_t g = ceil_div(n, int64_t(kStrNT) * 4);
    if (g > 8192) g = 8192;
    TQP_LAUNCH("str_match", k_str_match, dim3(unsigned(g)), dim3(kStrNT), 0, as_stream(stream), chars,
               n, int(m), pat, int(plen), int(mode), out);
    return check_launch("tqp_str_match");
}
