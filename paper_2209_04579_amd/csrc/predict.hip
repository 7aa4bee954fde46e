// PREDICT inside a query: an fp32 MLP with one ReLU hidden layer scores each
// row.  Every multiply-add is one fused fma, k and j ascending, relu(v) is
// (v > 0 ? v : 0) and ties go to the first class, so the class equals that
// of any implementation taking the same steps.  Each hidden unit feeds the
// logits as soon as it is computed; every logit's chain is still in
// ascending j.  The model is copied into LDS once per workgroup, W1 rows
// padded and W2 stored by hidden unit, so a hidden unit's weights come in a
// few 16-byte broadcast reads; the features of a row are loaded together,
// one aligned word per column.
#include "tqp_internal.hpp"

namespace tqp {

constexpr int kPredNT = 256;
constexpr int kMaxFeat = 16;
constexpr int kMaxHidden = 64;
constexpr int kMaxClasses = 8;

struct PredArgs {
    const void *feat[kMaxFeat];
    int64_t flen[kMaxFeat];
    int32_t fdt[kMaxFeat];
    int32_t nfeat, hidden, classes;
    const int32_t *rows;
    const float *model;
    int64_t n;
    const int64_t *d_n;
    int8_t *out;
};

// FM >= nfeat and CM >= classes are multiples of 4: the weights are padded
// with zeros to those bounds and every multiply-add runs to the bound, with
// no branch.  The padding changes nothing: x[k] = 0 and W1[j][k] = 0 for
// k >= nfeat, so those steps add +0, which leaves a nonzero sum unchanged
// and can only turn a -0 into +0, and relu maps both zeros to 0; logits past
// `classes` are never compared.
template <int FM, int CM>
__global__ __launch_bounds__(kPredNT) void k_mlp_predict(PredArgs a) {
    __shared__ float4 s_w1[kMaxHidden][FM / 4];      // W1[j][k], zero padded
    __shared__ float4 s_w2[kMaxHidden][CM / 4];      // W2[c][j] stored as [j][c]
    __shared__ float s_b1[kMaxHidden];
    __shared__ float s_b2[CM];
    const int64_t cnt = count_of(a.d_n, a.n);
    const int F = a.nfeat, H = a.hidden, C = a.classes;
    {
        const float *m = a.model;
        float *w1 = reinterpret_cast<float *>(s_w1), *w2 = reinterpret_cast<float *>(s_w2);
        for (int i = threadIdx.x; i < kMaxHidden * FM; i += kPredNT) {
            const int j = i / FM, k = i % FM;
            w1[i] = j < H && k < F ? m[j * F + k] : 0.0f;
        }
        for (int i = threadIdx.x; i < kMaxHidden * CM; i += kPredNT) {
            const int j = i / CM, c = i % CM;
            w2[i] = j < H && c < C ? m[H * F + H + c * H + j] : 0.0f;
        }
        for (int i = threadIdx.x; i < kMaxHidden; i += kPredNT) s_b1[i] = i < H ? m[H * F + i] : 0.0f;
        for (int i = threadIdx.x; i < CM; i += kPredNT) s_b2[i] = i < C ? m[H * F + H + C * H + i] : 0.0f;
    }
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * kPredNT;
    for (int64_t i = blockIdx.x * int64_t(kPredNT) + threadIdx.x; i < cnt; i += stride) {
        const int64_t r = a.rows ? a.rows[i] : i;
        uint64_t w[FM];
#pragma unroll
        for (int k = 0; k < FM; k++) {
            const bool in = k < F && r >= 0 && r < a.flen[k];
            w[k] = word_of(k < F ? a.feat[k] : a.feat[0], k < F ? dtype_lg(a.fdt[k]) : 0,
                           in ? r : 0);
        }
        float x[FM];
#pragma unroll
        for (int k = 0; k < FM; k++) {
            const bool in = k < F && r >= 0 && r < a.flen[k];
            x[k] = in ? float(sext_of(from_word(w[k], a.feat[k], dtype_lg(a.fdt[k]), r), a.fdt[k]))
                      : 0.0f;
        }
        float z[CM];
#pragma unroll
        for (int c = 0; c < CM; c++) z[c] = s_b2[c];
        for (int j = 0; j < H; j++) {
            float wr[FM], wc[CM];
#pragma unroll
            for (int q = 0; q < FM / 4; q++) {
                const float4 v = s_w1[j][q];
                wr[4 * q] = v.x; wr[4 * q + 1] = v.y; wr[4 * q + 2] = v.z; wr[4 * q + 3] = v.w;
            }
#pragma unroll
            for (int q = 0; q < CM / 4; q++) {
                const float4 v = s_w2[j][q];
                wc[4 * q] = v.x; wc[4 * q + 1] = v.y; wc[4 * q + 2] = v.z; wc[4 * q + 3] = v.w;
            }
            float acc = s_b1[j];
#pragma unroll
            for (int k = 0; k < FM; k++) acc = __builtin_fmaf(wr[k], x[k], acc);
            const float h = acc > 0.0f ? acc : 0.0f;
#pragma unroll
            for (int c = 0; c < CM; c++) z[c] = __builtin_fmaf(wc[c], h, z[c]);
        }
        int arg = 0;
        float best = z[0];
#pragma unroll
        for (int c = 1; c < CM; c++)
            if (c < C && z[c] > best) {
                best = z[c];
                arg = c;
            }
        a.out[i] = int8_t(arg);
    }
}

}  // namespace tqp

using namespace tqp;

TQP_API int tqp_mlp_predict(const tqp_col *feats, int nfeat, const int32_t *rows, int64_t n,
                            const int64_t *d_n, const float *model, int hidden, int classes,
                            int8_t *out, void *stream) {
    clear_error();
    if (!feats || nfeat < 1 || nfeat > kMaxFeat)
        return set_error(TQP_EINVAL, "tqp_mlp_predict: nfeat must be in [1, %d]", kMaxFeat);
    if (hidden < 1 || hidden > kMaxHidden || classes < 1 || classes > kMaxClasses)
        return set_error(TQP_EINVAL, "tqp_mlp_predict: hidden must be in [1, %d], classes in [1, %d]",
                         kMaxHidden, kMaxClasses);
    if (n < 0 || (n > 0 && (!model || !out)))
        return set_error(TQP_EINVAL, "tqp_mlp_predict: need n >= 0, a model and an output");
    if (rows && !col_aligned(rows, TQP_INT32))
        return set_error(TQP_EINVAL, "tqp_mlp_predict: rows must be 4-byte aligned");
    if (!col_aligned(model, TQP_INT32))
        return set_error(TQP_EINVAL, "tqp_mlp_predict: model must be 4-byte aligned");
    PredArgs a = {};
    for (int k = 0; k < nfeat; k++) {
        if (!dtype_ok(feats[k].dtype) || feats[k].len < 0 || (feats[k].len > 0 && !feats[k].data) ||
            !col_aligned(feats[k].data, feats[k].dtype))
            return set_error(TQP_EINVAL, "tqp_mlp_predict: feature %d is invalid or unaligned", k);
        if (!rows && feats[k].len < n)
            return set_error(TQP_EINVAL, "tqp_mlp_predict: feature %d is shorter than n", k);
        a.feat[k] = feats[k].len > 0 ? feats[k].data : model;   // never read when empty
        a.flen[k] = feats[k].len;
        a.fdt[k] = feats[k].dtype;
    }
    if (n == 0) return TQP_OK;
    a.nfeat = nfeat;
    a.hidden = hidden;
    a.classes = classes;
    a.rows = rows;
    a.model = model;
    a.n = n;
    a.d_n = d_n;
    a.out = out;
    int64_t g = ceil_div(n, int64_t(kPredNT) * 4);
    if (g > 8192) g = 8192;
    hipStream_t s = as_stream(stream);
    if (nfeat <= 8 && classes <= 4)
        TQP_LAUNCH("mlp_predict", (k_mlp_predict<8, 4>), dim3(unsigned(g)), dim3(kPredNT), 0, s, a);
    else if (nfeat <= 8)
        TQP_LAUNCH("mlp_predict", (k_mlp_predict<8, 8>), dim3(unsigned(g)), dim3(kPredNT), 0, s, a);
    else if (classes <= 4)
        TQP_LAUNCH("mlp_predict", (k_mlp_predict<16, 4>), dim3(unsigned(g)), dim3(kPredNT), 0, s, a);
    else
        TQP_LAUNCH("mlp_predict", (k_mlp_predict<16, 8>), dim3(unsigned(g)), dim3(kPredNT), 0, s, a);
    return check_launch("tqp_mlp_predict");
}
