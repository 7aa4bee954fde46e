// Learned CDF partitioner and the partition sort it drives.
//
// Model.  F(key) approximates the CDF of the key distribution:
//   x    = (key - kmin) / (kmax - kmin), computed in float64, then float32,
//   root = sum_j v_j * clamp(w_j * x + c_j, 0, 1) + d      (1 -> 32 -> 1 MLP)
//   leaf = clamp(floor(root * L), 0, L - 1)
//   F    = the leaf's piecewise-linear spline through kKnots knots (key, rank)
//          taken at evenly spaced points of the leaf's sorted sample, over the
//          key itself: the segment is found by int64 compares with the exact
//          knot keys and the position inside it is the exact int64 difference
//          (not x: a float32 x cannot tell apart keys closer than 2^-24 of the
//          key span, and a dense cluster of a million keys can sit inside
//          such a gap, as can a whole cluster inside one leaf)
// and, where a leaf holds a heavy key h (one that fills a run of the sorted
// sample), F jumps exactly at h: keys below h are held at or under the rank
// where h's copies start, keys above at or over the rank where they end, and
// h itself sits in the middle, so its copies get a bucket of their own.
// with w_j, v_j > 0.  Every step is monotone non-decreasing in x, under
// float rounding too (round-to-nearest is monotone), and the leaves' clamps
// are ordered (hi_k <= lo_{k+1}), so F is monotone: a bucket
// floor(F * 2^bits) is a contiguous key range.  That is the one property the
// partition sort needs; how well F fits only changes the speed.
//
// Training (all on the device, no host round trip): a strided 1% sample of
// the keys is sorted; the root's 32 ramps start on the sample's 32-quantiles
// and are refined by full-batch Adam on the mean squared error against the
// sample ranks; each leaf then takes its knots from the sample points the
// root routes to it, plus its most repeated sample key when that repeats at
// least kHeavyMin times.  Each ramp's
// centre is trained in units of its starting width (ramps on a dense part of
// the distribution can be 1e-9 wide in normalised key space, and Adam moves
// every parameter by about the learning rate at first), and the parameters
// with the lowest loss seen are the ones kept.
//
// Partition sort.  Every key's bucket number is evaluated once (the leaves
// held in LDS); stable radix passes on it group the keys by bucket (input
// order kept inside a bucket); then each window of whole buckets (at most
// 8192 keys) is sorted by one workgroup in LDS by (key, position), which is
// the stable order and, since buckets are key ranges, sorts every bucket in
// it.  A bucket too large for a window is left as is when all its keys are
// equal (already in stable order); the others are gathered, sorted together
// by the plain radix sort over their own key range and scattered back.  With
// bucket = top bits of (key - kmin) the same pipeline is the plain MSD radix
// partitioner the learned one is compared against.
#include <limits.h>
#include <stddef.h>
#include <math.h>
#include <algorithm>
#include <vector>

#include "radix.hpp"

namespace tqp {

constexpr int kHidden = 32;
constexpr int kKnots = 8;                    // spline knots per leaf
constexpr int kNParam = 3 * kHidden + 1;     // centre offset, log-width, log-height per ramp; d
constexpr int kTrainPoints = 4096;           // root training set (sample points, even ranks)
constexpr int kLeafMax = 65536;
// The root as a table: its breakpoints in [0, 1] (every ramp starts and ends
// at one), 0 and 1: at most 2 * kHidden + 2 points, searched as 128.
constexpr int kRootPts = 2 * kHidden + 2;
constexpr int kRootPad = 128;
constexpr int kHeavyMin = 4;                 // sample copies that make a key heavy
constexpr int64_t kOvfCap = 65536;           // overflow buckets re-sorted one by one

struct LcdfModel {
    int64_t kmin;
    double inv_span;
    int32_t nleaf;
    int32_t steps_done;
    float loss_first, loss_last, loss_best, pad0;
    // effective root parameters
    float w[kHidden], c[kHidden], v[kHidden], d;
    // the root as used for routing: points px (ascending, px[0] = 0, +inf past
    // the last), the root's values py there (non-decreasing) and the slopes
    // ps between them
    int32_t npts, pad1;
    float px[kRootPad], py[kRootPts], ps[kRootPts];
    // training state: ramp centre offset u (centre = c0 + s0 * u), log width,
    // log height, bias; Adam moments; the best parameters seen and their loss
    float theta[kNParam], m1[kNParam], m2[kNParam], best[kNParam];
    float c0[kHidden], s0[kHidden];
    // 96 bytes: exact knot keys, knot ranks as 16-bit fractions of the
    // leaf's rank range.  A heavy key h is a pair of knots (h, hlo), (h, hhi)
    // at indices hk, hk + 1, so keys below h stay at or under the rank where
    // its copies start and keys above at or over the rank where they end.
    struct alignas(16) Leaf {
        int64_t kx[kKnots];                   // knot keys, ascending; unused ones INT64_MAX
        uint16_t r[kKnots];                   // knot ranks: lo + (hi - lo) * r / 65535,
                                              // ascending; unused ones repeat the last
        float lo, hi;                         // the leaf's rank range
        uint16_t hlo, hhi;                    // the heavy key's ranks (r[hk], r[hk + 1])
        uint8_t nk, hk;                       // knots in use (0: constant lo); heavy pair
                                              // index, kNoHeavy when none
        uint16_t pad;
    } leaf[1];                                // nleaf entries
};
using Leaf = LcdfModel::Leaf;
constexpr int kNoHeavy = 0xff;
static_assert(sizeof(Leaf) == 96 && offsetof(Leaf, lo) == 80, "leaf layout");
// Leaves held in LDS at once while bucket numbers are evaluated (with the
// root's table, 160 KB); a model with more is evaluated in several passes
// over the keys, each holding the next kLdsLeafMax leaves.
constexpr int kLdsLeafMax = 1688;
constexpr int kRootTabBytes = int(sizeof(float)) * (kRootPad + 2 * kRootPts);   // 1040
static_assert(kRootTabBytes % 16 == 0, "leaves after the table stay 16-byte aligned");

static size_t model_bytes(int nleaf) {
    return sizeof(LcdfModel) + sizeof(Leaf) * size_t(nleaf > 0 ? nleaf - 1 : 0);
}

__device__ __forceinline__ float lcdf_x(const LcdfModel *m, int64_t key) {
    const uint64_t off = uint64_t(key) - uint64_t(m->kmin);
    double x = key < m->kmin ? 0.0 : double(off) * m->inv_span;
    x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
    return float(x);
}

// A ramp clamp(h, 0, 1) is one median-of-three (no NaN reaches it: x is a
// clamped finite value and the parameters are finite).
__device__ __forceinline__ float ramp(float h) { return __builtin_amdgcn_fmed3f(h, 0.f, 1.f); }

__device__ __forceinline__ float lcdf_root(const LcdfModel *m, float x) {
    float y = m->d;
#pragma unroll
    for (int j = 0; j < kHidden; j++) y = fmaf(m->v[j], ramp(fmaf(m->w[j], x, m->c[j])), y);
    return y;
}

// The root from its table: the last point at or below x (a branch-free
// search over the 128 padded points), then the straight line to the next
// point, clamped to the two points' values, so the result is monotone in x
// whatever the rounding.  The same function as the ramp sum up to rounding.
__device__ __forceinline__ float lcdf_root_tab(const float *px, const float *py, const float *ps,
                                               int npts, float x) {
    int k = 0;
#pragma unroll
    for (int h = kRootPad / 2; h >= 1; h >>= 1) k += px[k + h] <= x ? h : 0;
    if (k >= npts - 1) return py[npts - 1];
    const float y0 = py[k], y1 = py[k + 1];
    return __builtin_amdgcn_fmed3f(fmaf(ps[k], x - px[k], y0), y0, y1);
}

__device__ __forceinline__ float lcdf_root_tab(const LcdfModel *m, float x) {
    return lcdf_root_tab(m->px, m->py, m->ps, m->npts, x);
}

__device__ __forceinline__ int lcdf_leaf(const LcdfModel *m, float root) {
    float t = root * float(m->nleaf);
    int k = t <= 0.f ? 0 : (t >= float(m->nleaf) ? m->nleaf - 1 : int(t));
    return k;
}

// F of one key in its leaf.  The spline segment is the last knot at or below
// the key; each segment's value is clamped to its two knot ranks, so F is
// monotone across segments even with rounding.
__device__ __forceinline__ int lcdf_leaf_of(const LcdfModel *m, int64_t key) {
    return lcdf_leaf(m, lcdf_root_tab(m, lcdf_x(m, key)));
}

// lo + (hi - lo) * u / 65535: non-decreasing in u, at least lo (the sum of lo
// and a non-negative product never rounds below lo); callers clamp to hi.
__device__ __forceinline__ float leaf_rank(float lo, float span, uint32_t u) {
    return fmaf(span, float(u) * (1.f / 65535.f), lo);
}

// F of one key in its leaf.  The segment is the last knot at or below the
// key (a branch-free binary search over the eight ascending knot keys); the
// position inside it is the exact int64 offset from the segment's first knot
// over the segment's width (each converted to float, which is monotone), and
// the value is clamped to the segment's two knot ranks, so F is monotone
// across segments even with rounding.  A key below the first knot takes the
// first rank, one at or past the last knot the last rank, and the heavy key
// itself the middle of its pair's ranks.
__device__ __forceinline__ float lcdf_leaf_eval(const Leaf &L, int64_t key) {
    const float lo = L.lo, hi = L.hi, span = hi - lo;
    const int nk = L.nk;
    int c = L.kx[3] <= key ? 4 : 0;                  // knots at or below the key
    c += L.kx[c + 1] <= key ? 2 : 0;
    c += L.kx[c] <= key ? 1 : 0;
    c += L.kx[c] <= key ? 1 : 0;
    const int j = c > 0 ? c - 1 : 0;
    const int j1 = c < nk ? c : j;                   // j1 == j: no segment beyond j
    const int64_t kj = L.kx[j], kj1 = L.kx[j1];
    const float rj = leaf_rank(lo, span, L.r[j]), rj1 = leaf_rank(lo, span, L.r[j1]);
    // below the first knot d = 0, past the last rj1 = rj: both give rj
    const uint64_t d = c > 0 ? uint64_t(key) - uint64_t(kj) : 0;
    const uint64_t w = j1 != j ? uint64_t(kj1) - uint64_t(kj) : 1;
    const float g = fmaf(rj1 - rj, float(d) * __builtin_amdgcn_rcpf(float(w)), rj);
    float f = __builtin_amdgcn_fmed3f(g, rj, rj1);
    if (L.hk != kNoHeavy && j == int(L.hk) + 1 && kj == key)
        f = 0.5f * (leaf_rank(lo, span, L.hlo) + leaf_rank(lo, span, L.hhi));
    f = nk == 0 ? lo : f;
    return f < lo ? lo : (f > hi ? hi : f);
}

// Bucket ordinals: learned (the leaves read from LDS by the bucket-number
// kernel), or the top bits of key - kmin.
template <class K> struct LearnedOrd {
    const LcdfModel *m;
    const Leaf *leaves;                         // the model's leaves in memory
    float scale;                                // 2^bucket_bits
    uint32_t top;                               // 2^bucket_bits - 1
    __device__ __forceinline__ uint32_t bucket(float f) const {
        const float t = f * scale;
        const uint32_t b = t <= 0.f ? 0u : uint32_t(t);
        return b > top ? top : b;
    }
};

template <class K> struct MsdOrd {
    K key_min;
    int shift;
    uint32_t top;                               // 2^bucket_bits - 1
    __device__ __forceinline__ uint64_t operator()(K k) const {
        using U = typename KeyTraits<K>::U;
        const uint64_t b = uint64_t(U(U(k) - U(key_min))) >> shift;
        return b > top ? top : b;               // keys outside the stated range
    }
};

// ---- training ------------------------------------------------------------------

__global__ void k_lcdf_sample(const void *c0, int dt0, int64_t n0, const void *c1, int dt1,
                              int64_t n1, int64_t stride, int64_t *out) {
    const int64_t m0 = ceil_div(n0, stride), m1 = ceil_div(n1, stride);
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < m0 + m1;
         t += int64_t(gridDim.x) * blockDim.x)
        out[t] = t < m0 ? load_any(c0, dt0, t * stride) : load_any(c1, dt1, (t - m0) * stride);
}

// One workgroup: normalization from the sorted sample, the training points,
// and the ramps' starting positions on the sample's quantiles.
__global__ __launch_bounds__(256) void k_lcdf_init(const int64_t *sorted, int64_t m, int nleaf,
                                                   LcdfModel *mod, float *tx, float *tq, int T) {
    __shared__ int64_t s_min, s_max;
    if (threadIdx.x == 0) {
        s_min = sorted[0];
        s_max = sorted[m - 1];
        mod->kmin = s_min;
        const double span = double(uint64_t(s_max) - uint64_t(s_min));
        mod->inv_span = span > 0 ? 1.0 / span : 0.0;
        mod->nleaf = nleaf;
        mod->steps_done = 0;
    }
    __syncthreads();
    const double inv = s_max > s_min ? 1.0 / double(uint64_t(s_max) - uint64_t(s_min)) : 0.0;
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        const int64_t i = int64_t((double(t) + 0.5) * double(m) / double(T));
        tx[t] = float(double(uint64_t(sorted[i]) - uint64_t(s_min)) * inv);
        tq[t] = float((double(i) + 0.5) / double(m));
    }
    if (threadIdx.x < kHidden) {
        const int j = threadIdx.x;
        const int64_t ia = int64_t(double(j) * double(m - 1) / kHidden);
        const int64_t ib = int64_t(double(j + 1) * double(m - 1) / kHidden);
        const float xa = float(double(uint64_t(sorted[ia]) - uint64_t(s_min)) * inv);
        const float xb = float(double(uint64_t(sorted[ib]) - uint64_t(s_min)) * inv);
        float width = xb - xa;
        if (width < 1e-9f) width = 1e-9f;
        mod->c0[j] = 0.5f * (xa + xb);                       // starting centre
        mod->s0[j] = width;                                  // centre unit
        mod->theta[j] = 0.f;                                 // centre offset
        mod->theta[kHidden + j] = logf(width);               // log width
        mod->theta[2 * kHidden + j] = logf(1.0f / kHidden);  // log height
    }
    if (threadIdx.x == 0) {
        mod->theta[3 * kHidden] = 0.f;
        mod->loss_best = INFINITY;
    }
    for (int p = threadIdx.x; p < kNParam; p += blockDim.x) {
        mod->m1[p] = 0.f;
        mod->m2[p] = 0.f;
    }
}

// The whole training loop in one launch: one workgroup keeps the parameters,
// Adam's moments and the training points on chip and runs `steps`
// full-batch steps.  Each step: the per-ramp constants (inverse width,
// height, centre) once; a forward pass (thread t: points t + k * 1024) that
// leaves every point's scaled error in LDS; a backward pass in which thread
// t accumulates the three gradients of ramp t mod 32 over the points
// congruent to t / 32 mod 32; reductions in a fixed order (lanes by
// shuffles, then the waves in turn); one Adam step per parameter (b1 = 0.9,
// b2 = 0.999, bias-corrected).  The parameters with the lowest loss seen are
// kept.  The gradient is that of the mean squared error between the root
// and the sample ranks.
constexpr int kFitNT = 1024;
constexpr int kFitNW = kFitNT / kWave;
constexpr int kFitPer = kTrainPoints / kFitNT;              // forward points per thread
constexpr int kFitGroups = kFitNT / kHidden;                // threads per ramp in the backward pass
static_assert(kTrainPoints % kFitNT == 0 && kFitNT % kHidden == 0, "training layout");

__global__ __launch_bounds__(kFitNT) void k_lcdf_fit(LcdfModel *mod, const float *tx,
                                                     const float *tq, int T, int steps, float lr) {
    __shared__ float s_th[kNParam], s_m1[kNParam], s_m2[kNParam], s_best[kNParam];
    __shared__ float s_w[kHidden], s_v[kHidden], s_c[kHidden], s_c0[kHidden], s_s0[kHidden];
    __shared__ float s_x[kTrainPoints], s_e[kTrainPoints];
    __shared__ float s_red[kFitNW][3 * kHidden];
    __shared__ float s_red1[kFitNW][2];
    __shared__ float s_g[kNParam + 1];
    __shared__ float s_lbest, s_lfirst, s_llast;
    __shared__ int s_step;
    const int tid = threadIdx.x, w = wave_id(), lane = lane_id();
    for (int p = tid; p < kNParam; p += kFitNT) {
        s_th[p] = mod->theta[p];
        s_m1[p] = mod->m1[p];
        s_m2[p] = mod->m2[p];
        s_best[p] = mod->theta[p];
    }
    if (tid < kHidden) {
        s_c0[tid] = mod->c0[tid];
        s_s0[tid] = mod->s0[tid];
    }
    if (tid == 0) {
        s_lbest = mod->loss_best;
        s_lfirst = mod->loss_first;
        s_llast = mod->loss_last;
        s_step = mod->steps_done;
    }
    float pq[kFitPer];
#pragma unroll
    for (int k = 0; k < kFitPer; k++) {
        const int t = tid + k * kFitNT;
        s_x[t] = t < T ? tx[t] : 0.f;
        pq[k] = t < T ? tq[t] : 0.f;
    }
    const float inv_t = 2.0f / float(T);
    const int j = tid % kHidden, q = tid / kHidden;
    __syncthreads();
    for (int it = 0; it < steps; it++) {
        if (tid < kHidden) {
            s_w[tid] = __expf(-s_th[kHidden + tid]);
            s_v[tid] = __expf(s_th[2 * kHidden + tid]);
            s_c[tid] = s_c0[tid] + s_s0[tid] * s_th[tid];
        }
        __syncthreads();
        // forward: the root at this thread's points, their scaled errors
        float loss = 0.f, esum = 0.f;
#pragma unroll
        for (int k = 0; k < kFitPer; k++) {
            const int t = tid + k * kFitNT;
            const float x = s_x[t];
            float y = s_th[3 * kHidden];
#pragma unroll
            for (int r = 0; r < kHidden; r++) y += s_v[r] * ramp((x - s_c[r]) * s_w[r] + 0.5f);
            const float err = t < T ? y - pq[k] : 0.f;
            s_e[t] = err * inv_t;
            loss += err * err / float(T);
            esum += err * inv_t;
        }
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            loss += __shfl_xor(loss, o, kWave);
            esum += __shfl_xor(esum, o, kWave);
        }
        if (lane == 0) {
            s_red1[w][0] = loss;
            s_red1[w][1] = esum;
        }
        __syncthreads();
        // backward: ramp j over the points q, q + 32, ...
        {
            const float wj = s_w[j], vj = s_v[j], cj = s_c[j], sj = s_s0[j];
            float gc = 0.f, gw = 0.f, gv = 0.f;
            for (int p = q; p < T; p += kFitGroups) {
                const float z = (s_x[p] - cj) * wj + 0.5f;
                const float e = s_e[p];
                const float h = z < 0.f ? 0.f : (z > 1.f ? 1.f : z);
                if (z > 0.f && z < 1.f) {
                    gc += e * vj * (-wj) * sj;                    // d/du = s0 * d/dcentre
                    gw += e * vj * (-(z - 0.5f));
                }
                gv += e * vj * h;
            }
            // lanes l and l + 32 of a wave hold the same ramp
            gc += __shfl_xor(gc, kHidden, kWave);
            gw += __shfl_xor(gw, kHidden, kWave);
            gv += __shfl_xor(gv, kHidden, kWave);
            if (lane < kHidden) {
                s_red[w][j] = gc;
                s_red[w][kHidden + j] = gw;
                s_red[w][2 * kHidden + j] = gv;
            }
        }
        __syncthreads();
        if (tid <= kNParam) {
            float sum = 0.f;
            if (tid < 3 * kHidden) {
                for (int ww = 0; ww < kFitNW; ww++) sum += s_red[ww][tid];
            } else {
                const int c = tid == 3 * kHidden ? 1 : 0;        // bias gradient, then the loss
                for (int ww = 0; ww < kFitNW; ww++) sum += s_red1[ww][c];
            }
            s_g[tid] = sum;
        }
        __syncthreads();
        const float lossv = s_g[kNParam];
        const bool better = lossv < s_lbest;
        const int step = s_step + 1;
        if (tid < kNParam) {
            const int p = tid;
            if (better) s_best[p] = s_th[p];
            const float b1 = 0.9f, b2 = 0.999f, gp = s_g[p];
            const float m1 = b1 * s_m1[p] + (1.f - b1) * gp;
            const float m2 = b2 * s_m2[p] + (1.f - b2) * gp * gp;
            s_m1[p] = m1;
            s_m2[p] = m2;
            const float mh = m1 / (1.f - powf(b1, float(step)));
            const float vh = m2 / (1.f - powf(b2, float(step)));
            float th = s_th[p] - lr * mh / (sqrtf(vh) + 1e-12f);
            if (p >= kHidden && p < 2 * kHidden && th < -40.f) th = -40.f;    // width > 0
            s_th[p] = th;
        }
        __syncthreads();
        if (tid == 0) {
            if (step == 1) s_lfirst = lossv;
            s_llast = lossv;
            if (better) s_lbest = lossv;
            s_step = step;
        }
        __syncthreads();
    }
    for (int p = tid; p < kNParam; p += kFitNT) {
        mod->theta[p] = s_th[p];
        mod->m1[p] = s_m1[p];
        mod->m2[p] = s_m2[p];
        if (steps > 0) mod->best[p] = s_best[p];
    }
    if (tid == 0) {
        mod->loss_best = s_lbest;
        mod->loss_first = s_lfirst;
        mod->loss_last = s_llast;
        mod->steps_done = s_step;
    }
}

// Effective root parameters from the best parameters seen (the starting ones
// when no step was taken): w = 1 / width, c = 0.5 - centre * w, v = height;
// then the root's table, which routing uses.
__global__ void k_lcdf_finalize(LcdfModel *mod) {
    const int j = threadIdx.x;
    const bool trained = mod->loss_best < INFINITY;
    const float *th = trained ? mod->best : mod->theta;
    if (j < kHidden) {
        const float w = expf(-th[kHidden + j]);
        const float centre = mod->c0[j] + mod->s0[j] * th[j];
        mod->w[j] = w;
        mod->c[j] = 0.5f - centre * w;
        mod->v[j] = expf(th[2 * kHidden + j]);
    }
    if (j == 0) mod->d = th[3 * kHidden];
    __syncthreads();
    if (j != 0) return;
    // the root's table: breakpoints inside (0, 1), then 0 and 1, sorted and
    // without repeats; values from the ramp sum, made non-decreasing
    float pts[kRootPts];
    int np = 0;
    pts[np++] = 0.f;
    pts[np++] = 1.f;
    for (int q = 0; q < kHidden; q++) {
        const float a = -mod->c[q] / mod->w[q], b = (1.f - mod->c[q]) / mod->w[q];
        if (a > 0.f && a < 1.f) pts[np++] = a;
        if (b > 0.f && b < 1.f) pts[np++] = b;
    }
    for (int i = 1; i < np; i++)                  // insertion sort (at most 66 points)
        for (int t = i; t > 0 && pts[t - 1] > pts[t]; t--) {
            const float u = pts[t];
            pts[t] = pts[t - 1];
            pts[t - 1] = u;
        }
    int n = 0;
    for (int i = 0; i < np; i++)
        if (n == 0 || pts[i] > mod->px[n - 1]) mod->px[n++] = pts[i];
    for (int i = n; i < kRootPad; i++) mod->px[i] = INFINITY;
    float ymax = -INFINITY;
    for (int i = 0; i < n; i++) {
        const float y = lcdf_root(mod, mod->px[i]);
        ymax = y > ymax ? y : ymax;
        mod->py[i] = ymax;
    }
    for (int i = 0; i + 1 < n; i++)
        mod->ps[i] = (mod->py[i + 1] - mod->py[i]) / (mod->px[i + 1] - mod->px[i]);
    mod->ps[n - 1] = 0.f;
    mod->npts = n;
}

// lstart[l] = the first sorted sample point the root routes to leaf l or
// later (lstart[nleaf] = m): the routing is monotone along the sorted
// sample, so each point writes the starts of the leaves its step from the
// previous point passes, and every entry is written once.
__global__ __launch_bounds__(256) void k_leaf_starts(const LcdfModel *mod, const int64_t *sorted,
                                                     int64_t m, int64_t *lstart) {
    const int nl = mod->nleaf;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < m;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int l = lcdf_leaf_of(mod, sorted[i]);
        const int p = i > 0 ? lcdf_leaf_of(mod, sorted[i - 1]) : -1;
        for (int t = p + 1; t <= l; t++) lstart[t] = i;
        if (i == m - 1)
            for (int t = l + 1; t <= nl; t++) lstart[t] = m;
    }
}

// The spline through knots (kx, kr) at a key, in float64: the rank of the
// last knot at or below the key, moved linearly toward the next one.
__device__ __forceinline__ double knot_spline(const int64_t *kx, const double *kr, int nk,
                                              int64_t key) {
    int c = 0;
    while (c < nk && kx[c] <= key) c++;
    if (c == 0) return kr[0];
    if (c == nk) return kr[nk - 1];
    const double d = double(uint64_t(key) - uint64_t(kx[c - 1]));
    const double w = double(uint64_t(kx[c]) - uint64_t(kx[c - 1]));
    return kr[c - 1] + (kr[c] - kr[c - 1]) * (d / w);
}

// One workgroup per leaf: the contiguous run of sorted sample points the root
// routes to it (from lstart), its longest run of one key (a heavy key when it repeats at
// least kHeavyMin times), and the spline knots.  The knots start as the
// leaf's first and last sample points and the heavy key's pair; each further
// knot is the sample point where the spline so far misses the sample rank
// the most (so knots land on the edges of dense clusters, where a straight
// segment across a gap would put a whole cluster edge into one bucket).
__global__ __launch_bounds__(256) void k_lcdf_leaf_fit(LcdfModel *mod, const int64_t *sorted,
                                                       int64_t m, const int64_t *lstart) {
    __shared__ int64_t s_run[256 / kWave][2];
    __shared__ int64_t s_kx[kKnots];
    __shared__ double s_kr[kKnots];
    __shared__ int s_nk, s_hpos, s_done;
    __shared__ double s_err[256 / kWave];
    __shared__ int64_t s_arg[256 / kWave];
    const int leaf = blockIdx.x, tid = threadIdx.x;
    const int64_t a0 = lstart[leaf], a1 = lstart[leaf + 1];
    // longest run of equal keys: each run start finds its end by binary search
    int64_t best_len = 0, best_start = 0;
    for (int64_t i = a0 + tid; i < a1; i += blockDim.x) {
        const int64_t v = sorted[i];
        if (i > a0 && sorted[i - 1] == v) continue;
        int64_t lo = i + 1, hi = a1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (sorted[mid] == v) lo = mid + 1;
            else hi = mid;
        }
        if (lo - i > best_len) {
            best_len = lo - i;
            best_start = i;
        }
    }
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t ol = __shfl_xor(best_len, o, kWave);
        const int64_t os = __shfl_xor(best_start, o, kWave);
        if (ol > best_len || (ol == best_len && os < best_start)) {
            best_len = ol;
            best_start = os;
        }
    }
    if (lane_id() == 0) {
        s_run[wave_id()][0] = best_len;
        s_run[wave_id()][1] = best_start;
    }
    __syncthreads();
    int64_t rl = 0, rs = 0;
    for (int ww = 0; ww < 256 / kWave; ww++)
        if (s_run[ww][0] > rl || (s_run[ww][0] == rl && s_run[ww][1] < rs)) {
            rl = s_run[ww][0];
            rs = s_run[ww][1];
        }
    const bool heavy = a1 > a0 && rl >= kHeavyMin;
    if (tid == 0) {
        int nk = 0, hpos = -1;
        if (a1 > a0) {
            if (!(heavy && rs == a0)) {
                s_kx[nk] = sorted[a0];
                s_kr[nk++] = (double(a0) + 0.5) / double(m);
            }
            if (heavy) {
                hpos = nk;
                s_kx[nk] = sorted[rs];
                s_kr[nk++] = double(rs) / double(m);
                s_kx[nk] = sorted[rs];
                s_kr[nk++] = double(rs + rl) / double(m);
            }
            if (a1 - 1 > a0 && !(heavy && rs + rl == a1)) {
                s_kx[nk] = sorted[a1 - 1];
                s_kr[nk++] = (double(a1 - 1) + 0.5) / double(m);
            }
        }
        s_nk = nk;
        s_hpos = hpos;
        s_done = 0;
    }
    __syncthreads();
    // greedy knots: the point of largest rank error, until the knots run out
    while (!s_done && s_nk < kKnots) {
        const int nk = s_nk;
        double be = 0.0;
        int64_t ba = -1;
        for (int64_t i = a0 + tid; i < a1; i += blockDim.x) {
            if (heavy && i >= rs && i < rs + rl) continue;      // the pair places these exactly
            const double e = fabs(knot_spline(s_kx, s_kr, nk, sorted[i]) - (double(i) + 0.5) / double(m));
            if (e > be) {
                be = e;
                ba = i;
            }
        }
        for (int o = 1; o < kWave; o <<= 1) {
            const double oe = __shfl_xor(be, o, kWave);
            const int64_t oa = __shfl_xor(ba, o, kWave);
            if (oe > be || (oe == be && oa >= 0 && (ba < 0 || oa < ba))) {
                be = oe;
                ba = oa;
            }
        }
        if (lane_id() == 0) {
            s_err[wave_id()] = be;
            s_arg[wave_id()] = ba;
        }
        __syncthreads();
        if (tid == 0) {
            double e = 0.0;
            int64_t arg = -1;
            for (int ww = 0; ww < 256 / kWave; ww++)
                if (s_err[ww] > e || (s_err[ww] == e && s_arg[ww] >= 0 && (arg < 0 || s_arg[ww] < arg))) {
                    e = s_err[ww];
                    arg = s_arg[ww];
                }
            if (arg < 0 || !(e > 0.0)) {
                s_done = 1;                                    // exact already
            } else {
                // insert (key, rank) in (key, rank) order
                const int64_t key = sorted[arg];
                const double rank = (double(arg) + 0.5) / double(m);
                int at = nk;
                while (at > 0 && (s_kx[at - 1] > key || (s_kx[at - 1] == key && s_kr[at - 1] > rank))) {
                    s_kx[at] = s_kx[at - 1];
                    s_kr[at] = s_kr[at - 1];
                    at--;
                }
                s_kx[at] = key;
                s_kr[at] = rank;
                if (s_hpos >= at) s_hpos++;
                s_nk = nk + 1;
            }
        }
        __syncthreads();
    }
    if (tid != 0) return;
    Leaf o;
    o.hlo = o.hhi = 0;
    o.hk = uint8_t(kNoHeavy);
    o.pad = 0;
    const int nk = s_nk, hpos = s_hpos;
    if (nk == 0) {                                    // empty: range filled in later
        for (int t = 0; t < kKnots; t++) {
            o.kx[t] = INT64_MAX;
            o.r[t] = 0;
        }
        o.nk = 0;
        o.lo = o.hi = -1.f;
        mod->leaf[leaf] = o;
        return;
    }
    // the first leaf's range starts at 0 and the last one's ends at 1
    const float lo = leaf == 0 ? 0.f : float(s_kr[0]);
    const float hi = leaf == mod->nleaf - 1 ? 1.f : float(s_kr[nk - 1]);
    const double dlo = double(lo), dspan = double(hi) - double(lo);
    auto enc = [&](double v) -> uint16_t {          // nearest 16-bit fraction of [lo, hi]
        if (!(dspan > 0)) return 0;
        const double u = nearbyint((v - dlo) / dspan * 65535.0);
        return uint16_t(u < 0 ? 0 : (u > 65535 ? 65535 : u));
    };
    for (int t = 0; t < kKnots; t++) {
        o.kx[t] = t < nk ? s_kx[t] : INT64_MAX;
        o.r[t] = enc(s_kr[t < nk ? t : nk - 1]);
    }
    o.lo = lo;
    o.hi = hi;
    o.nk = uint8_t(nk);
    if (hpos >= 0) {
        o.hk = uint8_t(hpos);
        o.hlo = o.r[hpos];
        o.hhi = o.r[hpos + 1];
    }
    mod->leaf[leaf] = o;
}

// Empty leaves take the rank reached by the leaves before them, so the
// rank ranges stay ordered; the first leaf's range starts at 0, the last
// one's ends at 1.  One workgroup: each thread takes a run of consecutive
// leaves; the rank reached before a run is the last non-empty leaf's hi
// among the runs before it (a prefix "last value" scan over the runs).
constexpr int kFillNT = 256;

__global__ __launch_bounds__(kFillNT) void k_lcdf_leaf_fill(LcdfModel *mod) {
    __shared__ float s_last[kFillNT];
    __shared__ int s_has[kFillNT];
    const int nl = mod->nleaf;
    const int per = (nl + kFillNT - 1) / kFillNT;
    const int a = threadIdx.x * per, b = a + per < nl ? a + per : nl;
    float last = 0.f;
    int has = 0;
    for (int k = a; k < b; k++)
        if (mod->leaf[k].nk != 0) {
            last = mod->leaf[k].hi;
            has = 1;
        }
    s_last[threadIdx.x] = last;
    s_has[threadIdx.x] = has;
    __syncthreads();
    float prev = 0.f;
    for (int t = threadIdx.x - 1; t >= 0; t--)
        if (s_has[t]) {
            prev = s_last[t];
            break;
        }
    for (int k = a; k < b; k++) {
        Leaf &L = mod->leaf[k];
        if (L.nk == 0) {
            L.lo = L.hi = prev;
        } else {
            if (k == 0) L.lo = 0.f;
            prev = L.hi;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) mod->leaf[nl - 1].hi = 1.f;
}

// ---- per-bucket finishing sort -------------------------------------------------

struct BucketStats {
    unsigned long long max_bucket;
    unsigned long long nbig;            // entries of the big-bucket list
};

struct Overflow {
    int64_t start, len, kmin, kmax;
    int64_t off;                        // position in the gathered overflow keys
};

// Bucket number of every key, evaluated once (int32, in [0, nb)).
template <class K, class Ord>
__global__ __launch_bounds__(256) void k_bucket_ids(const K *__restrict__ keys, int64_t n, Ord ord,
                                                    int32_t *__restrict__ ids) {
    constexpr int R = 2;                // keys per thread per step, loads issued together
    const int64_t stride = int64_t(gridDim.x) * blockDim.x * R;
    for (int64_t base = blockIdx.x * int64_t(blockDim.x) * R + threadIdx.x; base < n;
         base += stride) {
        K k[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int64_t i = base + int64_t(r) * blockDim.x;
            k[r] = i < n ? keys[i] : K(0);
        }
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int64_t i = base + int64_t(r) * blockDim.x;
            if (i < n) ids[i] = int32_t(ord(k[r]));
        }
    }
}

// The same for a learned model, its leaves read from LDS: a key's leaf is a
// random one of thousands, and the handful of reads its evaluation makes
// cost far less from LDS than from the caches.  One workgroup per compute unit copies leaves
// [leaf0, leaf0 + kLdsLeafMax) into LDS and numbers the keys whose leaf is
// among them; a model with more leaves takes one such pass per group of
// leaves (the keys are read again, each number is written once).
constexpr int kBidNT = 1024;

template <class K>
__global__ __launch_bounds__(kBidNT) void k_bucket_ids_lds(const K *__restrict__ keys, int64_t n,
                                                           LearnedOrd<K> ord, int leaf0,
                                                           int32_t *__restrict__ ids) {
    extern __shared__ int4 s_dyn[];
    constexpr int Q = int(sizeof(Leaf) / 16);
    const LcdfModel *m = ord.m;
    const int nl = m->nleaf;
    const int cnt = nl - leaf0 < kLdsLeafMax ? nl - leaf0 : kLdsLeafMax;
    if (cnt <= 0) return;
    // the root's table, then the leaves of this pass
    float *s_px = reinterpret_cast<float *>(s_dyn);
    float *s_py = s_px + kRootPad, *s_ps = s_py + kRootPts;
    int4 *s_leaf = s_dyn + kRootTabBytes / 16;
    for (int i = threadIdx.x; i < kRootPad; i += kBidNT) s_px[i] = m->px[i];
    for (int i = threadIdx.x; i < kRootPts; i += kBidNT) {
        s_py[i] = m->py[i];
        s_ps[i] = m->ps[i];
    }
    const int4 *src = reinterpret_cast<const int4 *>(ord.leaves + leaf0);
    for (int i = threadIdx.x; i < cnt * Q; i += kBidNT) s_leaf[i] = src[i];
    __syncthreads();
    const Leaf *lds = reinterpret_cast<const Leaf *>(s_leaf);
    const int npts = m->npts;
    constexpr int R = 4;
    const int64_t stride = int64_t(gridDim.x) * kBidNT * R;
    for (int64_t base = blockIdx.x * int64_t(kBidNT) * R + threadIdx.x; base < n; base += stride) {
        K k[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int64_t i = base + int64_t(r) * kBidNT;
            k[r] = i < n ? keys[i] : K(0);
        }
        // all R evaluations issued together (their LDS reads overlap), then
        // only the keys whose leaf is in this pass's group are written
        int li[R];
        float f[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const float y = lcdf_root_tab(s_px, s_py, s_ps, npts, lcdf_x(m, int64_t(k[r])));
            li[r] = lcdf_leaf(m, y) - leaf0;
            f[r] = lcdf_leaf_eval(lds[li[r] >= 0 && li[r] < cnt ? li[r] : 0], int64_t(k[r]));
        }
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int64_t i = base + int64_t(r) * kBidNT;
            if (i < n && li[r] >= 0 && li[r] < cnt) ids[i] = int32_t(ord.bucket(f[r]));
        }
    }
}

template <class K, class Ord>
static int launch_bucket_ids(const K *keys, int64_t n, const Ord &ord, int32_t *ids, hipStream_t s) {
    int64_t g = ceil_div(n, 256);
    if (g > 16384) g = 16384;
    TQP_LAUNCH("bucket_ids", (k_bucket_ids<K, Ord>), dim3(unsigned(g)), dim3(256), 0, s, keys, n,
               ord, ids);
    return check_launch("bucket ids");
}

template <class K>
static int launch_bucket_ids(const K *keys, int64_t n, const LearnedOrd<K> &ord, int32_t *ids,
                             hipStream_t s) {
    int32_t nl = 0;
    hipError_t e = hipMemcpyAsync(&nl, &ord.m->nleaf, sizeof nl, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(TQP_EHIP, "bucket ids: model header: %s", hipGetErrorString(e));
    if (nl < 1 || nl > kLeafMax) return set_error(TQP_EINVAL, "bucket ids: the model has %d leaves", nl);
    const size_t lds = size_t(kRootTabBytes) + size_t(kLdsLeafMax) * sizeof(Leaf);
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_bucket_ids_lds<K>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess)
        return set_error(TQP_EHIP, "bucket ids: LDS of %zu bytes: %s", lds, hipGetErrorString(e));
    for (int leaf0 = 0; leaf0 < nl; leaf0 += kLdsLeafMax) {
        TQP_LAUNCH("bucket_ids", k_bucket_ids_lds<K>, dim3(unsigned(kComputeUnits)), dim3(kBidNT),
                   lds, s, keys, n, ord, leaf0, ids);
        int rc = check_launch("bucket ids");
        if (rc) return rc;
    }
    return TQP_OK;
}

// The buckets that occur are the runs of the grouped bucket numbers: run r
// starts at rs[r] and ends where run r + 1 starts (the last one at n).
__device__ __forceinline__ int64_t run_end(const int32_t *rs, int64_t nruns, int64_t r,
                                           int64_t n) {
    return r + 1 < nruns ? int64_t(rs[r + 1]) : n;
}

// ---- windows: every bucket of at most kWinCap keys, sorted in LDS ------------
//
// The grouped keys are cut into windows of whole buckets: slot w holds the
// buckets that start in [w * kWin, (w + 1) * kWin).  All of them but the
// last lie inside that range, so they span fewer than kWin positions; when
// the last one makes the slot wider than kWinCap = 2 kWin, the slot becomes
// two windows, the buckets before the last and the last one alone, and a
// last bucket of more than kWinCap keys goes to the big-bucket path instead.
// Buckets are disjoint key ranges in key order, so sorting a window's keys
// as one sequence sorts each of its buckets.
constexpr int kWin = 4096;
constexpr int kWinCap = 2 * kWin;
constexpr int kWinNT = 1024;
constexpr int kWinPer = kWinCap / kWinNT;        // elements per thread
constexpr int kWinIdxBits = 13;                  // local index in a packed value
static_assert((1 << kWinIdxBits) == kWinCap, "packed index width");

__device__ __forceinline__ int64_t runs_lower_bound(const int32_t *rs, int64_t nruns, int64_t pos) {
    int64_t lo = 0, hi = nruns;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (int64_t(rs[mid]) < pos) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void push_big(BucketStats *stats, Overflow *big, int64_t big_cap,
                                         int64_t start, int64_t len) {
    const unsigned long long slot = atomicAdd(&stats->nbig, 1ull);
    if (int64_t(slot) < big_cap) big[slot] = Overflow{start, len, 0, 0, 0};
}

// One thread per slot: its one or two windows, win[w] and win[nwin + w], as
// {start, end} (end <= start: nothing to sort), and the hand-off of a bucket
// of more than kWinCap keys to the big-bucket path.
__global__ __launch_bounds__(256) void k_window_plan(const int32_t *__restrict__ rs,
                                                     const int64_t *__restrict__ d_nruns, int64_t n,
                                                     int64_t nwin, int2 *win, BucketStats *stats,
                                                     Overflow *big, int64_t big_cap) {
    const int64_t nruns = *d_nruns;
    for (int64_t w = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; w < nwin;
         w += int64_t(gridDim.x) * blockDim.x) {
        const int64_t a = runs_lower_bound(rs, nruns, w * kWin);
        const int64_t b = runs_lower_bound(rs, nruns, (w + 1) * kWin);
        const int64_t s0 = a < nruns ? rs[a] : n, e0 = b < nruns ? rs[b] : n;
        if (e0 - s0 <= kWinCap) {
            win[w] = make_int2(int(s0), int(e0));
            win[nwin + w] = make_int2(0, 0);
            continue;
        }
        const int64_t sl = rs[b - 1];            // the last bucket: [sl, e0), longer than kWin
        win[w] = make_int2(int(s0), int(sl));
        if (e0 - sl <= kWinCap) {
            win[nwin + w] = make_int2(int(sl), int(e0));
        } else {
            win[nwin + w] = make_int2(0, 0);
            push_big(stats, big, big_cap, sl, e0 - sl);
        }
    }
}

// The largest bucket (reported by the partition sort).
__global__ __launch_bounds__(256) void k_run_max(const int32_t *__restrict__ rs,
                                                 const int64_t *__restrict__ d_nruns, int64_t n,
                                                 BucketStats *stats) {
    const int64_t nruns = *d_nruns;
    unsigned long long mx = 0;
    for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < nruns;
         r += int64_t(gridDim.x) * blockDim.x) {
        const unsigned long long len = (unsigned long long)(run_end(rs, nruns, r, n) - rs[r]);
        mx = len > mx ? len : mx;
    }
    for (int o = 1; o < kWave; o <<= 1) {
        const unsigned long long om = __shfl_xor(mx, o, kWave);
        mx = om > mx ? om : mx;
    }
    if (lane_id() == 0 && mx) atomicMax(&stats->max_bucket, mx);
}

// Compare-exchange of two registers (ascending).
__device__ __forceinline__ void cx(uint64_t &a, uint64_t &b) {
    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// LDS index of element i of a window buffer: one padding slot per 8, so the
// 8 consecutive elements a thread reads or writes do not all fall on the
// same banks as its neighbours'.
__device__ __forceinline__ int wphys(int i) { return i + (i >> 3); }
constexpr int kWinPhys = kWinCap + kWinCap / 8;

// Persistent workgroups over the windows.  A window of m keys whose key span
// (max - min) is below 2^51 is sorted as packed values
// ((key - min) << 13 | local index), all distinct, by a merge sort in LDS:
// runs of 8 sorted in registers, then merge levels 8, 16, ... where each
// thread finds its 8 outputs by a merge-path search (the last run of a level
// may be short: nothing is padded beyond a multiple of 8).  Ties cannot
// occur, so the order is (key, position), the stable one.  A wider window is
// sorted by a bitonic network on (key, local index) in LDS.  Row ids are read
// through the local indices and written back in place.
template <class K>
__device__ __forceinline__ void window_load(const K *keys, const int32_t *rows, const int2 *win,
                                            int64_t w, int64_t nwin, int2 &se, K (&k)[kWinPer],
                                            int32_t (&r)[kWinPer]) {
    se = w < nwin ? win[w] : make_int2(0, 0);
    const int m = se.y - se.x;
#pragma unroll
    for (int i = 0; i < kWinPer; i++) {
        const int j = threadIdx.x + i * kWinNT;
        k[i] = j < m ? keys[int64_t(se.x) + j] : K(0);
        r[i] = j < m ? rows[int64_t(se.x) + j] : 0;
    }
}

template <class K>
__global__ __launch_bounds__(kWinNT) void k_window_sort(K *keys, int32_t *rows,
                                                        const int2 *__restrict__ win, int64_t nwin) {
    __shared__ uint64_t s_a[kWinPhys], s_b[kWinPhys];
    __shared__ int64_t s_lo[kWinNT / kWave], s_hi[kWinNT / kWave];
    const int tid = threadIdx.x;
    for (int64_t w = blockIdx.x; w < nwin; w += gridDim.x) {
        int2 se;
        K k[kWinPer];
        int32_t rw[kWinPer];
        window_load(keys, rows, win, w, nwin, se, k, rw);
        const int64_t s0 = se.x;
        const int m = se.y - se.x;
        if (m > 1) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
#pragma unroll
        for (int i = 0; i < kWinPer; i++) {
            const int j = tid + i * kWinNT;
            if (j < m) {
                lo = int64_t(k[i]) < lo ? int64_t(k[i]) : lo;
                hi = int64_t(k[i]) > hi ? int64_t(k[i]) : hi;
            }
        }
        for (int o = 1; o < kWave; o <<= 1) {
            const int64_t ol = shfl_xor(lo, o), oh = shfl_xor(hi, o);
            lo = ol < lo ? ol : lo;
            hi = oh > hi ? oh : hi;
        }
        if (lane_id() == 0) {
            s_lo[wave_id()] = lo;
            s_hi[wave_id()] = hi;
        }
        __syncthreads();
        lo = s_lo[0];
        hi = s_hi[0];
        for (int ww = 1; ww < kWinNT / kWave; ww++) {
            lo = s_lo[ww] < lo ? s_lo[ww] : lo;
            hi = s_hi[ww] > hi ? s_hi[ww] : hi;
        }
        const int m8 = (m + 7) & ~7;
        const bool packed = (uint64_t(hi) - uint64_t(lo)) < (uint64_t(1) << (64 - kWinIdxBits));
        uint64_t *res = nullptr;
        if (packed) {
#pragma unroll
            for (int i = 0; i < kWinPer; i++) {
                const int j = tid + i * kWinNT;
                if (j < m8)
                    s_a[wphys(j)] = j < m ? ((uint64_t(int64_t(k[i])) - uint64_t(lo)) << kWinIdxBits) |
                                                uint64_t(j)
                                          : ~uint64_t(0);
            }
            __syncthreads();
            // runs of 8 in registers
            if (tid * 8 < m8) {
                uint64_t v[8];
#pragma unroll
                for (int i = 0; i < 8; i++) v[i] = s_a[wphys(tid * 8 + i)];
#pragma unroll
                for (int r = 0; r < 8; r++)
#pragma unroll
                    for (int i = r & 1; i + 1 < 8; i += 2) cx(v[i], v[i + 1]);
#pragma unroll
                for (int i = 0; i < 8; i++) s_a[wphys(tid * 8 + i)] = v[i];
            }
            __syncthreads();
            uint64_t *src = s_a, *dst = s_b;
            for (int L = 8; L < m8; L <<= 1) {
                if (tid * 8 < m8) {
                    const int out0 = tid * 8;
                    const int base = (out0 / (2 * L)) * (2 * L);
                    const int d = out0 - base;
                    const int la = m8 - base < L ? m8 - base : L;
                    const int lb = m8 - base - L < 0 ? 0 : (m8 - base - L < L ? m8 - base - L : L);
                    const int pa = base, pb = base + L;          // run starts (logical)
                    int a = d - lb > 0 ? d - lb : 0, hb = d < la ? d : la;
                    while (a < hb) {
                        const int mid = (a + hb) >> 1;
                        if (src[wphys(pa + mid)] <= src[wphys(pb + d - 1 - mid)]) a = mid + 1;
                        else hb = mid;
                    }
                    int b = d - a;
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        const uint64_t va = a < la ? src[wphys(pa + a)] : ~uint64_t(0);
                        const uint64_t vb = b < lb ? src[wphys(pb + b)] : ~uint64_t(0);
                        const bool takeA = a < la && (b >= lb || va <= vb);
                        dst[wphys(out0 + i)] = takeA ? va : vb;
                        a += takeA ? 1 : 0;
                        b += takeA ? 0 : 1;
                    }
                }
                __syncthreads();
                uint64_t *t = src;
                src = dst;
                dst = t;
            }
            res = src;
        } else {
            // bitonic on (key, local index): keys in s_a, indices in s_b
            int P = 8;
            while (P < m) P <<= 1;
            K *sk = reinterpret_cast<K *>(s_a);
            uint16_t *sx = reinterpret_cast<uint16_t *>(s_b);
#pragma unroll
            for (int i = 0; i < kWinPer; i++) {
                const int j = tid + i * kWinNT;
                if (j < P) {
                    sk[j] = j < m ? k[i] : (sizeof(K) == 4 ? K(INT32_MAX) : K(INT64_MAX));
                    sx[j] = j < m ? uint16_t(j) : uint16_t(0xffff);
                }
            }
            __syncthreads();
            for (int kk = 2; kk <= P; kk <<= 1) {
                for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (int i = tid; i < P; i += kWinNT) {
                        const int l = i ^ jj;
                        if (l > i) {
                            const K ki = sk[i], kl = sk[l];
                            const uint16_t xi = sx[i], xl = sx[l];
                            const bool gt = ki > kl || (ki == kl && xi > xl);
                            if (gt == ((i & kk) == 0)) {
                                sk[i] = kl;
                                sk[l] = ki;
                                sx[i] = xl;
                                sx[l] = xi;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
        }
        // sorted keys and local indices into registers, then the row ids
        // permuted through LDS (the buffer the sort no longer uses)
        K ok[kWinPer];
        int idx[kWinPer];
#pragma unroll
        for (int i = 0; i < kWinPer; i++) {
            const int j = tid + i * kWinNT;
            idx[i] = 0;
            if (j < m) {
                if (packed) {
                    const uint64_t v = res[wphys(j)];
                    idx[i] = int(v & uint64_t(kWinCap - 1));
                    ok[i] = K(int64_t(uint64_t(lo) + (v >> kWinIdxBits)));
                } else {
                    idx[i] = reinterpret_cast<uint16_t *>(s_b)[j];
                    ok[i] = reinterpret_cast<K *>(s_a)[j];
                }
            }
        }
        __syncthreads();
        int32_t *srow = reinterpret_cast<int32_t *>(packed && res == s_a ? s_b : s_a);
        if (!packed) srow = reinterpret_cast<int32_t *>(s_b) + kWinCap;   // past the indices
#pragma unroll
        for (int i = 0; i < kWinPer; i++) {
            const int j = tid + i * kWinNT;
            if (j < m) srow[j] = rw[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kWinPer; i++) {
            const int j = tid + i * kWinNT;
            if (j < m) {
                keys[s0 + j] = ok[i];
                rows[s0 + j] = srow[idx[i]];
            }
        }
        __syncthreads();                 // LDS is reused by the next window
        }
    }
}

// Min and max key of the big buckets, in chunks of at most kChunk keys per
// workgroup: chunk c covers keys [cs[c].start, cs[c].start + cs[c].len) of big
// bucket cs[c].kmin (its index); one atomic min and max per chunk.
constexpr int64_t kChunk = 65536;

template <class K>
__global__ __launch_bounds__(256) void k_big_minmax(const K *__restrict__ keys,
                                                    const Overflow *__restrict__ cs,
                                                    long long *__restrict__ mm) {
    __shared__ long long s_lo[256 / kWave], s_hi[256 / kWave];
    const Overflow c = cs[blockIdx.x];
    long long lo = LLONG_MAX, hi = LLONG_MIN;
    for (int64_t i = c.start + threadIdx.x; i < c.start + c.len; i += blockDim.x) {
        const long long x = keys[i];
        lo = x < lo ? x : lo;
        hi = x > hi ? x : hi;
    }
    for (int o = 1; o < kWave; o <<= 1) {
        const long long ol = __shfl_xor(lo, o, kWave), oh = __shfl_xor(hi, o, kWave);
        lo = ol < lo ? ol : lo;
        hi = oh > hi ? oh : hi;
    }
    if (lane_id() == 0) {
        s_lo[wave_id()] = lo;
        s_hi[wave_id()] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / kWave; w++) {
            lo = s_lo[w] < lo ? s_lo[w] : lo;
            hi = s_hi[w] > hi ? s_hi[w] : hi;
        }
        atomicMin(&mm[2 * c.kmin], lo);
        atomicMax(&mm[2 * c.kmin + 1], hi);
    }
}

// The overflow buckets (sorted by start, off = prefix sum of len) are
// gathered into one contiguous run, sorted together, and scattered back.
// Buckets are disjoint key ranges in key order, so sorting their
// concatenation sorts each of them in place.  Element t of the run belongs to
// the last bucket whose off <= t.
__device__ __forceinline__ int64_t ovf_src(const Overflow *list, int nlist, int64_t t) {
    int lo = 0, hi = nlist - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (list[mid].off <= t) lo = mid;
        else hi = mid - 1;
    }
    return list[lo].start + (t - list[lo].off);
}

template <class K>
__global__ void k_ovf_gather(const K *keys, const int32_t *rows, const Overflow *list, int nlist,
                             int64_t total, K *kd, int32_t *rd) {
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t src = ovf_src(list, nlist, t);
        kd[t] = keys[src];
        rd[t] = rows[src];
    }
}

template <class K>
__global__ void k_ovf_scatter(const K *ks, const int32_t *rs, const Overflow *list, int nlist,
                              int64_t total, K *keys, int32_t *rows) {
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t dst = ovf_src(list, nlist, t);
        keys[dst] = ks[t];
        rows[dst] = rs[t];
    }
}

// ---- host -----------------------------------------------------------------------

struct TrainLayout {
    int64_t *sample, *sorted;
    void *rws;
    size_t rws_bytes;
    float *tx, *tq;
    int64_t *lstart;                    // kLeafMax + 1 leaf starts
    size_t bytes;
};

static TrainLayout train_layout(void *ws, int64_t m) {
    TrainLayout L = {};
    Carver c(ws);
    const int64_t mm = m > 0 ? m : 1;
    L.sample = c.take<int64_t>(size_t(mm));
    L.sorted = c.take<int64_t>(size_t(mm));
    L.rws_bytes = radix_ws_bytes(mm, 8, 8, 0);
    L.rws = c.take<char>(L.rws_bytes);
    L.tx = c.take<float>(kTrainPoints);
    L.tq = c.take<float>(kTrainPoints);
    L.lstart = c.take<int64_t>(size_t(kLeafMax) + 1);
    L.bytes = c.bytes();
    return L;
}

static int64_t sample_count(const tqp_col *cols, int ncols, int64_t stride) {
    int64_t m = 0;
    for (int i = 0; i < ncols; i++) m += ceil_div(cols[i].len, stride);
    return m;
}

struct PartLayout {
    BucketStats *stats;
    Overflow *ovf;                      // big buckets, then the overflow list
    int64_t ovf_cap;
    Overflow *chunks;                   // min/max chunks of the big buckets
    int64_t chunk_cap;
    long long *mm;                      // min, max per big bucket
    int32_t *ids, *ids_sorted;          // bucket number of every key, before / after grouping
    int2 *win;                          // windows of whole buckets
    int32_t *ruk, *rus;                 // runs of the grouped bucket numbers: value, start
    int64_t *d_nruns;
    uint64_t *rle_ws;
    void *rws;
    size_t rws_bytes;
    void *tmp_k, *tmp2_k;
    int32_t *tmp_r, *tmp2_r;
    void *fws;
    size_t fws_bytes;
    size_t bytes;
};

static PartLayout part_layout(void *ws, int64_t n, int ksize, int bucket_bits) {
    PartLayout L = {};
    Carver c(ws);
    const int64_t nn = n > 0 ? n : 1;
    L.stats = c.take<BucketStats>(1);
    L.ovf_cap = (int64_t(1) << bucket_bits) < kOvfCap ? (int64_t(1) << bucket_bits) : kOvfCap;
    L.ovf = c.take<Overflow>(size_t(L.ovf_cap));
    L.chunk_cap = nn / kChunk + 1 + L.ovf_cap;
    L.chunks = c.take<Overflow>(size_t(L.chunk_cap));
    L.mm = c.take<long long>(size_t(2 * L.ovf_cap));
    L.ids = c.take<int32_t>(size_t(nn));
    L.ids_sorted = c.take<int32_t>(size_t(nn));
    L.win = c.take<int2>(size_t(2 * ceil_div(nn, kWin)));
    L.ruk = c.take<int32_t>(size_t(nn));
    L.rus = c.take<int32_t>(size_t(nn));
    L.d_nruns = c.take<int64_t>(1);
    L.rle_ws = c.take<uint64_t>(rle_words(nn));
    L.rws_bytes = radix_ws_bytes(nn, 4, npass_for(bucket_bits), ksize);
    L.rws = c.take<char>(L.rws_bytes);
    // fallback: the gathered overflow keys, their sorted copy, the radix workspace
    L.tmp_k = c.take<char>(size_t(nn) * ksize);
    L.tmp_r = c.take<int32_t>(size_t(nn));
    L.tmp2_k = c.take<char>(size_t(nn) * ksize);
    L.tmp2_r = c.take<int32_t>(size_t(nn));
    L.fws_bytes = radix_ws_bytes(nn, ksize, ksize, 0);
    L.fws = c.take<char>(L.fws_bytes);
    L.bytes = c.bytes();
    return L;
}

// Copies host -> device on s and waits, so the host buffer may go away.
static int upload(void *dst, const void *src, size_t bytes, hipStream_t s, const char *what) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? TQP_OK : set_error(TQP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static int download(void *dst, const void *src, size_t bytes, hipStream_t s, const char *what) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? TQP_OK : set_error(TQP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

template <class K, class Ord>
static int partition_sort_typed(const K *key, const int32_t *in_rows, int64_t n, Ord ord,
                                int bucket_bits, K *out_key, int32_t *out_rows, int64_t *h_stats,
                                void *ws, hipStream_t s) {
    PartLayout L = part_layout(ws, n, sizeof(K), bucket_bits);
    int rc = fill_u64(L.stats, 0, sizeof(BucketStats) / 8, s);
    if (rc) return rc;
    // 1. every key's bucket number, once
    if ((rc = launch_bucket_ids(key, n, ord, L.ids, s))) return rc;
    // 2. group the keys by bucket: stable radix passes over the bucket
    // number, the key and its row id moving along
    SortCols sc = {};
    sc.rows_in = in_rows;
    sc.rows_out = out_rows;
    sc.npay = 1;
    sc.pin[0] = key;
    sc.pout[0] = out_key;
    sc.pdt[0] = sizeof(K) == 4 ? TQP_INT32 : TQP_INT64;
    rc = run_radix<int32_t, KeyOrd<int32_t>>(L.ids, n, nullptr, bucket_bits, KeyOrd<int32_t>{0},
                                             L.ids_sorted, sc, L.rws, s);
    if (rc) return rc;
    // 3. the buckets that occur (runs of the grouped bucket numbers), then
    // each one sorted: short ones in registers, the rest by a workgroup in LDS
    if ((rc = rle_i32(L.ids_sorted, n, L.ruk, L.rus, L.d_nruns, L.rle_ws, s))) return rc;
    {
        const int64_t nwin = ceil_div(n, kWin);
        int64_t g = ceil_div(n, 256);
        if (g > 4096) g = 4096;
        TQP_LAUNCH("run_max", k_run_max, dim3(unsigned(g)), dim3(256), 0, s, L.rus, L.d_nruns, n,
                   L.stats);
        if ((rc = check_launch("bucket sizes"))) return rc;
        g = ceil_div(nwin, 256);
        TQP_LAUNCH("window_plan", k_window_plan, dim3(unsigned(g)), dim3(256), 0, s, L.rus,
                   L.d_nruns, n, nwin, L.win, L.stats, L.ovf, L.ovf_cap);
        if ((rc = check_launch("window plan"))) return rc;
        TQP_LAUNCH("window_sort", k_window_sort<K>, dim3(unsigned(kComputeUnits)), dim3(kWinNT), 0,
                   s, out_key, out_rows, L.win, 2 * nwin);
        if ((rc = check_launch("window sort"))) return rc;
    }
    BucketStats hs;
    if ((rc = download(&hs, L.stats, sizeof hs, s, "partition stats"))) return rc;
    int64_t n_ovf = 0, ovf_keys = 0, single = 0;
    const int64_t cap = tune(kTunePartOvfCap) < L.ovf_cap ? tune(kTunePartOvfCap) : L.ovf_cap;
    if (int64_t(hs.nbig) > cap) {
        // More big buckets than the list holds: the partition is useless for
        // these keys, so sort the whole input by the plain radix sort.
        SortCols fc = {};
        fc.rows_in = in_rows;
        fc.rows_out = out_rows;
        rc = run_radix<K, KeyOrd<K>>(key, n, nullptr, int(8 * sizeof(K)),
                                     KeyOrd<K>{sizeof(K) == 4 ? K(INT32_MIN) : K(INT64_MIN)},
                                     out_key, fc, L.fws, s);
        if (rc) return rc;
        n_ovf = int64_t(hs.nbig);
        ovf_keys = n;
    } else if (hs.nbig > 0) {
        // 3. min and max of each big bucket: equal means one key, already in
        // stable order; the others are re-sorted together
        const size_t nbig = size_t(hs.nbig);
        std::vector<Overflow> big(nbig);
        if ((rc = download(big.data(), L.ovf, sizeof(Overflow) * nbig, s, "big buckets"))) return rc;
        std::vector<Overflow> chunks;
        for (size_t j = 0; j < nbig; j++)
            for (int64_t o = 0; o < big[j].len; o += kChunk)
                chunks.push_back(Overflow{big[j].start + o,
                                          big[j].len - o < kChunk ? big[j].len - o : kChunk,
                                          int64_t(j), 0, 0});
        if (int64_t(chunks.size()) > L.chunk_cap)
            return set_error(TQP_EHIP, "partition sort: %zu chunks exceed %lld", chunks.size(),
                             (long long)L.chunk_cap);
        std::vector<long long> mm(2 * nbig);
        for (size_t j = 0; j < nbig; j++) {
            mm[2 * j] = LLONG_MAX;
            mm[2 * j + 1] = LLONG_MIN;
        }
        if ((rc = upload(L.chunks, chunks.data(), sizeof(Overflow) * chunks.size(), s, "chunks")))
            return rc;
        if ((rc = upload(L.mm, mm.data(), sizeof(long long) * mm.size(), s, "min/max"))) return rc;
        TQP_LAUNCH("big_minmax", k_big_minmax<K>, dim3(unsigned(chunks.size())), dim3(256), 0, s,
                   out_key, L.chunks, L.mm);
        if ((rc = check_launch("big bucket min/max"))) return rc;
        if ((rc = download(mm.data(), L.mm, sizeof(long long) * mm.size(), s, "min/max"))) return rc;
        std::vector<Overflow> list;
        for (size_t j = 0; j < nbig; j++) {
            if (mm[2 * j] == mm[2 * j + 1]) {
                single++;
                continue;
            }
            list.push_back(Overflow{big[j].start, big[j].len, int64_t(mm[2 * j]),
                                    int64_t(mm[2 * j + 1]), 0});
            ovf_keys += big[j].len;
        }
        n_ovf = int64_t(list.size());
        if (!list.empty()) {
            // 4. gather the overflowing buckets, sort them together, scatter back
            std::sort(list.begin(), list.end(),
                      [](const Overflow &a, const Overflow &b) { return a.start < b.start; });
            int64_t total = 0, kmin = list[0].kmin, kmax = list[0].kmax;
            for (Overflow &o : list) {
                o.off = total;
                total += o.len;
                kmin = o.kmin < kmin ? o.kmin : kmin;
                kmax = o.kmax > kmax ? o.kmax : kmax;
            }
            if ((rc = upload(L.ovf, list.data(), sizeof(Overflow) * list.size(), s, "overflow list")))
                return rc;
            int64_t g = ceil_div(total, 256);
            if (g > 8192) g = 8192;
            K *tk = static_cast<K *>(L.tmp_k), *tk2 = static_cast<K *>(L.tmp2_k);
            TQP_LAUNCH("ovf_gather", k_ovf_gather<K>, dim3(unsigned(g)), dim3(256), 0, s, out_key,
                       out_rows, L.ovf, int(list.size()), total, tk, L.tmp_r);
            if ((rc = check_launch("overflow gather"))) return rc;
            const uint64_t span = uint64_t(kmax) - uint64_t(kmin);
            int bits = 0;
            while (bits < 64 && (span >> bits) != 0) bits++;
            SortCols fc = {};
            fc.rows_in = L.tmp_r;
            fc.rows_out = L.tmp2_r;
            rc = run_radix<K, KeyOrd<K>>(tk, total, nullptr, bits, KeyOrd<K>{K(kmin)}, tk2, fc,
                                         L.fws, s);
            if (rc) return rc;
            TQP_LAUNCH("ovf_scatter", k_ovf_scatter<K>, dim3(unsigned(g)), dim3(256), 0, s, tk2,
                       L.tmp2_r, L.ovf, int(list.size()), total, out_key, out_rows);
            if ((rc = check_launch("overflow scatter"))) return rc;
        }
    }
    if (h_stats) {
        h_stats[0] = int64_t(hs.max_bucket);
        h_stats[1] = n_ovf;
        h_stats[2] = ovf_keys;
        h_stats[3] = single;
    }
    return TQP_OK;
}

}  // namespace tqp

using namespace tqp;

TQP_API size_t tqp_lcdf_model_bytes(int nleaf) {
    if (nleaf < 1 || nleaf > kLeafMax) return 0;
    return model_bytes(nleaf);
}

TQP_API size_t tqp_lcdf_train_workspace_bytes(int64_t total_keys, int sample_stride) {
    if (total_keys < 0 || sample_stride < 1) return 0;
    return train_layout(nullptr, ceil_div(total_keys, sample_stride) + 2).bytes;
}

TQP_API int tqp_lcdf_train(const tqp_col *cols, int ncols, int sample_stride, int nleaf, int steps,
                           float lr, void *model, size_t model_size, void *ws, size_t ws_bytes,
                           void *stream) {
    clear_error();
    if (!cols || ncols < 1 || ncols > 2 || sample_stride < 1 || nleaf < 1 || nleaf > kLeafMax ||
        steps < 0 || !model)
        return set_error(TQP_EINVAL, "tqp_lcdf_train: bad argument");
    for (int i = 0; i < ncols; i++)
        if ((cols[i].dtype != TQP_INT32 && cols[i].dtype != TQP_INT64) || cols[i].len < 0 ||
            (cols[i].len > 0 && !cols[i].data))
            return set_error(TQP_EINVAL, "tqp_lcdf_train: column %d is invalid", i);
    if (model_size < model_bytes(nleaf))
        return set_error(TQP_ECAPACITY, "tqp_lcdf_train: model needs %zu bytes", model_bytes(nleaf));
    int64_t total = 0;
    for (int i = 0; i < ncols; i++) total += cols[i].len;
    const int64_t m = sample_count(cols, ncols, sample_stride);
    if (m < 2) return set_error(TQP_EINVAL, "tqp_lcdf_train: fewer than two sample keys");
    if (m > (int64_t(1) << 30) - 1)
        return set_error(TQP_EINVAL, "tqp_lcdf_train: more than 2^30 - 1 sample keys");
    const size_t need = tqp_lcdf_train_workspace_bytes(total, sample_stride);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "tqp_lcdf_train: workspace needs %zu bytes", need);
    hipStream_t s = as_stream(stream);
    TrainLayout L = train_layout(ws, m);
    LcdfModel *mod = static_cast<LcdfModel *>(model);
    int rc;
    {
        int64_t g = ceil_div(m, 256);
        if (g > 4096) g = 4096;
        TQP_LAUNCH("lcdf_sample", k_lcdf_sample, dim3(unsigned(g)), dim3(256), 0, s, cols[0].data,
                   cols[0].dtype, cols[0].len, ncols > 1 ? cols[1].data : nullptr,
                   ncols > 1 ? cols[1].dtype : TQP_INT64, ncols > 1 ? cols[1].len : 0,
                   int64_t(sample_stride), L.sample);
        if ((rc = check_launch("lcdf sample"))) return rc;
    }
    SortCols none = {};
    rc = run_radix<int64_t, KeyOrd<int64_t>>(L.sample, m, nullptr, 64, KeyOrd<int64_t>{INT64_MIN},
                                             L.sorted, none, L.rws, s);
    if (rc) return rc;
    const int T = int(m < kTrainPoints ? m : kTrainPoints);
    TQP_LAUNCH("lcdf_init", k_lcdf_init, dim3(1), dim3(256), 0, s, L.sorted, m, nleaf, mod, L.tx,
               L.tq, T);
    if ((rc = check_launch("lcdf init"))) return rc;
    if (steps > 0)
        TQP_LAUNCH("lcdf_fit", k_lcdf_fit, dim3(1), dim3(kFitNT), 0, s, mod, L.tx, L.tq, T, steps, lr);
    if ((rc = check_launch("lcdf train"))) return rc;
    TQP_LAUNCH("lcdf_finalize", k_lcdf_finalize, dim3(1), dim3(64), 0, s, mod);
    {
        int64_t g = ceil_div(m, 256);
        if (g > 4096) g = 4096;
        TQP_LAUNCH("lcdf_leaf_starts", k_leaf_starts, dim3(unsigned(g)), dim3(256), 0, s, mod,
                   L.sorted, m, L.lstart);
    }
    TQP_LAUNCH("lcdf_leaf_fit", k_lcdf_leaf_fit, dim3(unsigned(nleaf)), dim3(256), 0, s, mod,
               L.sorted, m, L.lstart);
    TQP_LAUNCH("lcdf_leaf_fill", k_lcdf_leaf_fill, dim3(1), dim3(kFillNT), 0, s, mod);
    return check_launch("lcdf leaves");
}

TQP_API int tqp_lcdf_buckets(const void *model, const tqp_col *keys, int bucket_bits,
                             int32_t *out_bucket, void *stream) {
    clear_error();
    if (!model || !keys || bucket_bits < 1 || bucket_bits > 24 ||
        (keys->dtype != TQP_INT32 && keys->dtype != TQP_INT64) ||
        (keys->len > 0 && (!keys->data || !out_bucket)))
        return set_error(TQP_EINVAL, "tqp_lcdf_buckets: bad argument");
    if (keys->len == 0) return TQP_OK;
    hipStream_t s = as_stream(stream);
    const LcdfModel *m = static_cast<const LcdfModel *>(model);
    const float scale = float(1u << bucket_bits);
    const uint32_t top = (1u << bucket_bits) - 1;
    if (keys->dtype == TQP_INT32)
        return launch_bucket_ids(static_cast<const int32_t *>(keys->data), keys->len,
                                 LearnedOrd<int32_t>{m, m->leaf, scale, top}, out_bucket, s);
    return launch_bucket_ids(static_cast<const int64_t *>(keys->data), keys->len,
                             LearnedOrd<int64_t>{m, m->leaf, scale, top}, out_bucket, s);
}

TQP_API size_t tqp_partition_sort_workspace_bytes(int64_t n, int dtype, int bucket_bits) {
    if (n < 0 || (dtype != TQP_INT32 && dtype != TQP_INT64) || bucket_bits < 1 || bucket_bits > 24)
        return 0;
    Carver c(nullptr);
    c.take<int64_t>(2);
    c.take<char>(part_layout(nullptr, n, dtype_size(dtype), bucket_bits).bytes);
    return c.bytes();
}

TQP_API int tqp_partition_sort(const tqp_col *key, const int32_t *in_rows, uint32_t mode,
                               const void *model, int bucket_bits, int key_bits, int64_t key_min,
                               const tqp_col *out_key, int32_t *out_rows, int64_t *h_stats,
                               void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!key || !out_key || (key->len > 0 && (!key->data || !out_key->data || !out_rows)))
        return set_error(TQP_EINVAL, "tqp_partition_sort: null argument");
    if ((key->dtype != TQP_INT32 && key->dtype != TQP_INT64) || out_key->dtype != key->dtype)
        return set_error(TQP_EINVAL, "tqp_partition_sort: keys must be int32 or int64");
    if (mode != TQP_PART_LEARNED && mode != TQP_PART_RADIX)
        return set_error(TQP_EINVAL, "tqp_partition_sort: unknown mode");
    if (mode == TQP_PART_LEARNED && !model)
        return set_error(TQP_EINVAL, "tqp_partition_sort: learned mode needs a model");
    if (bucket_bits < 1 || bucket_bits > 24 || key_bits < 0 || key_bits > 64)
        return set_error(TQP_EINVAL, "tqp_partition_sort: bucket_bits in [1, 24], key_bits in [0, 64]");
    const int64_t n = key->len;
    if (n > (int64_t(1) << 30) - 1 || out_key->len < n)
        return set_error(TQP_EINVAL, "tqp_partition_sort: n must be in [0, 2^30 - 1], out >= n");
    const size_t need = tqp_partition_sort_workspace_bytes(n, key->dtype, bucket_bits);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "tqp_partition_sort: workspace needs %zu bytes", need);
    if (n == 0) {
        if (h_stats) h_stats[0] = h_stats[1] = h_stats[2] = h_stats[3] = 0;
        return TQP_OK;
    }
    hipStream_t s = as_stream(stream);
    Carver c(ws);
    void *scratch = c.take<int64_t>(2);
    void *pws = c.take<char>(part_layout(nullptr, n, dtype_size(key->dtype), bucket_bits).bytes);
    if (mode == TQP_PART_RADIX && key_bits == 0) {
        int rc = derive_key_range(key->data, key->dtype, n, nullptr, scratch, s, &key_min, &key_bits);
        if (rc) return rc;
    }
    const int shift = key_bits > bucket_bits ? key_bits - bucket_bits : 0;
    if (key->dtype == TQP_INT32) {
        const int32_t *k = static_cast<const int32_t *>(key->data);
        int32_t *ok = static_cast<int32_t *>(out_key->data);
        if (mode == TQP_PART_LEARNED)
            return partition_sort_typed(k, in_rows, n,
                                        LearnedOrd<int32_t>{static_cast<const LcdfModel *>(model),
                                                            static_cast<const LcdfModel *>(model)->leaf,
                                                            float(1u << bucket_bits),
                                                            (1u << bucket_bits) - 1},
                                        bucket_bits, ok, out_rows, h_stats, pws, s);
        return partition_sort_typed(k, in_rows, n, MsdOrd<int32_t>{int32_t(key_min), shift, (1u << bucket_bits) - 1},
                                    bucket_bits, ok, out_rows, h_stats, pws, s);
    }
    const int64_t *k = static_cast<const int64_t *>(key->data);
    int64_t *ok = static_cast<int64_t *>(out_key->data);
    if (mode == TQP_PART_LEARNED)
        return partition_sort_typed(k, in_rows, n,
                                    LearnedOrd<int64_t>{static_cast<const LcdfModel *>(model),
                                                        static_cast<const LcdfModel *>(model)->leaf,
                                                        float(1u << bucket_bits),
                                                        (1u << bucket_bits) - 1},
                                    bucket_bits, ok, out_rows, h_stats, pws, s);
    return partition_sort_typed(k, in_rows, n, MsdOrd<int64_t>{key_min, shift, (1u << bucket_bits) - 1}, bucket_bits, ok,
                                out_rows, h_stats, pws, s);
}
