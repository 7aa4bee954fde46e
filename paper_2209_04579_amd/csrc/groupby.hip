// GROUP BY with SUM / COUNT / SUM of products, int64 exact modulo 2^64.
//
// Sort-based path (general).  After the keys are sorted, every group is a run.
// Because int64 addition modulo 2^64 is a group operation, the sum of a run
// equals the difference of the running prefix sum at its last row and at the
// last row of the run before it.  One single-pass scan over the sorted rows
// (block scan + decoupled look-back carrying the head count and one running
// sum per aggregate) writes, at every run end, the running sums and the
// unique key; a second, small kernel over the groups takes adjacent
// differences.  No atomics, so the output is the same bytes on every run.
//
// Dense path.  When the caller bounds the key to a small domain
// [key_lo, key_lo + span), each workgroup accumulates into LDS counters
// indexed by key - key_lo and adds its totals to device accumulators; a final
// one-workgroup kernel emits the non-empty keys in ascending order.  Integer
// addition is order-free, so this path is bit-identical to the sorted one.
#include "tqp_internal.hpp"

namespace tqp {

constexpr int kGbNT = 512;
constexpr int kGbIPT = 8;
constexpr int kGbTile = kGbNT * kGbIPT;
constexpr int kMaxAgg = 4;
constexpr int kMaxVals = 8;
constexpr int kNV = kMaxAgg + 1;        // head count + one running sum per aggregate

struct AggArgs {
    const void *val[kMaxVals];
    int64_t vlen[kMaxVals];
    int32_t vdt[kMaxVals];
    int32_t op[kMaxAgg];
    int32_t ia[kMaxAgg];
    int32_t ib[kMaxAgg];
    int64_t ic[kMaxAgg];
    int32_t nagg;
    const int32_t *val_rows;
};

// The second factor of a product aggregate: vals[b] itself (SUM_PRODUCT) or
// c - vals[b] (SUM_DIFF_PRODUCT), in wrapping int64 arithmetic, so the product
// is the exact one modulo 2^64.
__device__ __forceinline__ int64_t agg_second(const AggArgs &a, int g, int64_t y) {
    return a.op[g] == TQP_AGG_SUM_PRODUCT ? y : int64_t(uint64_t(a.ic[g]) - uint64_t(y));
}

__device__ __forceinline__ int64_t agg_term(const AggArgs &a, int g, int64_t row) {
    if (a.op[g] == TQP_AGG_COUNT) return 1;
    const int x = a.ia[g];
    const int64_t vx = (row >= 0 && row < a.vlen[x]) ? load_any(a.val[x], a.vdt[x], row) : 0;
    if (a.op[g] == TQP_AGG_SUM) return vx;
    const int y = a.ib[g];
    const int64_t vy = (row >= 0 && row < a.vlen[y]) ? load_any(a.val[y], a.vdt[y], row) : 0;
    return int64_t(uint64_t(vx) * uint64_t(agg_second(a, g, vy)));
}

// Look-back over kNV int64 values.  Each tile owns 2 * kNV status words; word
// 2k holds the low 32 bits of value k and word 2k+1 the high 32 bits, each
// tagged in its top bits with 1 (tile aggregate) or 2 (inclusive prefix); 0
// means not written yet.  Every word is a single relaxed agent-scope atomic,
// so no fence orders one against another: a reader accepts a tile's record
// only when all the words it needs carry the same non-zero tag, and otherwise
// reads again.  An aggregate, once written, never changes until the same
// words are rewritten as the inclusive prefix.
__device__ __forceinline__ uint64_t tag_word(uint64_t tag, uint32_t half) {
    return (tag << 62) | half;
}

template <int NV>
__device__ __forceinline__ void publish_multi(uint64_t *rec, uint64_t tag, const int64_t (&v)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
        st_relaxed(&rec[2 * k], tag_word(tag, uint32_t(uint64_t(v[k]))));
        st_relaxed(&rec[2 * k + 1], tag_word(tag, uint32_t(uint64_t(v[k]) >> 32)));
    }
}

// Look-back over NV values (records of 2 * kNV words per tile; the first
// 2 * NV are used), one predecessor per lane per round trip.
template <int NV>
__device__ __forceinline__ void lookback_multi(uint64_t *status, int64_t tile,
                                               const int64_t (&agg)[NV], int64_t (&excl)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; k++) excl[k] = 0;
    if (tile == 0) {
        if (lane_id() == 0) publish_multi<NV>(status, 2, agg);
        return;
    }
    if (lane_id() == 0) publish_multi<NV>(status + tile * 2 * kNV, 1, agg);
    int64_t base = tile - 1;
    while (true) {
        const int64_t idx = base - lane_id();
        uint64_t tag = 2;
        int64_t v[NV];
#pragma unroll
        for (int k = 0; k < NV; k++) v[k] = 0;
        if (idx >= 0) {
            const uint64_t *rec = status + idx * 2 * kNV;
            while (true) {
                // all words are read independently (no early exit), then checked
                uint64_t w[2 * NV];
#pragma unroll
                for (int k = 0; k < 2 * NV; k++) w[k] = ld_relaxed(&rec[k]);
                const uint64_t first = w[0] >> 62;
                bool ok = first != 0;
#pragma unroll
                for (int k = 0; k < NV; k++) {
                    ok = ok && (w[2 * k] >> 62) == first && (w[2 * k + 1] >> 62) == first;
                    v[k] = int64_t((w[2 * k + 1] << 32) | (w[2 * k] & 0xffffffffu));
                }
                if (ok) {
                    tag = first;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        const uint64_t inc = ballot(tag == 2);
        const int stop = inc ? (__ffsll(static_cast<long long>(inc)) - 1) : (kWave - 1);
#pragma unroll
        for (int k = 0; k < NV; k++) {
            const int64_t x = lane_id() <= stop ? v[k] : 0;
            excl[k] += wave_sum(x);
        }
        if (inc) break;
        base -= kWave;
    }
    if (lane_id() == 0) {
        int64_t incl[NV];
#pragma unroll
        for (int k = 0; k < NV; k++) incl[k] = int64_t(uint64_t(excl[k]) + uint64_t(agg[k]));
        publish_multi<NV>(status + tile * 2 * kNV, 2, incl);
    }
}

// Reads the value column of N rows (row ids in rows[]; 0 where the bit of
// valid is clear or the row is outside the column).  One dtype test for all
// N and no predicated loads (such rows read element 0), so the N loads issue
// back to back and the sign extension waits for all of them at once.
template <int N>
__device__ __forceinline__ void load_vals(const void *col, int dt, int64_t len,
                                          const int32_t (&rows)[N], uint32_t valid,
                                          int64_t (&out)[N]) {
    if (len <= 0) {
#pragma unroll
        for (int r = 0; r < N; r++) out[r] = 0;
        return;
    }
    bool ok[N];
    int32_t li[N];
    uint64_t raw[N];
#pragma unroll
    for (int r = 0; r < N; r++) {
        ok[r] = ((valid >> r) & 1) && rows[r] >= 0 && rows[r] < len;
        li[r] = ok[r] ? rows[r] : 0;
    }
    load_raw<N>(col, dt, li, raw);
#pragma unroll
    for (int r = 0; r < N; r++) out[r] = ok[r] ? sext_of(raw[r], dt) : 0;
}

// Value-row ids of positions idx[] (position i itself without val_rows; 0
// past cnt), all loads issued together; needs cnt >= 1.
template <int N>
__device__ __forceinline__ void load_rows(const int32_t *val_rows, const int64_t (&idx)[N], int64_t cnt,
                                          int32_t (&row)[N]) {
    if (val_rows) {
        int64_t li[N];
        uint64_t rr[N];
#pragma unroll
        for (int r = 0; r < N; r++) li[r] = idx[r] < cnt ? idx[r] : 0;
#pragma unroll
        for (int r = 0; r < N; r++) rr[r] = uint32_t(val_rows[li[r]]);
#pragma unroll
        for (int r = 0; r < N; r++) row[r] = idx[r] < cnt ? int32_t(uint32_t(rr[r])) : 0;
    } else {
#pragma unroll
        for (int r = 0; r < N; r++) row[r] = idx[r] < cnt ? int32_t(idx[r]) : 0;
    }
}

// Exclusive prefix sums of N values per thread across the block, with one
// pair of barriers for all N.  lds holds (NT / 64) * N entries.
template <int NT, int N>
__device__ __forceinline__ void block_excl_scan_n(const int64_t (&v)[N], int64_t (&ex)[N],
                                                  int64_t (&tot)[N], int64_t *lds) {
    constexpr int NW = NT / kWave;
    int64_t inc[N];
#pragma unroll
    for (int k = 0; k < N; k++) inc[k] = wave_incl_scan(v[k]);
    const int w = wave_id();
    if (lane_id() == kWave - 1) {
#pragma unroll
        for (int k = 0; k < N; k++) lds[w * N + k] = inc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; k++) {
        int64_t pre = 0, t = 0;
#pragma unroll
        for (int i = 0; i < NW; i++) {
            const int64_t x = lds[i * N + k];
            if (i < w) pre += x;
            t += x;
        }
        ex[k] = pre + inc[k] - v[k];
        tot[k] = t;
    }
    __syncthreads();
}

// One single-pass scan over sorted keys for NAGG aggregates: head count and
// running sums carried across tiles by look-back; run ends write the running
// sums, run heads write the key.  Every value is loaded once, into registers.
template <class K, int NAGG>
__global__ __launch_bounds__(kGbNT, 4) void k_gb_scan(const K *__restrict__ keys, int64_t n,
                                                   const int64_t *d_n, AggArgs a,
                                                   K *__restrict__ out_key, int64_t key_cap,
                                                   int64_t *__restrict__ ends /* [NAGG][n] */,
                                                   int64_t ends_stride, int64_t *d_ngroups,
                                                   uint32_t *ticket, uint64_t *status) {
    __shared__ int64_t s_tile;
    __shared__ int64_t s_scan[(kGbNT / kWave) * (NAGG + 1)];
    __shared__ int64_t s_term[NAGG * kGbIPT * kGbNT];   // [NAGG][kGbIPT][kGbNT]
    __shared__ int64_t s_excl[kNV];
    const int64_t cnt = count_of(d_n, n);
    const int64_t ntiles = ceil_div(cnt, kGbTile);
    const bool kvec = reinterpret_cast<uintptr_t>(keys) % 16 == 0;
    const bool rvec = a.val_rows && reinterpret_cast<uintptr_t>(a.val_rows) % 16 == 0;
    for (;;) {
    const int64_t tile = take_tile(ticket, &s_tile);
    if (tile >= ntiles) {
        if (tile == 0 && threadIdx.x == 0) *d_ngroups = 0;
        break;
    }
    const int64_t row0 = tile * kGbTile + int64_t(threadIdx.x) * kGbIPT;
    constexpr int R = kGbIPT;
    const bool full = row0 + R <= cnt;
    K v[R];
    if (kvec && full) {
        constexpr int kPer = 16 / sizeof(K);
        const int4 *q = reinterpret_cast<const int4 *>(keys + row0);
#pragma unroll
        for (int j = 0; j < R / kPer; j++) {
            int4 x = q[j];
            const K *e = reinterpret_cast<const K *>(&x);
#pragma unroll
            for (int t = 0; t < kPer; t++) v[j * kPer + t] = e[t];
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; r++) v[r] = row0 + r < cnt ? keys[row0 + r] : K(0);
    }
    int32_t rows[R];
    if (rvec && full) {
        const int4 *q = reinterpret_cast<const int4 *>(a.val_rows + row0);
#pragma unroll
        for (int j = 0; j < R / 4; j++) {
            int4 x = q[j];
            rows[4 * j + 0] = x.x;
            rows[4 * j + 1] = x.y;
            rows[4 * j + 2] = x.z;
            rows[4 * j + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; r++)
            rows[r] = row0 + r < cnt ? (a.val_rows ? a.val_rows[row0 + r] : int32_t(row0 + r)) : 0;
    }
    const K before = row0 > 0 && row0 <= cnt ? keys[row0 - 1] : K(0);
    const K after = row0 + R < cnt ? keys[row0 + R] : K(0);
    uint32_t head = 0, end = 0, valid = 0;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int64_t i = row0 + r;
        if (i < cnt) {
            valid |= 1u << r;
            const K prv = r == 0 ? before : v[r - 1];
            const K nxt = r == R - 1 ? after : v[r + 1];
            if (i == 0 || v[r] != prv) head |= 1u << r;
            if (i == cnt - 1 || v[r] != nxt) end |= 1u << r;
        }
    }
    // per-row aggregate terms, loaded once
    int64_t term[NAGG][R];
#pragma unroll
    for (int g = 0; g < NAGG; g++) {
        if (a.op[g] == TQP_AGG_COUNT) {
#pragma unroll
            for (int r = 0; r < R; r++) term[g][r] = (valid >> r) & 1;
        } else {
            const int x = a.ia[g];
            load_vals<R>(a.val[x], a.vdt[x], a.vlen[x], rows, valid, term[g]);
            if (a.op[g] >= TQP_AGG_SUM_PRODUCT) {
                int64_t other[R];
                const int y = a.ib[g];
                load_vals<R>(a.val[y], a.vdt[y], a.vlen[y], rows, valid, other);
#pragma unroll
                for (int r = 0; r < R; r++)
                    term[g][r] = int64_t(uint64_t(term[g][r]) * uint64_t(agg_second(a, g, other[r])));
            }
        }
    }
    // the terms wait in LDS (conflict-free: row r of thread t at r * kGbNT + t)
    // while the block scan and the look-back run, so they hold no registers
#pragma unroll
    for (int g = 0; g < NAGG; g++) {
#pragma unroll
        for (int r = 0; r < R; r++) s_term[(g * R + r) * kGbNT + threadIdx.x] = term[g][r];
    }
    int64_t agg[NAGG + 1], excl[NAGG + 1], tot[NAGG + 1];
    agg[0] = __popc(head);
#pragma unroll
    for (int g = 0; g < NAGG; g++) {
        uint64_t s = 0;
#pragma unroll
        for (int r = 0; r < R; r++) s += uint64_t(term[g][r]);
        agg[g + 1] = int64_t(s);
    }
    block_excl_scan_n<kGbNT, NAGG + 1>(agg, excl, tot, s_scan);
    if (wave_id() == 0) {
        int64_t pre[NAGG + 1];
        lookback_multi<NAGG + 1>(status, tile, tot, pre);
        if (lane_id() == 0)
            for (int k = 0; k <= NAGG; k++) s_excl[k] = pre[k];
    }
    __syncthreads();
    if (tile == ntiles - 1 && threadIdx.x == 0) *d_ngroups = s_excl[0] + tot[0];
    int64_t hc = s_excl[0] + excl[0];
    uint64_t run[NAGG];
#pragma unroll
    for (int g = 0; g < NAGG; g++) run[g] = uint64_t(s_excl[g + 1]) + uint64_t(excl[g + 1]);
#pragma unroll
    for (int r = 0; r < R; r++) {
        if ((valid >> r) & 1) {
            if (head & (1u << r)) {
                if (hc < key_cap) out_key[hc] = v[r];
                hc++;
            }
#pragma unroll
            for (int g = 0; g < NAGG; g++) run[g] += uint64_t(s_term[(g * R + r) * kGbNT + threadIdx.x]);
            if (end & (1u << r)) {
#pragma unroll
                for (int g = 0; g < NAGG; g++) ends[g * ends_stride + (hc - 1)] = int64_t(run[g]);
            }
        }
    }
    __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_gb_diff(const int64_t *__restrict__ ends,
                                                 int64_t ends_stride, int nagg,
                                                 const int64_t *d_ngroups, int64_t cap,
                                                 int64_t *o0, int64_t *o1, int64_t *o2,
                                                 int64_t *o3) {
    const int64_t ng0 = *d_ngroups;
    const int64_t ng = ng0 < cap ? ng0 : cap;
    int64_t *outs[4] = {o0, o1, o2, o3};
    for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < ng;
         g += int64_t(gridDim.x) * blockDim.x) {
        for (int k = 0; k < nagg; k++) {
            const int64_t *e = ends + k * ends_stride;
            const uint64_t hi = uint64_t(e[g]);
            const uint64_t lo = g > 0 ? uint64_t(e[g - 1]) : 0;
            outs[k][g] = int64_t(hi - lo);
        }
    }
}

// ---- dense key domain ------------------------------------------------------

constexpr int kDenseR = 4;                  // rows per thread per step (loads issued together)

// Where a dense group-by reads its keys: a key column, or a packed key built
// from other columns on the fly (never written to memory).
template <class K> struct ColKeys {
    const K *keys;
    template <int R>
    __device__ __forceinline__ void get(const int64_t (&idx)[R], int64_t cnt, int64_t (&v)[R]) const {
        K k[R];
#pragma unroll
        for (int r = 0; r < R; r++) k[r] = keys[idx[r] < cnt ? idx[r] : 0];   // cnt >= 1 here
#pragma unroll
        for (int r = 0; r < R; r++) v[r] = idx[r] < cnt ? int64_t(k[r]) : 0;
    }
};
struct TermKeys {
    PackArgs a;
    template <int R>
    __device__ __forceinline__ void get(const int64_t (&idx)[R], int64_t cnt, int64_t (&v)[R]) const {
        uint64_t acc[R];
        pack_keys<R>(a, idx, cnt, acc);
#pragma unroll
        for (int r = 0; r < R; r++) v[r] = int64_t(acc[r]);
    }
};

template <class KS>
__global__ __launch_bounds__(kGbNT) void k_gb_dense(KS ks, int64_t n,
                                                    const int64_t *d_n, int64_t key_lo,
                                                    int64_t span, AggArgs a,
                                                    unsigned long long *__restrict__ gacc) {
    extern __shared__ unsigned long long s_acc[];   // [(nagg + 1)][span], count last
    const int nagg = a.nagg;
    const int64_t cells = int64_t(nagg + 1) * span;
    for (int64_t i = threadIdx.x; i < cells; i += kGbNT) s_acc[i] = 0;
    __syncthreads();
    const int64_t cnt = count_of(d_n, n);
    constexpr int R = kDenseR;
    const int64_t stride = int64_t(gridDim.x) * kGbNT * R;
    for (int64_t base = blockIdx.x * int64_t(kGbNT) * R; base < cnt; base += stride) {
        uint32_t ok = 0;
        uint64_t b[R];
        int32_t row[R];
        int64_t idx[R], kv[R];
#pragma unroll
        for (int r = 0; r < R; r++) idx[r] = base + r * kGbNT + threadIdx.x;
        load_rows<R>(a.val_rows, idx, cnt, row);
        ks.template get<R>(idx, cnt, kv);
#pragma unroll
        for (int r = 0; r < R; r++)
            b[r] = idx[r] < cnt ? uint64_t(kv[r]) - uint64_t(key_lo) : uint64_t(span);
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (b[r] < uint64_t(span)) {
                ok |= 1u << r;
                atomicAdd(&s_acc[nagg * span + b[r]], 1ull);
            }
        }
        for (int g = 0; g < nagg; g++) {
            if (a.op[g] == TQP_AGG_COUNT) {
#pragma unroll
                for (int r = 0; r < R; r++)
                    if ((ok >> r) & 1) atomicAdd(&s_acc[g * span + b[r]], 1ull);
                continue;
            }
            int64_t v[R];
            load_vals<R>(a.val[a.ia[g]], a.vdt[a.ia[g]], a.vlen[a.ia[g]], row, ok, v);
            if (a.op[g] >= TQP_AGG_SUM_PRODUCT) {
                int64_t vy[R];
                load_vals<R>(a.val[a.ib[g]], a.vdt[a.ib[g]], a.vlen[a.ib[g]], row, ok, vy);
#pragma unroll
                for (int r = 0; r < R; r++) v[r] = int64_t(uint64_t(v[r]) * uint64_t(agg_second(a, g, vy[r])));
            }
#pragma unroll
            for (int r = 0; r < R; r++)
                if ((ok >> r) & 1) atomicAdd(&s_acc[g * span + b[r]], (unsigned long long)v[r]);
        }
    }
    __syncthreads();
    for (int64_t c = threadIdx.x; c < span; c += kGbNT) {
        if (s_acc[nagg * span + c] == 0) continue;
        for (int g = 0; g <= nagg; g++) atomicAdd(&gacc[g * span + c], s_acc[g * span + c]);
    }
}

// Domains of at most kTinySpan keys: every thread keeps all the groups'
// accumulators in registers (selecting, not indexing, the group), so no two
// lanes ever contend for one counter; waves then reduce with shuffles.  Each
// thread takes kTinyR rows per step and issues all their loads (keys, row ids,
// then values) before using any, so a wave has kTinyR dependent gathers in
// flight instead of one.
constexpr int kTinySpan = 8;
constexpr int kTinyR = 4;

template <class KS, int NAGG>
__global__ __launch_bounds__(kGbNT) void k_gb_tiny(KS ks, int64_t n,
                                                   const int64_t *d_n, int64_t key_lo, int span,
                                                   AggArgs a, unsigned long long *__restrict__ gacc) {
    constexpr int R = kTinyR;
    __shared__ int64_t s_red[kGbNT / kWave][kTinySpan][NAGG + 1];
    int64_t acc[kTinySpan][NAGG];
    int64_t cnt_b[kTinySpan];
#pragma unroll
    for (int b = 0; b < kTinySpan; b++) {
        cnt_b[b] = 0;
#pragma unroll
        for (int g = 0; g < NAGG; g++) acc[b][g] = 0;
    }
    const int64_t cnt = count_of(d_n, n);
    const int64_t stride = int64_t(gridDim.x) * kGbNT * R;
    for (int64_t base = blockIdx.x * int64_t(kGbNT) * R; base < cnt; base += stride) {
        uint32_t ok = 0;
        uint64_t b[R];
        int32_t row[R];
        int64_t idx[R], kv[R];
#pragma unroll
        for (int r = 0; r < R; r++) idx[r] = base + r * kGbNT + threadIdx.x;
        load_rows<R>(a.val_rows, idx, cnt, row);
        ks.template get<R>(idx, cnt, kv);
#pragma unroll
        for (int r = 0; r < R; r++)
            b[r] = idx[r] < cnt ? uint64_t(kv[r]) - uint64_t(key_lo) : uint64_t(span);
#pragma unroll
        for (int r = 0; r < R; r++) ok |= (b[r] < uint64_t(span) ? 1u : 0u) << r;
        int64_t t[NAGG][R];
#pragma unroll
        for (int g = 0; g < NAGG; g++) {
            if (a.op[g] == TQP_AGG_COUNT) {
#pragma unroll
                for (int r = 0; r < R; r++) t[g][r] = 1;
                continue;
            }
            const int x = a.ia[g];
            load_vals<R>(a.val[x], a.vdt[x], a.vlen[x], row, ok, t[g]);
            if (a.op[g] >= TQP_AGG_SUM_PRODUCT) {
                const int y = a.ib[g];
                int64_t vy[R];
                load_vals<R>(a.val[y], a.vdt[y], a.vlen[y], row, ok, vy);
#pragma unroll
                for (int r = 0; r < R; r++) t[g][r] = int64_t(uint64_t(t[g][r]) * uint64_t(agg_second(a, g, vy[r])));
            }
        }
#pragma unroll
        for (int r = 0; r < R; r++) {
#pragma unroll
            for (int bb = 0; bb < kTinySpan; bb++) {
                const bool hit = ((ok >> r) & 1) && uint64_t(bb) == b[r];
                cnt_b[bb] += hit ? 1 : 0;
#pragma unroll
                for (int g = 0; g < NAGG; g++) acc[bb][g] += hit ? t[g][r] : 0;
            }
        }
    }
    const int w = wave_id();
#pragma unroll
    for (int bb = 0; bb < kTinySpan; bb++) {
#pragma unroll
        for (int g = 0; g < NAGG; g++) {
            const int64_t sv = wave_sum(acc[bb][g]);
            if (lane_id() == 0) s_red[w][bb][g] = sv;
        }
        const int64_t c = wave_sum(cnt_b[bb]);
        if (lane_id() == 0) s_red[w][bb][NAGG] = c;
    }
    __syncthreads();
    if (threadIdx.x < kTinySpan * (NAGG + 1)) {
        const int bb = threadIdx.x / (NAGG + 1), g = threadIdx.x % (NAGG + 1);
        int64_t sv = 0;
#pragma unroll
        for (int ww = 0; ww < kGbNT / kWave; ww++) sv += s_red[ww][bb][g];
        if (bb < span && sv != 0) atomicAdd(&gacc[g * span + bb], (unsigned long long)sv);
    }
}

template <class K>
__global__ __launch_bounds__(1024) void k_gb_dense_emit(const unsigned long long *__restrict__ gacc,
                                                        int64_t key_lo, int64_t span, int nagg,
                                                        K *out_key, int64_t cap, int64_t *o0,
                                                        int64_t *o1, int64_t *o2, int64_t *o3,
                                                        int64_t *d_ngroups) {
    // 1024 threads x 4 consecutive bins each covers span <= 4096.
    __shared__ int64_t s_scan[1024 / kWave];
    int64_t *outs[4] = {o0, o1, o2, o3};
    const int64_t c0 = int64_t(threadIdx.x) * 4;
    uint32_t live = 0;
    for (int r = 0; r < 4; r++)
        if (c0 + r < span && gacc[nagg * span + c0 + r] != 0) live |= 1u << r;
    int64_t total;
    int64_t q = block_excl_scan<1024>(int64_t(__popc(live)), &total, s_scan);
    for (int r = 0; r < 4; r++) {
        if (!(live & (1u << r))) continue;
        if (q < cap) {
            out_key[q] = K(key_lo + c0 + r);
            for (int g = 0; g < nagg; g++) outs[g][q] = int64_t(gacc[g * span + c0 + r]);
        }
        q++;
    }
    if (threadIdx.x == 0) *d_ngroups = total;
}

struct GbLayout {
    int64_t *scratch;
    void *skey;
    int32_t *srows;
    void *sort_ws;
    size_t sort_ws_bytes;
    int64_t *ends;
    uint64_t *words;          // ticket word, then 2 * kNV status words per tile
    int64_t nwords;
    int64_t ntiles;
    unsigned long long *gacc;
    size_t bytes;
};

static bool dense_ok(uint32_t flags, int64_t span, int nagg) {
    return (flags & TQP_GB_DENSE) && span > 0 && span <= TQP_GB_DENSE_MAX &&
           int64_t(nagg + 1) * span * 8 <= 48 * 1024;
}

static GbLayout gb_layout(void *ws, int64_t n, int dtype, int nagg, uint32_t flags, int64_t span) {
    GbLayout L = {};
    Carver c(ws);
    const int ks = dtype_size(dtype);
    L.scratch = c.take<int64_t>(2);
    if (dense_ok(flags, span, nagg)) {
        L.gacc = c.take<unsigned long long>(size_t(nagg + 1) * span);
        L.bytes = c.bytes();
        return L;
    }
    const int64_t nn = n > 0 ? n : 1;
    if (!(flags & TQP_GB_SORTED)) {
        L.skey = c.take<char>(size_t(nn) * ks);
        L.srows = c.take<int32_t>(size_t(nn));
        L.sort_ws_bytes = sort_ws_bytes(nn, dtype, ks * 8);
        L.sort_ws = c.take<char>(L.sort_ws_bytes);
    }
    L.ends = c.take<int64_t>(size_t(kMaxAgg) * nn);
    L.ntiles = ceil_div(nn, kGbTile);
    L.nwords = 1 + L.ntiles * 2 * kNV;
    L.words = c.take<uint64_t>(size_t(L.nwords));
    L.bytes = c.bytes();
    return L;
}

// Dense domains: zero the accumulators, aggregate (registers for at most
// kTinySpan keys, LDS otherwise), emit the groups that occur.  KS gives the
// keys (a column, or a packed key built on the fly); OK is the output key type.
template <class OK, class KS>
static int dense_groupby(const KS &ks, int64_t n, const int64_t *d_n, int64_t key_lo,
                         int64_t key_span, const AggArgs &args, unsigned long long *gacc,
                         OK *out_key, int64_t out_cap, int64_t *const *o, int64_t *d_ngroups,
                         hipStream_t s) {
    const int nagg = args.nagg;
    int rc = fill_u64(gacc, 0, int64_t(nagg + 1) * key_span, s);
    if (rc) return rc;
    if (n > 0 && key_span <= kTinySpan) {
        // no more workgroups than are resident at once (4 per CU at this
        // kernel's register count): measured 4% faster than twice as many
        int64_t g = ceil_div(n, int64_t(kGbNT) * kTinyR * 8);
        if (g > int64_t(kComputeUnits) * 4) g = int64_t(kComputeUnits) * 4;
        switch (nagg) {
        case 1:
            TQP_LAUNCH("gb_tiny", (k_gb_tiny<KS, 1>), dim3(unsigned(g)), dim3(kGbNT), 0, s, ks, n,
                       d_n, key_lo, int(key_span), args, gacc);
            break;
        case 2:
            TQP_LAUNCH("gb_tiny", (k_gb_tiny<KS, 2>), dim3(unsigned(g)), dim3(kGbNT), 0, s, ks, n,
                       d_n, key_lo, int(key_span), args, gacc);
            break;
        case 3:
            TQP_LAUNCH("gb_tiny", (k_gb_tiny<KS, 3>), dim3(unsigned(g)), dim3(kGbNT), 0, s, ks, n,
                       d_n, key_lo, int(key_span), args, gacc);
            break;
        default:
            TQP_LAUNCH("gb_tiny", (k_gb_tiny<KS, 4>), dim3(unsigned(g)), dim3(kGbNT), 0, s, ks, n,
                       d_n, key_lo, int(key_span), args, gacc);
            break;
        }
        if ((rc = check_launch("group-by tiny"))) return rc;
    } else if (n > 0) {
        int64_t g = ceil_div(n, int64_t(kGbNT) * 64);
        if (g > 2048) g = 2048;
        const size_t lds = size_t(nagg + 1) * key_span * 8;
        TQP_LAUNCH("gb_dense", k_gb_dense<KS>, dim3(unsigned(g)), dim3(kGbNT), lds, s, ks, n, d_n,
                   key_lo, key_span, args, gacc);
        if ((rc = check_launch("group-by dense"))) return rc;
    }
    TQP_LAUNCH("gb_dense_emit", k_gb_dense_emit<OK>, dim3(1), dim3(1024), 0, s, gacc, key_lo,
               key_span, nagg, out_key, out_cap, o[0], o[1], o[2], o[3], d_ngroups);
    return check_launch("group-by dense emit");
}

template <class K>
static int groupby_typed(const tqp_col *key, const int64_t *d_n, uint32_t flags, int64_t key_lo,
                         int64_t key_span, const AggArgs &args, const tqp_col *out_key,
                         int64_t *const *out_aggs, int64_t *d_ngroups, void *ws, hipStream_t s) {
    const int64_t n = key->len;
    const int nagg = args.nagg;
    GbLayout L = gb_layout(ws, n, key->dtype, nagg, flags, key_span);
    int64_t *o[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int g = 0; g < nagg; g++) o[g] = out_aggs[g];
    int rc;
    if (dense_ok(flags, key_span, nagg))
        return dense_groupby<K>(ColKeys<K>{static_cast<const K *>(key->data)}, n, d_n, key_lo,
                                key_span, args, L.gacc, static_cast<K *>(out_key->data),
                                out_key->len, o, d_ngroups, s);
    const K *k = static_cast<const K *>(key->data);
    AggArgs a = args;
    if (!(flags & TQP_GB_SORTED)) {
        int64_t kmin = key_lo;
        int kbits = 0;
        if (key_span > 0) {
            while (kbits < 64 && (uint64_t(key_span - 1) >> kbits) != 0) kbits++;
        } else {
            rc = derive_key_range(k, key->dtype, n, d_n, L.scratch, s, &kmin, &kbits);
            if (rc) return rc;
        }
        rc = sort_impl(k, key->dtype, args.val_rows, n, d_n, kbits, kmin, L.skey, L.srows,
                       L.sort_ws, L.sort_ws_bytes, s);
        if (rc) return rc;
        k = static_cast<const K *>(L.skey);
        a.val_rows = L.srows;
    }
    rc = fill_u64(L.words, 0, L.nwords, s);
    if (rc) return rc;
    const unsigned grid = persistent_grid(L.ntiles, tune(kTuneGbScanPerCu));
    K *ok = static_cast<K *>(out_key->data);
    const int64_t es = n > 0 ? n : int64_t(1);
    uint32_t *tk = reinterpret_cast<uint32_t *>(L.words);
    switch (nagg) {
    case 1:
        TQP_LAUNCH("gb_scan", (k_gb_scan<K, 1>), dim3(grid), dim3(kGbNT), 0, s, k, n, d_n, a, ok,
                   out_key->len, L.ends, es, d_ngroups, tk, L.words + 1);
        break;
    case 2:
        TQP_LAUNCH("gb_scan", (k_gb_scan<K, 2>), dim3(grid), dim3(kGbNT), 0, s, k, n, d_n, a, ok,
                   out_key->len, L.ends, es, d_ngroups, tk, L.words + 1);
        break;
    case 3:
        TQP_LAUNCH("gb_scan", (k_gb_scan<K, 3>), dim3(grid), dim3(kGbNT), 0, s, k, n, d_n, a, ok,
                   out_key->len, L.ends, es, d_ngroups, tk, L.words + 1);
        break;
    default:
        TQP_LAUNCH("gb_scan", (k_gb_scan<K, 4>), dim3(grid), dim3(kGbNT), 0, s, k, n, d_n, a, ok,
                   out_key->len, L.ends, es, d_ngroups, tk, L.words + 1);
        break;
    }
    if ((rc = check_launch("group-by scan"))) return rc;
    int64_t g = ceil_div(out_key->len > 0 ? out_key->len : 1, 256);
    if (g > 4096) g = 4096;
    TQP_LAUNCH("gb_diff", k_gb_diff, dim3(unsigned(g)), dim3(256), 0, s, L.ends,
                       n > 0 ? n : int64_t(1), nagg, d_ngroups, out_key->len, o[0], o[1], o[2],
                       o[3]);
    return check_launch("group-by diff");
}

}  // namespace tqp

using namespace tqp;

// Checks the value columns and aggregates of a group-by call and fills
// AggArgs; n is the row count value columns must cover without val_rows.
static int agg_args(const tqp_col *vals, int nvals, const int32_t *val_rows, const tqp_agg *aggs,
                    int nagg, int64_t n, int64_t out_cap, int64_t *const *out_aggs, AggArgs *a,
                    const char *who) {
    *a = AggArgs{};
    for (int c = 0; c < nvals; c++) {
        if (!dtype_ok(vals[c].dtype) || (vals[c].len > 0 && !vals[c].data) ||
            !col_aligned(vals[c].data, vals[c].dtype))
            return set_error(TQP_EINVAL, "%s: value column %d is invalid or unaligned", who, c);
        if (!val_rows && vals[c].len < n)
            return set_error(TQP_EINVAL, "%s: value column %d is shorter than keys", who, c);
        a->val[c] = vals[c].data;
        a->vlen[c] = vals[c].len;
        a->vdt[c] = vals[c].dtype;
    }
    for (int g = 0; g < nagg; g++) {
        const tqp_agg &x = aggs[g];
        if (x.op < TQP_AGG_SUM || x.op > TQP_AGG_SUM_DIFF_PRODUCT)
            return set_error(TQP_EINVAL, "%s: aggregate %d has a bad op", who, g);
        if (x.op != TQP_AGG_COUNT && (x.a < 0 || x.a >= nvals))
            return set_error(TQP_EINVAL, "%s: aggregate %d names a missing column", who, g);
        if (x.op >= TQP_AGG_SUM_PRODUCT && (x.b < 0 || x.b >= nvals))
            return set_error(TQP_EINVAL, "%s: aggregate %d names a missing column", who, g);
        if (out_cap > 0 && !out_aggs[g]) return set_error(TQP_EINVAL, "%s: output %d is null", who, g);
        a->op[g] = x.op;
        a->ia[g] = x.a;
        a->ib[g] = x.b;
        a->ic[g] = x.c;
    }
    if (val_rows && !col_aligned(val_rows, TQP_INT32))
        return set_error(TQP_EINVAL, "%s: val_rows must be 4-byte aligned", who);
    a->nagg = nagg;
    a->val_rows = val_rows;
    return TQP_OK;
}

TQP_API size_t tqp_groupby_workspace_bytes(int64_t n, int dtype, int nagg, uint32_t flags,
                                           int64_t key_span) {
    if (n < 0 || (dtype != TQP_INT32 && dtype != TQP_INT64) || nagg < 1 || nagg > kMaxAgg)
        return 0;
    return gb_layout(nullptr, n, dtype, nagg, flags, key_span).bytes;
}

TQP_API int tqp_groupby_agg(const tqp_col *key, const int64_t *d_n, uint32_t flags, int64_t key_lo,
                            int64_t key_span, const tqp_col *vals, int nvals,
                            const int32_t *val_rows, const tqp_agg *aggs, int nagg,
                            const tqp_col *out_key, int64_t *const *out_aggs, int64_t *d_ngroups,
                            void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!key || !out_key || !aggs || !out_aggs || !d_ngroups)
        return set_error(TQP_EINVAL, "tqp_groupby_agg: null argument");
    if (key->dtype != TQP_INT32 && key->dtype != TQP_INT64)
        return set_error(TQP_EINVAL, "tqp_groupby_agg: keys must be int32 or int64");
    if (out_key->dtype != key->dtype)
        return set_error(TQP_EINVAL, "tqp_groupby_agg: out_key dtype must equal the key dtype");
    if (nagg < 1 || nagg > kMaxAgg)
        return set_error(TQP_EINVAL, "tqp_groupby_agg: nagg must be in [1, %d]", kMaxAgg);
    if (nvals < 0 || nvals > kMaxVals || (nvals > 0 && !vals))
        return set_error(TQP_EINVAL, "tqp_groupby_agg: nvals must be in [0, %d]", kMaxVals);
    if (flags & ~(TQP_GB_SORTED | TQP_GB_DENSE))
        return set_error(TQP_EINVAL, "tqp_groupby_agg: unknown flag bits");
    if ((flags & TQP_GB_DENSE) && (key_span < 1 || key_span > TQP_GB_DENSE_MAX))
        return set_error(TQP_EINVAL, "tqp_groupby_agg: dense needs 1 <= key_span <= %d",
                         TQP_GB_DENSE_MAX);
    if (key_span < 0) return set_error(TQP_EINVAL, "tqp_groupby_agg: negative key_span");
    const int64_t n = key->len;
    if (n < 0 || n > (int64_t(1) << 30) - 1)
        return set_error(TQP_EINVAL, "tqp_groupby_agg: n must be in [0, 2^30 - 1]");
    if ((n > 0 && !key->data) || (out_key->len > 0 && !out_key->data))
        return set_error(TQP_EINVAL, "tqp_groupby_agg: null key data");
    AggArgs a = {};
    int rc = agg_args(vals, nvals, val_rows, aggs, nagg, n, out_key->len, out_aggs, &a,
                      "tqp_groupby_agg");
    if (rc) return rc;
    const size_t need = tqp_groupby_workspace_bytes(n, key->dtype, nagg, flags, key_span);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "tqp_groupby_agg: workspace needs %zu bytes", need);
    hipStream_t s = as_stream(stream);
    if (key->dtype == TQP_INT32)
        return groupby_typed<int32_t>(key, d_n, flags, key_lo, key_span, a, out_key, out_aggs,
                                      d_ngroups, ws, s);
    return groupby_typed<int64_t>(key, d_n, flags, key_lo, key_span, a, out_key, out_aggs,
                                  d_ngroups, ws, s);
}

TQP_API size_t tqp_groupby_terms_workspace_bytes(int nagg, int64_t key_span) {
    if (nagg < 1 || nagg > kMaxAgg || !dense_ok(TQP_GB_DENSE, key_span, nagg)) return 0;
    Carver c(nullptr);
    c.take<unsigned long long>(size_t(nagg + 1) * size_t(key_span));
    return c.bytes();
}

TQP_API int tqp_groupby_agg_terms(const tqp_keyterm *terms, int nterms, int64_t n,
                                  const int64_t *d_n, int64_t key_lo, int64_t key_span,
                                  const tqp_col *vals, int nvals, const int32_t *val_rows,
                                  const tqp_agg *aggs, int nagg, const tqp_col *out_key,
                                  int64_t *const *out_aggs, int64_t *d_ngroups, void *ws,
                                  size_t ws_bytes, void *stream) {
    clear_error();
    if (!terms || !out_key || !aggs || !out_aggs || !d_ngroups)
        return set_error(TQP_EINVAL, "tqp_groupby_agg_terms: null argument");
    if (nterms < 1 || nterms > 4)
        return set_error(TQP_EINVAL, "tqp_groupby_agg_terms: nterms must be in [1, 4]");
    if (out_key->dtype != TQP_INT32 && out_key->dtype != TQP_INT64)
        return set_error(TQP_EINVAL, "tqp_groupby_agg_terms: out_key must be int32 or int64");
    if (out_key->len > 0 && !out_key->data)
        return set_error(TQP_EINVAL, "tqp_groupby_agg_terms: null out_key data");
    if (nagg < 1 || nagg > kMaxAgg)
        return set_error(TQP_EINVAL, "tqp_groupby_agg_terms: nagg must be in [1, %d]", kMaxAgg);
    if (nvals < 0 || nvals > kMaxVals || (nvals > 0 && !vals))
        return set_error(TQP_EINVAL, "tqp_groupby_agg_terms: nvals must be in [0, %d]", kMaxVals);
    if (!dense_ok(TQP_GB_DENSE, key_span, nagg))
        return set_error(TQP_EINVAL,
                         "tqp_groupby_agg_terms: need 1 <= key_span and (nagg + 1) * key_span <= 6144");
    if (out_key->dtype == TQP_INT32 &&
        (key_lo < INT32_MIN || key_lo + key_span - 1 > INT32_MAX))
        return set_error(TQP_EINVAL, "tqp_groupby_agg_terms: the key range does not fit int32");
    if (n < 0 || n > (int64_t(1) << 30) - 1)
        return set_error(TQP_EINVAL, "tqp_groupby_agg_terms: n must be in [0, 2^30 - 1]");
    PackArgs p;
    int rc = pack_args(terms, nterms, n, &p, "tqp_groupby_agg_terms");
    if (rc) return rc;
    AggArgs a;
    rc = agg_args(vals, nvals, val_rows, aggs, nagg, n, out_key->len, out_aggs, &a,
                  "tqp_groupby_agg_terms");
    if (rc) return rc;
    const size_t need = tqp_groupby_terms_workspace_bytes(nagg, key_span);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "tqp_groupby_agg_terms: workspace needs %zu bytes", need);
    int64_t *o[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int g = 0; g < nagg; g++) o[g] = out_aggs[g];
    hipStream_t s = as_stream(stream);
    unsigned long long *gacc = static_cast<unsigned long long *>(ws);
    if (out_key->dtype == TQP_INT32)
        return dense_groupby<int32_t>(TermKeys{p}, n, d_n, key_lo, key_span, a, gacc,
                                      static_cast<int32_t *>(out_key->data), out_key->len, o,
                                      d_ngroups, s);
    return dense_groupby<int64_t>(TermKeys{p}, n, d_n, key_lo, key_span, a, gacc,
                                  static_cast<int64_t *>(out_key->data), out_key->len, o,
                                  d_ngroups, s);
}
