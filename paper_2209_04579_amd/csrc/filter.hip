// WHERE with stream compaction, single pass.
//
// Each workgroup takes a 4096-row tile (256 threads x 16 consecutive rows),
// evaluates the predicate conjunction with wide vector loads and counts its
// kept rows with a block scan.  A sparse tile stages its kept row ids in LDS
// in ascending order; its output offset comes from a decoupled look-back over
// the tiles before it, resolved while the workgroup's next tile is loading,
// and the staged row ids, with the payload columns read through them, are
// written at that offset by consecutive threads.  A dense tile resolves its
// offset at once and writes each column through LDS.  Every predicate byte is
// read once, payload only where rows are kept; output is written once, in
// ascending row id order.
#include "tqp_internal.hpp"

namespace tqp {

constexpr int kFilterNT = 256;
constexpr int kFilterIPT = 16;
constexpr int kFilterTile = kFilterNT * kFilterIPT;
constexpr int kMaxPred = 8;
constexpr int kMaxPay = 8;

struct FilterArgs {
    const void *pcol[kMaxPred];
    int64_t plit[kMaxPred];
    int32_t pdt[kMaxPred];
    int32_t pop[kMaxPred];
    int32_t pcolid[kMaxPred];
    const void *pin[kMaxPay];
    void *pout[kMaxPay];
    int32_t paydt[kMaxPay];
    int32_t npred;
    int32_t npay;
    int32_t vec;          // every column base is 16-byte aligned
    int32_t *out_rows;
    int64_t *d_count;
    int64_t n;
    uint32_t *ticket;
    uint64_t *status;
};

// Loads 16 consecutive elements starting at row0 (sign-extended to int64).
__device__ __forceinline__ void load16(const void *p, int dt, int64_t row0, int64_t n,
                                       bool vec, int64_t (&v)[16]) {
    if (vec && row0 + 16 <= n) {
        if (dt == TQP_INT8) {
            int4 x = *reinterpret_cast<const int4 *>(static_cast<const int8_t *>(p) + row0);
            const int w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int r = 0; r < 16; r++)
                v[r] = static_cast<int8_t>(static_cast<uint32_t>(w[r >> 2]) >> (8 * (r & 3)));
        } else if (dt == TQP_INT32) {
            const int4 *q = reinterpret_cast<const int4 *>(static_cast<const int32_t *>(p) + row0);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                int4 x = q[k];
                v[4 * k + 0] = x.x;
                v[4 * k + 1] = x.y;
                v[4 * k + 2] = x.z;
                v[4 * k + 3] = x.w;
            }
        } else {
            const longlong2 *q =
                reinterpret_cast<const longlong2 *>(static_cast<const int64_t *>(p) + row0);
#pragma unroll
            for (int k = 0; k < 8; k++) {
                longlong2 x = q[k];
                v[2 * k + 0] = x.x;
                v[2 * k + 1] = x.y;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; r++)
            v[r] = (row0 + r < n) ? load_any(p, dt, row0 + r) : 0;
    }
}

// Loads 8 consecutive elements starting at row0 (sign-extended to int64).
__device__ __forceinline__ void load8(const void *p, int dt, int64_t row0, int64_t n, bool vec,
                                      int64_t (&v)[8]) {
    if (vec && row0 + 8 <= n) {
        if (dt == TQP_INT8) {
            int2 x = *reinterpret_cast<const int2 *>(static_cast<const int8_t *>(p) + row0);
            const int w[2] = {x.x, x.y};
#pragma unroll
            for (int r = 0; r < 8; r++)
                v[r] = static_cast<int8_t>(static_cast<uint32_t>(w[r >> 2]) >> (8 * (r & 3)));
        } else if (dt == TQP_INT32) {
            const int4 *q = reinterpret_cast<const int4 *>(static_cast<const int32_t *>(p) + row0);
#pragma unroll
            for (int k = 0; k < 2; k++) {
                int4 x = q[k];
                v[4 * k + 0] = x.x;
                v[4 * k + 1] = x.y;
                v[4 * k + 2] = x.z;
                v[4 * k + 3] = x.w;
            }
        } else {
            const longlong2 *q =
                reinterpret_cast<const longlong2 *>(static_cast<const int64_t *>(p) + row0);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                longlong2 x = q[k];
                v[2 * k + 0] = x.x;
                v[2 * k + 1] = x.y;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 8; r++)
            v[r] = (row0 + r < n) ? load_any(p, dt, row0 + r) : 0;
    }
}

// Element v (zero-extended) of a column of element size 1 << lg, stored at i.
__device__ __forceinline__ void store_lg(void *out, int lg, int64_t i, uint64_t v) {
    if (lg == 0) static_cast<uint8_t *>(out)[i] = uint8_t(v);
    else if (lg == 2) static_cast<uint32_t *>(out)[i] = uint32_t(v);
    else static_cast<uint64_t *>(out)[i] = v;
}

// Writes a staged tile's kept rows from slot base on: the row ids, then
// every payload column read through them, consecutive threads taking
// consecutive slots (so the writes are coalesced, and so are the payload
// reads where the kept rows are dense).  Each thread takes kWriteU slots per
// pass with every column's loads issued before the first store, so a dense
// tile costs few memory round trips.  The staging writes and the prefix in
// LDS must be visible: callers come here after a barrier that follows both.
constexpr int kWriteU = 2;
__device__ __forceinline__ void filter_write_staged(const FilterArgs &a, const int32_t *srow,
                                                    int64_t base, int cnt, bool last_tile) {
    if (last_tile && threadIdx.x == 0) *a.d_count = base + cnt;
    int lg[kMaxPay];
#pragma unroll
    for (int c = 0; c < kMaxPay; c++) lg[c] = c < a.npay ? dtype_lg(a.paydt[c]) : 0;
    for (int i0 = threadIdx.x; i0 < cnt; i0 += kWriteU * kFilterNT) {
        int32_t row[kWriteU];
#pragma unroll
        for (int u = 0; u < kWriteU; u++) {
            const int i = i0 + u * kFilterNT;
            row[u] = i < cnt ? srow[i] : -1;
        }
        uint64_t w[kWriteU][kMaxPay];
#pragma unroll
        for (int c = 0; c < kMaxPay; c++)
#pragma unroll
            for (int u = 0; u < kWriteU; u++)
                if (c < a.npay && row[u] >= 0) w[u][c] = word_of(a.pin[c], lg[c], row[u]);
#pragma unroll
        for (int u = 0; u < kWriteU; u++) {
            if (row[u] < 0) continue;
            const int64_t slot = base + i0 + u * kFilterNT;
            if (a.out_rows) a.out_rows[slot] = row[u];
#pragma unroll
            for (int c = 0; c < kMaxPay; c++)
                if (c < a.npay) store_lg(a.pout[c], lg[c], slot, from_word(w[u][c], a.pin[c], lg[c], row[u]));
        }
    }
}

// A tile keeping at most this many rows defers its look-back and writes
// (its row ids wait in LDS); a denser one resolves its offset at once and
// writes each column from LDS, where a column's values are staged straight
// from its vector loads.
constexpr int kFilterDefer = 1024;

__global__ __launch_bounds__(kFilterNT) void k_filter(FilterArgs a) {
    __shared__ int64_t s_tile;
    __shared__ int64_t s_prefix, s_pprefix;
    __shared__ int32_t s_scan[kFilterNT / kWave];
    // Two buffers of a tile's kept row ids (ascending): one filled by the
    // current tile while the previous tile's rows are written from the
    // other.  A dense tile uses the whole array for one column at a time.
    __shared__ int64_t s_stage[kFilterTile];
    int32_t *const s_rows = reinterpret_cast<int32_t *>(s_stage);

    const int64_t n = a.n;
    const int64_t ntiles = ceil_div(n, kFilterTile);
    const bool vec = a.vec != 0;
    int64_t pend_tile = -1;      // the tile whose kept rows wait in LDS
    int pend_total = 0, pb = 0;
    // Persistent workgroups: each takes tiles in ticket order until none are
    // left.  A sparse tile publishes its count as soon as it is known; its
    // prefix is resolved while the workgroup's next tile is being loaded, and
    // its rows are written after that tile's scan.
    for (;;) {
        const int64_t tile = take_tile(a.ticket, &s_tile);
        const bool last = tile >= ntiles;
        if (last && tile == 0 && threadIdx.x == 0) *a.d_count = 0;   // empty input
        const int64_t row0 = tile * kFilterTile + int64_t(threadIdx.x) * kFilterIPT;
        int64_t v[16];
        if (!last) load16(a.pcol[0], a.pdt[0], row0, n, vec, v);
        if (pend_tile >= 0 && wave_id() == 0) {
            const int64_t pre = lookback_resolve(a.status, pend_tile, pend_total);
            if (lane_id() == 0) s_pprefix = pre;
        }
        uint32_t mask = 0;
        int32_t total = 0, excl = 0;
        bool defer = true;
        int cb = pb;
        if (!last) {       // (uniform across the workgroup)
#pragma unroll
            for (int r = 0; r < 16; r++)
                if (row0 + r < n) mask |= 1u << r;
            int loaded = a.pcolid[0];
            for (int p = 0; p < a.npred; p++) {
                if (a.pcolid[p] != loaded) {
                    load16(a.pcol[p], a.pdt[p], row0, n, vec, v);
                    loaded = a.pcolid[p];
                }
                const int op = a.pop[p];
                const int64_t lit = a.plit[p];
                uint32_t m = 0;
#pragma unroll
                for (int r = 0; r < 16; r++)
                    if (cmp_holds(v[r], op, lit)) m |= 1u << r;
                mask &= m;
            }
            excl = block_excl_scan<kFilterNT>(int32_t(__popc(mask)), &total, s_scan);
            defer = total <= kFilterDefer;
            if (defer) {
                if (wave_id() == 0) lookback_publish(a.status, tile, total);
                cb = pend_tile >= 0 ? pb ^ 1 : pb;
                int32_t *st = s_rows + cb * kFilterTile;
                int q = excl;
#pragma unroll
                for (int r = 0; r < 16; r++)
                    if (mask & (1u << r)) st[q++] = static_cast<int32_t>(row0 + r);
            } else if (wave_id() == 0) {
                // dense tile: its offset now
                const int64_t pre = lookback_count(a.status, tile, total);
                if (lane_id() == 0) s_prefix = pre;
            }
        } else {
            __syncthreads();     // s_pprefix
        }
        if (pend_tile >= 0)
            filter_write_staged(a, s_rows + pb * kFilterTile, s_pprefix, pend_total,
                                pend_tile == ntiles - 1);
        if (last) break;
        if (defer) {
            pend_tile = tile;
            pend_total = total;
            pb = cb;
            continue;
        }

        // dense tile, with the pending tile's rows out: every column through LDS
        pend_tile = -1;
        __syncthreads();
        const int64_t base = s_prefix;
        if (tile == ntiles - 1 && threadIdx.x == 0) *a.d_count = base + total;
        // each output column goes through LDS in kept order, then out with
        // consecutive threads on consecutive addresses
        if (a.out_rows) {
            int q = excl;
#pragma unroll
            for (int r = 0; r < 16; r++)
                if (mask & (1u << r)) s_rows[q++] = static_cast<int32_t>(row0 + r);
            __syncthreads();
            for (int i = threadIdx.x; i < total; i += kFilterNT) a.out_rows[base + i] = s_rows[i];
            __syncthreads();
        }
        for (int c = 0; c < a.npay; c++) {
            const int dt = a.paydt[c];
            // only threads with kept rows read the column (v is overwritten
            // either way, so the predicate values are dead by now)
            if (mask) {
                load16(a.pin[c], dt, row0, n, vec, v);
            } else {
#pragma unroll
                for (int r = 0; r < 16; r++) v[r] = 0;
            }
            int q = excl;
            if (dt == TQP_INT8) {
                int8_t *st = reinterpret_cast<int8_t *>(s_stage);
#pragma unroll
                for (int r = 0; r < 16; r++)
                    if (mask & (1u << r)) st[q++] = static_cast<int8_t>(v[r]);
                __syncthreads();
                int8_t *out = static_cast<int8_t *>(a.pout[c]);
                for (int i = threadIdx.x; i < total; i += kFilterNT) out[base + i] = st[i];
            } else if (dt == TQP_INT32) {
                int32_t *st = reinterpret_cast<int32_t *>(s_stage);
#pragma unroll
                for (int r = 0; r < 16; r++)
                    if (mask & (1u << r)) st[q++] = static_cast<int32_t>(v[r]);
                __syncthreads();
                int32_t *out = static_cast<int32_t *>(a.pout[c]);
                for (int i = threadIdx.x; i < total; i += kFilterNT) out[base + i] = st[i];
            } else {
                int64_t *st = s_stage;
#pragma unroll
                for (int r = 0; r < 16; r++)
                    if (mask & (1u << r)) st[q++] = v[r];
                __syncthreads();
                int64_t *out = static_cast<int64_t *>(a.pout[c]);
                for (int i = threadIdx.x; i < total; i += kFilterNT) out[base + i] = st[i];
            }
            __syncthreads();
        }
    }
}

// WHERE + aggregate without compaction: the predicate pass of k_filter (8
// consecutive rows per thread here, which halves the registers a column
// takes and doubles the loads in flight), then SUM(a * b) and COUNT over the
// kept rows.  The predicates come grouped by column; with at most
// kSumMaxCols distinct columns, every column of a tile is loaded before the
// first test (one memory round trip per tile instead of one per column), and
// a value operand that is also a predicate column is taken from those loads.
// Other value columns are read only by threads holding a kept row, so at low
// selectivity most of their cache lines are never fetched.  Partial sums are
// reduced per workgroup and added with one device atomic each; int64
// addition wraps modulo 2^64, so every order gives the same bytes.
constexpr int kSumMaxCols = 4;
struct FilterSumArgs {
    const void *pcol[kMaxPred];      // per predicate, grouped by column
    int64_t plit[kMaxPred];
    int32_t pdt[kMaxPred];
    int32_t pop[kMaxPred];
    int32_t pcolid[kMaxPred];
    int32_t npred;
    int32_t vec;
    const void *dcol[kMaxPred];      // the distinct predicate columns
    int32_t ddt[kMaxPred];
    int32_t pbeg[kMaxPred + 1];      // column d's predicates: pbeg[d] .. pbeg[d + 1] - 1
    int32_t nd;
    int32_t aslot, bslot;            // the distinct column that a / b is, or -1
    const void *a;        // null: the sum is 0
    const void *b;        // null: SUM(a)
    int32_t adt, bdt;
    int64_t n;
    unsigned long long *d_sum;
    unsigned long long *d_count;
};

__global__ void k_zero2(unsigned long long *p, unsigned long long *q) {
    if (threadIdx.x == 0) {
        *p = 0;
        *q = 0;
    }
}

constexpr int kSumIPT = 8;
constexpr int kSumTile = kFilterNT * kSumIPT;

// ND distinct predicate columns (1 .. kSumMaxCols) loaded together; ND = 0:
// each column loaded when its first predicate is reached.
template <int ND>
__global__ __launch_bounds__(kFilterNT) void k_filter_sum(FilterSumArgs f) {
    __shared__ unsigned long long s_red[2][kFilterNT / kWave];
    const int64_t n = f.n;
    const int64_t ntiles = ceil_div(n, kSumTile);
    const bool vec = f.vec != 0;
    uint64_t sum = 0, cnt = 0;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t row0 = tile * kSumTile + int64_t(threadIdx.x) * kSumIPT;
        uint32_t mask = 0;
#pragma unroll
        for (int r = 0; r < kSumIPT; r++)
            if (row0 + r < n) mask |= 1u << r;
        if constexpr (ND > 0) {
            int64_t d[ND][kSumIPT];
#pragma unroll
            for (int c = 0; c < ND; c++) load8(f.dcol[c], f.ddt[c], row0, n, vec, d[c]);
#pragma unroll
            for (int c = 0; c < ND; c++) {
                for (int p = f.pbeg[c]; p < f.pbeg[c + 1]; p++) {
                    const int op = f.pop[p];
                    const int64_t lit = f.plit[p];
                    uint32_t m = 0;
#pragma unroll
                    for (int r = 0; r < kSumIPT; r++)
                        if (cmp_holds(d[c][r], op, lit)) m |= 1u << r;
                    mask &= m;
                }
            }
            cnt += __popc(mask);
            if (mask && f.a) {
                int64_t x[kSumIPT], y[kSumIPT];
                if (f.aslot >= 0) {
#pragma unroll
                    for (int c = 0; c < ND; c++)
                        if (c == f.aslot) {
#pragma unroll
                            for (int r = 0; r < kSumIPT; r++) x[r] = d[c][r];
                        }
                } else {
                    load8(f.a, f.adt, row0, n, vec, x);
                }
                if (f.b) {
                    if (f.bslot >= 0) {
#pragma unroll
                        for (int c = 0; c < ND; c++)
                            if (c == f.bslot) {
#pragma unroll
                                for (int r = 0; r < kSumIPT; r++) y[r] = d[c][r];
                            }
                    } else {
                        load8(f.b, f.bdt, row0, n, vec, y);
                    }
#pragma unroll
                    for (int r = 0; r < kSumIPT; r++)
                        if (mask & (1u << r)) sum += uint64_t(x[r]) * uint64_t(y[r]);
                } else {
#pragma unroll
                    for (int r = 0; r < kSumIPT; r++)
                        if (mask & (1u << r)) sum += uint64_t(x[r]);
                }
            }
            continue;
        }
        int64_t v[kSumIPT];
        int loaded = -1;
        for (int p = 0; p < f.npred; p++) {
            if (f.pcolid[p] != loaded) {
                load8(f.pcol[p], f.pdt[p], row0, n, vec, v);
                loaded = f.pcolid[p];
            }
            const int op = f.pop[p];
            const int64_t lit = f.plit[p];
            uint32_t m = 0;
#pragma unroll
            for (int r = 0; r < kSumIPT; r++)
                if (cmp_holds(v[r], op, lit)) m |= 1u << r;
            mask &= m;
        }
        cnt += __popc(mask);
        if (mask && f.a) {
            int64_t x[kSumIPT];
            load8(f.a, f.adt, row0, n, vec, x);
            if (f.b) {
                load8(f.b, f.bdt, row0, n, vec, v);
#pragma unroll
                for (int r = 0; r < kSumIPT; r++)
                    if (mask & (1u << r)) sum += uint64_t(x[r]) * uint64_t(v[r]);
            } else {
#pragma unroll
                for (int r = 0; r < kSumIPT; r++)
                    if (mask & (1u << r)) sum += uint64_t(x[r]);
            }
        }
    }
    const uint64_t ws = uint64_t(wave_sum(int64_t(sum)));
    const uint64_t wc = uint64_t(wave_sum(int64_t(cnt)));
    if (lane_id() == 0) {
        s_red[0][wave_id()] = ws;
        s_red[1][wave_id()] = wc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long ts = 0, tc = 0;
#pragma unroll
        for (int w = 0; w < kFilterNT / kWave; w++) {
            ts += s_red[0][w];
            tc += s_red[1][w];
        }
        if (ts) atomicAdd(f.d_sum, ts);
        if (tc) atomicAdd(f.d_count, tc);
    }
}

// Tiles are dealt to workgroups statically, so the grid holds no more
// workgroups than can be resident at once (their count depends on the
// variant's registers; looked up once per variant): a second round of
// late-starting workgroups would each still take a full share of tiles.
template <class Kern>
static int launch_filter_sum(Kern kern, int nd, int64_t n, hipStream_t s, const FilterSumArgs &f) {
    static int resident[kSumMaxCols + 1] = {};
    if (resident[nd] == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern),
                                                         kFilterNT, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        resident[nd] = per_cu;
    }
    int per_cu = 2 * tune(kTuneFilterPerCu);
    if (per_cu > resident[nd]) per_cu = resident[nd];
    const unsigned grid = persistent_grid(ceil_div(n, kSumTile), per_cu);
    TQP_LAUNCH("filter_sum", kern, dim3(grid), dim3(kFilterNT), 0, s, f);
    return check_launch("tqp_filter_sum");
}

static size_t filter_ws(int64_t n) {
    Carver c(nullptr);
    c.take<uint64_t>(1 + (n > 0 ? ceil_div(n, kFilterTile) : 1));
    return c.bytes();
}

}  // namespace tqp

using namespace tqp;

TQP_API size_t tqp_filter_workspace_bytes(int64_t n) { return filter_ws(n < 0 ? 0 : n); }

TQP_API int tqp_filter(const tqp_col *cols, int ncols, const tqp_pred *preds, int npred,
                       const tqp_col *pay_in, const tqp_col *pay_out, int npay,
                       int32_t *out_rows, int64_t *d_count, void *ws, size_t ws_bytes,
                       void *stream) {
    clear_error();
    if (!cols || ncols < 1 || ncols > kMaxPred)
        return set_error(TQP_EINVAL, "tqp_filter: ncols must be in [1, %d]", kMaxPred);
    if (!preds || npred < 1 || npred > kMaxPred)
        return set_error(TQP_EINVAL, "tqp_filter: npred must be in [1, %d]", kMaxPred);
    if (npay < 0 || npay > kMaxPay || (npay > 0 && (!pay_in || !pay_out)))
        return set_error(TQP_EINVAL, "tqp_filter: npay must be in [0, %d] with both arrays", kMaxPay);
    if (!d_count) return set_error(TQP_EINVAL, "tqp_filter: d_count is required");
    const int64_t n = cols[0].len;
    if (n < 0 || n > INT32_MAX) return set_error(TQP_EINVAL, "tqp_filter: bad row count %lld", (long long)n);
    FilterArgs a = {};
    bool vec = true;
    for (int c = 0; c < ncols; c++) {
        if (!dtype_ok(cols[c].dtype) || cols[c].len != n || (n > 0 && !cols[c].data))
            return set_error(TQP_EINVAL, "tqp_filter: column %d has a bad dtype, length or pointer", c);
        if (!col_aligned(cols[c].data, cols[c].dtype))
            return set_error(TQP_EINVAL, "tqp_filter: column %d is unaligned", c);
        vec = vec && (reinterpret_cast<uintptr_t>(cols[c].data) % 16 == 0);
    }
    for (int p = 0; p < npred; p++) {
        if (preds[p].col < 0 || preds[p].col >= ncols || preds[p].op < TQP_LT || preds[p].op > TQP_NE)
            return set_error(TQP_EINVAL, "tqp_filter: predicate %d is invalid", p);
        a.pcol[p] = cols[preds[p].col].data;
        a.pdt[p] = cols[preds[p].col].dtype;
        a.pcolid[p] = preds[p].col;
        a.pop[p] = preds[p].op;
        a.plit[p] = preds[p].literal;
    }
    for (int c = 0; c < npay; c++) {
        if (!dtype_ok(pay_in[c].dtype) || pay_in[c].dtype != pay_out[c].dtype ||
            pay_in[c].len != n || pay_out[c].len < n || (n > 0 && (!pay_in[c].data || !pay_out[c].data)))
            return set_error(TQP_EINVAL, "tqp_filter: payload %d has a bad dtype, length or pointer", c);
        // (kept rows' payload is read as the aligned 8-byte word holding it)
        if (!col_aligned(pay_in[c].data, pay_in[c].dtype) || !col_aligned(pay_out[c].data, pay_out[c].dtype))
            return set_error(TQP_EINVAL, "tqp_filter: payload %d is unaligned", c);
        vec = vec && (reinterpret_cast<uintptr_t>(pay_in[c].data) % 16 == 0);
        a.pin[c] = pay_in[c].data;
        a.pout[c] = pay_out[c].data;
        a.paydt[c] = pay_in[c].dtype;
    }
    const size_t need = filter_ws(n);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "tqp_filter: workspace needs %zu bytes", need);
    hipStream_t s = as_stream(stream);
    Carver cv(ws);
    const int64_t ntiles = ceil_div(n, kFilterTile);
    uint64_t *words = cv.take<uint64_t>(1 + (ntiles > 0 ? ntiles : 1));
    int rc = fill_u64(words, 0, 1 + (ntiles > 0 ? ntiles : 1), s);
    if (rc) return rc;
    a.npred = npred;
    a.npay = npay;
    a.vec = vec ? 1 : 0;
    a.out_rows = out_rows;
    a.d_count = d_count;
    a.n = n;
    a.ticket = reinterpret_cast<uint32_t *>(words);
    a.status = words + 1;
    const unsigned grid = persistent_grid(ntiles, tune(kTuneFilterPerCu));
    TQP_LAUNCH("filter", k_filter, dim3(grid), dim3(kFilterNT), 0, s, a);
    return check_launch("tqp_filter");
}

TQP_API int tqp_filter_sum(const tqp_col *cols, int ncols, const tqp_pred *preds, int npred,
                           const tqp_col *a, const tqp_col *b, int64_t *d_sum, int64_t *d_count,
                           void *stream) {
    clear_error();
    if (!cols || ncols < 1 || ncols > kMaxPred)
        return set_error(TQP_EINVAL, "tqp_filter_sum: ncols must be in [1, %d]", kMaxPred);
    if (npred < 0 || npred > kMaxPred || (npred > 0 && !preds))
        return set_error(TQP_EINVAL, "tqp_filter_sum: npred must be in [0, %d]", kMaxPred);
    if (!d_sum || !d_count) return set_error(TQP_EINVAL, "tqp_filter_sum: d_sum and d_count are required");
    if (b && !a) return set_error(TQP_EINVAL, "tqp_filter_sum: b needs a");
    const int64_t n = cols[0].len;
    if (n < 0 || n > INT32_MAX) return set_error(TQP_EINVAL, "tqp_filter_sum: bad row count %lld", (long long)n);
    FilterSumArgs f = {};
    bool vec = true;
    for (int c = 0; c < ncols; c++) {
        if (!dtype_ok(cols[c].dtype) || cols[c].len != n || (n > 0 && !cols[c].data) ||
            !col_aligned(cols[c].data, cols[c].dtype))
            return set_error(TQP_EINVAL, "tqp_filter_sum: column %d has a bad dtype, length or pointer", c);
        vec = vec && (reinterpret_cast<uintptr_t>(cols[c].data) % 16 == 0);
    }
    for (int p = 0; p < npred; p++)
        if (preds[p].col < 0 || preds[p].col >= ncols || preds[p].op < TQP_LT || preds[p].op > TQP_NE)
            return set_error(TQP_EINVAL, "tqp_filter_sum: predicate %d is invalid", p);
    // predicates grouped by column, columns in order of first use (a
    // conjunction does not depend on the order of its terms)
    int np = 0;
    f.nd = 0;
    for (int p = 0; p < npred; p++) {
        const int col = preds[p].col;
        bool seen = false;
        for (int q = 0; q < p; q++) seen = seen || preds[q].col == col;
        if (seen) continue;
        f.dcol[f.nd] = cols[col].data;
        f.ddt[f.nd] = cols[col].dtype;
        f.pbeg[f.nd] = np;
        f.nd++;
        for (int q = p; q < npred; q++) {
            if (preds[q].col != col) continue;
            f.pcol[np] = cols[col].data;
            f.pdt[np] = cols[col].dtype;
            f.pcolid[np] = col;
            f.pop[np] = preds[q].op;
            f.plit[np] = preds[q].literal;
            np++;
        }
    }
    f.pbeg[f.nd] = np;
    const tqp_col *vals[2] = {a, b};
    for (int k = 0; k < 2; k++) {
        const tqp_col *v = vals[k];
        if (!v) continue;
        if (!dtype_ok(v->dtype) || v->len < n || (n > 0 && !v->data) || !col_aligned(v->data, v->dtype))
            return set_error(TQP_EINVAL, "tqp_filter_sum: value column %c has a bad dtype, length or pointer",
                             k ? 'b' : 'a');
        vec = vec && (reinterpret_cast<uintptr_t>(v->data) % 16 == 0);
    }
    f.npred = npred;
    f.vec = vec ? 1 : 0;
    f.a = a ? a->data : nullptr;
    f.b = b ? b->data : nullptr;
    f.adt = a ? a->dtype : 0;
    f.bdt = b ? b->dtype : 0;
    // a value operand that is one of the loaded predicate columns
    f.aslot = f.bslot = -1;
    for (int c = 0; c < f.nd; c++) {
        if (a && f.aslot < 0 && f.dcol[c] == a->data && f.ddt[c] == a->dtype) f.aslot = c;
        if (b && f.bslot < 0 && f.dcol[c] == b->data && f.ddt[c] == b->dtype) f.bslot = c;
    }
    f.n = n;
    f.d_sum = reinterpret_cast<unsigned long long *>(d_sum);
    f.d_count = reinterpret_cast<unsigned long long *>(d_count);
    hipStream_t s = as_stream(stream);
    TQP_LAUNCH("filter_sum_init", k_zero2, dim3(1), dim3(64), 0, s, f.d_sum, f.d_count);
    int rc = check_launch("tqp_filter_sum");
    if (rc || n == 0) return rc;
    const int nd = f.nd <= kSumMaxCols ? f.nd : 0;
    switch (nd) {
    case 1: return launch_filter_sum(k_filter_sum<1>, nd, n, s, f);
    case 2: return launch_filter_sum(k_filter_sum<2>, nd, n, s, f);
    case 3: return launch_filter_sum(k_filter_sum<3>, nd, n, s, f);
    case 4: return launch_filter_sum(k_filter_sum<4>, nd, n, s, f);
    default: return launch_filter_sum(k_filter_sum<0>, nd, n, s, f);
    }
}
