// Semi-join reduction in front of a star join.
//
// An inner join of a fact row with a dimension can only produce output when
// the row's foreign key occurs among the dimension's (filtered) keys, so the
// fact rows that fail that test for any dimension can be dropped before the
// sort-merge joins without changing their result (the relational semi-join
// of the fact table with each dimension side).
//
// A dimension side is reduced to a key set: a bitmap over its key range
// (tqp_keyset_build).  The fact table is then scanned once.  Each workgroup
// takes a tile of rows; every key column is read with 16-byte loads that are
// consecutive across the lanes of the workgroup (each load instruction of a
// wave covers 1 KiB of one column), all of them issued before the first
// test.  Sets small enough are staged in LDS once per workgroup; larger ones
// are read from memory (they stay in L2) for the rows still alive after the
// LDS tests.  The surviving rows are compacted in ascending order: a block
// scan inside the tile and a decoupled look-back across tiles give each its
// output slot, where it is written straight from registers.
#include <mutex>

#include "tqp_internal.hpp"

namespace tqp {

constexpr int kSjNT = 256;
constexpr int kSjMaxSets = 4;
constexpr int kSjMaxPay = 4;
// Words of key sets staged in LDS per 256 threads of workgroup (36 KiB): a
// 1024-thread workgroup, alone on its compute unit, stages up to 144 KiB.
constexpr int kSjLdsWordsPer256 = 9216;
// Kept rows of a tile staged in LDS (row ids and keys) so that the tile's
// look-back and writes can wait until the next tile's loads are in flight;
// a tile keeping more is written at once from registers instead.
constexpr int kSjStage = 256;
template <class K> constexpr int sj_stage_words(int ns) {
    return 2 * kSjStage * (1 + ns * int(sizeof(K) / 4));     // two buffers, in 4-byte words
}
// Tiles are handed out in groups of kSjGroup consecutive tiles per XCD
// counter (workgroup b draws from counter b % kSjXcds), so that no single
// ticket address takes every workgroup's atomic.
constexpr int kSjXcds = 8;
constexpr int kSjGroup = 8;

struct SemiArgs {
    const void *key[kSjMaxSets];
    const uint32_t *bits[kSjMaxSets];
    int64_t lo[kSjMaxSets];
    uint64_t nbits[kSjMaxSets];
    int32_t lds_off[kSjMaxSets];     // word offset of a set staged in LDS; -1: read from memory
    int32_t lds_len[kSjMaxSets];
    void *key_out[kSjMaxSets];
    const void *pin[kSjMaxPay];
    void *pout[kSjMaxPay];
    int32_t paylg[kSjMaxPay];
    int32_t npay;
    int32_t lds_words;
    int32_t vec;                     // every key column is 16-byte aligned
    int32_t *out_rows;
    int64_t *d_count;
    int64_t n;
    uint32_t *ticket;                // kSjXcds counters
    uint64_t *status;                // one look-back status per tile
};

// Rows per thread per tile: up to 16, fewer with more sets or wider keys
// (three steps of 16-byte loads per set with three or four sets), so that a
// tile's keys and the staging of the previous tile's kept rows fit the
// registers.  Each step is one 16-byte load per set.
template <class K, int NS> struct SjShape {
    static constexpr int V = 16 / int(sizeof(K));     // keys per 16-byte load
    static constexpr int Steps = (16 / V) < (NS >= 3 ? 3 : 12 / NS) ? (16 / V) : (NS >= 3 ? 3 : 12 / NS);
    static constexpr int R = V * Steps;               // rows per thread per tile
};
// the smallest tile of any set count and workgroup size (sizes the
// look-back statuses)
template <class K> constexpr int64_t sj_min_tile() {
    return int64_t(kSjNT) * SjShape<K, kSjMaxSets>::R;
}

// Stores element value v of a payload column of element size 1 << lg.
__device__ __forceinline__ void sj_store(void *out, int lg, int64_t i, uint64_t v) {
    if (lg == 0) static_cast<uint8_t *>(out)[i] = uint8_t(v);
    else if (lg == 2) static_cast<uint32_t *>(out)[i] = uint32_t(v);
    else static_cast<uint64_t *>(out)[i] = v;
}

// Tiles of one XCD counter come in groups of kSjGroup consecutive tiles.
__device__ __forceinline__ int64_t sj_tile_of(int64_t ticket, int xcd) {
    return ((ticket / kSjGroup) * kSjXcds + xcd) * kSjGroup + ticket % kSjGroup;
}

// Writes a staged tile's kept rows (row ids, keys, then the payload read
// through the row ids) to their slots from base, consecutive threads taking
// consecutive slots.  The staging writes and the prefix in LDS must be
// visible: callers come here after a barrier that follows both.
template <class K, int NS, int NT>
__device__ __forceinline__ void sj_write_staged(const SemiArgs &a, const int32_t *srow,
                                                int64_t base, int cnt, bool last_tile) {
    const K *skey = reinterpret_cast<const K *>(srow + kSjStage);
    if (last_tile && threadIdx.x == 0) *a.d_count = base + cnt;
    for (int i = threadIdx.x; i < cnt; i += NT) {
        const int32_t row = srow[i];
        if (a.out_rows) a.out_rows[base + i] = row;
#pragma unroll
        for (int s = 0; s < NS; s++)
            if (a.key_out[s]) static_cast<K *>(a.key_out[s])[base + i] = skey[s * kSjStage + i];
#pragma unroll 1
        for (int c = 0; c < a.npay; c++) {
            const int lg = a.paylg[c];
            sj_store(a.pout[c], lg, base + i, from_word(word_of(a.pin[c], lg, row), a.pin[c], lg, row));
        }
    }
}

// NT threads per workgroup; a tile is NT * R rows.  Larger workgroups take
// larger tiles, so the per-tile ticket, scan and look-back are paid over
// more rows.
template <class K, int NS, int NT>
__global__ __launch_bounds__(NT) void k_semijoin(SemiArgs a) {
    using S = SjShape<K, NS>;
    constexpr int V = S::V;
    constexpr int R = S::R;
    constexpr int64_t Tile = int64_t(NT) * R;
    constexpr int64_t Step = int64_t(NT) * V;
    constexpr int NW = S::Steps > 4 ? 2 : 1;       // words of packed step counts
    static_assert(R <= 32, "keep bits of a thread fit one word");
    __shared__ int64_t s_tile;
    __shared__ int64_t s_prefix, s_pprefix;
    __shared__ uint64_t s_scan[NT / kWave];
    extern __shared__ uint32_t s_sets[];

    const int64_t n = a.n;
    const int64_t ntiles = ceil_div(n, Tile);
    const bool vec = a.vec != 0;
    const int tid = threadIdx.x;
    const int xcd = int(blockIdx.x % kSjXcds);
    const uint32_t full = R == 32 ? ~0u : (1u << R) - 1u;

    // stage the small sets once per workgroup
    for (int s = 0; s < NS; s++) {
        if (a.lds_off[s] < 0) continue;
        uint32_t *dst = s_sets + a.lds_off[s];
        for (int i = tid; i < a.lds_len[s]; i += NT) dst[i] = a.bits[s][i];
    }
    __syncthreads();
    // the kept rows waiting to be written, after the sets: two buffers, each
    // row ids then each set's keys.  A tile stages into one while the
    // previous tile's rows are written from the other.
    int32_t *s_stage = reinterpret_cast<int32_t *>(s_sets + ((a.lds_words + 3) & ~3));
    const int stage_half = sj_stage_words<K>(NS) / 2;
    int64_t pend_tile = -1;              // the tile whose kept rows wait in LDS
    int pend_total = 0, pb = 0;
    // A tile's ticket is drawn only when the workgroup is ready to work on
    // it: every tile handed out is in progress, so the look-backs of later
    // tiles never wait on a tile that is merely reserved.
    for (;;) {
        const int64_t tile = sj_tile_of(take_tile(a.ticket + xcd, &s_tile), xcd);
        const bool last = tile >= ntiles;
        if (last && tile == 0 && tid == 0) *a.d_count = 0;    // empty input
        const int64_t row0 = tile * Tile;
        // item r = k * V + jj of this thread is row trow + k * Step + jj
        const int64_t trow = row0 + int64_t(tid) * V;
        K v[NS][R];
        uint32_t alive = full;
        if (vec && row0 + Tile <= n) {
            // a whole tile (the same branch for the workgroup): every load is
            // one 16-byte vector, all issued before the first test
#pragma unroll
            for (int s = 0; s < NS; s++) {
                const K *p = static_cast<const K *>(a.key[s]);
#pragma unroll
                for (int k = 0; k < S::Steps; k++) {
                    if constexpr (sizeof(K) == 4) {
                        const int4 x = *reinterpret_cast<const int4 *>(p + trow + k * Step);
                        v[s][k * V + 0] = x.x; v[s][k * V + 1] = x.y;
                        v[s][k * V + 2] = x.z; v[s][k * V + 3] = x.w;
                    } else {
                        const longlong2 x = *reinterpret_cast<const longlong2 *>(p + trow + k * Step);
                        v[s][k * V + 0] = x.x; v[s][k * V + 1] = x.y;
                    }
                }
            }
        } else {
            alive = 0;
#pragma unroll
            for (int s = 0; s < NS; s++) {
                const K *p = static_cast<const K *>(a.key[s]);
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const int64_t row = trow + (r / V) * Step + (r % V);
                    v[s][r] = row < n ? p[row] : K(0);
                }
            }
#pragma unroll
            for (int r = 0; r < R; r++)
                if (trow + (r / V) * Step + (r % V) < n) alive |= 1u << r;
        }
        // the previous tile's look-back while these loads are in flight (its
        // predecessors have long posted their counts); its rows are written
        // at the end of this tile, once this tile's keys are no longer held
        if (pend_tile >= 0 && wave_id() == 0) {
            const int64_t pre = lookback_resolve(a.status, pend_tile, pend_total);
            if (lane_id() == 0) s_pprefix = pre;
        }
        if (last) {
            if (pend_tile >= 0) {
                __syncthreads();
                sj_write_staged<K, NS, NT>(a, s_stage + pb * stage_half, s_pprefix, pend_total,
                                           pend_tile == ntiles - 1);
            }
            break;
        }
        // sets in LDS: every row tested (LDS reads are cheap); a set of at
        // most 64 keys is held in a register instead
#pragma unroll
        for (int s = 0; s < NS; s++) {
            if (a.lds_off[s] < 0) continue;
            const uint32_t *w = s_sets + a.lds_off[s];
            const uint64_t lo = uint64_t(a.lo[s]);
            const uint64_t nb = a.nbits[s];
            uint32_t m = 0;
            if (nb <= 64) {
                const uint64_t bits = uint64_t(w[0]) | (nb > 32 ? uint64_t(w[1]) << 32 : 0);
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const uint64_t idx = uint64_t(int64_t(v[s][r])) - lo;
                    if (idx < nb && ((bits >> idx) & 1u)) m |= 1u << r;
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const uint64_t idx = uint64_t(int64_t(v[s][r])) - lo;
                    const bool in = idx < nb;
                    const uint32_t word = w[in ? uint32_t(idx >> 5) : 0u];
                    if (in && ((word >> (idx & 31)) & 1u)) m |= 1u << r;
                }
            }
            alive &= m;
        }
        // sets in memory: only the rows still alive read their word
#pragma unroll
        for (int s = 0; s < NS; s++) {
            if (a.lds_off[s] >= 0) continue;
            const uint32_t *w = a.bits[s];
            const uint64_t lo = uint64_t(a.lo[s]);
            const uint64_t nb = a.nbits[s];
            uint32_t word[R];
            uint32_t need = 0;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const uint64_t idx = uint64_t(int64_t(v[s][r])) - lo;
                const bool in = ((alive >> r) & 1u) && idx < nb;
                if (in) need |= 1u << r;
                word[r] = in ? w[idx >> 5] : 0u;
            }
            uint32_t m = 0;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const uint64_t idx = uint64_t(int64_t(v[s][r])) - lo;
                if (((need >> r) & 1u) && ((word[r] >> (idx & 31)) & 1u)) m |= 1u << r;
            }
            alive &= m;
        }

        // slots: kept items are ordered by (step k, thread, jj) = by row.
        // Per-step counts are packed 16 bits apiece, four steps per word
        // (a step keeps at most NT * V <= 4096 rows).
        uint64_t packed[NW], excl[NW], tot[NW];
#pragma unroll
        for (int w = 0; w < NW; w++) packed[w] = 0;
#pragma unroll
        for (int k = 0; k < S::Steps; k++) {
            const uint32_t mk = (alive >> (k * V)) & ((1u << V) - 1u);
            packed[k / 4] += uint64_t(__popc(mk)) << (16 * (k % 4));
        }
#pragma unroll
        for (int w = 0; w < NW; w++) excl[w] = block_excl_scan<NT>(packed[w], &tot[w], s_scan);
        int total = 0;
        int first[S::Steps];                     // slot of the thread's first kept item of step k
#pragma unroll
        for (int k = 0; k < S::Steps; k++) {
            first[k] = total + int((excl[k / 4] >> (16 * (k % 4))) & 0xffff);
            total += int((tot[k / 4] >> (16 * (k % 4))) & 0xffff);
        }
        if (wave_id() == 0) lookback_publish(a.status, tile, total);
        const bool stage = total <= kSjStage;
        const int cb = pend_tile >= 0 ? pb ^ 1 : pb;
        if (stage) {
            // stage the kept rows in slot order; written during the next tile
            int32_t *srow = s_stage + cb * stage_half;
            K *skey = reinterpret_cast<K *>(srow + kSjStage);
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int k = r / V, jj = r % V;
                const uint32_t mk = (alive >> (k * V)) & ((1u << V) - 1u);
                if (!((mk >> jj) & 1u)) continue;
                const int local = first[k] + __popc(mk & ((1u << jj) - 1u));
                srow[local] = int32_t(trow + k * Step + jj);
#pragma unroll
                for (int s = 0; s < NS; s++) skey[s * kSjStage + local] = v[s][r];
            }
        } else {
            // too many kept rows to stage: this tile's prefix now, its rows
            // straight from registers (each column's writes of a tile cover
            // one contiguous run, which the L2 merges into whole lines)
            if (wave_id() == 0) {
                const int64_t pre = lookback_resolve(a.status, tile, total);
                if (lane_id() == 0) s_prefix = pre;
            }
            __syncthreads();
            const int64_t base = s_prefix;
            if (tile == ntiles - 1 && tid == 0) *a.d_count = base + total;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int k = r / V, jj = r % V;
                const uint32_t mk = (alive >> (k * V)) & ((1u << V) - 1u);
                if (!((mk >> jj) & 1u)) continue;
                const int64_t slot = base + first[k] + __popc(mk & ((1u << jj) - 1u));
                if (a.out_rows) a.out_rows[slot] = int32_t(trow + k * Step + jj);
#pragma unroll
                for (int s = 0; s < NS; s++)
                    if (a.key_out[s]) static_cast<K *>(a.key_out[s])[slot] = v[s][r];
            }
            // payload: only kept rows are read, four loads in flight at a time
            for (int c = 0; c < a.npay; c++) {
                const int lg = a.paylg[c];
                const void *src = a.pin[c];
#pragma unroll
                for (int r0 = 0; r0 < R; r0 += 4) {
                    uint64_t val[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int r = r0 + q;
                        const int64_t row = trow + (r / V) * Step + (r % V);
                        val[q] = ((alive >> r) & 1u) ? word_of(src, lg, row) : 0;
                    }
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int r = r0 + q, k = r / V, jj = r % V;
                        if (!((alive >> r) & 1u)) continue;
                        const uint32_t mk = (alive >> (k * V)) & ((1u << V) - 1u);
                        const int64_t row = trow + k * Step + jj;
                        const int64_t slot = base + first[k] + __popc(mk & ((1u << jj) - 1u));
                        sj_store(a.pout[c], lg, slot, from_word(val[q], src, lg, row));
                    }
                }
            }
        }
        // the previous tile's rows, now that this tile's keys are no longer
        // needed (its prefix was posted before this tile's block scan)
        if (pend_tile >= 0)
            sj_write_staged<K, NS, NT>(a, s_stage + pb * stage_half, s_pprefix, pend_total,
                                       pend_tile == ntiles - 1);
        pend_tile = stage ? tile : -1;
        pend_total = total;
        pb = cb;
    }
}

// Sets the bit of every key (of the first count) that falls in the set's
// range [lo, lo + nbits).
__global__ __launch_bounds__(256) void k_keyset_set(const void *key, int dt, int64_t n,
                                                    const int64_t *d_n, int64_t lo,
                                                    uint64_t nbits, uint32_t *bits) {
    const int64_t cnt = count_of(d_n, n);
    const int lg = dtype_lg(dt);
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < cnt;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t v = sext_of(load_word(key, lg, i), dt);
        const uint64_t idx = uint64_t(v) - uint64_t(lo);
        if (idx < nbits) atomicOr(&bits[idx >> 5], 1u << (idx & 31));
    }
}

static size_t semijoin_ws(int64_t n, int dtype) {
    const int64_t tile = dtype == TQP_INT32 ? sj_min_tile<int32_t>() : sj_min_tile<int64_t>();
    Carver c(nullptr);
    c.take<uint64_t>(kSjXcds / 2 + (n > 0 ? ceil_div(n, tile) : 1));
    return c.bytes();
}

// Dynamic LDS beyond 64 KiB has to be allowed per kernel.
template <class F> static int sj_allow_lds(F kern, size_t lds) {
    if (lds <= 65536) return TQP_OK;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    return e == hipSuccess ? TQP_OK
                           : set_error(TQP_EHIP, "tqp_semijoin: LDS of %zu bytes: %s", lds,
                                       hipGetErrorString(e));
}

template <class K, int NT>
static int launch_semijoin_nt(int ns, unsigned grid, size_t lds, hipStream_t s, const SemiArgs &a) {
    int rc = TQP_OK;
    switch (ns) {
    case 1: rc = sj_allow_lds(k_semijoin<K, 1, NT>, lds); break;
    case 2: rc = sj_allow_lds(k_semijoin<K, 2, NT>, lds); break;
    case 3: rc = sj_allow_lds(k_semijoin<K, 3, NT>, lds); break;
    default: rc = sj_allow_lds(k_semijoin<K, 4, NT>, lds); break;
    }
    if (rc) return rc;
    switch (ns) {
    case 1: TQP_LAUNCH("semijoin", (k_semijoin<K, 1, NT>), dim3(grid), dim3(NT), lds, s, a); break;
    case 2: TQP_LAUNCH("semijoin", (k_semijoin<K, 2, NT>), dim3(grid), dim3(NT), lds, s, a); break;
    case 3: TQP_LAUNCH("semijoin", (k_semijoin<K, 3, NT>), dim3(grid), dim3(NT), lds, s, a); break;
    default: TQP_LAUNCH("semijoin", (k_semijoin<K, 4, NT>), dim3(grid), dim3(NT), lds, s, a); break;
    }
    return TQP_OK;
}

// The workgroup size in units of kSjNT threads (1, 2 or 4) from the
// "semijoin.wg" knob.  A 1024-thread workgroup allows 128 registers per
// thread; only three 4-byte key sets and three or four 8-byte ones (12 and
// 6 rows per thread) fit it without spilling, the other shapes stop at 512.
static int sj_wg(int dtype, int ns) {
    const int wg = tune(kTuneSemiWg);
    const bool fits = dtype == TQP_INT32 ? ns == 3 : ns >= 3;
    if (wg >= 4) return fits ? 4 : 2;
    return wg >= 2 ? 2 : 1;
}

template <class K>
static int launch_semijoin(int ns, int wg, unsigned grid, size_t lds, hipStream_t s,
                           const SemiArgs &a) {
    if (wg >= 4) return launch_semijoin_nt<K, 4 * kSjNT>(ns, grid, lds, s, a);
    if (wg >= 2) return launch_semijoin_nt<K, 2 * kSjNT>(ns, grid, lds, s, a);
    return launch_semijoin_nt<K, kSjNT>(ns, grid, lds, s, a);
}

}  // namespace tqp

using namespace tqp;

TQP_API int tqp_keyset_build(const tqp_col *key, const int64_t *d_n, int64_t lo, int64_t nbits,
                             uint32_t *bits, void *stream) {
    clear_error();
    if (!key || !dtype_ok(key->dtype) || key->len < 0 || (key->len > 0 && !key->data) ||
        !col_aligned(key->data, key->dtype))
        return set_error(TQP_EINVAL, "tqp_keyset_build: bad key column");
    if (nbits < 0 || nbits > TQP_KEYSET_MAX_BITS)
        return set_error(TQP_EINVAL, "tqp_keyset_build: nbits must be in [0, 2^36]");
    if (nbits > 0 && !bits) return set_error(TQP_EINVAL, "tqp_keyset_build: bits is required");
    if (nbits > 0 && lo > INT64_MAX - nbits + 1)
        return set_error(TQP_EINVAL, "tqp_keyset_build: lo + nbits - 1 exceeds the int64 range");
    if (nbits == 0) return TQP_OK;
    hipStream_t s = as_stream(stream);
    int rc = fill_u32(bits, 0, ceil_div(nbits, 32), s);
    if (rc || key->len == 0) return rc;
    int64_t blocks = ceil_div(key->len, 256 * 8);
    if (blocks > 2048) blocks = 2048;
    TQP_LAUNCH("keyset_set", k_keyset_set, dim3(unsigned(blocks)), dim3(256), 0, s, key->data,
               key->dtype, key->len, d_n, lo, uint64_t(nbits), bits);
    return check_launch("tqp_keyset_build");
}

TQP_API size_t tqp_semijoin_workspace_bytes(int64_t n, int dtype) {
    return semijoin_ws(n < 0 ? 0 : n, dtype);
}

// Validates the arguments, then clears the tickets and look-back statuses in
// `words` (the caller's workspace, or the library's static scratch) and
// launches the scan.  words_cap: uint64 words available at `words`.
static int semijoin_run(const char *who, const tqp_col *keys, const tqp_keyset *sets, int nsets,
                        const tqp_col *keys_out, const tqp_col *pay_in, const tqp_col *pay_out,
                        int npay, int32_t *out_rows, int64_t *d_count, uint64_t *words,
                        int64_t words_cap, void *stream) {
    if (!keys || !sets || nsets < 1 || nsets > kSjMaxSets)
        return set_error(TQP_EINVAL, "%s: nsets must be in [1, %d] with keys and sets", who,
                         kSjMaxSets);
    if (npay < 0 || npay > kSjMaxPay || (npay > 0 && (!pay_in || !pay_out)))
        return set_error(TQP_EINVAL, "%s: npay must be in [0, %d] with both arrays", who,
                         kSjMaxPay);
    if (!d_count) return set_error(TQP_EINVAL, "%s: d_count is required", who);
    const int64_t n = keys[0].len;
    const int dt = keys[0].dtype;
    if (n < 0 || n > INT32_MAX)
        return set_error(TQP_EINVAL, "%s: bad row count %lld", who, (long long)n);
    if (dt != TQP_INT32 && dt != TQP_INT64)
        return set_error(TQP_EINVAL, "%s: key columns must be int32 or int64", who);
    SemiArgs a = {};
    bool vec = true;
    int lds_words = 0;
    const int wg = sj_wg(dt, nsets);
    const int lds_budget = kSjLdsWordsPer256 * wg;
    for (int s = 0; s < nsets; s++) {
        if (keys[s].dtype != dt || keys[s].len != n || (n > 0 && !keys[s].data) ||
            !col_aligned(keys[s].data, dt))
            return set_error(TQP_EINVAL,
                             "%s: key column %d differs in dtype or length, or is unaligned", who, s);
        if (sets[s].nbits < 0 || sets[s].nbits > TQP_KEYSET_MAX_BITS || (sets[s].nbits > 0 && !sets[s].bits) ||
            (sets[s].nbits > 0 && sets[s].lo > INT64_MAX - sets[s].nbits + 1))
            return set_error(TQP_EINVAL, "%s: key set %d is invalid", who, s);
        vec = vec && reinterpret_cast<uintptr_t>(keys[s].data) % 16 == 0;
        a.key[s] = keys[s].data;
        a.bits[s] = sets[s].bits;
        a.lo[s] = sets[s].lo;
        a.nbits[s] = uint64_t(sets[s].nbits);
        const int64_t words_s = ceil_div(sets[s].nbits, 32);
        if (words_s > 0 && lds_words + words_s <= lds_budget) {
            a.lds_off[s] = lds_words;
            a.lds_len[s] = int32_t(words_s);
            lds_words += int(words_s);
        } else {
            a.lds_off[s] = -1;
            a.lds_len[s] = 0;
        }
        if (keys_out && keys_out[s].data) {
            if (keys_out[s].dtype != dt || keys_out[s].len < n)
                return set_error(TQP_EINVAL, "%s: keys_out[%d] has a bad dtype or length", who, s);
            a.key_out[s] = keys_out[s].data;
        }
    }
    for (int c = 0; c < npay; c++) {
        if (!dtype_ok(pay_in[c].dtype) || pay_in[c].dtype != pay_out[c].dtype ||
            pay_in[c].len < n || pay_out[c].len < n ||
            (n > 0 && (!pay_in[c].data || !pay_out[c].data)) ||
            !col_aligned(pay_in[c].data, pay_in[c].dtype) ||
            !col_aligned(pay_out[c].data, pay_out[c].dtype))
            return set_error(TQP_EINVAL, "%s: payload %d has a bad dtype, length or pointer", who, c);
        a.pin[c] = pay_in[c].data;
        a.pout[c] = pay_out[c].data;
        a.paylg[c] = pay_in[c].dtype == TQP_INT8 ? 0 : pay_in[c].dtype == TQP_INT32 ? 2 : 3;
    }
    const int64_t tile = dt == TQP_INT32 ? sj_min_tile<int32_t>() : sj_min_tile<int64_t>();
    const int64_t ntiles = ceil_div(n, tile);        // an upper bound for every set count
    const int64_t nwords = kSjXcds / 2 + (ntiles > 0 ? ntiles : 1);
    if (!words || words_cap < nwords)
        return set_error(TQP_ECAPACITY, "%s: scratch needs %lld bytes", who,
                         (long long)(nwords * 8));
    hipStream_t s = as_stream(stream);
    int rc = fill_u64(words, 0, nwords, s);
    if (rc) return rc;
    a.npay = npay;
    a.lds_words = lds_words;
    a.vec = vec ? 1 : 0;
    a.out_rows = out_rows;
    a.d_count = d_count;
    a.n = n;
    a.ticket = reinterpret_cast<uint32_t *>(words);
    a.status = words + kSjXcds / 2;
    // workgroups per CU count 256-thread units: a 1024-thread workgroup takes four
    const int per_cu = tune(kTuneSemiPerCu) / wg > 0 ? tune(kTuneSemiPerCu) / wg : 1;
    const unsigned grid = persistent_grid(ntiles, per_cu);
    // the sets, then (16-byte aligned) the staging of kept rows
    const int stage_words = dt == TQP_INT32 ? sj_stage_words<int32_t>(nsets)
                                            : sj_stage_words<int64_t>(nsets);
    const size_t lds = size_t(((lds_words + 3) & ~3) + stage_words) * 4;
    rc = dt == TQP_INT32 ? launch_semijoin<int32_t>(nsets, wg, grid, lds, s, a)
                         : launch_semijoin<int64_t>(nsets, wg, grid, lds, s, a);
    if (rc) return rc;
    return check_launch(who);
}

TQP_API int tqp_semijoin(const tqp_col *keys, const tqp_keyset *sets, int nsets,
                         const tqp_col *keys_out, const tqp_col *pay_in, const tqp_col *pay_out,
                         int npay, int32_t *out_rows, int64_t *d_count, void *ws, size_t ws_bytes,
                         void *stream) {
    clear_error();
    if (reinterpret_cast<uintptr_t>(ws) % 8 != 0)
        return set_error(TQP_EINVAL, "tqp_semijoin: the workspace must be 8-byte aligned");
    return semijoin_run("tqp_semijoin", keys, sets, nsets, keys_out, pay_in, pay_out, npay,
                        out_rows, d_count, static_cast<uint64_t *>(ws), int64_t(ws_bytes / 8),
                        stream);
}

// ---- the same scan with library-held scratch ------------------------------
// For callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid allocation): the tickets and
// look-back statuses live in a file-scope device array instead of a
// caller's workspace.  Each device the library runs on holds its own copy
// until the process ends.
constexpr int64_t kSjScratchWords = int64_t(1) << 20;       // 8 MiB
static __device__ __align__(256) uint64_t scratch[kSjScratchWords];
constexpr int kSjMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint64_t *g_scratch_ptr[kSjMaxDevices];

// The device address of this device's scratch (the host-side name of the
// array is not one), looked up on the first call on each device.
static int sj_scratch(uint64_t **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return set_error(TQP_EHIP, "tqp_semijoin_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kSjMaxDevices)
        return set_error(TQP_EINVAL, "tqp_semijoin_noalloc: device %d beyond the %d supported", dev,
                         kSjMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(TQP_EHIP, "tqp_semijoin_noalloc: scratch address: %s",
                             hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<uint64_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return TQP_OK;
}

TQP_API int64_t tqp_semijoin_noalloc_max_rows(int dtype) {
    if (dtype != TQP_INT32 && dtype != TQP_INT64) return 0;
    const int64_t tile = dtype == TQP_INT32 ? sj_min_tile<int32_t>() : sj_min_tile<int64_t>();
    const int64_t rows = (kSjScratchWords - kSjXcds / 2) * tile;
    return rows < INT32_MAX ? rows : INT32_MAX;
}

TQP_API int tqp_semijoin_noalloc(const tqp_col *keys, const tqp_keyset *sets, int nsets,
                                 const tqp_col *keys_out, const tqp_col *pay_in,
                                 const tqp_col *pay_out, int npay, int32_t *out_rows,
                                 int64_t *d_count, void *stream) {
    clear_error();
    if (keys && (keys[0].dtype == TQP_INT32 || keys[0].dtype == TQP_INT64) &&
        keys[0].len > tqp_semijoin_noalloc_max_rows(keys[0].dtype))
        return set_error(TQP_ECAPACITY,
                         "tqp_semijoin_noalloc: %lld rows exceed the static scratch's %lld",
                         (long long)keys[0].len,
                         (long long)tqp_semijoin_noalloc_max_rows(keys[0].dtype));
    uint64_t *words = nullptr;
    int rc = sj_scratch(&words);
    if (rc) return rc;
    return semijoin_run("tqp_semijoin_noalloc", keys, sets, nsets, keys_out, pay_in, pay_out,
                        npay, out_rows, d_count, words, kSjScratchWords, stream);
}
