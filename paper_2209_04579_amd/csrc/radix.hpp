#pragma once
// Stable LSD radix passes over an ordinal of each key, carrying row ids and up
// to four payload columns.  The ordinal is a functor: the key itself (minus
// its minimum) for the sort, or a bucket number for a partitioner.
//
// Keys are ranked on u = key - key_min (unsigned), which orders signed keys
// correctly and drops the bits that never vary.  The b significant bits are
// cut into ceil(b / 8) digits of equal width (at most 8 bits: 21 bits take
// three 7-bit digits, not 8 + 8 + 5), so each pass has as few bins, and as
// long runs per bin, as its pass count allows.  One sweep builds the
// histograms of every digit at once; each digit then takes one pass:
//   * a workgroup takes a 4096-key tile (dynamic tile id),
//   * ranks its keys stably: each wave walks its items in input order, finds
//     the lanes holding the same digit with one ballot per digit bit, and
//     bumps a per-wave LDS counter once per distinct digit,
//   * publishes its digit counts and looks back over earlier tiles (one
//     thread per digit) for the global start of each digit run,
//   * then, column by column (keys, row ids, payloads), stages the tile in LDS
//     in digit order and writes each digit run out with consecutive threads on
//     consecutive addresses.
// Carrying the payload through the passes keeps every later read of it
// sequential, instead of a random gather through a permutation.
#include "tqp_internal.hpp"

namespace tqp {

constexpr int kSortNT = 512;
constexpr int kSortIPT = 8;
constexpr int kSortTile = kSortNT * kSortIPT;
constexpr int kRadixBits = 8;
constexpr int kBins = 1 << kRadixBits;
constexpr int kSortNW = kSortNT / kWave;
constexpr int kMaxSortPay = 4;
constexpr int kMaxPassCols = kMaxSortPay + 1;   // payload columns + row ids
constexpr int kMaxSortPred = 4;            // predicates of a filtered first pass
constexpr int kHistNT = 256;
constexpr int kHistIPT = 16;
constexpr int kLookAhead = 4;             // predecessor statuses fetched per round trip
// Tiles are handed out in groups of kTileGroup consecutive tiles per XCD:
// workgroups are dispatched to the chip's 8 XCDs round robin by index, so
// workgroup b draws from counter b % kXcds, which owns the groups g with
// g % kXcds == b % kXcds.  Consecutive tiles write adjacent parts of every
// digit run, so the cache lines they share are mostly completed in one
// XCD's L2 instead of being written partially from two.  (Correctness does
// not depend on the placement; every counter's groups are taken in order by
// resident workgroups, so the look-back always finds its predecessors.)
constexpr int kXcds = 8;
constexpr int kTileGroup = 8;
constexpr uint32_t kSFlagAgg = 1u << 30;
constexpr uint32_t kSFlagInc = 2u << 30;
constexpr uint32_t kSValMask = (1u << 30) - 1;

// The conjunction a filtered sort applies before its first pass: item i is
// kept when col[q][i] op[q] lit[q] holds for every q < npred.  Columns are
// naturally aligned, of run-time dtype, read as aligned words.
struct PassPred {
    const void *col[kMaxSortPred];
    int64_t lit[kMaxSortPred];
    int32_t dt[kMaxSortPred];
    int32_t op[kMaxSortPred];
    int32_t npred;
};

// Bit r of the result: item idx[r] satisfies every predicate (no item past
// cnt is tested; their bits are 0).  One predicate's N loads go out together.
template <int N, class I>
__device__ __forceinline__ uint32_t keep_mask(const PassPred &f, const I (&idx)[N], int64_t cnt) {
    uint32_t m = 0;
    I li[N];
#pragma unroll
    for (int r = 0; r < N; r++) {
        m |= (int64_t(idx[r]) < cnt ? 1u : 0u) << r;
        li[r] = int64_t(idx[r]) < cnt ? idx[r] : I(0);
    }
#pragma unroll
    for (int q = 0; q < kMaxSortPred; q++) {
        if (q >= f.npred) break;
        uint64_t raw[N];
        load_raw<N>(f.col[q], f.dt[q], li, raw);
#pragma unroll
        for (int r = 0; r < N; r++)
            if (!cmp_holds(sext_of(raw[r], f.dt[q]), f.op[q], f.lit[q])) m &= ~(1u << r);
    }
    return m;
}

// Counts the ordinal u of every valid lane into the wave's LDS histograms
// h[pass][digit].  Skewed keys put many lanes of a wave on one counter, and
// LDS atomics on one address serialize: the lanes sharing the first valid
// lane's digit are counted by one ballot and one add.
__device__ __forceinline__ void count_digits(uint32_t (*h)[kBins], bool valid, uint64_t u,
                                             int npass, int dbits, uint32_t dmask) {
    const uint64_t vm = ballot(valid);
    if (vm == 0) return;
    const int first = __builtin_ctzll(vm);
    for (int p = 0; p < npass; p++) {
        const uint32_t d = uint32_t(u >> (p * dbits)) & dmask;
        const uint32_t f = uint32_t(__builtin_amdgcn_readlane(int(d), first));
        const bool same = valid && d == f;
        const uint64_t sm = ballot(same);
        if (lane_id() == first) atomicAdd(&h[p][f], uint32_t(__popcll(sm)));
        else if (valid && !same) atomicAdd(&h[p][d], 1u);
    }
}

// 256-bin histograms of every digit in one sweep: each thread reads 16
// consecutive keys with 16-byte loads and counts them into its wave's LDS
// histograms; the workgroup then adds its totals to the device histogram.
template <class K, class Ord>
__global__ __launch_bounds__(kHistNT) void k_radix_hist(const K *__restrict__ keys, int64_t n,
                                                        const int64_t *d_n, Ord ord, int npass,
                                                        int dbits, uint32_t *__restrict__ ghist) {
    const uint32_t dmask = (1u << dbits) - 1;
    constexpr int kMaxPass = KeyTraits<K>::kBits / kRadixBits;
    constexpr int NW = kHistNT / kWave;
    __shared__ uint32_t s_h[NW][kMaxPass][kBins];
    for (int i = threadIdx.x; i < NW * kMaxPass * kBins; i += kHistNT) (&s_h[0][0][0])[i] = 0;
    __syncthreads();
    const int64_t cnt = count_of(d_n, n);
    const int w = wave_id();
    const int64_t chunk = int64_t(kHistNT) * kHistIPT;
    const bool vec = reinterpret_cast<uintptr_t>(keys) % 16 == 0;
    for (int64_t base = blockIdx.x * chunk; base < cnt; base += int64_t(gridDim.x) * chunk) {
        const int64_t row0 = base + int64_t(threadIdx.x) * kHistIPT;
        K v[kHistIPT];
        if (vec && row0 + kHistIPT <= cnt) {
            constexpr int kPer = 16 / sizeof(K);
            const int4 *q = reinterpret_cast<const int4 *>(keys + row0);
#pragma unroll
            for (int j = 0; j < kHistIPT / kPer; j++) {
                int4 x = q[j];
                const K *e = reinterpret_cast<const K *>(&x);
#pragma unroll
                for (int t = 0; t < kPer; t++) v[j * kPer + t] = e[t];
            }
        } else {
#pragma unroll
            for (int r = 0; r < kHistIPT; r++) v[r] = row0 + r < cnt ? keys[row0 + r] : K(0);
        }
#pragma unroll
        for (int r = 0; r < kHistIPT; r++)
            count_digits(s_h[w], row0 + r < cnt, ord(v[r]), npass, dbits, dmask);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < npass * kBins; i += kHistNT) {
        const int p = i / kBins, d = i % kBins;
        uint32_t t = 0;
#pragma unroll
        for (int ww = 0; ww < NW; ww++) t += s_h[ww][p][d];
        if (t) atomicAdd(&ghist[p * kBins + d], t);
    }
}

// The histograms of a filtered sort, over the items the predicates flt keep
// (n items, no device count).  Each step a wave tests 8 items per lane
// (item r of lane l: base + r * kHistNT + 64 * wave + l, so each r covers
// 64 consecutive items, one word of keep_bits), writes the keep bits, and
// queues its kept keys in LDS; it then counts the queue 64 keys at a time, so
// rejected items cost no counting.  Also adds the kept count to *d_kept and
// sets bit i % 64 of keep_bits[i / 64] for each kept item i (every word up to
// item n - 1 is written).
constexpr int kHistFIPT = 8;
template <class K, class Ord>
__global__ __launch_bounds__(kHistNT) void k_radix_hist_filt(const K *__restrict__ keys, int64_t n,
                                                             Ord ord, int npass, int dbits,
                                                             uint32_t *__restrict__ ghist,
                                                             PassPred flt, int64_t *d_kept,
                                                             uint64_t *__restrict__ keep_bits) {
    const uint32_t dmask = (1u << dbits) - 1;
    constexpr int kMaxPass = KeyTraits<K>::kBits / kRadixBits;
    constexpr int NW = kHistNT / kWave;
    __shared__ uint32_t s_h[NW][kMaxPass][kBins];
    __shared__ K s_q[NW][kWave * kHistFIPT];      // one wave's kept keys of one step
    for (int i = threadIdx.x; i < NW * kMaxPass * kBins; i += kHistNT) (&s_h[0][0][0])[i] = 0;
    __syncthreads();
    const int w = wave_id();
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int64_t chunk = int64_t(kHistNT) * kHistFIPT;
    uint32_t kept = 0;
    for (int64_t base = blockIdx.x * chunk; base < n; base += int64_t(gridDim.x) * chunk) {
        const int64_t w0 = base + int64_t(w) * kWave;
        int64_t ri[kHistFIPT];
        K v[kHistFIPT];
#pragma unroll
        for (int r = 0; r < kHistFIPT; r++) ri[r] = w0 + int64_t(r) * kHistNT + lane;
#pragma unroll
        for (int r = 0; r < kHistFIPT; r++) v[r] = keys[ri[r] < n ? ri[r] : 0];
        const uint32_t keep = keep_mask<kHistFIPT>(flt, ri, n);
        kept += __popc(keep);
        uint32_t qn = 0;                            // the same in every lane
#pragma unroll
        for (int r = 0; r < kHistFIPT; r++) {
            const bool kr = (keep >> r) & 1;
            const uint64_t m = ballot(kr);
            if (lane == 0 && w0 + int64_t(r) * kHistNT < n)
                keep_bits[(w0 + int64_t(r) * kHistNT) >> 6] = m;
            if (kr) s_q[w][qn + __popcll(m & lt)] = v[r];
            qn += __popcll(m);
        }
        __syncthreads();                            // the queue is written
        for (uint32_t j0 = 0; j0 < qn; j0 += kWave) {
            const uint32_t j = j0 + lane;
            const bool valid = j < qn;
            const K key = s_q[w][valid ? j : 0];
            count_digits(s_h[w], valid, ord(key), npass, dbits, dmask);
        }
        __syncthreads();                            // ... and read before it is reused
    }
    for (int i = threadIdx.x; i < npass * kBins; i += kHistNT) {
        const int p = i / kBins, d = i % kBins;
        uint32_t t = 0;
#pragma unroll
        for (int ww = 0; ww < NW; ww++) t += s_h[ww][p][d];
        if (t) atomicAdd(&ghist[p * kBins + d], t);
    }
    const uint64_t wk = wave_sum(uint64_t(kept));
    if (lane == 0 && wk) atomicAdd(reinterpret_cast<unsigned long long *>(d_kept), (unsigned long long)wk);
}

// The columns a pass moves with its keys: the payload columns, then the row
// ids when they are produced.  A null source is the item's position (the row
// ids of a first pass).
struct PassCols {
    const void *pin[kMaxPassCols];
    void *pout[kMaxPassCols];
    int32_t pdt[kMaxPassCols];
    int32_t ncols;
};

// Column p of the items at positions lidx[]: the aligned 8-byte words that
// hold them (word_of; from_word extracts the elements when they are staged,
// so nothing waits for these loads before then).  A null source (the items'
// positions, filled in at staging) reads the words of `alt` instead, so the
// same loads are issued on every path and the compiler's wait counts stay
// exact.
// The row-id column (ROWID) is int32 by construction and read with 4-byte
// loads.
template <bool ROWID>
__device__ __forceinline__ void load_col(const PassCols &c, int p, const void *alt,
                                         const uint32_t (&lidx)[kSortIPT], uint64_t (&out)[kSortIPT]) {
    const void *src = c.pin[p] ? c.pin[p] : alt;
    if constexpr (ROWID) {
#pragma unroll
        for (int k = 0; k < kSortIPT; k++) out[k] = static_cast<const uint32_t *>(src)[lidx[k]];
    } else {
        const int lg = c.pin[p] ? dtype_lg(c.pdt[p]) : 0;
#pragma unroll
        for (int k = 0; k < kSortIPT; k++) out[k] = word_of(src, lg, lidx[k]);
    }
}

// Writes one staged column of the tile (in digit order) to its runs: thread
// t writes tile positions t, t + kSortNT, ... to the global positions in
// pos[] (computed once per tile; -1 past the tile's end).  Row counts are
// below 2^30, so positions fit int32.
template <class T>
__device__ __forceinline__ void flush_stage(const uint64_t *s_stage, const int32_t (&pos)[kSortIPT],
                                            T *dst) {
    const T *st = reinterpret_cast<const T *>(s_stage);
#pragma unroll
    for (int k = 0; k < kSortIPT; k++)
        if (pos[k] >= 0) dst[pos[k]] = st[threadIdx.x + k * kSortNT];
}

// One LSD pass.  NPAY payload columns (a compile-time count; dtypes at run
// time) and, with ROWS, the int32 row ids after them move with the keys: the
// first column is read into registers together with the keys, so its latency
// overlaps the ranking and look-back, and each later one while its
// predecessor is written.
// At least 4 waves per SIMD (<= 128 VGPRs) so two workgroups share a CU.
// LB: the global start of each digit run comes from a decoupled look-back
// over earlier tiles (persistent workgroups, tiles by ticket); otherwise one
// workgroup per tile reads it from toff[digit * tstride + tile], the tile
// offsets k_radix_tilescan computed from every tile's digit counts.
// FILT (with LB only): items whose bit in keep_bits is clear (bit i % 64 of
// word i / 64, written by the filtered histogram) are dropped, as items past
// the end are, so the pass also compacts: its output holds the kept items,
// sorted by the digit, in their input order within a digit.
template <class K, int NPAY, class Ord, bool LB, bool ROWS, bool FILT>
__global__ __launch_bounds__(kSortNT, 4) void k_onesweep(
    const K *__restrict__ keys_in, K *__restrict__ keys_out, PassCols c, int64_t n,
    const int64_t *d_n, Ord ord, int shift, int dbits, const uint32_t *__restrict__ ghist,
    uint32_t *status, uint32_t *ticket, int64_t tstride, const uint64_t *__restrict__ keep_bits) {
    static_assert(LB || !FILT, "a filtered pass takes its offsets from the look-back");
    const uint32_t nbins = 1u << dbits;
    __shared__ uint32_t s_hist[kSortNW][kBins];
    __shared__ uint32_t s_local[kBins];      // tile-local start of each digit run
    __shared__ int64_t s_gbase[kBins];       // global start of the run minus its local start
    __shared__ uint64_t s_stage[kSortTile];  // one column of the tile, in digit order
    __shared__ uint64_t s_stage2[kSortTile]; // the next column (staging alternates)
    __shared__ uint8_t s_dig[kSortTile];     // digit of each sorted tile position
    __shared__ uint32_t s_scan[kSortNW];
    __shared__ uint32_t s_kept;
    __shared__ int64_t s_tile;

    const int64_t cnt = count_of(d_n, n);
    const int64_t ntiles = ceil_div(cnt, kSortTile);
    const int tid = threadIdx.x;
    const int w = wave_id();
    const int lane = lane_id();
    // LB: persistent workgroups, each taking its XCD's tiles in order until
    // none are left.  Otherwise: tile = blockIdx.x, once.
    const int xcd = int(blockIdx.x % kXcds);
    // LB: the global start of every digit (the same for all tiles)
    uint32_t gstart = 0;
    if constexpr (LB) {
        uint32_t gtot;
        gstart = block_excl_scan<kSortNT>(tid < kBins ? ghist[tid] : 0u, &gtot, s_scan);
    }
    for (int it = 0;; it++) {
    int64_t tile;
    if constexpr (LB) {
        const int64_t j = take_tile(ticket + xcd, &s_tile);
        tile = ((j / kTileGroup) * kXcds + xcd) * kTileGroup + j % kTileGroup;
    } else {
        if (it > 0) break;
        tile = blockIdx.x;
    }
    if (tile >= ntiles) break;
    const int64_t wbase = tile * kSortTile + int64_t(w) * (kWave * kSortIPT);

    // Issue the tile's loads before the first wait: keys and the first moved
    // column.  Positions past the end read the last item instead (a tile
    // exists only if cnt >= 1); those items are marked missing below.
    // Positions are below 2^30 (the callers' row limit), so 32 bits hold them.
    uint32_t lidx[kSortIPT];
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        const int64_t idx = wbase + k * kWave + lane;
        lidx[k] = uint32_t(idx < cnt ? idx : cnt - 1);
    }
    K key[kSortIPT];
    uint64_t cur[kSortIPT];       // the column being moved (column 0 first)
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) key[k] = keys_in[lidx[k]];
    uint32_t keep = 0xffffffffu;
    if constexpr (FILT) {
        // item k of every lane lies in one 64-item word (wbase is a multiple of 64)
        const int64_t last = (cnt - 1) >> 6;
        uint64_t kw[kSortIPT];
#pragma unroll
        for (int k = 0; k < kSortIPT; k++) {
            const int64_t wi = (wbase + k * kWave) >> 6;
            kw[k] = keep_bits[wi < last ? wi : last];
        }
        keep = 0;
#pragma unroll
        for (int k = 0; k < kSortIPT; k++) keep |= uint32_t((kw[k] >> lane) & 1) << k;
    }
    constexpr int NC = NPAY + (ROWS ? 1 : 0);   // moved columns, row ids last
    if (NC > 0) load_col<NPAY == 0>(c, 0, keys_in, lidx, cur);
    for (int i = tid; i < kSortNW * kBins; i += kSortNT) (&s_hist[0][0])[i] = 0;
    __syncthreads();
    // pd[k] = digit << 16 | position (digit kBins marks a missing item; a
    // position is below the tile size, 4096).
    uint32_t pd[kSortIPT];
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        const int64_t idx = wbase + k * kWave + lane;
        const bool in = idx < cnt && ((keep >> k) & 1);
        pd[k] = (in ? uint32_t(ord(key[k]) >> shift) & (nbins - 1) : kBins) << 16;
    }

    // Stable rank of each item among the items of this wave with its digit.
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        const uint32_t d = pd[k] >> 16;
        const bool valid = d < kBins;
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; b++) {
            if (b >= dbits) break;                   // higher digit bits are all zero
            const bool bit = (d >> b) & 1;
            const uint64_t bb = ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t old = 0;
        if (valid) old = s_hist[w][d];
        pd[k] |= old + __popcll(peers & lt);
        if (valid && (peers & lt) == 0) s_hist[w][d] = old + __popcll(peers);
    }
    __syncthreads();

    // Per digit (threads below kBins): offsets across waves and tile total.
    uint32_t tot = 0;
    if (tid < kBins) {
#pragma unroll
        for (int ww = 0; ww < kSortNW; ww++) {
            const uint32_t cw = s_hist[ww][tid];
            s_hist[ww][tid] = tot;
            tot += cw;
        }
    }
    uint32_t tile_total;
    const uint32_t local = block_excl_scan<kSortNT>(tot, &tile_total, s_scan);
    if (FILT && tid == 0) s_kept = tile_total;
    if (!LB) {
        if (tid < int(nbins)) {
            s_local[tid] = local;
            s_gbase[tid] = int64_t(status[int64_t(tid) * tstride + tile]) - int64_t(local);
        }
    } else if (tid < int(nbins)) {
        s_local[tid] = local;
        // Decoupled look-back for digit tid across earlier tiles.
        uint32_t *st = status + tile * kBins + tid;
        int64_t prefix = 0;
        if (tile == 0) {
            st_relaxed(st, kSFlagInc | tot);
        } else {
            st_relaxed(st, kSFlagAgg | tot);
            // Walk back kLookAhead tiles per memory round trip: the statuses
            // of the next kLookAhead predecessors are fetched together, then
            // consumed in order until an inclusive prefix is met.
            bool done = false;
            for (int64_t t = tile - 1; !done; t -= kLookAhead) {
                uint32_t sv[kLookAhead];
#pragma unroll
                for (int j = 0; j < kLookAhead; j++)
                    sv[j] = t - j >= 0 ? ld_relaxed(status + (t - j) * kBins + tid) : kSFlagInc;
#pragma unroll
                for (int j = 0; j < kLookAhead; j++) {
                    if (done) break;
                    while ((sv[j] >> 30) == 0) {
                        __builtin_amdgcn_s_sleep(1);
                        sv[j] = ld_relaxed(status + (t - j) * kBins + tid);
                    }
                    prefix += sv[j] & kSValMask;
                    if ((sv[j] >> 30) == 2) done = true;
                }
            }
            st_relaxed(st, kSFlagInc | uint32_t(prefix + tot));
        }
        s_gbase[tid] = int64_t(gstart) + prefix - int64_t(local);
    }
    __syncthreads();

    // Tile position of each item; stage the keys in digit order.
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        const uint32_t d = pd[k] >> 16;
        if (d < kBins) {
            const uint32_t p = (pd[k] & 0xffffu) + s_local[d] + s_hist[w][d];
            pd[k] = (d << 16) | p;
            reinterpret_cast<K *>(s_stage)[p] = key[k];
            s_dig[p] = uint8_t(d);
        }
    }
    __syncthreads();
    // the tile's items that are not missing (FILT: as counted by the scan,
    // kept in LDS rather than a register through the look-back)
    const int tile_cnt = FILT ? int(s_kept)
                              : int(cnt - tile * kSortTile < kSortTile ? cnt - tile * kSortTile : kSortTile);
    int32_t gpos[kSortIPT];
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        const int i = tid + k * kSortNT;
        gpos[k] = i < tile_cnt ? int32_t(s_gbase[s_dig[i]] + i) : -1;
    }
    flush_stage<K>(s_stage, gpos, keys_out);

    // Moved columns one after another: column p + 1 is loaded while column p
    // is staged and written, so at most two are held in registers.  Staging
    // alternates between two buffers, so one barrier per column suffices: the
    // barrier after staging column p also ends every thread's writes of
    // column p - 1, whose buffer column p + 1 then reuses.
#pragma unroll
    for (int p = 0; p < NC; p++) {
        uint64_t nxt[kSortIPT];
        if (p + 1 < NC) {               // both tests fold once the loop is unrolled
            if (p + 1 == NPAY) load_col<true>(c, p + 1, keys_in, lidx, nxt);
            else load_col<false>(c, p + 1, keys_in, lidx, nxt);
        }
        const int dt = c.pdt[p];
        {
            const void *src = c.pin[p];
            const int lg = dtype_lg(dt);
#pragma unroll
            for (int k = 0; k < kSortIPT; k++)
                cur[k] = !src ? uint64_t(lidx[k]) : p == NPAY ? cur[k] : from_word(cur[k], src, lg, lidx[k]);
        }
        uint64_t *buf = (p & 1) ? s_stage : s_stage2;
        if (dt == TQP_INT8) {
#pragma unroll
            for (int k = 0; k < kSortIPT; k++)
                if ((pd[k] >> 16) < kBins) reinterpret_cast<int8_t *>(buf)[pd[k] & 0xffffu] = int8_t(cur[k]);
            __syncthreads();
            flush_stage<int8_t>(buf, gpos, static_cast<int8_t *>(c.pout[p]));
        } else if (dt == TQP_INT32) {
#pragma unroll
            for (int k = 0; k < kSortIPT; k++)
                if ((pd[k] >> 16) < kBins) reinterpret_cast<int32_t *>(buf)[pd[k] & 0xffffu] = int32_t(cur[k]);
            __syncthreads();
            flush_stage<int32_t>(buf, gpos, static_cast<int32_t *>(c.pout[p]));
        } else {
#pragma unroll
            for (int k = 0; k < kSortIPT; k++)
                if ((pd[k] >> 16) < kBins) reinterpret_cast<uint64_t *>(buf)[pd[k] & 0xffffu] = cur[k];
            __syncthreads();
            flush_stage<int64_t>(buf, gpos, static_cast<int64_t *>(c.pout[p]));
        }
        if (p + 1 < NC) {
#pragma unroll
            for (int k = 0; k < kSortIPT; k++) cur[k] = nxt[k];
        }
    }
    __syncthreads();
    }
}

// Digit counts of every occupied tile for one pass (the tiles
// k_onesweep<..., false> will take): counts[digit * tstride + tile].  Lanes
// sharing the first valid lane's digit are counted with one ballot (skewed
// keys otherwise serialize on one LDS address).
template <class K, class Ord>
__global__ __launch_bounds__(kSortNT) void k_radix_tilecount(const K *__restrict__ keys, int64_t n,
                                                             const int64_t *d_n, Ord ord, int shift,
                                                             int dbits, uint32_t *counts,
                                                             int64_t tstride) {
    __shared__ uint32_t s_c[kSortNW][kBins];
    const uint32_t nbins = 1u << dbits;
    const int64_t cnt = count_of(d_n, n);
    const int64_t tile = blockIdx.x;
    if (tile * kSortTile >= cnt) return;
    const int tid = threadIdx.x, w = wave_id(), lane = lane_id();
    for (int i = tid; i < kSortNW * kBins; i += kSortNT) (&s_c[0][0])[i] = 0;
    const int64_t wbase = tile * kSortTile + int64_t(w) * (kWave * kSortIPT);
    K key[kSortIPT];
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        const int64_t idx = wbase + k * kWave + lane;
        key[k] = keys[idx < cnt ? idx : cnt - 1];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        const bool valid = wbase + k * kWave + lane < cnt;
        const uint64_t vm = ballot(valid);
        if (vm == 0) continue;
        const int first = __builtin_ctzll(vm);
        const uint32_t d = uint32_t(ord(key[k]) >> shift) & (nbins - 1);
        const uint32_t f = uint32_t(__builtin_amdgcn_readlane(int(d), first));
        const bool same = valid && d == f;
        const uint64_t sm = ballot(same);
        if (lane == first) atomicAdd(&s_c[w][f], uint32_t(__popcll(sm)));
        else if (valid && !same) atomicAdd(&s_c[w][d], 1u);
    }
    __syncthreads();
    for (int d = tid; d < int(nbins); d += kSortNT) {
        uint32_t t = 0;
#pragma unroll
        for (int ww = 0; ww < kSortNW; ww++) t += s_c[ww][d];
        counts[int64_t(d) * tstride + tile] = t;
    }
}

// One workgroup per digit: turns that digit's row of tile counts (occupied
// tiles only) into the global position of each tile's run, in place: the
// digit's start (counts of all smaller digits, from the pass histogram) plus
// the counts of the tiles before it.  Each thread scans kScanIPT consecutive
// tiles.
constexpr int kScanNT = 1024;
constexpr int kScanIPT = 8;
static __global__ __launch_bounds__(kScanNT) void k_radix_tilescan(uint32_t *counts, int64_t tstride,
                                                            const uint32_t *__restrict__ ghist,
                                                            int64_t n, const int64_t *d_n) {
    __shared__ uint32_t s_scan[kScanNT / kWave];
    __shared__ uint32_t s_base;
    const int d = blockIdx.x;
    const int64_t ntiles = ceil_div(count_of(d_n, n), kSortTile);
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (int e = 0; e < d; e++) b += ghist[e];
        s_base = b;
    }
    __syncthreads();
    uint32_t carry = s_base;
    uint32_t *row = counts + int64_t(d) * tstride;
    for (int64_t t0 = 0; t0 < ntiles; t0 += int64_t(kScanNT) * kScanIPT) {
        const int64_t tb = t0 + int64_t(threadIdx.x) * kScanIPT;
        uint32_t v[kScanIPT], sum = 0;
#pragma unroll
        for (int j = 0; j < kScanIPT; j++) {
            v[j] = tb + j < ntiles ? row[tb + j] : 0u;
            sum += v[j];
        }
        uint32_t total;
        uint32_t ex = carry + block_excl_scan<kScanNT>(sum, &total, s_scan);
#pragma unroll
        for (int j = 0; j < kScanIPT; j++) {
            if (tb + j < ntiles) row[tb + j] = ex;
            ex += v[j];
        }
        carry += total;
    }
}

template <class K>
__global__ __launch_bounds__(256) void k_copy_sorted(const K *__restrict__ keys_in, K *__restrict__ keys_out,
                                                     PassCols c, int64_t n, const int64_t *d_n) {
    const int64_t cnt = count_of(d_n, n);
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < cnt;
         i += int64_t(gridDim.x) * blockDim.x) {
        keys_out[i] = keys_in[i];
        for (int p = 0; p < c.ncols; p++)
            store_any(c.pout[p], c.pdt[p], i, c.pin[p] ? load_any(c.pin[p], c.pdt[p], i) : i);
    }
}


// Ordinal of a key for the plain sort: its offset from the smallest key.
template <class K> struct KeyOrd {
    K key_min;
    __device__ __forceinline__ uint64_t operator()(K k) const {
        using U = typename KeyTraits<K>::U;
        return uint64_t(U(U(k) - U(key_min)));
    }
};

struct SortCols {
    const int32_t *rows_in;
    int32_t *rows_out;
    const void *pin[kMaxSortPay];
    void *pout[kMaxSortPay];
    int32_t pdt[kMaxSortPay];
    int32_t npay;
};

inline int npass_for(int key_bits) { return (key_bits + kRadixBits - 1) / kRadixBits; }
// Equal digit widths: the fewest bits per digit that keep npass_for's count.
inline int digit_bits_for(int key_bits) {
    const int np = npass_for(key_bits);
    return np ? (key_bits + np - 1) / np : 0;
}

// Workspace of run_radix: ping-pong buffers (when more than one pass), the
// digit histograms, tickets and look-back statuses.
inline size_t radix_ws_bytes(int64_t n, int key_size, int npass, int pay_bytes) {
    const int64_t ntiles = n > 0 ? ceil_div(n, kSortTile) : 1;
    Carver c(nullptr);
    if (npass > 1) {
        c.take<char>(size_t(n) * key_size);
        c.take<int32_t>(size_t(n));
        for (int b = 0; b < pay_bytes; b++) c.take<char>(size_t(n));
    }
    c.take<uint32_t>(size_t(npass) * kBins + size_t(npass) * kXcds + size_t(npass) * ntiles * kBins);
    c.take<uint64_t>(size_t(ceil_div(n > 0 ? n : 1, 64)));     // keep bits of a filtered sort
    return c.bytes();
}

template <class K, int NPAY, class Ord, bool LB, bool ROWS, bool FILT>
static int launch_pass(unsigned grid, hipStream_t s, const K *src, K *dst, const PassCols &x,
                       int64_t n, const int64_t *d_n, Ord ord, int shift, int dbits,
                       const uint32_t *gh, uint32_t *st, uint32_t *ticket, int64_t tstride,
                       const uint64_t *keep_bits) {
    TQP_LAUNCH("onesweep", (k_onesweep<K, NPAY, Ord, LB, ROWS, FILT>), dim3(grid), dim3(kSortNT), 0, s,
               src, dst, x, n, d_n, ord, shift, dbits, gh, st, ticket, tstride, keep_bits);
    return TQP_OK;
}

// The instantiation for npay payload columns and (rows) row ids: row ids
// alone take the typed 4-byte path (ROWS); next to payload columns they are
// one more column of the generic path, which needs fewer registers there.
template <class K, class Ord, bool LB, bool FILT = false>
static int launch_cols(int npay, bool rows, unsigned grid, hipStream_t s, const K *src, K *dst,
                       const PassCols &x, int64_t n, const int64_t *d_n, Ord ord, int shift,
                       int dbits, const uint32_t *gh, uint32_t *st, uint32_t *ticket, int64_t tstride,
                       const uint64_t *keep_bits = nullptr) {
#define TQP_PASS(NP, R) launch_pass<K, NP, Ord, LB, R, FILT>(grid, s, src, dst, x, n, d_n, ord, shift, \
                                                             dbits, gh, st, ticket, tstride, keep_bits)
    if (rows && npay == 0) return TQP_PASS(0, true);
    switch (npay + (rows ? 1 : 0)) {
    case 0: return TQP_PASS(0, false);
    case 1: return TQP_PASS(1, false);
    case 2: return TQP_PASS(2, false);
    case 3: return TQP_PASS(3, false);
    case 4: return TQP_PASS(4, false);
    default: return TQP_PASS(5, false);
    }
#undef TQP_PASS
}

// Sorts by the low `bits` bits of the ordinal: npass_for(bits) stable passes
// over equal-width digits (least significant first) from key_in into key_out
// (they must not overlap), with the columns of sc moving along.  bits == 0
// copies.  With pred (then bits >= 1 and d_n null): only the items the
// predicates keep are sorted -- the histogram counts only them and writes
// their number to *d_kept, the first pass drops the others (always by
// look-back), and the later passes run over *d_kept items.
template <class K, class Ord>
int run_radix(const K *key_in, int64_t n, const int64_t *d_n, int bits, Ord ord, K *key_out,
              const SortCols &sc, void *ws, hipStream_t s, const PassPred *pred = nullptr,
              int64_t *d_kept = nullptr) {
    if (pred && (bits < 1 || d_n || !d_kept))
        return set_error(TQP_EINVAL, "radix: a filtered sort needs key bits and a kept counter");
    const int npass = npass_for(bits);
    const int dbits = digit_bits_for(bits);
    const unsigned grid_all = unsigned(ceil_div(n > 0 ? n : 1, kSortTile));
    const unsigned grid_pass = persistent_grid(grid_all, tune(kTuneSortPerCu));
    const int mode = tune(kTuneSortMode);
    // every tile group's counter needs a workgroup (true for these grids)
    const int64_t groups = ceil_div(int64_t(grid_all), int64_t(kTileGroup));
    if (int64_t(grid_pass) < (groups < kXcds ? groups : int64_t(kXcds)))
        return set_error(TQP_EINVAL, "radix: grid %u too small for its tile groups", grid_pass);
    PassCols pc = {};
    for (int p = 0; p < sc.npay; p++) {
        pc.pin[p] = sc.pin[p];
        pc.pout[p] = sc.pout[p];
        pc.pdt[p] = sc.pdt[p];
    }
    pc.ncols = sc.npay;
    if (sc.rows_out) {
        pc.pin[pc.ncols] = sc.rows_in;
        pc.pout[pc.ncols] = sc.rows_out;
        pc.pdt[pc.ncols] = TQP_INT32;
        pc.ncols++;
    }
    if (npass == 0) {
        unsigned g = grid_all > 4096 ? 4096 : grid_all;
        TQP_LAUNCH("copy_sorted", k_copy_sorted<K>, dim3(g), dim3(256), 0, s, key_in, key_out, pc, n, d_n);
        return check_launch("sort copy");
    }
    const int64_t ntiles = n > 0 ? ceil_div(n, kSortTile) : 1;
    Carver cv(ws);
    K *tmp_keys = nullptr;
    int32_t *tmp_rows = nullptr;
    void *tmp_col[kMaxPassCols] = {};
    if (npass > 1) {
        tmp_keys = reinterpret_cast<K *>(cv.take<char>(size_t(n) * sizeof(K)));
        tmp_rows = cv.take<int32_t>(size_t(n));
        for (int p = 0; p < sc.npay; p++) tmp_col[p] = cv.take<char>(size_t(n) * dtype_size(sc.pdt[p]));
        if (sc.rows_out) tmp_col[sc.npay] = tmp_rows;
    }
    const size_t nwords = size_t(npass) * kBins + size_t(npass) * kXcds + size_t(npass) * ntiles * kBins;
    uint32_t *words = cv.take<uint32_t>(nwords);
    uint32_t *ghist = words;
    uint32_t *tickets = words + npass * kBins;
    uint32_t *status = tickets + npass * kXcds;
    uint64_t *keep_bits = cv.take<uint64_t>(size_t(ceil_div(n > 0 ? n : 1, 64)));
    // histograms and tickets, then (contiguous with them) the per-pass tile
    // statuses over the tiles the actual count needs (a plan sized for a
    // large capacity does not pay for clearing all of it), in one launch
    const int64_t head = int64_t(npass) * (kBins + kXcds);
    int rc = (d_n && !pred)
                 ? clear_sections(status, head, npass, ntiles * kBins, d_n, n, kSortTile, kBins, s)
                 : fill_u32(words, 0, head + int64_t(npass) * ntiles * kBins, s);
    if (rc) return rc;
    if (pred && (rc = fill_u64(reinterpret_cast<uint64_t *>(d_kept), 0, 1, s))) return rc;
    {
        // a few workgroups per CU: each merges its counters into the device
        // histogram once, so fewer workgroups mean fewer device atomics
        int64_t g = ceil_div(n > 0 ? n : 1, int64_t(kHistNT) * kHistIPT);
        if (g > int64_t(kComputeUnits) * 4) g = int64_t(kComputeUnits) * 4;
        if (pred) {
            // as many workgroups as are resident at once: registers allow 5
            // per CU with 4-byte keys, LDS 3 with 8-byte keys (measured 5%
            // faster than 4 per CU on the star query's 60M rows)
            const int64_t per_cu = sizeof(K) == 4 ? 5 : 3;
            g = ceil_div(n > 0 ? n : 1, int64_t(kHistNT) * kHistFIPT);
            if (g > int64_t(kComputeUnits) * per_cu) g = int64_t(kComputeUnits) * per_cu;
            TQP_LAUNCH("radix_hist", (k_radix_hist_filt<K, Ord>), dim3(unsigned(g)), dim3(kHistNT), 0,
                       s, key_in, n, ord, npass, dbits, ghist, *pred, d_kept, keep_bits);
        } else {
            TQP_LAUNCH("radix_hist", (k_radix_hist<K, Ord>), dim3(unsigned(g)), dim3(kHistNT), 0, s,
                       key_in, n, d_n, ord, npass, dbits, ghist);
        }
        rc = check_launch("radix histogram");
        if (rc) return rc;
    }
    const K *src_k = key_in;
    PassCols cur = pc;
    const int64_t *pass_n = pred ? d_kept : d_n;   // item count of the passes after a filtered one
    for (int p = 0; p < npass; p++) {
        const bool to_out = ((npass - 1 - p) % 2) == 0;
        K *dk = to_out ? key_out : tmp_keys;
        PassCols x = cur;
        for (int q = 0; q < pc.ncols; q++) x.pout[q] = to_out ? pc.pout[q] : tmp_col[q];
        uint32_t *st = status + size_t(p) * ntiles * kBins;
        const int shift = p * dbits;
        const uint32_t *gh = ghist + p * kBins;
        if (pred && p == 0) {
            rc = launch_cols<K, Ord, true, true>(sc.npay, sc.rows_out != nullptr, grid_pass, s, src_k,
                                                 dk, x, n, nullptr, ord, shift, dbits, gh, st,
                                                 tickets, 0, keep_bits);
        } else if (mode == 0) {
            rc = launch_cols<K, Ord, true>(sc.npay, sc.rows_out != nullptr, grid_pass, s, src_k, dk, x, n,
                                           pass_n, ord, shift, dbits, gh, st, tickets + p * kXcds, 0);
        } else {
            // tile counts, their scan per digit, then one workgroup per tile
            uint32_t *tc = status;                    // ntiles * kBins words, reused per pass
            TQP_LAUNCH("radix_tilecount", (k_radix_tilecount<K, Ord>), dim3(grid_all), dim3(kSortNT), 0, s,
                       src_k, n, pass_n, ord, shift, dbits, tc, ntiles);
            if ((rc = check_launch("radix tile counts"))) return rc;
            TQP_LAUNCH("radix_tilescan", k_radix_tilescan, dim3(1u << dbits), dim3(kScanNT), 0, s, tc,
                       ntiles, gh, n, pass_n);
            if ((rc = check_launch("radix tile scan"))) return rc;
            rc = launch_cols<K, Ord, false>(sc.npay, sc.rows_out != nullptr, grid_all, s, src_k, dk, x, n,
                                            pass_n, ord, shift, dbits, gh, tc, nullptr, ntiles);
        }
        if (rc) return rc;
        rc = check_launch("radix pass");
        if (rc) return rc;
        src_k = dk;
        for (int q = 0; q < pc.ncols; q++) cur.pin[q] = x.pout[q];
    }
    return TQP_OK;
}

}  // namespace tqp
