// Sort-merge inner equi-join over two ascending key columns.
//
//  1. Run-length encode each sorted side: one single-pass compaction of the
//     run heads gives (unique key, run start) and the number of runs.
//  2. Match: for each left run, find the right run with the same key
//     (binary search over the right run keys); a matched key becomes one range
//     (key, lstart, lcnt, rstart, rcnt).  Two decoupled look-backs in the same
//     kernel give each range its slot and its first output pair (the running
//     sum of lcnt * rcnt), so the pair total is known on the device.
//     It also records, for every tile of output pairs, the range holding the
//     tile's first pair.
//  3. Expand: output pairs are split into equal tiles, whatever the key skew;
//     a tile stages the pair offsets of its (at most tile-size) ranges in LDS,
//     each pair finds its range there and takes (i, j) = row-major position
//     within the range, which is the canonical (key, i, j) order.
#include "tqp_internal.hpp"

namespace tqp {

constexpr int kJoinNT = 256;
constexpr int kJoinIPT = 16;
constexpr int kJoinTile = kJoinNT * kJoinIPT;
constexpr int kExpandPer = 8;
constexpr int kExpandTile = kJoinNT * kExpandPer;   // output pairs per expand tile
// Consecutive left runs per thread of the match: 4 when either side is
// below 2^25 rows (each lane's ranges 32 bytes apart, so a store covers few
// cache lines when most left runs match, as against a dimension), 16 when
// both sides are large (a quarter of the tiles, tickets and look-backs).  The
// tile count and the workspace are sized for the smaller tile.
constexpr int kMatchIPTSmall = 4;
constexpr int kMatchIPTLarge = 16;
constexpr int64_t kMatchLargeRows = int64_t(1) << 25;
constexpr int kMatchTile = kJoinNT * kMatchIPTSmall;
__host__ __device__ constexpr int match_ipt(int64_t nl) {
    return nl >= kMatchLargeRows ? kMatchIPTLarge : kMatchIPTSmall;
}
constexpr int kMatchWindow = 4096;      // right keys staged in LDS per match tile
constexpr int kRleNT = 1024;
constexpr int kRleTile = kRleNT * kJoinIPT;

template <class K>
__device__ __forceinline__ void load_keys16(const K *p, int64_t row0, int64_t cnt, K (&v)[16]) {
    if (row0 + 16 <= cnt) {
        if (sizeof(K) == 4) {
            const int4 *q = reinterpret_cast<const int4 *>(p + row0);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                int4 x = q[k];
                v[4 * k + 0] = K(x.x);
                v[4 * k + 1] = K(x.y);
                v[4 * k + 2] = K(x.z);
                v[4 * k + 3] = K(x.w);
            }
        } else {
            const longlong2 *q = reinterpret_cast<const longlong2 *>(p + row0);
#pragma unroll
            for (int k = 0; k < 8; k++) {
                longlong2 x = q[k];
                v[2 * k + 0] = K(x.x);
                v[2 * k + 1] = K(x.y);
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; r++) v[r] = row0 + r < cnt ? p[row0 + r] : K(0);
    }
}

// Run heads of a sorted column -> (unique key, run start), count in *d_nu.
// Tiles of 1024 threads x 16 keys: the keys are only 4-8 bytes each, so a
// large tile keeps the per-tile ticket and look-back cost small next to the
// tile's own traffic.  A wave takes 16 rows of 64 consecutive keys, one key
// per lane and row, and compacts each row's heads by ballot, so the heads of
// a row are written by consecutive lanes to consecutive places (per-thread
// runs of 16 keys made each store touch 64 cache lines).
template <class K>
__global__ __launch_bounds__(kRleNT) void k_rle(const K *__restrict__ keys, int64_t n,
                                                const int64_t *d_n, K *__restrict__ ukey,
                                                int32_t *__restrict__ ustart, int64_t *d_nu,
                                                uint32_t *ticket, uint64_t *status) {
    __shared__ int64_t s_tile, s_prefix;
    __shared__ int32_t s_wcnt[kRleNT / kWave];
    const int64_t cnt = count_of(d_n, n);
    const int64_t ntiles = ceil_div(cnt, kRleTile);
    const int w = wave_id(), lane = lane_id();
    const uint64_t lt = lanemask_lt();
    for (;;) {
    const int64_t tile = take_tile(ticket, &s_tile);
    if (tile >= ntiles) {
        if (tile == 0 && threadIdx.x == 0) *d_nu = 0;
        break;
    }
    const int64_t wbase = tile * kRleTile + int64_t(w) * (kWave * kJoinIPT);
    K v[kJoinIPT], pv[kJoinIPT];
#pragma unroll
    for (int r = 0; r < kJoinIPT; r++) {
        const int64_t i = wbase + r * kWave + lane;
        v[r] = i < cnt ? keys[i] : K(0);
        pv[r] = i > 0 && i - 1 < cnt ? keys[i - 1] : K(0);
    }
    uint64_t hm[kJoinIPT];
    int32_t wc = 0;
#pragma unroll
    for (int r = 0; r < kJoinIPT; r++) {
        const int64_t i = wbase + r * kWave + lane;
        hm[r] = ballot(i < cnt && (i == 0 || v[r] != pv[r]));
        wc += __popcll(hm[r]);
    }
    if (lane == 0) s_wcnt[w] = wc;
    __syncthreads();
    int32_t wex = 0, total = 0;
#pragma unroll
    for (int ww = 0; ww < kRleNT / kWave; ww++) {
        const int32_t c = s_wcnt[ww];
        wex += ww < w ? c : 0;
        total += c;
    }
    if (w == 0) {
        int64_t pre = lookback_count(status, tile, total);
        if (lane == 0) s_prefix = pre;
    }
    __syncthreads();
    if (tile == ntiles - 1 && threadIdx.x == 0) *d_nu = s_prefix + total;
    int64_t q = s_prefix + wex;
#pragma unroll
    for (int r = 0; r < kJoinIPT; r++) {
        if ((hm[r] >> lane) & 1) {
            const int64_t pos = q + __popcll(hm[r] & lt);
            ukey[pos] = v[r];
            ustart[pos] = int32_t(wbase + r * kWave + lane);
        }
        q += __popcll(hm[r]);
    }
    __syncthreads();
    }
}

// Run heads of a sorted int32 column for other operators (the partition
// sort): ukey / ustart receive each run's value and first position, *d_nu
// the run count.  words: rle_words(n) zeroed-here uint64 words (ticket and
// look-back statuses).
size_t rle_words(int64_t n) { return size_t(1 + ceil_div(n > 0 ? n : 1, kRleTile)); }

int rle_i32(const int32_t *keys, int64_t n, int32_t *ukey, int32_t *ustart, int64_t *d_nu,
            uint64_t *words, hipStream_t s) {
    int rc = fill_u64(words, 0, int64_t(rle_words(n)), s);
    if (rc) return rc;
    const unsigned g = persistent_grid(ceil_div(n > 0 ? n : 1, kRleTile), tune(kTuneRlePerCu));
    TQP_LAUNCH("rle", k_rle<int32_t>, dim3(g), dim3(kRleNT), 0, s, keys, n, nullptr, ukey, ustart,
               d_nu, reinterpret_cast<uint32_t *>(words), words + 1);
    return check_launch("run-length encoding");
}

struct MatchArgs {
    const void *uL;
    const int32_t *sL;
    const int64_t *d_nuL;
    const int64_t *d_nl;     // left row count (device), or null => nl
    int64_t nl;
    const void *uR;
    const int32_t *sR;
    const int64_t *d_nuR;
    const int64_t *d_nr;
    int64_t nr;
    int64_t *rkey, *rls, *rlc, *rrs, *rrc;   // ranges (workspace), capacity min(nl, nr)
    int64_t *off;                            // first pair of each range
    int64_t *ukey, *uls, *ulc, *urs, *urc;   // optional user copies
    int64_t ucap;
    int64_t *d_nranges_ws;
    int64_t *d_nranges_user;
    int64_t *d_count;
    int64_t *tile_first;     // optional: range holding the first pair of each output tile
    int64_t ntiles_out;
    const int64_t *bounds;   // per match tile: its window [bounds[2t], bounds[2t + 1]) of right runs
    uint32_t *ticket;
    uint64_t *status_m;
    uint64_t *status_p;
};

// The right runs a match tile can meet lie in [lower_bound of its first left
// key, upper_bound of its last): one thread per tile, all tiles at once, so no
// tile waits on a search over the whole right side.
template <class K>
__global__ __launch_bounds__(256) void k_match_bounds(const K *__restrict__ uL,
                                                      const int64_t *d_nuL, const K *__restrict__ uR,
                                                      const int64_t *d_nuR, int64_t tile_runs,
                                                      int64_t cap_tiles, int64_t *bounds) {
    const int64_t nuL = *d_nuL, nuR = *d_nuR;
    const int64_t ntiles = ceil_div(nuL, tile_runs);
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < ntiles && t < cap_tiles;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t u0 = t * tile_runs;
        const int64_t u1 = (u0 + tile_runs < nuL ? u0 + tile_runs : nuL) - 1;
        const K k0 = uL[u0], k1 = uL[u1];
        int64_t lo = 0, hi = nuR;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (uR[mid] < k0) lo = mid + 1;
            else hi = mid;
        }
        const int64_t wl = lo;
        hi = nuR;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (!(k1 < uR[mid])) lo = mid + 1;
            else hi = mid;
        }
        bounds[2 * t] = wl;
        bounds[2 * t + 1] = lo;
    }
}

// Lower bound of k among wkeys[pos, wn), keys at or after pos: a gallop from
// pos, then a binary search inside the last step (a few reads when the two
// sides' keys interleave evenly).
template <class K, class P>
__device__ __forceinline__ int64_t gallop_lower(P wkeys, int64_t pos, int64_t wn, K k) {
    int64_t lo = pos, hi = pos, step = 1;
    while (hi < wn && wkeys[hi] < k) {
        lo = hi + 1;
        hi = lo + step;
        step <<= 1;
    }
    if (hi > wn) hi = wn;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (wkeys[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Each thread takes IPT consecutive left runs and finds each one's key
// among the tile's right window (staged in LDS when it fits) by galloping
// from the previous key's position.  A first sweep counts the matched runs
// and their pairs; after the two look-backs, a second sweep writes the
// ranges of the matched runs from the window positions kept in registers.
template <class K, int IPT>
__global__ __launch_bounds__(kJoinNT) void k_join_match(MatchArgs a) {
    constexpr int kTileRuns = kJoinNT * IPT;
    __shared__ int64_t s_tile, s_pm, s_pp;
    __shared__ int64_t s_win[2];
    __shared__ K s_rkeys[kMatchWindow];
    __shared__ int32_t s_scan32[kJoinNT / kWave];
    __shared__ int64_t s_scan64[kJoinNT / kWave];
    const int64_t nuL = count_of(a.d_nuL, a.nl);
    const int64_t nuR = count_of(a.d_nuR, a.nr);
    const int64_t nl = count_of(a.d_nl, a.nl);
    const int64_t nr = count_of(a.d_nr, a.nr);
    const int64_t ntiles = ceil_div(nuL, kTileRuns);
    const K *uL = static_cast<const K *>(a.uL);
    const K *uR = static_cast<const K *>(a.uR);
    for (;;) {
    const int64_t tile = take_tile(a.ticket, &s_tile);
    if (tile >= ntiles) {
        if (tile == 0 && threadIdx.x == 0) {
            *a.d_nranges_ws = 0;
            if (a.d_nranges_user) *a.d_nranges_user = 0;
            *a.d_count = 0;
        }
        break;
    }
    if (threadIdx.x < 2) s_win[threadIdx.x] = a.bounds[2 * tile + threadIdx.x];
    __syncthreads();
    const int64_t w_lo = s_win[0], w_hi = s_win[1];
    const int64_t wn = w_hi - w_lo;
    const bool in_lds = wn <= kMatchWindow;
    if (in_lds)
        for (int64_t i = threadIdx.x; i < wn; i += kJoinNT) s_rkeys[i] = uR[w_lo + i];
    // this thread's left runs: keys and starts (one more start for the counts)
    const int64_t u0 = tile * kTileRuns + int64_t(threadIdx.x) * IPT;
    K key[IPT];
    if (u0 + IPT <= nuL && reinterpret_cast<uintptr_t>(uL) % 16 == 0) {
        // u0 is a multiple of IPT, so whole 16-byte groups
        constexpr int kPer = 16 / sizeof(K);
        const int4 *q = reinterpret_cast<const int4 *>(uL + u0);
#pragma unroll
        for (int j = 0; j < IPT / kPer; j++) {
            const int4 x = q[j];
            const K *e = reinterpret_cast<const K *>(&x);
#pragma unroll
            for (int t = 0; t < kPer; t++) key[j * kPer + t] = e[t];
        }
    } else {
#pragma unroll
        for (int r = 0; r < IPT; r++) key[r] = u0 + r < nuL ? uL[u0 + r] : K(0);
    }
    int32_t st[IPT + 1];
#pragma unroll
    for (int r = 0; r <= IPT; r++) st[r] = u0 + r < nuL ? a.sL[u0 + r] : int32_t(nl);
    __syncthreads();
    uint32_t hit = 0;
    int32_t widx[IPT];
    int64_t pairs = 0;
    int64_t from = 0;
#pragma unroll
    for (int r = 0; r < IPT; r++) {
        widx[r] = 0;
        if (u0 + r < nuL) {
            const K k = key[r];
            const int64_t lo = in_lds ? gallop_lower(static_cast<const K *>(s_rkeys), from, wn, k)
                                      : gallop_lower(uR + w_lo, from, wn, k);
            from = lo;
            const K rk = lo < wn ? (in_lds ? s_rkeys[lo] : uR[w_lo + lo]) : k;
            if (lo < wn && rk == k) {
                hit |= 1u << r;
                widx[r] = int32_t(lo);
                const int64_t g = w_lo + lo;
                const int64_t rs = a.sR[g];
                const int64_t rc = (g + 1 < nuR ? int64_t(a.sR[g + 1]) : nr) - rs;
                pairs += int64_t(st[r + 1] - st[r]) * rc;
            }
        }
    }
    int32_t tot_m;
    int64_t tot_p;
    const int32_t ex_m = block_excl_scan<kJoinNT>(int32_t(__popc(hit)), &tot_m, s_scan32);
    const int64_t ex_p = block_excl_scan<kJoinNT>(pairs, &tot_p, s_scan64);
    if (wave_id() == 0) {
        int64_t pm = lookback_count(a.status_m, tile, tot_m);
        int64_t pp = lookback_count(a.status_p, tile, tot_p);
        if (lane_id() == 0) { s_pm = pm; s_pp = pp; }
    }
    __syncthreads();
    if (tile == ntiles - 1 && threadIdx.x == 0) {
        *a.d_nranges_ws = s_pm + tot_m;
        if (a.d_nranges_user) *a.d_nranges_user = s_pm + tot_m;
        *a.d_count = s_pp + tot_p;
    }
    int64_t q = s_pm + ex_m;
    int64_t o = s_pp + ex_p;
#pragma unroll
    for (int r = 0; r < IPT; r++) {
        if (!(hit & (1u << r))) continue;
        const int64_t g = w_lo + widx[r];
        const int64_t rs = a.sR[g];
        const int64_t rc = (g + 1 < nuR ? int64_t(a.sR[g + 1]) : nr) - rs;
        const int64_t ls = st[r], lc = int64_t(st[r + 1]) - ls;
        if (a.rkey) {
            a.rkey[q] = int64_t(key[r]);
            a.rls[q] = ls;
            a.rlc[q] = lc;
            a.rrs[q] = rs;
            a.rrc[q] = rc;
            a.off[q] = o;
        }
        if (a.ukey && q < a.ucap) {
            a.ukey[q] = int64_t(key[r]);
            a.uls[q] = ls;
            a.ulc[q] = lc;
            a.urs[q] = rs;
            a.urc[q] = rc;
        }
        const int64_t p = lc * rc;
        if (a.tile_first) {
            // this range holds the first pair of every output tile starting in it
            for (int64_t t = ceil_div(o, kExpandTile); t * kExpandTile < o + p && t < a.ntiles_out; t++)
                a.tile_first[t] = q;
        }
        o += p;
        q++;
    }
    __syncthreads();
    }
}

// Output tile t (kExpandTile pairs) starts in range tile_first[t] and ends at
// most kExpandTile ranges later; those ranges' first-pair offsets are staged in
// LDS, and each output finds its range there by binary search.  Consecutive
// threads write consecutive pairs.
template <class K>
__global__ __launch_bounds__(kJoinNT) void k_join_expand(
    const int64_t *__restrict__ rkey, const int64_t *__restrict__ rls,
    const int64_t *__restrict__ rlc, const int64_t *__restrict__ rrs,
    const int64_t *__restrict__ rrc, const int64_t *__restrict__ off,
    const int64_t *__restrict__ tile_first, const int64_t *d_nranges, const int64_t *d_count,
    int64_t cap, const int32_t *__restrict__ lrows, const int32_t *__restrict__ rrows,
    int32_t *__restrict__ out_l, int32_t *__restrict__ out_r, K *__restrict__ out_key) {
    __shared__ int64_t s_off[kExpandTile + 1];
    const int64_t nranges = *d_nranges;
    const int64_t total = *d_count;
    const int64_t limit = total < cap ? total : cap;
    const int64_t ntiles = ceil_div(limit, kExpandTile);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t o_begin = t * kExpandTile;
        const int64_t o_end = o_begin + kExpandTile < limit ? o_begin + kExpandTile : limit;
        const int64_t m0 = tile_first[t];
        int64_t m1 = t + 1 < ntiles ? tile_first[t + 1] : nranges - 1;
        if (m1 > m0 + kExpandTile) m1 = m0 + kExpandTile;
        const int nm = int(m1 - m0 + 1);
        for (int i = threadIdx.x; i < nm; i += kJoinNT) s_off[i] = off[m0 + i];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kExpandPer; k++) {
            const int64_t o = o_begin + k * kJoinNT + threadIdx.x;
            if (o < o_end) {
                int lo = 0, hi = nm;               // last local range with offset <= o
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_off[mid] <= o) lo = mid;
                    else hi = mid;
                }
                const int64_t m = m0 + lo;
                const uint64_t tt = uint64_t(o - s_off[lo]);
                const uint64_t rc = uint64_t(rrc[m]);
                uint64_t i, j;
                if (rc == 1) {
                    i = tt;
                    j = 0;
                } else if ((tt >> 32) == 0 && (rc >> 32) == 0) {
                    i = uint32_t(tt) / uint32_t(rc);
                    j = tt - i * rc;
                } else {
                    i = tt / rc;
                    j = tt - i * rc;
                }
                const int64_t li = rls[m] + int64_t(i), rj = rrs[m] + int64_t(j);
                if (out_l) out_l[o] = lrows ? lrows[li] : int32_t(li);
                if (out_r) out_r[o] = rrows ? rrows[rj] : int32_t(rj);
                if (out_key) out_key[o] = K(rkey[m]);
            }
        }
        __syncthreads();
    }
}

struct JoinLayout {
    void *sl_key, *sr_key;
    int32_t *sl_rows, *sr_rows;
    void *sort_ws;
    size_t sort_ws_bytes;
    void *uL, *uR;
    int32_t *sL, *sR;
    int64_t *rng[5];
    int64_t *off;
    int64_t *tile_first;     // per output tile of the expand: its first range
    int64_t ntiles_out;
    int64_t *bounds;         // per match tile: its window of right runs
    int64_t ntiles_match;
    int64_t *counters;       // nuL, nuR, nranges
    uint64_t *words;         // tickets + statuses
    int64_t nwords;
    uint64_t *stL, *stR, *stM, *stP;
    size_t bytes;
};

static JoinLayout join_layout(void *ws, int64_t nl, int64_t nr, int dtype, uint32_t flags,
                              int64_t cap) {
    JoinLayout L = {};
    Carver c(ws);
    const int ks = dtype_size(dtype);
    if (!(flags & TQP_JOIN_SORTED)) {
        L.sl_key = c.take<char>(size_t(nl) * ks);
        L.sl_rows = c.take<int32_t>(size_t(nl));
        L.sr_key = c.take<char>(size_t(nr) * ks);
        L.sr_rows = c.take<int32_t>(size_t(nr));
        const int64_t nmax = nl > nr ? nl : nr;
        L.sort_ws_bytes = sort_ws_bytes(nmax, dtype, ks * 8);
        L.sort_ws = c.take<char>(L.sort_ws_bytes);
    }
    L.uL = c.take<char>(size_t(nl > 0 ? nl : 1) * ks);
    L.sL = c.take<int32_t>(size_t(nl > 0 ? nl : 1));
    L.uR = c.take<char>(size_t(nr > 0 ? nr : 1) * ks);
    L.sR = c.take<int32_t>(size_t(nr > 0 ? nr : 1));
    const int64_t nm = (nl < nr ? nl : nr) > 0 ? (nl < nr ? nl : nr) : 1;
    for (int k = 0; k < 5; k++) L.rng[k] = c.take<int64_t>(size_t(nm));
    L.off = c.take<int64_t>(size_t(nm));
    L.ntiles_out = ceil_div(cap > 0 ? cap : 1, kExpandTile);
    L.tile_first = c.take<int64_t>(size_t(L.ntiles_out));
    L.ntiles_match = ceil_div(nl > 0 ? nl : 1, kMatchTile);
    L.bounds = c.take<int64_t>(size_t(2 * L.ntiles_match));
    L.counters = c.take<int64_t>(4);
    const int64_t tl = ceil_div(nl > 0 ? nl : 1, kRleTile);
    const int64_t tr = ceil_div(nr > 0 ? nr : 1, kRleTile);
    const int64_t tm = ceil_div(nl > 0 ? nl : 1, kMatchTile);
    L.nwords = 4 + tl + tr + 2 * tm;
    L.words = c.take<uint64_t>(size_t(L.nwords));
    if (L.words) {
        L.stL = L.words + 4;
        L.stR = L.stL + tl;
        L.stM = L.stR + tr;
        L.stP = L.stM + tm;
    }
    L.bytes = c.bytes();
    return L;
}

template <class K>
static int join_typed(const tqp_col *lkey, const int32_t *lrows, const int64_t *d_nl,
                      const tqp_col *rkey, const int32_t *rrows, const int64_t *d_nr,
                      uint32_t flags, int32_t *out_l, int32_t *out_r, void *out_pair_key,
                      int64_t cap, int64_t *d_count, const tqp_ranges *ranges, int64_t range_cap,
                      int64_t *d_nranges, void *ws, hipStream_t s) {
    const int64_t nl = lkey->len, nr = rkey->len;
    const bool want_pairs = (out_l || out_r || out_pair_key) && cap > 0;
    JoinLayout L = join_layout(ws, nl, nr, lkey->dtype, flags, want_pairs ? cap : 0);
    const K *lk = static_cast<const K *>(lkey->data);
    const K *rk = static_cast<const K *>(rkey->data);
    int rc;
    if (!(flags & TQP_JOIN_SORTED)) {
        int64_t kmin;
        int kbits;
        rc = derive_key_range(lk, lkey->dtype, nl, d_nl, L.sort_ws, s, &kmin, &kbits);
        if (rc) return rc;
        rc = sort_impl(lk, lkey->dtype, lrows, nl, d_nl, kbits, kmin, L.sl_key, L.sl_rows,
                       L.sort_ws, L.sort_ws_bytes, s);
        if (rc) return rc;
        rc = derive_key_range(rk, rkey->dtype, nr, d_nr, L.sort_ws, s, &kmin, &kbits);
        if (rc) return rc;
        rc = sort_impl(rk, rkey->dtype, rrows, nr, d_nr, kbits, kmin, L.sr_key, L.sr_rows,
                       L.sort_ws, L.sort_ws_bytes, s);
        if (rc) return rc;
        lk = static_cast<const K *>(L.sl_key);
        rk = static_cast<const K *>(L.sr_key);
        lrows = L.sl_rows;
        rrows = L.sr_rows;
    }
    rc = fill_u64(L.words, 0, L.nwords, s);
    if (rc) return rc;
    uint32_t *tickets = reinterpret_cast<uint32_t *>(L.words);
    const unsigned gl = persistent_grid(ceil_div(nl > 0 ? nl : 1, kRleTile), tune(kTuneRlePerCu));
    const unsigned gr = persistent_grid(ceil_div(nr > 0 ? nr : 1, kRleTile), tune(kTuneRlePerCu));
    TQP_LAUNCH("rle", k_rle<K>, dim3(gl), dim3(kRleNT), 0, s, lk, nl, d_nl,
                       static_cast<K *>(L.uL), L.sL, &L.counters[0], tickets + 0, L.stL);
    if ((rc = check_launch("join rle left"))) return rc;
    TQP_LAUNCH("rle", k_rle<K>, dim3(gr), dim3(kRleNT), 0, s, rk, nr, d_nr,
                       static_cast<K *>(L.uR), L.sR, &L.counters[1], tickets + 2, L.stR);
    if ((rc = check_launch("join rle right"))) return rc;
    MatchArgs a = {};
    a.uL = L.uL;
    a.sL = L.sL;
    a.d_nuL = &L.counters[0];
    a.d_nl = d_nl;
    a.nl = nl;
    a.uR = L.uR;
    a.sR = L.sR;
    a.d_nuR = &L.counters[1];
    a.d_nr = d_nr;
    a.nr = nr;
    a.rkey = L.rng[0];
    a.rls = L.rng[1];
    a.rlc = L.rng[2];
    a.rrs = L.rng[3];
    a.rrc = L.rng[4];
    a.off = L.off;
    if (flags & TQP_JOIN_RANGES) {
        a.ukey = ranges->key;
        a.uls = ranges->lstart;
        a.ulc = ranges->lcnt;
        a.urs = ranges->rstart;
        a.urc = ranges->rcnt;
        a.ucap = range_cap;
        a.d_nranges_user = d_nranges;
    }
    a.d_nranges_ws = &L.counters[2];
    a.d_count = d_count;
    if (want_pairs) {
        a.tile_first = L.tile_first;
        a.ntiles_out = L.ntiles_out;
    }
    if (!want_pairs) a.rkey = nullptr;      // only the expand reads the workspace copy
    a.ticket = tickets + 4;
    a.status_m = L.stM;
    a.status_p = L.stP;
    a.bounds = L.bounds;
    {
        int64_t g = ceil_div(L.ntiles_match, 256);
        if (g > 1024) g = 1024;
        TQP_LAUNCH("match_bounds", k_match_bounds<K>, dim3(unsigned(g)), dim3(256), 0, s,
                   static_cast<const K *>(L.uL), &L.counters[0], static_cast<const K *>(L.uR),
                   &L.counters[1], int64_t(kJoinNT) * match_ipt(nl < nr ? nl : nr), L.ntiles_match,
                   L.bounds);
        if ((rc = check_launch("join match bounds"))) return rc;
    }
    const int ipt = match_ipt(nl < nr ? nl : nr);
    const unsigned gm = persistent_grid(ceil_div(nl > 0 ? nl : 1, int64_t(kJoinNT) * ipt),
                                        tune(kTuneMatchPerCu));
    if (ipt == kMatchIPTLarge)
        TQP_LAUNCH("join_match", (k_join_match<K, kMatchIPTLarge>), dim3(gm), dim3(kJoinNT), 0, s, a);
    else
        TQP_LAUNCH("join_match", (k_join_match<K, kMatchIPTSmall>), dim3(gm), dim3(kJoinNT), 0, s, a);
    if ((rc = check_launch("join match"))) return rc;
    if (want_pairs) {
        int64_t g = L.ntiles_out;
        if (g > 16384) g = 16384;
        TQP_LAUNCH("join_expand", k_join_expand<K>, dim3(unsigned(g)), dim3(kJoinNT), 0, s,
                   L.rng[0], L.rng[1], L.rng[2], L.rng[3], L.rng[4], L.off, L.tile_first,
                   &L.counters[2], d_count, cap, lrows, rrows, out_l, out_r,
                   static_cast<K *>(out_pair_key));
        if ((rc = check_launch("join expand"))) return rc;
    }
    return TQP_OK;
}

}  // namespace tqp

using namespace tqp;

TQP_API size_t tqp_join_workspace_bytes(int64_t nl, int64_t nr, int dtype, uint32_t flags,
                                        int64_t cap) {
    if (nl < 0 || nr < 0 || cap < 0 || (dtype != TQP_INT32 && dtype != TQP_INT64)) return 0;
    return join_layout(nullptr, nl, nr, dtype, flags, cap).bytes;
}

TQP_API int tqp_join(const tqp_col *lkey, const int32_t *lrows, const int64_t *d_nl,
                     const tqp_col *rkey, const int32_t *rrows, const int64_t *d_nr,
                     uint32_t flags, int32_t *out_l, int32_t *out_r, void *out_pair_key,
                     int64_t cap, int64_t *d_count, const tqp_ranges *ranges, int64_t range_cap,
                     int64_t *d_nranges, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!lkey || !rkey || !d_count) return set_error(TQP_EINVAL, "tqp_join: null argument");
    if (lkey->dtype != rkey->dtype || (lkey->dtype != TQP_INT32 && lkey->dtype != TQP_INT64))
        return set_error(TQP_EINVAL, "tqp_join: keys must share dtype int32 or int64");
    if (flags & ~(TQP_JOIN_SORTED | TQP_JOIN_RANGES))
        return set_error(TQP_EINVAL, "tqp_join: unknown flag bits");
    const int64_t nl = lkey->len, nr = rkey->len;
    if (nl < 0 || nr < 0 || nl > (int64_t(1) << 30) - 1 || nr > (int64_t(1) << 30) - 1)
        return set_error(TQP_EINVAL, "tqp_join: sides must hold [0, 2^30 - 1] rows");
    if ((nl > 0 && !lkey->data) || (nr > 0 && !rkey->data))
        return set_error(TQP_EINVAL, "tqp_join: null key data");
    if (cap < 0) return set_error(TQP_EINVAL, "tqp_join: negative cap");
    if ((flags & TQP_JOIN_RANGES) &&
        (!ranges || !d_nranges || range_cap < 0 ||
         (range_cap > 0 && (!ranges->key || !ranges->lstart || !ranges->lcnt || !ranges->rstart ||
                            !ranges->rcnt))))
        return set_error(TQP_EINVAL, "tqp_join: ranges mode needs five arrays and d_nranges");
    const bool want_pairs = (out_l || out_r || out_pair_key) && cap > 0;
    const size_t need = tqp_join_workspace_bytes(nl, nr, lkey->dtype, flags, want_pairs ? cap : 0);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "tqp_join: workspace needs %zu bytes", need);
    hipStream_t s = as_stream(stream);
    if (lkey->dtype == TQP_INT32)
        return join_typed<int32_t>(lkey, lrows, d_nl, rkey, rrows, d_nr, flags, out_l, out_r,
                                   out_pair_key, cap, d_count, ranges, range_cap, d_nranges, ws, s);
    return join_typed<int64_t>(lkey, lrows, d_nl, rkey, rrows, d_nr, flags, out_l, out_r,
                               out_pair_key, cap, d_count, ranges, range_cap, d_nranges, ws, s);
}
