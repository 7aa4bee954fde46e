// Stable LSD radix sort of signed int32 / int64 keys carrying int32 row ids.
//
// Keys are ranked on u = key - key_min (unsigned), which orders signed keys
// correctly and drops the bits that never vary.  One sweep builds the 256-bin
// histograms of every 8-bit digit at once; each digit then takes one pass:
//   * a workgroup takes a 4096-key tile (dynamic tile id),
//   * ranks its keys stably: each wave walks its items in input order, finds
//     the lanes holding the same digit with eight ballots, and bumps a per-wave
//     LDS counter once per distinct digit,
//   * publishes its 256 digit counts and looks back over earlier tiles (one
//     thread per digit) for the global start of each digit run,
//   * stages the tile in LDS in digit order and writes each digit run out
//     with consecutive threads on consecutive addresses.
#include "tqp_internal.hpp"

namespace tqp {

constexpr int kSortNT = 256;
constexpr int kSortIPT = 16;
constexpr int kSortTile = kSortNT * kSortIPT;
constexpr int kRadixBits = 8;
constexpr int kBins = 1 << kRadixBits;
constexpr int kSortNW = kSortNT / kWave;
constexpr uint32_t kSFlagAgg = 1u << 30;
constexpr uint32_t kSFlagInc = 2u << 30;
constexpr uint32_t kSValMask = (1u << 30) - 1;

template <class K>
__global__ __launch_bounds__(kSortNT) void k_radix_hist(const K *__restrict__ keys, int64_t n,
                                                        const int64_t *d_n, K key_min, int npass,
                                                        uint32_t *__restrict__ ghist) {
    using U = typename KeyTraits<K>::U;
    constexpr int kMaxPass = KeyTraits<K>::kBits / kRadixBits;
    __shared__ uint32_t s_h[kSortNW][kMaxPass][kBins];
    for (int i = threadIdx.x; i < kSortNW * kMaxPass * kBins; i += kSortNT)
        (&s_h[0][0][0])[i] = 0;
    __syncthreads();
    const int64_t cnt = count_of(d_n, n);
    const int w = wave_id();
    const int64_t stride = int64_t(gridDim.x) * kSortNT;
    for (int64_t i = blockIdx.x * int64_t(kSortNT) + threadIdx.x; i < cnt; i += stride) {
        const U u = U(keys[i]) - U(key_min);
        for (int p = 0; p < npass; p++)
            atomicAdd(&s_h[w][p][(u >> (p * kRadixBits)) & (kBins - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < npass * kBins; i += kSortNT) {
        const int p = i / kBins, d = i % kBins;
        uint32_t t = 0;
#pragma unroll
        for (int ww = 0; ww < kSortNW; ww++) t += s_h[ww][p][d];
        if (t) atomicAdd(&ghist[p * kBins + d], t);
    }
}

template <class K>
__global__ __launch_bounds__(kSortNT) void k_onesweep(
    const K *__restrict__ keys_in, const int32_t *__restrict__ rows_in, K *__restrict__ keys_out,
    int32_t *__restrict__ rows_out, int64_t n, const int64_t *d_n, K key_min, int shift,
    const uint32_t *__restrict__ ghist, uint32_t *status, uint32_t *ticket) {
    using U = typename KeyTraits<K>::U;
    __shared__ uint32_t s_hist[kSortNW][kBins];
    __shared__ uint32_t s_local[kBins];      // tile-local start of each digit run
    __shared__ int64_t s_gbase[kBins];       // global start of each digit run of this tile
    __shared__ K s_keys[kSortTile];
    __shared__ int32_t s_rows[kSortTile];
    __shared__ uint32_t s_scan[kSortNW];
    __shared__ int64_t s_tile;

    const int64_t cnt = count_of(d_n, n);
    const int64_t ntiles = ceil_div(cnt, kSortTile);
    const int64_t tile = take_tile(ticket, &s_tile);
    if (tile >= ntiles) return;

    const int d0 = threadIdx.x;               // the digit this thread stands for
    for (int ww = 0; ww < kSortNW; ww++) s_hist[ww][d0] = 0;
    // global exclusive start of digit d0 over the whole input
    uint32_t gtot;
    const uint32_t gstart = block_excl_scan<kSortNT>(ghist[d0], &gtot, s_scan);

    const int w = wave_id();
    const int lane = lane_id();
    const int64_t wbase = tile * kSortTile + int64_t(w) * (kWave * kSortIPT);
    K key[kSortIPT];
    int32_t row[kSortIPT];
    uint32_t dig[kSortIPT];
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        const int64_t idx = wbase + k * kWave + lane;
        const bool valid = idx < cnt;
        key[k] = valid ? keys_in[idx] : K(0);
        row[k] = valid ? (rows_in ? rows_in[idx] : int32_t(idx)) : 0;
        dig[k] = valid ? uint32_t((U(key[k]) - U(key_min)) >> shift) & (kBins - 1) : kBins;
    }

    // Stable rank of each item among the items of this wave with its digit.
    uint32_t rank[kSortIPT];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        const bool valid = dig[k] < kBins;
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; b++) {
            const bool bit = (dig[k] >> b) & 1;
            const uint64_t bb = ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t old = 0;
        if (valid) old = s_hist[w][dig[k]];
        rank[k] = old + __popcll(peers & lt);
        if (valid && (peers & lt) == 0) s_hist[w][dig[k]] = old + __popcll(peers);
    }
    __syncthreads();

    // Per digit: exclusive offsets across waves and the tile total.
    uint32_t tot = 0;
#pragma unroll
    for (int ww = 0; ww < kSortNW; ww++) {
        const uint32_t c = s_hist[ww][d0];
        s_hist[ww][d0] = tot;
        tot += c;
    }
    uint32_t tile_total;
    const uint32_t local = block_excl_scan<kSortNT>(tot, &tile_total, s_scan);
    s_local[d0] = local;

    // Decoupled look-back for digit d0 across earlier tiles.
    uint32_t *st = status + tile * kBins + d0;
    int64_t prefix = 0;
    if (tile == 0) {
        st_relaxed(st, kSFlagInc | tot);
    } else {
        st_relaxed(st, kSFlagAgg | tot);
        for (int64_t t = tile - 1; t >= 0; t--) {
            const uint32_t *sp = status + t * kBins + d0;
            uint32_t s = ld_relaxed(sp);
            while ((s >> 30) == 0) {
                __builtin_amdgcn_s_sleep(1);
                s = ld_relaxed(sp);
            }
            prefix += s & kSValMask;
            if ((s >> 30) == 2) break;
        }
        st_relaxed(st, kSFlagInc | uint32_t(prefix + tot));
    }
    s_gbase[d0] = int64_t(gstart) + prefix - int64_t(local);
    __syncthreads();

    // Stage the tile in digit order.
#pragma unroll
    for (int k = 0; k < kSortIPT; k++) {
        if (dig[k] < kBins) {
            const uint32_t pos = s_local[dig[k]] + s_hist[w][dig[k]] + rank[k];
            s_keys[pos] = key[k];
            s_rows[pos] = row[k];
        }
    }
    __syncthreads();

    const int64_t tile_cnt = cnt - tile * kSortTile < kSortTile ? cnt - tile * kSortTile : kSortTile;
    for (int i = threadIdx.x; i < tile_cnt; i += kSortNT) {
        const K kk = s_keys[i];
        const uint32_t d = uint32_t((U(kk) - U(key_min)) >> shift) & (kBins - 1);
        const int64_t dest = s_gbase[d] + i;
        keys_out[dest] = kk;
        rows_out[dest] = s_rows[i];
    }
}

template <class K>
__global__ __launch_bounds__(256) void k_copy_sorted(const K *__restrict__ keys_in,
                                                     const int32_t *__restrict__ rows_in,
                                                     K *__restrict__ keys_out,
                                                     int32_t *__restrict__ rows_out, int64_t n,
                                                     const int64_t *d_n) {
    const int64_t cnt = count_of(d_n, n);
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < cnt;
         i += int64_t(gridDim.x) * blockDim.x) {
        keys_out[i] = keys_in[i];
        rows_out[i] = rows_in ? rows_in[i] : int32_t(i);
    }
}

static int npass_for(int key_bits) { return (key_bits + kRadixBits - 1) / kRadixBits; }

size_t sort_ws_bytes(int64_t n, int dtype, int key_bits) {
    const int npass = npass_for(key_bits);
    const int64_t ntiles = n > 0 ? ceil_div(n, kSortTile) : 1;
    Carver c(nullptr);
    c.take<int64_t>(2);                                   // key-range scratch
    if (npass > 1) {
        c.take<char>(size_t(n) * dtype_size(dtype));      // ping-pong keys
        c.take<int32_t>(size_t(n));                       // ping-pong rows
    }
    c.take<uint32_t>(size_t(npass) * kBins + npass + size_t(npass) * ntiles * kBins);
    return c.bytes();
}

template <class K>
static int sort_typed(const K *key_in, const int32_t *rows_in, int64_t n, const int64_t *d_n,
                      int key_bits, int64_t key_min, K *key_out, int32_t *rows_out, void *ws,
                      hipStream_t s) {
    const int npass = npass_for(key_bits);
    const unsigned grid_all = unsigned(ceil_div(n > 0 ? n : 1, kSortTile));
    if (npass == 0) {
        unsigned g = grid_all > 4096 ? 4096 : grid_all;
        TQP_LAUNCH("copy_sorted", k_copy_sorted<K>, dim3(g), dim3(256), 0, s, key_in, rows_in, key_out,
                           rows_out, n, d_n);
        return check_launch("sort copy");
    }
    const int64_t ntiles = n > 0 ? ceil_div(n, kSortTile) : 1;
    Carver c(ws);
    c.take<int64_t>(2);
    K *tmp_keys = nullptr;
    int32_t *tmp_rows = nullptr;
    if (npass > 1) {
        tmp_keys = reinterpret_cast<K *>(c.take<char>(size_t(n) * sizeof(K)));
        tmp_rows = c.take<int32_t>(size_t(n));
    }
    const size_t nwords = size_t(npass) * kBins + npass + size_t(npass) * ntiles * kBins;
    uint32_t *words = c.take<uint32_t>(nwords);
    uint32_t *ghist = words;
    uint32_t *tickets = words + npass * kBins;
    uint32_t *status = tickets + npass;
    int rc = fill_u32(words, 0, int64_t(nwords), s);
    if (rc) return rc;
    {
        unsigned g = grid_all > 1024 ? 1024 : grid_all;
        TQP_LAUNCH("radix_hist", k_radix_hist<K>, dim3(g), dim3(kSortNT), 0, s, key_in, n, d_n,
                           K(key_min), npass, ghist);
        rc = check_launch("radix histogram");
        if (rc) return rc;
    }
    const K *src_k = key_in;
    const int32_t *src_r = rows_in;
    for (int p = 0; p < npass; p++) {
        const bool to_out = ((npass - 1 - p) % 2) == 0;
        K *dk = to_out ? key_out : tmp_keys;
        int32_t *dr = to_out ? rows_out : tmp_rows;
        TQP_LAUNCH("onesweep", k_onesweep<K>, dim3(grid_all), dim3(kSortNT), 0, s, src_k, src_r, dk,
                           dr, n, d_n, K(key_min), p * kRadixBits, ghist + p * kBins,
                           status + size_t(p) * ntiles * kBins, tickets + p);
        rc = check_launch("radix pass");
        if (rc) return rc;
        src_k = dk;
        src_r = dr;
    }
    return TQP_OK;
}

int sort_impl(const void *key_in, int dtype, const int32_t *rows_in, int64_t n, const int64_t *d_n,
              int key_bits, int64_t key_min, void *key_out, int32_t *rows_out, void *ws,
              size_t ws_bytes, hipStream_t s) {
    const int width = dtype == TQP_INT32 ? 32 : 64;
    if (key_bits > width) key_bits = width;
    if (key_bits < 0) key_bits = 0;
    const size_t need = sort_ws_bytes(n, dtype, key_bits);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "sort: workspace needs %zu bytes", need);
    if (dtype == TQP_INT32)
        return sort_typed<int32_t>(static_cast<const int32_t *>(key_in), rows_in, n, d_n, key_bits,
                                   key_min, static_cast<int32_t *>(key_out), rows_out, ws, s);
    return sort_typed<int64_t>(static_cast<const int64_t *>(key_in), rows_in, n, d_n, key_bits,
                               key_min, static_cast<int64_t *>(key_out), rows_out, ws, s);
}

}  // namespace tqp

using namespace tqp;

TQP_API size_t tqp_sort_workspace_bytes(int64_t n, int dtype) {
    if (!dtype_ok(dtype) || n < 0) return 0;
    return sort_ws_bytes(n, dtype, dtype == TQP_INT32 ? 32 : 64);
}

TQP_API int tqp_sort(const tqp_col *key, const int32_t *in_rows, int64_t n, const int64_t *d_n,
                     int key_bits, int64_t key_min, const tqp_col *out_key, int32_t *out_rows,
                     void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!key || !out_key || (n > 0 && (!key->data || !out_key->data || !out_rows)))
        return set_error(TQP_EINVAL, "tqp_sort: null argument");
    if (key->dtype != TQP_INT32 && key->dtype != TQP_INT64)
        return set_error(TQP_EINVAL, "tqp_sort: keys must be int32 or int64");
    if (out_key->dtype != key->dtype)
        return set_error(TQP_EINVAL, "tqp_sort: out_key dtype differs from key dtype");
    if (n < 0 || n > (int64_t(1) << 30) - 1)
        return set_error(TQP_EINVAL, "tqp_sort: n must be in [0, 2^30 - 1]");
    if (key->len < n || out_key->len < n)
        return set_error(TQP_ECAPACITY, "tqp_sort: key or out_key shorter than n");
    if (key_bits < 0 || key_bits > 64)
        return set_error(TQP_EINVAL, "tqp_sort: key_bits must be in [0, 64]");
    const size_t need = tqp_sort_workspace_bytes(n, key->dtype);
    if (!ws || ws_bytes < need)
        return set_error(TQP_ECAPACITY, "tqp_sort: workspace needs %zu bytes", need);
    if (n == 0) return TQP_OK;
    hipStream_t s = as_stream(stream);
    if (key_bits == 0) {
        int rc = derive_key_range(key->data, key->dtype, n, d_n, ws, s, &key_min, &key_bits);
        if (rc) return rc;
    }
    return sort_impl(key->data, key->dtype, in_rows, n, d_n, key_bits, key_min, out_key->data,
                     out_rows, ws, ws_bytes, s);
}
