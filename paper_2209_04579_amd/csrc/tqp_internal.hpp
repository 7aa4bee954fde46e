// Internal helpers shared by the libtqp translation units: error reporting,
// launch checks, wave64 primitives and the decoupled look-back used by every
// single-pass scan (filter compaction, run-length encoding, join offsets,
// group-by prefix sums, radix scatter).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "tqp.h"

#define TQP_API extern "C" __attribute__((visibility("default")))

namespace tqp {

constexpr int kWave = 64;

// ---- host side ---------------------------------------------------------

int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
// Reports a failed launch (hipGetLastError) as TQP_EHIP.
int check_launch(const char *what);
int dtype_size(int dtype);
bool dtype_ok(int dtype);
// data is aligned to the element size (kernels read whole aligned words)
bool col_aligned(const void *p, int dtype);
inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Carves aligned sub-buffers out of a caller-provided workspace.  With a null
// base it only measures.
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T> T *take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (used + 255) & ~size_t(255); }
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Grid of a persistent tile loop: at most `per_cu` workgroups per compute
// unit, never more than there are tiles.  Every tile id comes from one
// device-wide ticket counter, whose atomic serializes (about 11 ns per ticket
// on MI355X), so a grid of idle workgroups is not free: size it to the
// machine, not to the capacity.
constexpr int kComputeUnits = 256;

// Tuning knobs (set through tqp_tune_set, read at launch time on the host).
enum TuneKnob {
    kTuneFilterPerCu = 0,   // workgroups per CU of the filter's persistent grid
    kTuneSortPerCu,         // ... of each radix pass
    kTuneRlePerCu,          // ... of run-length encoding
    kTuneMatchPerCu,        // ... of the join match
    kTuneGbScanPerCu,       // ... of the sorted group-by scan
    kTunePartOvfCap,        // overflowing buckets a partition sort re-sorts before it
                            // sorts the whole input instead
    kTuneSortMode,          // radix pass: 0 = decoupled look-back, 1 = tile counts + scan
    kTuneSemiPerCu,         // 256-thread units per CU of the semi-join scan
    kTuneSemiWg,            // its workgroup size, in 256-thread units (1, 2, 4)
    kTuneCount
};
int tune(TuneKnob k);

inline unsigned persistent_grid(int64_t tiles, int per_cu) {
    int64_t g = int64_t(kComputeUnits) * per_cu;
    if (tiles < g) g = tiles;
    return unsigned(g > 0 ? g : 1);
}

// Per-kernel timing (see profile.hip).  A scope records one event before and
// one after the launches it encloses, on the launch stream, when enabled.
bool profile_on();
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
  private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// Launches a kernel inside a timing scope named after it.
#define TQP_LAUNCH(name, kern, grid, block, lds, stream, ...)                  \
    do {                                                                       \
        ::tqp::ProfScope tqp_prof_scope_(name, stream);                        \
        hipLaunchKernelGGL(kern, grid, block, lds, stream, __VA_ARGS__);       \
    } while (0)

// Enqueues a fill of `count` 64-bit words (a kernel, not a memset node, so
// that captured graphs replay it faithfully).
int fill_u64(void *dst, uint64_t value, int64_t count, hipStream_t s);
// Run heads of a sorted int32 column (join.hip): value and first position of
// each run, run count in *d_nu; words: rle_words(n) uint64 of workspace.
size_t rle_words(int64_t n);
int rle_i32(const int32_t *keys, int64_t n, int32_t *ukey, int32_t *ustart, int64_t *d_nu,
            uint64_t *words, hipStream_t s);
int fill_u32(void *dst, uint32_t value, int64_t count, hipStream_t s);
// Zeroes the head words before dst, then nsec sections (section k at dst +
// k * stride words), each over its first ceil(count / per) * width words
// with count = min(*d_n, n) read on the device (d_n NULL: count = n).  One
// launch for both.
int clear_sections(uint32_t *dst, int64_t head, int nsec, int64_t stride, const int64_t *d_n,
                   int64_t n, int64_t per, int64_t width, hipStream_t s);

// Device-side min / max of a key column over min(*d_n, n) entries, written to
// out[0] = min, out[1] = max (int64).
int launch_minmax(const void *key, int dtype, int64_t n, const int64_t *d_n,
                  int64_t *out, hipStream_t s);

// Internal entry used by join and group-by: LSD radix sort with known range.
int sort_impl(const void *key_in, int dtype, const int32_t *rows_in, int64_t n,
              const int64_t *d_n, int key_bits, int64_t key_min, void *key_out,
              int32_t *rows_out, void *ws, size_t ws_bytes, hipStream_t s);
size_t sort_ws_bytes(int64_t n, int dtype, int key_bits);
size_t sort_ws_bytes(int64_t n, int dtype, int key_bits, int pay_bytes);
// Host-synchronizing derivation of (key_min, key_bits) for a column.
int derive_key_range(const void *key, int dtype, int64_t n, const int64_t *d_n,
                     void *scratch16, hipStream_t s, int64_t *key_min, int *key_bits);

// ---- device side --------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }
__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << lane_id()) - 1;
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int64_t count_of(const int64_t *d_n, int64_t n) {
    if (d_n) {
        int64_t v = *d_n;
        return v < n ? (v < 0 ? 0 : v) : n;
    }
    return n;
}

template <class T> __device__ __forceinline__ T shfl_up(T v, int d) {
    return __shfl_up(v, d, kWave);
}
template <> __device__ __forceinline__ int64_t shfl_up<int64_t>(int64_t v, int d) {
    int lo = __shfl_up(static_cast<int>(v & 0xffffffff), d, kWave);
    int hi = __shfl_up(static_cast<int>(v >> 32), d, kWave);
    return (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
}
template <> __device__ __forceinline__ uint64_t shfl_up<uint64_t>(uint64_t v, int d) {
    return static_cast<uint64_t>(shfl_up<int64_t>(static_cast<int64_t>(v), d));
}
template <class T> __device__ __forceinline__ T shfl_xor(T v, int m) {
    return __shfl_xor(v, m, kWave);
}
template <> __device__ __forceinline__ int64_t shfl_xor<int64_t>(int64_t v, int m) {
    int lo = __shfl_xor(static_cast<int>(v & 0xffffffff), m, kWave);
    int hi = __shfl_xor(static_cast<int>(v >> 32), m, kWave);
    return (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
}
template <class T> __device__ __forceinline__ T shfl(T v, int src) {
    return __shfl(v, src, kWave);
}
template <> __device__ __forceinline__ int64_t shfl<int64_t>(int64_t v, int src) {
    int lo = __shfl(static_cast<int>(v & 0xffffffff), src, kWave);
    int hi = __shfl(static_cast<int>(v >> 32), src, kWave);
    return (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
}

// Inclusive prefix sum across the 64 lanes of a wave (wrapping arithmetic).
template <class T> __device__ __forceinline__ T wave_incl_scan(T v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = shfl_up(v, d);
        if (lane_id() >= d) v += u;
    }
    return v;
}

template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += shfl_xor(v, m);
    return v;
}

// Exclusive prefix sum across a block of NT threads.  `lds` holds NT/64
// entries of T.  Returns the exclusive prefix; *total receives the block sum.
template <int NT, class T>
__device__ __forceinline__ T block_excl_scan(T v, T *total, T *lds) {
    constexpr int NW = NT / kWave;
    T inc = wave_incl_scan(v);
    const int w = wave_id();
    if (lane_id() == kWave - 1) lds[w] = inc;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        T x = lds[i];
        if (i < w) pre += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

// ---- agent-scope atomics ------------------------------------------------

template <class T> __device__ __forceinline__ T ld_acquire(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ T ld_relaxed(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ void st_release(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ void st_relaxed(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Dynamic tile id: tiles are handed out in launch order, so every tile's
// predecessors belong to workgroups that are already running.  That is what
// lets a look-back wait on them without deadlock.
__device__ __forceinline__ int64_t take_tile(uint32_t *ticket, int64_t *lds_slot) {
    if (threadIdx.x == 0) *lds_slot = atomicAdd(ticket, 1u);
    __syncthreads();
    return *lds_slot;
}

// ---- decoupled look-back over one non-negative count -----------------------
// status[t] = flag << 62 | value, flag 0 = not ready, 1 = tile aggregate,
// 2 = inclusive prefix.  Called by all 64 lanes of one wave of tile `tile`
// with the tile aggregate `agg` (< 2^62).  Returns the exclusive prefix of
// the tile; publishes the inclusive prefix.
constexpr uint64_t kFlagAgg = uint64_t(1) << 62;
constexpr uint64_t kFlagInc = uint64_t(2) << 62;
constexpr uint64_t kValMask = (uint64_t(1) << 62) - 1;

__device__ __forceinline__ int64_t lookback_count(uint64_t *status, int64_t tile,
                                                  int64_t agg) {
    if (tile == 0) {
        if (lane_id() == 0) st_relaxed(&status[0], kFlagInc | uint64_t(agg));
        return 0;
    }
    if (lane_id() == 0) st_relaxed(&status[tile], kFlagAgg | uint64_t(agg));
    int64_t excl = 0;
    int64_t base = tile - 1;
    while (true) {
        const int64_t idx = base - lane_id();
        uint64_t s = kFlagInc;
        if (idx >= 0) {
            s = ld_relaxed(&status[idx]);
            while ((s >> 62) == 0) {
                __builtin_amdgcn_s_sleep(1);
                s = ld_relaxed(&status[idx]);
            }
        }
        const uint64_t inc = ballot((s >> 62) == 2);
        const int stop = inc ? (__ffsll(static_cast<long long>(inc)) - 1) : (kWave - 1);
        int64_t v = lane_id() <= stop ? int64_t(s & kValMask) : 0;
        excl += wave_sum(v);
        if (inc) break;
        base -= kWave;
    }
    if (lane_id() == 0) st_relaxed(&status[tile], kFlagInc | uint64_t(excl + agg));
    return excl;
}

// The same look-back in two halves, for a tile whose prefix is wanted later
// than its count is known: lookback_publish posts the tile's aggregate (the
// inclusive prefix for tile 0) as soon as it is counted; lookback_resolve,
// called later by one whole wave, walks back to the exclusive prefix and
// posts the inclusive one.  A successor only ever needs aggregates, which
// are posted before any wait, so deferring the resolution cannot deadlock.
__device__ __forceinline__ void lookback_publish(uint64_t *status, int64_t tile, int64_t agg) {
    if (lane_id() == 0) st_relaxed(&status[tile], (tile == 0 ? kFlagInc : kFlagAgg) | uint64_t(agg));
}

__device__ __forceinline__ int64_t lookback_resolve(uint64_t *status, int64_t tile, int64_t agg) {
    if (tile == 0) return 0;
    int64_t excl = 0;
    int64_t base = tile - 1;
    while (true) {
        const int64_t idx = base - lane_id();
        uint64_t s = kFlagInc;
        if (idx >= 0) {
            s = ld_relaxed(&status[idx]);
            while ((s >> 62) == 0) {
                __builtin_amdgcn_s_sleep(1);
                s = ld_relaxed(&status[idx]);
            }
        }
        const uint64_t inc = ballot((s >> 62) == 2);
        const int stop = inc ? (__ffsll(static_cast<long long>(inc)) - 1) : (kWave - 1);
        int64_t v = lane_id() <= stop ? int64_t(s & kValMask) : 0;
        excl += wave_sum(v);
        if (inc) break;
        base -= kWave;
    }
    if (lane_id() == 0) st_relaxed(&status[tile], kFlagInc | uint64_t(excl + agg));
    return excl;
}

// ---- key/value element access ------------------------------------------------

template <class T> struct KeyTraits;
template <> struct KeyTraits<int32_t> {
    using U = uint32_t;
    static constexpr int kBits = 32;
};
template <> struct KeyTraits<int64_t> {
    using U = uint64_t;
    static constexpr int kBits = 64;
};

__device__ __forceinline__ int64_t load_any(const void *p, int dtype, int64_t i) {
    switch (dtype) {
    case TQP_INT8: return static_cast<const int8_t *>(p)[i];
    case TQP_INT32: return static_cast<const int32_t *>(p)[i];
    default: return static_cast<const int64_t *>(p)[i];
    }
}
// log2 of the element size of a column dtype.
__device__ __forceinline__ int dtype_lg(int dtype) {
    return dtype == TQP_INT8 ? 0 : dtype == TQP_INT32 ? 2 : 3;
}

// Element i of a naturally aligned column of 1-, 4- or 8-byte integers,
// zero-extended: one 8-byte load of the aligned word that holds it
// (word_of), then a shift and a mask (from_word).  The same instruction
// serves every dtype, so a kernel reading columns whose dtypes are known only
// at run time needs no branch and keeps all its loads in flight together.
// The aligned word lies in the element's own page, so it is always readable;
// its other bytes are dropped.
__device__ __forceinline__ uint64_t word_of(const void *p, int lg, int64_t i) {
    const char *e = static_cast<const char *>(p) + (i << lg);
    return *reinterpret_cast<const uint64_t *>(e - (reinterpret_cast<uintptr_t>(e) & 7));
}
__device__ __forceinline__ uint64_t from_word(uint64_t w, const void *p, int lg, int64_t i) {
    const uint64_t mis = (reinterpret_cast<uintptr_t>(p) + (uint64_t(i) << lg)) & 7;
    const uint64_t v = w >> (mis * 8);
    return lg == 3 ? v : v & ((uint64_t(1) << (8 << lg)) - 1);
}
__device__ __forceinline__ uint64_t load_word(const void *p, int lg, int64_t i) {
    return from_word(word_of(p, lg, i), p, lg, i);
}

// N elements of one column at valid positions idx[], zero-extended to 64
// bits, all N loads issued before any result is used.
template <int N, class I>
__device__ __forceinline__ void load_raw(const void *p, int dtype, const I (&idx)[N],
                                         uint64_t (&out)[N]) {
    const int lg = dtype_lg(dtype);
#pragma unroll
    for (int r = 0; r < N; r++) out[r] = word_of(p, lg, int64_t(idx[r]));
#pragma unroll
    for (int r = 0; r < N; r++) out[r] = from_word(out[r], p, lg, int64_t(idx[r]));
}
// The signed value of a zero-extended element of the given dtype.
__device__ __forceinline__ int64_t sext_of(uint64_t v, int dtype) {
    return dtype == TQP_INT8 ? int64_t(int8_t(v)) : dtype == TQP_INT32 ? int64_t(int32_t(v)) : int64_t(v);
}
__device__ __forceinline__ void store_any(void *p, int dtype, int64_t i, int64_t v) {
    switch (dtype) {
    case TQP_INT8: static_cast<int8_t *>(p)[i] = static_cast<int8_t>(v); break;
    case TQP_INT32: static_cast<int32_t *>(p)[i] = static_cast<int32_t>(v); break;
    default: static_cast<int64_t *>(p)[i] = v; break;
    }
}

// `v op lit` for a tqp_cmp code, compared as mathematical integers.
__device__ __forceinline__ bool cmp_holds(int64_t v, int op, int64_t lit) {
    switch (op) {
    case TQP_LT: return v < lit;
    case TQP_LE: return v <= lit;
    case TQP_GT: return v > lit;
    case TQP_GE: return v >= lit;
    case TQP_EQ: return v == lit;
    default: return v != lit;
    }
}

// ---- packed multi-column keys ---------------------------------------------
// key(i) = sum over terms of mul * f(col[rows ? rows[i] : i]) mod 2^64, with
// f(v) = v mod m in [0, m) when m > 0, f(v) = v otherwise; a term without a
// column adds mul; a row outside the column reads 0.
struct PackArgs {
    const void *col[4];
    const int32_t *rows[4];
    int64_t len[4];
    int64_t mod[4];
    int64_t mul[4];
    int32_t dt[4];
    int32_t nterms;
};

// The keys of R positions (positions >= cnt give 0), term by term: each
// term's R row-id loads go out together, then its R value loads.  Loads are
// never predicated: a position past cnt reads row 0 and a row outside the
// column reads element 0 (both exist whenever cnt >= 1, as in every caller's
// loop), and the result is then replaced.  A power-of-two modulus is a mask
// (v mod 2^k in [0, 2^k) is v & (2^k - 1) in two's complement).
template <int R>
__device__ __forceinline__ void pack_keys(const PackArgs &a, const int64_t (&idx)[R], int64_t cnt,
                                          uint64_t (&acc)[R]) {
#pragma unroll
    for (int r = 0; r < R; r++) acc[r] = 0;
    for (int t = 0; t < a.nterms; t++) {
        if (!a.col[t]) {                       // constant term
#pragma unroll
            for (int r = 0; r < R; r++) acc[r] += uint64_t(a.mul[t]);
            continue;
        }
        int64_t row[R];
        if (a.rows[t]) {
            int64_t li[R];
            uint64_t rr[R];
#pragma unroll
            for (int r = 0; r < R; r++) li[r] = idx[r] < cnt ? idx[r] : 0;
#pragma unroll
            for (int r = 0; r < R; r++) rr[r] = uint32_t(a.rows[t][li[r]]);
#pragma unroll
            for (int r = 0; r < R; r++) row[r] = idx[r] < cnt ? int64_t(int32_t(uint32_t(rr[r]))) : -1;
        } else {
#pragma unroll
            for (int r = 0; r < R; r++) row[r] = idx[r] < cnt ? idx[r] : -1;
        }
        const int64_t len = a.len[t];
        const int dt = a.dt[t];
        int64_t v[R];
        if (len > 0) {
            int64_t li[R];
            uint64_t raw[R];
#pragma unroll
            for (int r = 0; r < R; r++) li[r] = row[r] >= 0 && row[r] < len ? row[r] : 0;
            load_raw<R>(a.col[t], dt, li, raw);
#pragma unroll
            for (int r = 0; r < R; r++) v[r] = row[r] >= 0 && row[r] < len ? sext_of(raw[r], dt) : 0;
        } else {
#pragma unroll
            for (int r = 0; r < R; r++) v[r] = 0;
        }
        const int64_t m = a.mod[t];
        if (m > 0 && (m & (m - 1)) == 0) {
#pragma unroll
            for (int r = 0; r < R; r++) v[r] &= m - 1;
        } else if (m > 0) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                v[r] %= m;
                if (v[r] < 0) v[r] += m;
            }
        }
#pragma unroll
        for (int r = 0; r < R; r++) acc[r] += uint64_t(a.mul[t]) * uint64_t(v[r]);
    }
}

// Fills PackArgs from the C-ABI terms; n is the row count a term without row
// ids must cover.  Returns TQP_OK or an error (message set).
int pack_args(const tqp_keyterm *terms, int nterms, int64_t n, PackArgs *a, const char *who);

}  // namespace tqp
