/*
 * tqp.h -- C ABI of the MI355X relational hot path (libtqp.so).
 *
 * The operation set is the relational core of a tensor query processor
 * (arXiv 2209.04579): tables are columnar, one contiguous (n x 1) device array
 * per numeric column (Section 2.1), and the executor turns input columns into
 * result columns (Section 2.2, "Execution").  The operators are the ones the
 * paper's TPC-H workload exercises (Section 2.3): predicate filters (also
 * fused with an aggregate, Q6's shape), an equi-join and SUM/COUNT
 * aggregation, here with a group-by (Fig. 4); LIKE over string columns, which
 * Section 2.1 stores as zero-padded (n x m) byte tensors (Q14's CASE); and a
 * model's prediction inside a query (Section 3.3).  The sort is the step a
 * sort-merge join and a sort-based group-by rest on; tqp_filter_sort fuses a
 * filter with it, so that the filtered table is never materialised.
 *
 * Conventions for every entry point:
 *  - Every pointer to column data, row ids, counts, outputs and workspace is
 *    DEVICE memory on the current HIP device, unless the argument is a
 *    descriptor array (tqp_col*, tqp_pred*, tqp_agg*, tqp_keyterm*,
 *    tqp_ranges*): those descriptor structs live in HOST memory and are read
 *    before the call returns.
 *  - The caller allocates and owns every buffer, including the workspace
 *    (size from the matching *_workspace_bytes call).  The library keeps no
 *    device memory between calls.  Input and output buffers must not overlap.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    the call returns without waiting, unless it says it synchronizes.
 *    Result counts are written to device memory (int64_t *d_...), so calls can
 *    be chained, and captured in a graph, without host round trips.
 *  - `n` arguments are host-side capacities.  Where a `const int64_t *d_n`
 *    is accepted and non-NULL, the actual count is min(*d_n, n), read on the
 *    device; NULL means the count is n.
 *  - Row ids are int32; a call accepts at most 2^31 - 1 rows (sort: 2^30 - 1).
 *  - Return value: TQP_OK, or an error code with a message retrievable from
 *    tqp_last_error() (thread-local).  Argument errors are reported before
 *    anything is enqueued; nothing aborts the process.
 */
#ifndef TQP_H
#define TQP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TQP_OK        0
#define TQP_EINVAL    1   /* bad argument: null pointer, size, dtype, flag   */
#define TQP_ECAPACITY 2   /* an output or workspace buffer is too small       */
#define TQP_EHIP      3   /* the HIP runtime reported an error                */

/* Column element types.  Money is int64 fixed-point cents, so sums are exact. */
typedef enum { TQP_INT8 = 1, TQP_INT32 = 2, TQP_INT64 = 3 } tqp_dtype;

/* A non-owning 1-D device column: `len` elements of `dtype` at `data`, which
 * is aligned to the element size (entry points that read columns of run-time
 * dtype check this and return TQP_EINVAL otherwise). */
typedef struct {
    void    *data;
    int64_t  len;
    int32_t  dtype;
    int32_t  reserved;
} tqp_col;

/* Predicate `cols[col] op literal`, compared as mathematical integers. */
typedef enum { TQP_LT = 0, TQP_LE = 1, TQP_GT = 2, TQP_GE = 3, TQP_EQ = 4, TQP_NE = 5 } tqp_cmp;
typedef struct {
    int32_t col;
    int32_t op;
    int64_t literal;
} tqp_pred;

/* Aggregates over value columns: SUM(vals[a]), COUNT(*), SUM(vals[a]*vals[b]),
 * SUM(vals[a] * (c - vals[b])) with c a constant (Section 2.3's Q14 revenue,
 * price * (100 - discount) in cents and hundredths).  Sums are int64 two's
 * complement, i.e. exact modulo 2^64.  c is read by SUM_DIFF_PRODUCT only. */
typedef enum {
    TQP_AGG_SUM = 0, TQP_AGG_COUNT = 1, TQP_AGG_SUM_PRODUCT = 2, TQP_AGG_SUM_DIFF_PRODUCT = 3
} tqp_agg_op;
typedef struct {
    int32_t op;
    int32_t a;
    int32_t b;
    int32_t c;
} tqp_agg;

/* One term of a packed key: mul * f(col[rows ? rows[i] : i]) where
 * f(v) = v mod m in [0, m) when m > 0, and f(v) = v when m == 0. */
typedef struct {
    tqp_col        col;
    const int32_t *rows;
    int64_t        mod;
    int64_t        mul;
} tqp_keyterm;

/* Join result in ranges form: five device int64 arrays of capacity range_cap. */
typedef struct {
    int64_t *key;
    int64_t *lstart;
    int64_t *lcnt;
    int64_t *rstart;
    int64_t *rcnt;
} tqp_ranges;

/* Thread-local text of the last error reported on this thread ("" if none). */
const char *tqp_last_error(void);

/* Library version string. */
const char *tqp_version(void);

/* Per-kernel timing, off by default.  While enabled, every kernel the library
 * enqueues is bracketed by two HIP events on its stream.  tqp_profile_collect
 * waits for the pending events, accumulates them and writes one line per
 * kernel name, "name launches total_ms\n", into buf (HOST memory, truncated to
 * len); it returns the length the full text needs, including the final NUL.
 * tqp_profile_reset drops all pending and accumulated timings. */
void tqp_profile_enable(int on);
int tqp_profile_collect(char *buf, size_t len);
void tqp_profile_reset(void);

/* Launch knobs, the control surface of the autotuner (an extension of this
 * library; the paper tunes nothing at this level).  Each knob is an integer in a
 * fixed range with a default: "filter.per_cu", "sort.per_cu", "rle.per_cu",
 * "match.per_cu", "gbscan.per_cu" are workgroups per compute unit of one
 * persistent kernel's grid; "part.ovf_cap" is how many overflowing buckets
 * tqp_partition_sort re-sorts before it sorts the whole input instead;
 * "sort.mode" picks how a radix pass finds where each tile's digit runs go:
 * 0 = decoupled look-back over earlier tiles, 1 = every tile's digit counts
 * first, then a scan per digit (one more read of the keys, no waiting);
 * "semijoin.wg" is tqp_semijoin's workgroup size in units of 256 threads
 * (1, 2 or 4; a larger workgroup takes a larger tile) and "semijoin.per_cu"
 * its threads per compute unit in the same units.
 * Knobs change how the work is done, never results.  They are process-wide
 * and read when a call enqueues its kernels; setting them concurrently with
 * calls on other threads is a race.
 *   tqp_tune_set: TQP_EINVAL for an unknown name or a value out of range.
 *   tqp_tune_get: writes value / lo / hi (each pointer may be NULL).
 *   tqp_tune_name: name of knob `index` (0-based), NULL past the last one. */
int tqp_tune_set(const char *name, int value);
int tqp_tune_get(const char *name, int *value, int *lo, int *hi);
const char *tqp_tune_name(int index);

/* ------------------------------------------------------------------------
 * tqp_minmax -- the value range of a column: d_out[0] = min and d_out[1] =
 * max of the first count keys (count = min(*d_n, key->len) with d_n, else
 * key->len), as int64; with no keys, d_out = {INT64_MAX, INT64_MIN}.  The
 * statistics a planner keeps per column (Section 2.2 compiles a query into
 * an operator plan): they fix a sort's pass count, a dense group-by's domain
 * and a key set's range.  key: any integer dtype.  d_out: device, 2 int64s.
 * Nothing is synchronized.
 * ---------------------------------------------------------------------- */
int tqp_minmax(const tqp_col *key, const int64_t *d_n, int64_t *d_out, void *stream);

/* ------------------------------------------------------------------------
 * tqp_filter -- WHERE with stream compaction (Section 2.3: Q6's filters).
 * Keeps row i of an n-row table when every predicate holds; n = cols[0].len
 * and every cols[c] and pay_in[c] has len n.  npred in [1, 8], ncols in
 * [1, 8], npay in [0, 8].
 *   out_rows  : optional, capacity n; kept row ids, ascending.
 *   pay_out[c]: optional payload columns (same dtype as pay_in[c], capacity
 *               n): pay_out[c][k] = pay_in[c][out_rows[k]].
 *   d_count   : required; receives the number of kept rows.
 * Workspace: tqp_filter_workspace_bytes(n).
 * ---------------------------------------------------------------------- */
size_t tqp_filter_workspace_bytes(int64_t n);
int tqp_filter(const tqp_col *cols, int ncols, const tqp_pred *preds, int npred,
               const tqp_col *pay_in, const tqp_col *pay_out, int npay,
               int32_t *out_rows, int64_t *d_count,
               void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * tqp_filter_sum -- WHERE + aggregate without compaction (Section 2.3: TPC-H
 * Q6 is four filters over columns of different types feeding one SUM).
 * Over the rows of an n-row table (n = cols[0].len, every cols[c] of len n)
 * where every predicate holds:
 *   *d_sum   = SUM(a[i] * b[i])  (b NULL: SUM(a[i]); a NULL: 0), int64 two's
 *              complement, i.e. exact modulo 2^64;
 *   *d_count = COUNT(*).
 * a and b, when given, hold >= n elements.  ncols in [1, 8]; npred in [0, 8]
 * (none keeps every row).  d_sum and d_count are device int64s, overwritten.
 * No workspace; nothing is synchronized.
 * ---------------------------------------------------------------------- */
int tqp_filter_sum(const tqp_col *cols, int ncols, const tqp_pred *preds, int npred,
                   const tqp_col *a, const tqp_col *b, int64_t *d_sum, int64_t *d_count,
                   void *stream);

/* ------------------------------------------------------------------------
 * tqp_str_match -- LIKE over a string column.  Section 2.1 stores a string
 * column as an (n x m) tensor of UTF-8 bytes, one row per value, zero-padded
 * to m.  out[i] = 1 when row i starts with pattern[0..plen)
 * (TQP_STR_PREFIX: LIKE 'pattern%') or is exactly the pattern
 * (TQP_STR_EQUAL: those bytes, then only zero padding), else 0.
 *   chars  : device, n * m bytes, row-major;
 *   pattern: host, plen in [0, 64] bytes (copied into the launch);
 *   out    : device int8, n entries (a flag column for later operators).
 * m >= 1; a pattern longer than m matches nothing.  Nothing is synchronized.
 * ---------------------------------------------------------------------- */
#define TQP_STR_PREFIX 0
#define TQP_STR_EQUAL  1
int tqp_str_match(const uint8_t *chars, int64_t n, int32_t m, const uint8_t *pattern,
                  int32_t plen, int32_t mode, int8_t *out, void *stream);

/* ------------------------------------------------------------------------
 * tqp_mlp_predict -- PREDICT inside a query (Section 3.3's prediction query: a
 * model scores each row, then a group-by with a CASE compares the
 * predictions with the ratings).  For i < count (*d_n when d_n is given,
 * else n), with row = rows[i] (rows NULL: row = i) and x[k] =
 * feats[k][row] converted to float:
 *   h[j]  = relu(b1[j] + sum_k W1[j][k] x[k])   k ascending
 *   z[c]  = b2[c] + sum_j W2[c][j] h[j]          j ascending
 *   out[i] = the first c with the largest z[c]
 * in fp32, every multiply-add one fused fma in the order shown, relu(v) =
 * (v > 0 ? v : 0); integer features convert exactly below 2^24.
 *   feats : nfeat in [1, 16] columns of any integer dtype; a row outside a
 *           column reads 0;
 *   model : device fp32 [W1 (hidden x nfeat, row-major), b1 (hidden),
 *           W2 (classes x hidden), b2 (classes)]; hidden in [1, 64],
 *           classes in [1, 8];
 *   out   : device int8, n entries.
 * Nothing is synchronized.
 * ---------------------------------------------------------------------- */
int tqp_mlp_predict(const tqp_col *feats, int nfeat, const int32_t *rows, int64_t n,
                    const int64_t *d_n, const float *model, int hidden, int classes,
                    int8_t *out, void *stream);

/* ------------------------------------------------------------------------
 * tqp_gather -- out[i] = src[idx[i]] for i < count (Fig. 3's index_select).
 * src and dst share a dtype; dst->len >= n.  idx is 16-byte aligned (it is
 * read four ids at a time; TQP_EINVAL otherwise).  An index outside
 * [0, src->len) yields 0 instead of a read.
 * ---------------------------------------------------------------------- */
int tqp_gather(const tqp_col *src, const int32_t *idx, int64_t n,
               const int64_t *d_n, const tqp_col *dst, void *stream);

/* ------------------------------------------------------------------------
 * tqp_pack_key -- out[i] = sum over terms of mul * f(col[row]) (mod 2^64,
 * then truncated to out's dtype, int32 or int64) for i < count: the packed
 * multi-column group key, e.g. flag * 2 + (cat mod 2), or an instance prefix
 * (inst << 20) + fk.  A term whose column has no data (col.data NULL) adds
 * the constant mul.  Each term's rows (if given) hold >= count entries.
 * nterms in [1, 4].  Row ids outside the column read as 0.  out->len >= n.
 * ---------------------------------------------------------------------- */
int tqp_pack_key(const tqp_keyterm *terms, int nterms, int64_t n,
                 const int64_t *d_n, const tqp_col *out, void *stream);

/* ------------------------------------------------------------------------
 * tqp_sort -- stable ascending sort of signed int32/int64 keys (LSD radix),
 * the step under the sort-merge join and the sort-based group-by.
 *   key      : input keys, key->len >= n (n = capacity, d_n = actual count).
 *   in_rows  : optional row id carried with each key (NULL = 0, 1, 2, ...).
 *   key_bits : 0 = derive the key range on the device and read it back
 *              (this SYNCHRONIZES the stream); 1..64 = the caller guarantees
 *              0 <= key - key_min < 2^key_bits for every key.
 *   out_key  : sorted keys (capacity n).  Ties keep input order.
 *   out_rows : optional (capacity n); the row id carried with each key.
 *   pay_in / pay_out : npay in [0, 4] payload columns (any dtype, len >= n)
 *              moved with the keys: pay_out[c][i] = pay_in[c][perm[i]].
 * Workspace: tqp_sort_workspace_bytes(n, dtype, pay_bytes) where pay_bytes is
 * the sum of the payload element sizes.
 * ---------------------------------------------------------------------- */
size_t tqp_sort_workspace_bytes(int64_t n, int dtype, int pay_bytes);
int tqp_sort(const tqp_col *key, const int32_t *in_rows, int64_t n,
             const int64_t *d_n, int key_bits, int64_t key_min,
             const tqp_col *out_key, int32_t *out_rows,
             const tqp_col *pay_in, const tqp_col *pay_out, int npay,
             void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * tqp_filter_sort -- WHERE, then the stable sort, in one go: the result of
 * tqp_filter (Section 2.3's predicate filters) carrying the key and payload
 * columns, then tqp_sort of the kept rows, without the filtered table ever
 * being written.  The table has n = key->len rows; every cols[c] and
 * pay_in[c] has len >= n.  Row i is kept when every predicate holds on it
 * (ncols in [1, 8], npred in [1, 4]).  With k = *d_count kept rows (written
 * to device memory), for j < k:
 *   out_key[j]    : the kept keys, ascending; ties keep row order;
 *   out_rows[j]   : optional (capacity n); the row id (in the table) of j;
 *   pay_out[c][j] = pay_in[c][out_rows[j]], npay in [0, 4].
 * key_bits / key_min as for tqp_sort, bounding every key of the table
 * (0 = derive over all n keys, which SYNCHRONIZES the stream).  Outputs have
 * capacity n.  Workspace: tqp_sort_workspace_bytes(n, key dtype, pay_bytes).
 * ---------------------------------------------------------------------- */
int tqp_filter_sort(const tqp_col *cols, int ncols, const tqp_pred *preds, int npred,
                    const tqp_col *key, int key_bits, int64_t key_min,
                    const tqp_col *out_key, int32_t *out_rows,
                    const tqp_col *pay_in, const tqp_col *pay_out, int npay,
                    int64_t *d_count, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * tqp_join -- inner equi-join, bag semantics, sort-merge (Section 2.3: Q14).
 *   lkey/rkey : same dtype (int32 or int64).  With TQP_JOIN_SORTED both are
 *               ascending and lrows/rrows (optional; NULL = position) give the
 *               row id of each position; without it the library sorts both
 *               sides first (stable, key range derived on the device, which
 *               synchronizes the stream) and lrows/rrows are the row ids of
 *               the unsorted inputs.
 *   Pairs     : every (i, j) with lkey[i] == rkey[j], ordered by (key, i, j)
 *               over sorted positions, written as out_l = lrows[i],
 *               out_r = rrows[j], out_pair_key (optional, key dtype) = key.
 *               d_count (required) receives the pair count, even when it
 *               exceeds cap; then pairs past cap are not written.  Pass
 *               out_l = out_r = NULL to skip pairs.
 *   Ranges    : with TQP_JOIN_RANGES, for each key present on both sides,
 *               ascending: key, lstart, lcnt, rstart, rcnt, indexing the
 *               sorted sides; d_nranges receives their number (at most
 *               range_cap are written).
 * Workspace: tqp_join_workspace_bytes(nl, nr, dtype, flags, cap), with cap
 * 0 when no pairs are requested.
 * ---------------------------------------------------------------------- */
#define TQP_JOIN_SORTED 1u
#define TQP_JOIN_RANGES 2u
size_t tqp_join_workspace_bytes(int64_t nl, int64_t nr, int dtype, uint32_t flags,
                                int64_t cap);
int tqp_join(const tqp_col *lkey, const int32_t *lrows, const int64_t *d_nl,
             const tqp_col *rkey, const int32_t *rrows, const int64_t *d_nr,
             uint32_t flags,
             int32_t *out_l, int32_t *out_r, void *out_pair_key, int64_t cap,
             int64_t *d_count,
             const tqp_ranges *ranges, int64_t range_cap, int64_t *d_nranges,
             void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Semi-join reduction (in front of the joins of a star query, Section 2.3's
 * join queries).  A fact row can only join (inner) with a dimension when its
 * foreign key occurs among that dimension's keys, so rows failing the test
 * for any dimension are dropped before the sort-merge joins; the joins'
 * result is unchanged.
 *
 * A key set is a bitmap over the key range [lo, lo + nbits): bit (k - lo) of
 * bits (word (k - lo) / 32, bit (k - lo) % 32) is set when key k is in the
 * set.  bits is device memory of ceil(nbits / 32) uint32 words, owned by the
 * caller; nbits in [0, TQP_KEYSET_MAX_BITS] (0 = the empty set), and
 * lo + nbits - 1 <= INT64_MAX.  Both calls return TQP_EINVAL otherwise.
 *
 * tqp_keyset_build: clears bits, then sets the bit of each of the first
 *   count keys (count = min(*d_n, key->len) with d_n, else key->len) that lies
 *   in the range; keys outside it are ignored.  key: any integer dtype.
 * tqp_semijoin: keeps row i of an n-row table (n = keys[0].len) when
 *   keys[s][i] is in sets[s] for every s < nsets (nsets in [1, 4]).  The key
 *   columns share one dtype (int32 or int64) and length n.
 *   out_rows   : optional, capacity n; kept row ids, ascending.
 *   keys_out   : optional array of nsets columns (an entry with data NULL is
 *                skipped): keys_out[s][k] = keys[s][out_rows[k]], capacity n.
 *   pay_out[c] : pay_out[c][k] = pay_in[c][out_rows[k]] (npay in [0, 4],
 *                same dtype, len >= n); only kept rows of pay_in are read.
 *   d_count    : required; receives the number of kept rows.
 * Sets are staged in on-chip memory while they fit (up to 36864 words in all
 * with 1024-thread workgroups, a quarter of that per 256 threads with
 * smaller ones); the others are read from device memory.  Workspace:
 * tqp_semijoin_workspace_bytes(n, key dtype).  Nothing is synchronized.
 * ---------------------------------------------------------------------- */
#define TQP_KEYSET_MAX_BITS (1ll << 36)
typedef struct {
    const uint32_t *bits;
    int64_t         lo;
    int64_t         nbits;
} tqp_keyset;
int tqp_keyset_build(const tqp_col *key, const int64_t *d_n, int64_t lo, int64_t nbits,
                     uint32_t *bits, void *stream);
size_t tqp_semijoin_workspace_bytes(int64_t n, int dtype);
int tqp_semijoin(const tqp_col *keys, const tqp_keyset *sets, int nsets,
                 const tqp_col *keys_out, const tqp_col *pay_in, const tqp_col *pay_out,
                 int npay, int32_t *out_rows, int64_t *d_count,
                 void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * tqp_semijoin_noalloc -- tqp_semijoin without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation).  Same arguments, results
 * and errors as tqp_semijoin; its tickets and look-back statuses live in a
 * static 8 MiB device array of the library (one per device, held until the
 * process ends, located on the first call on each device), cleared by a
 * kernel at the start of every call.  It allocates nothing and calls no
 * allocating routine.  Tables of more than
 * tqp_semijoin_noalloc_max_rows(dtype) rows (every int32 table up to
 * 2^31 - 1 rows; about 1.6e9 rows of int64 keys) are rejected with
 * TQP_ECAPACITY.  All calls on one device share the array: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialized by the caller.
 * ---------------------------------------------------------------------- */
int64_t tqp_semijoin_noalloc_max_rows(int dtype);
int tqp_semijoin_noalloc(const tqp_col *keys, const tqp_keyset *sets, int nsets,
                         const tqp_col *keys_out, const tqp_col *pay_in, const tqp_col *pay_out,
                         int npay, int32_t *out_rows, int64_t *d_count, void *stream);

/* ------------------------------------------------------------------------
 * tqp_groupby_agg -- GROUP BY key with SUM / COUNT / SUM of products
 * (Section 2.3 aggregates; Fig. 4's group-by aggregate).
 *   key       : int32/int64 keys, capacity key->len, actual count d_n.
 *   vals      : nvals value columns (int8/int32/int64, each len >= count or
 *               >= max row id + 1 when val_rows is given).
 *   val_rows  : optional; the values of row i are vals[c][val_rows[i]].
 *   aggs      : nagg in [1, 4] aggregates.
 *   flags     : TQP_GB_SORTED  -- keys are already ascending (no sort);
 *               TQP_GB_DENSE   -- the caller guarantees
 *                                 key_lo <= key < key_lo + key_span with
 *                                 key_span <= TQP_GB_DENSE_MAX: direct
 *                                 aggregation, no sort.
 *               otherwise the keys are sorted first; key_span > 0 bounds the
 *               key range as above, key_span == 0 derives it on the device
 *               (synchronizes the stream).
 *   Output    : the groups that occur, ascending by key: out_key (capacity
 *               out_key->len) and out_aggs[a] (int64, same capacity);
 *               d_ngroups receives the group count.
 * Workspace: tqp_groupby_workspace_bytes(n, key dtype, nagg, flags, key_span).
 * ---------------------------------------------------------------------- */
#define TQP_GB_SORTED 1u
#define TQP_GB_DENSE  2u
#define TQP_GB_DENSE_MAX 4096
size_t tqp_groupby_workspace_bytes(int64_t n, int dtype, int nagg, uint32_t flags,
                                   int64_t key_span);
int tqp_groupby_agg(const tqp_col *key, const int64_t *d_n, uint32_t flags,
                    int64_t key_lo, int64_t key_span,
                    const tqp_col *vals, int nvals, const int32_t *val_rows,
                    const tqp_agg *aggs, int nagg,
                    const tqp_col *out_key, int64_t *const *out_aggs,
                    int64_t *d_ngroups,
                    void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * tqp_groupby_agg_terms -- the dense GROUP BY of tqp_groupby_agg
 * (TQP_GB_DENSE) over a packed key that is never written to memory: the key of
 * row i is the tqp_pack_key value of `terms` (nterms in [1, 4]) at i, for
 * i < count (d_n, else n), computed as the rows are aggregated.  The caller
 * guarantees key_lo <= key < key_lo + key_span; (nagg + 1) * key_span must be
 * at most 6144 (the accumulators live in LDS).  out_key is int32 or int64
 * (the key range must fit it); outputs as tqp_groupby_agg.  Workspace:
 * tqp_groupby_terms_workspace_bytes(nagg, key_span).
 * ---------------------------------------------------------------------- */
size_t tqp_groupby_terms_workspace_bytes(int nagg, int64_t key_span);
int tqp_groupby_agg_terms(const tqp_keyterm *terms, int nterms, int64_t n, const int64_t *d_n,
                          int64_t key_lo, int64_t key_span,
                          const tqp_col *vals, int nvals, const int32_t *val_rows,
                          const tqp_agg *aggs, int nagg,
                          const tqp_col *out_key, int64_t *const *out_aggs,
                          int64_t *d_ngroups, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * tqp_lower_bound -- out[i] = the number of the first count keys of `sorted`
 * (ascending; count = min(*d_n, sorted->len) with d_n, else sorted->len)
 * that are below queries[i], for i < queries->len: where each query would be
 * inserted.  sorted: int32 or int64; queries: any integer dtype; out: device
 * int64, queries->len entries.  Splits a batched, sorted result by instance.
 * ---------------------------------------------------------------------- */
int tqp_lower_bound(const tqp_col *sorted, const int64_t *d_n, const tqp_col *queries,
                    int64_t *out, void *stream);

/* ------------------------------------------------------------------------
 * Batched execution (an extension of the executor of Section 2.2: many
 * independent queries of one shape run as one plan).  The instances' tables
 * are laid end to end in one columnar arena; every join key carries its
 * instance number in its high bits (key' = i << key_shift | key) and every
 * category likewise (cat' = i << cat_shift | cat), so keys of different
 * instances never meet and instance i's groups precede instance i+1's.  The
 * whole plan over the arena is then captured once and replayed as one graph.
 *
 * tqp_batch_plan: HOST only.  From k instances' fact and dimension row
 *   counts and the largest join key and category over all of them (both
 *   >= 0), writes the arena offsets out->fact_off[0..k] and dim_off[0..k]
 *   (caller-owned host arrays of k + 1), the shifts and the arena's sizes.
 *   TQP_EINVAL when the prefixed keys or categories would not fit int32.
 * tqp_batch_capture_begin / tqp_batch_capture_end: every library call
 *   enqueued on `stream` (not the null stream) in between is recorded into
 *   one graph instead of running; end instantiates it and returns an opaque
 *   handle in *graph.  Calls that synchronize (key-range derivation,
 *   tqp_partition_sort) must not be captured.  Buffers and workspaces
 *   named by the captured calls must stay allocated while the graph lives.
 * tqp_batch_run: launches the captured graph on `stream` (one launch).
 * tqp_batch_destroy: releases the handle (NULL is a no-op).
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t *fact_off;      /* host, k + 1 entries (filled) */
    int64_t *dim_off;       /* host, k + 1 entries (filled) */
    int32_t  key_shift;     /* instance number position in join keys */
    int32_t  cat_shift;     /* instance number position in categories */
    int64_t  fact_rows;     /* arena sizes */
    int64_t  dim_rows;
} tqp_batch_layout;
int tqp_batch_plan(int k, const int64_t *fact_rows, const int64_t *dim_rows, int64_t max_key,
                   int64_t max_cat, tqp_batch_layout *out);
int tqp_batch_capture_begin(void *stream);
int tqp_batch_capture_end(void *stream, void **graph);
int tqp_batch_run(void *graph, void *stream);
int tqp_batch_destroy(void *graph);

/* ------------------------------------------------------------------------
 * Learned CDF partitioner.  A model F maps a key to [0, 1], monotone
 * non-decreasing: a 1 -> 32 -> 1 FP32 network (ramp units clamp(w x + c, 0, 1),
 * positive weights) over the key normalised to [0, 1], refined by nleaf
 * piecewise-linear leaves.  Buckets floor(F * 2^bits) are contiguous key
 * ranges, so grouping keys by bucket and sorting inside each bucket sorts
 * them; the model only decides how balanced the buckets are.
 *
 * tqp_lcdf_train: samples every sample_stride-th key of ncols (1 or 2)
 *   int32/int64 device columns, sorts the sample, fits the network by `steps`
 *   full-batch Adam steps (learning rate lr, e.g. 1e-2) on the squared error
 *   against the sample ranks, keeps the parameters with the lowest loss seen,
 *   then fits the leaves.  `model` is a device buffer of
 *   tqp_lcdf_model_bytes(nleaf) bytes (nleaf in [1, 65536]); its first 36
 *   bytes are int64 kmin, float64 1/span, int32 nleaf, int32 steps, float32
 *   loss at the first step, at the last step, and the lowest.  No host sync.
 *   Leaves are 96 bytes (eight exact int64 knots); bucket numbers are
 *   evaluated with the leaves held in LDS, 1688 leaves per pass over the
 *   keys, so nleaf <= 1688 takes one pass (the fast case).
 * tqp_lcdf_buckets: out_bucket[i] = bucket of keys[i] for 2^bucket_bits
 *   buckets (bits in [1, 24]); for inspection and tests.  Synchronizes the
 *   stream once (to read the model's leaf count).
 * ---------------------------------------------------------------------- */
size_t tqp_lcdf_model_bytes(int nleaf);
size_t tqp_lcdf_train_workspace_bytes(int64_t total_keys, int sample_stride);
int tqp_lcdf_train(const tqp_col *cols, int ncols, int sample_stride, int nleaf, int steps,
                   float lr, void *model, size_t model_bytes, void *ws, size_t ws_bytes,
                   void *stream);
int tqp_lcdf_buckets(const void *model, const tqp_col *keys, int bucket_bits,
                     int32_t *out_bucket, void *stream);

/* ------------------------------------------------------------------------
 * tqp_partition_sort -- the same stable ascending sort as tqp_sort (same
 * out_key and out_rows bytes), by partitioning into 2^bucket_bits key-range
 * buckets (bucket_bits in [1, 24]; at most about 3000 keys per bucket on
 * average, so that windows of whole buckets fit the 8192-key LDS sort) and
 * sorting windows of whole buckets in LDS.
 *   mode TQP_PART_LEARNED: buckets from `model` (trained by tqp_lcdf_train);
 *   mode TQP_PART_RADIX:   buckets = top bucket_bits of key - key_min over
 *                          key_bits bits (key_bits 0 = derive on the device).
 *   in_rows  : optional row ids (NULL = positions); out_rows required.
 *   h_stats  : optional HOST array of 4: largest bucket, buckets sorted by
 *              the radix fallback, keys in them, single-valued large buckets.
 * Buckets of more than 8192 keys with distinct keys fall back to the radix
 * sort over their own key range (all of them gathered into one sort); if
 * more than 65536 buckets (the "part.ovf_cap" knob) overflow, the whole input
 * is sorted by the radix sort instead.  SYNCHRONIZES the stream
 * (to read the model's leaf count and the fallback list).  Workspace:
 * tqp_partition_sort_workspace_bytes.
 * ---------------------------------------------------------------------- */
#define TQP_PART_LEARNED 1u
#define TQP_PART_RADIX   2u
size_t tqp_partition_sort_workspace_bytes(int64_t n, int dtype, int bucket_bits);
int tqp_partition_sort(const tqp_col *key, const int32_t *in_rows, uint32_t mode,
                       const void *model, int bucket_bits, int key_bits, int64_t key_min,
                       const tqp_col *out_key, int32_t *out_rows, int64_t *h_stats,
                       void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TQP_H */
