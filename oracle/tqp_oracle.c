/*
 * tqp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU statement of what the relational hot
 * path computes: SQL WHERE over columnar tables (paper Section 2.1: one
 * (n x 1) tensor per numeric column), a stable ascending key sort, an inner
 * equi-join with bag semantics, and GROUP BY with SUM / COUNT (Section 2.3:
 * TPC-H Q6 is filters plus an aggregate, Q14 a join plus an aggregate; Fig. 4
 * a group-by aggregate).  Every result here has a plain definition, so each
 * function is that definition written out with loops, a hash table and the C
 * library's qsort -- no blocking, no fusion, nothing shared with the GPU
 * library.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load this file; the product path never does.
 *
 * Conventions fixed where the paper is silent:
 *  - filter output is ascending row id;
 *  - sort is stable and ascending on the signed integer value;
 *  - join output is every (i, j) with L[i] == R[j], ordered by (key, i, j);
 *  - group-by emits only groups that occur, in ascending key order;
 *  - SUM is int64 two's complement (mod 2^64); the exact sum is also kept in
 *    __int128 so a caller can see whether it ever left the int64 range.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { DT_I8 = 1, DT_I32 = 2, DT_I64 = 3 };
enum { OP_LT = 0, OP_LE = 1, OP_GT = 2, OP_GE = 3, OP_EQ = 4, OP_NE = 5 };
enum { AGG_SUM = 0, AGG_COUNT = 1, AGG_SUM_PRODUCT = 2, AGG_SUM_DIFF_PRODUCT = 3 };

static int64_t value_at(const void *col, int dtype, int64_t i)
{
    switch (dtype) {
    case DT_I8:  return ((const int8_t *)col)[i];
    case DT_I32: return ((const int32_t *)col)[i];
    default:     return ((const int64_t *)col)[i];
    }
}

static void store_at(void *col, int dtype, int64_t i, int64_t v)
{
    switch (dtype) {
    case DT_I8:  ((int8_t *)col)[i] = (int8_t)v; break;
    case DT_I32: ((int32_t *)col)[i] = (int32_t)v; break;
    default:     ((int64_t *)col)[i] = v; break;
    }
}

/* Mathematical comparison of two integers. */
static int holds(int64_t v, int op, int64_t lit)
{
    switch (op) {
    case OP_LT: return v < lit;
    case OP_LE: return v <= lit;
    case OP_GT: return v > lit;
    case OP_GE: return v >= lit;
    case OP_EQ: return v == lit;
    default:    return v != lit;
    }
}

/* ------------------------------------------------------------------------
 * WHERE: row i is kept when every predicate (column op literal) holds.
 * Returns the number of kept rows; writes their ids ascending.
 * ---------------------------------------------------------------------- */
int64_t orc_filter(int64_t n, const void *const *cols, const int *dtypes,
                   int npred, const int *pcol, const int *pop,
                   const int64_t *plit, int32_t *out_rows)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; i++) {
        int keep = 1;
        for (int p = 0; p < npred; p++)
            if (!holds(value_at(cols[pcol[p]], dtypes[pcol[p]], i), pop[p], plit[p]))
                keep = 0;
        if (keep)
            out_rows[cnt++] = (int32_t)i;
    }
    return cnt;
}

/* out[i] = src[idx[i]] */
void orc_gather(int64_t n, const void *src, int dtype, const int32_t *idx,
                void *out)
{
    for (int64_t i = 0; i < n; i++)
        store_at(out, dtype, i, value_at(src, dtype, idx[i]));
}

/* ------------------------------------------------------------------------
 * Stable ascending sort: order rows by (key, original position).  Sorting the
 * pairs lexicographically is the definition of a stable sort.
 * ---------------------------------------------------------------------- */
typedef struct { int64_t key; int64_t pos; } keypos;

static int cmp_keypos(const void *a, const void *b)
{
    const keypos *x = (const keypos *)a, *y = (const keypos *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
    return 0;
}

int orc_sort(int64_t n, const void *keys, int dtype, void *out_keys,
             int32_t *out_perm)
{
    keypos *kp = (keypos *)malloc((size_t)(n > 0 ? n : 1) * sizeof(keypos));
    if (!kp) return -1;
    for (int64_t i = 0; i < n; i++) {
        kp[i].key = value_at(keys, dtype, i);
        kp[i].pos = i;
    }
    qsort(kp, (size_t)n, sizeof(keypos), cmp_keypos);
    for (int64_t i = 0; i < n; i++) {
        if (out_keys) store_at(out_keys, dtype, i, kp[i].key);
        if (out_perm) out_perm[i] = (int32_t)kp[i].pos;
    }
    free(kp);
    return 0;
}

/* ------------------------------------------------------------------------
 * A plain open-addressing hash map from int64 key to a slot number.
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t *keys;
    int64_t *slot;      /* -1 = empty */
    uint64_t mask;
    uint64_t used;
} hmap;

static uint64_t mix(uint64_t x)
{
    /* Fibonacci hashing of the key followed by a xor-shift. */
    x *= 11400714819323198485ull;
    return x ^ (x >> 29);
}

static int hmap_init(hmap *h, int64_t expected)
{
    uint64_t cap = 16;
    while (cap < (uint64_t)expected * 2 + 16) cap <<= 1;
    h->keys = (int64_t *)malloc(cap * sizeof(int64_t));
    h->slot = (int64_t *)malloc(cap * sizeof(int64_t));
    if (!h->keys || !h->slot) return -1;
    for (uint64_t i = 0; i < cap; i++) h->slot[i] = -1;
    h->mask = cap - 1;
    h->used = 0;
    return 0;
}

static void hmap_free(hmap *h) { free(h->keys); free(h->slot); }

/* Returns the slot stored for key, or -1. */
static int64_t hmap_get(const hmap *h, int64_t key)
{
    uint64_t p = mix((uint64_t)key) & h->mask;
    while (h->slot[p] != -1) {
        if (h->keys[p] == key) return h->slot[p];
        p = (p + 1) & h->mask;
    }
    return -1;
}

static void hmap_insert_new(hmap *h, int64_t key, int64_t slot)
{
    uint64_t p = mix((uint64_t)key) & h->mask;
    while (h->slot[p] != -1) p = (p + 1) & h->mask;
    h->keys[p] = key;
    h->slot[p] = slot;
    h->used++;
}

/* Doubles the table when it is half full, so probing always ends. */
static void hmap_grow(hmap *h)
{
    hmap old = *h;
    uint64_t cap = (old.mask + 1) * 2;
    h->keys = (int64_t *)malloc(cap * sizeof(int64_t));
    h->slot = (int64_t *)malloc(cap * sizeof(int64_t));
    for (uint64_t i = 0; i < cap; i++) h->slot[i] = -1;
    h->mask = cap - 1;
    h->used = 0;
    for (uint64_t i = 0; i <= old.mask; i++)
        if (old.slot[i] != -1) hmap_insert_new(h, old.keys[i], old.slot[i]);
    hmap_free(&old);
}

/* Inserts key -> slot if absent; returns the slot stored for key. */
static int64_t hmap_put(hmap *h, int64_t key, int64_t slot)
{
    uint64_t p = mix((uint64_t)key) & h->mask;
    while (h->slot[p] != -1) {
        if (h->keys[p] == key) return h->slot[p];
        p = (p + 1) & h->mask;
    }
    if ((h->used + 1) * 2 > h->mask + 1) {
        hmap_grow(h);
        hmap_insert_new(h, key, slot);
        return slot;
    }
    h->keys[p] = key;
    h->slot[p] = slot;
    h->used++;
    return slot;
}

/* ------------------------------------------------------------------------
 * Semi-join: row i of the left table is kept when, for every set s, its key
 * keys[s][i] equals at least one of the set_n[s] keys of the other side
 * (setkeys[s]).  This is the relational definition of L semi-join R on an
 * equality, taken over several right sides at once (a conjunction).  Returns
 * the number of kept rows; writes their ids ascending.  Each right side is
 * put in a hash set first; lookups are exact integer comparisons.
 * ---------------------------------------------------------------------- */
int64_t orc_semijoin(int64_t n, int nsets, const void *const *keys, const int *dtypes,
                     const void *const *setkeys, const int *setdt, const int64_t *set_n,
                     int32_t *out_rows)
{
    hmap *h = (hmap *)malloc((size_t)(nsets > 0 ? nsets : 1) * sizeof(hmap));
    for (int s = 0; s < nsets; s++) {
        hmap_init(&h[s], set_n[s]);
        for (int64_t j = 0; j < set_n[s]; j++)
            hmap_put(&h[s], value_at(setkeys[s], setdt[s], j), j);
    }
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; i++) {
        int keep = 1;
        for (int s = 0; s < nsets && keep; s++)
            if (hmap_get(&h[s], value_at(keys[s], dtypes[s], i)) < 0)
                keep = 0;
        if (keep)
            out_rows[cnt++] = (int32_t)i;
    }
    for (int s = 0; s < nsets; s++) hmap_free(&h[s]);
    free(h);
    return cnt;
}

/* ------------------------------------------------------------------------
 * Inner equi-join, bag semantics, as a hash join: a chained hash table over R
 * (chains in ascending j), probed by every L row in order.  The pairs are then
 * put in the canonical order (key, i, j).  Returns the pair count; writes the
 * pairs only if they fit in cap.
 * ---------------------------------------------------------------------- */
typedef struct { int64_t key; int64_t i; int64_t j; } triple;

static int cmp_triple(const void *a, const void *b)
{
    const triple *x = (const triple *)a, *y = (const triple *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    return 0;
}

int64_t orc_join(int64_t nl, const void *lk, int64_t nr, const void *rk,
                 int dtype, int64_t cap, int32_t *out_l, int32_t *out_r)
{
    hmap h;
    int64_t *head, *next;
    if (hmap_init(&h, nr) != 0) return -1;
    head = (int64_t *)malloc((size_t)(nr + 1) * sizeof(int64_t));
    next = (int64_t *)malloc((size_t)(nr + 1) * sizeof(int64_t));
    int64_t ndist = 0;
    for (int64_t j = nr - 1; j >= 0; j--) {      /* push front: chains ascend */
        int64_t key = value_at(rk, dtype, j);
        int64_t s = hmap_put(&h, key, ndist);
        if (s == ndist) { head[s] = -1; ndist++; }
        next[j] = head[s];
        head[s] = j;
    }
    int64_t count = 0;
    for (int64_t i = 0; i < nl; i++) {
        int64_t s = hmap_get(&h, value_at(lk, dtype, i));
        if (s < 0) continue;
        for (int64_t j = head[s]; j != -1; j = next[j]) count++;
    }
    if (count <= cap && count > 0) {
        triple *t = (triple *)malloc((size_t)count * sizeof(triple));
        int64_t k = 0;
        for (int64_t i = 0; i < nl; i++) {
            int64_t key = value_at(lk, dtype, i);
            int64_t s = hmap_get(&h, key);
            if (s < 0) continue;
            for (int64_t j = head[s]; j != -1; j = next[j]) {
                t[k].key = key; t[k].i = i; t[k].j = j; k++;
            }
        }
        qsort(t, (size_t)count, sizeof(triple), cmp_triple);
        for (int64_t q = 0; q < count; q++) {
            out_l[q] = (int32_t)t[q].i;
            out_r[q] = (int32_t)t[q].j;
        }
        free(t);
    }
    free(head); free(next); hmap_free(&h);
    return count;
}

/* ------------------------------------------------------------------------
 * Join in ranges form.  For every key k present on both sides, ascending:
 *   lstart = #{i : L[i] < k}, lcnt = #{i : L[i] == k}, and the same for R.
 * These index the stably sorted sides.  *total = sum of lcnt * rcnt (exact
 * in __int128; *total_overflow set if it does not fit int64).
 * Returns the number of matched keys, writing at most cap of them.
 * ---------------------------------------------------------------------- */
typedef struct { int64_t key; int64_t cnt; } keycnt;

static int cmp_keycnt(const void *a, const void *b)
{
    const keycnt *x = (const keycnt *)a, *y = (const keycnt *)b;
    return x->key < y->key ? -1 : (x->key > y->key ? 1 : 0);
}

/* Distinct keys with multiplicities, ascending by key. */
static keycnt *histogram(int64_t n, const void *k, int dtype, int64_t *ndist)
{
    hmap h;
    keycnt *kc = (keycnt *)malloc((size_t)(n > 0 ? n : 1) * sizeof(keycnt));
    hmap_init(&h, n);
    int64_t d = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t key = value_at(k, dtype, i);
        int64_t s = hmap_put(&h, key, d);
        if (s == d) { kc[d].key = key; kc[d].cnt = 0; d++; }
        kc[s].cnt++;
    }
    hmap_free(&h);
    qsort(kc, (size_t)d, sizeof(keycnt), cmp_keycnt);
    *ndist = d;
    return kc;
}

int64_t orc_join_ranges(int64_t nl, const void *lk, int64_t nr, const void *rk,
                        int dtype, int64_t cap, int64_t *o_key,
                        int64_t *o_lstart, int64_t *o_lcnt, int64_t *o_rstart,
                        int64_t *o_rcnt, int64_t *total, int *total_overflow)
{
    int64_t dl, dr;
    keycnt *hl = histogram(nl, lk, dtype, &dl);
    keycnt *hr = histogram(nr, rk, dtype, &dr);
    /* rank of each distinct R key: number of R rows with a smaller key */
    hmap rpos;
    hmap_init(&rpos, dr);
    int64_t *rstart = (int64_t *)malloc((size_t)(dr + 1) * sizeof(int64_t));
    int64_t acc = 0;
    for (int64_t q = 0; q < dr; q++) {
        rstart[q] = acc;
        acc += hr[q].cnt;
        hmap_put(&rpos, hr[q].key, q);
    }
    __int128 tot = 0;
    int64_t m = 0, lacc = 0;
    for (int64_t q = 0; q < dl; q++) {
        int64_t s = hmap_get(&rpos, hl[q].key);
        if (s >= 0) {
            if (m < cap) {
                o_key[m] = hl[q].key;
                o_lstart[m] = lacc;
                o_lcnt[m] = hl[q].cnt;
                o_rstart[m] = rstart[s];
                o_rcnt[m] = hr[s].cnt;
            }
            tot += (__int128)hl[q].cnt * (__int128)hr[s].cnt;
            m++;
        }
        lacc += hl[q].cnt;
    }
    *total = (int64_t)tot;
    *total_overflow = (tot > (__int128)INT64_MAX);
    hmap_free(&rpos);
    free(rstart); free(hl); free(hr);
    return m;
}

/* ------------------------------------------------------------------------
 * GROUP BY key: per distinct key, each aggregate over its rows.
 *   AGG_SUM(a)          = sum of vals[a][i]
 *   AGG_COUNT           = number of rows
 *   AGG_SUM_PRODUCT(a,b)= sum of vals[a][i] * vals[b][i]
 *   AGG_SUM_DIFF_PRODUCT(a,b,c) = sum of vals[a][i] * (c - vals[b][i]), c a
 *                         constant (Q14's revenue, price * (100 - discount)
 *                         in cents and hundredths, Section 2.3)
 * Accumulated exactly in __int128; the stored int64 is the value mod 2^64.
 * *overflow is set if any exact value left the int64 range.
 * ---------------------------------------------------------------------- */
int64_t orc_groupby(int64_t n, const void *keys, int kdtype,
                    const void *const *vals, const int *vdtypes,
                    int nagg, const int *aop, const int *aa, const int *ab,
                    const int64_t *ac,
                    int64_t cap, int64_t *out_keys, int64_t *const *out_aggs,
                    int *overflow)
{
    hmap h;
    hmap_init(&h, n);
    int64_t *gkey = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    __int128 *acc = (__int128 *)calloc((size_t)(n > 0 ? n : 1) * (size_t)(nagg > 0 ? nagg : 1),
                                       sizeof(__int128));
    int64_t ng = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t key = value_at(keys, kdtype, i);
        int64_t g = hmap_put(&h, key, ng);
        if (g == ng) { gkey[g] = key; ng++; }
        for (int a = 0; a < nagg; a++) {
            __int128 v;
            if (aop[a] == AGG_COUNT) v = 1;
            else if (aop[a] == AGG_SUM) v = value_at(vals[aa[a]], vdtypes[aa[a]], i);
            else if (aop[a] == AGG_SUM_PRODUCT)
                v = (__int128)value_at(vals[aa[a]], vdtypes[aa[a]], i) *
                    (__int128)value_at(vals[ab[a]], vdtypes[ab[a]], i);
            else
                v = (__int128)value_at(vals[aa[a]], vdtypes[aa[a]], i) *
                    ((__int128)ac[a] - (__int128)value_at(vals[ab[a]], vdtypes[ab[a]], i));
            acc[g * nagg + a] += v;
        }
    }
    hmap_free(&h);
    /* ascending key order */
    keycnt *order = (keycnt *)malloc((size_t)(ng > 0 ? ng : 1) * sizeof(keycnt));
    for (int64_t g = 0; g < ng; g++) { order[g].key = gkey[g]; order[g].cnt = g; }
    qsort(order, (size_t)ng, sizeof(keycnt), cmp_keycnt);
    int ovf = 0;
    for (int64_t q = 0; q < ng; q++) {
        int64_t g = order[q].cnt;
        for (int a = 0; a < nagg; a++) {
            __int128 v = acc[g * nagg + a];
            if (v > (__int128)INT64_MAX || v < (__int128)INT64_MIN) ovf = 1;
        }
        if (q < cap) {
            out_keys[q] = order[q].key;
            for (int a = 0; a < nagg; a++)
                out_aggs[a][q] = (int64_t)(uint64_t)(unsigned __int128)acc[g * nagg + a];
        }
    }
    *overflow = ovf;
    free(order); free(gkey); free(acc);
    return ng;
}

/* ------------------------------------------------------------------------
 * Whole queries, written directly as nested loops with hash lookups rather
 * than composed from the operator functions above: a second, structurally
 * different statement of the same results.
 * ---------------------------------------------------------------------- */

/* Chained index over a dimension's primary-key column (bag semantics). */
typedef struct { hmap h; int64_t *head; int64_t *next; } dimindex;

static void dimindex_build(dimindex *d, int64_t n, const int32_t *pk)
{
    hmap_init(&d->h, n);
    d->head = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    d->next = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int64_t nd = 0;
    for (int64_t j = n - 1; j >= 0; j--) {
        int64_t s = hmap_put(&d->h, pk[j], nd);
        if (s == nd) { d->head[s] = -1; nd++; }
        d->next[j] = d->head[s];
        d->head[s] = j;
    }
}

static void dimindex_free(dimindex *d) { hmap_free(&d->h); free(d->head); free(d->next); }

/* Group accumulator keyed by int64, up to three exact sums. */
typedef struct { hmap h; int64_t *key; __int128 *s; int64_t ng; int64_t cap; } groups;

static void groups_init(groups *g, int64_t expected)
{
    hmap_init(&g->h, expected);
    g->cap = expected + 1;
    g->key = (int64_t *)malloc((size_t)g->cap * sizeof(int64_t));
    g->s = (__int128 *)calloc((size_t)g->cap * 3, sizeof(__int128));
    g->ng = 0;
}

static void groups_add(groups *g, int64_t key, __int128 a, __int128 b, __int128 c)
{
    int64_t s = hmap_put(&g->h, key, g->ng);
    if (s == g->ng) {
        if (g->ng == g->cap) {               /* grow the group arrays */
            int64_t nc = g->cap * 2;
            g->key = (int64_t *)realloc(g->key, (size_t)nc * sizeof(int64_t));
            g->s = (__int128 *)realloc(g->s, (size_t)nc * 3 * sizeof(__int128));
            memset(g->s + 3 * g->cap, 0, (size_t)(nc - g->cap) * 3 * sizeof(__int128));
            g->cap = nc;
        }
        g->key[s] = key;
        g->ng++;
    }
    g->s[3 * s] += a; g->s[3 * s + 1] += b; g->s[3 * s + 2] += c;
}

/* Emits groups ascending by key; returns group count, sets *ovf. */
static int64_t groups_emit(groups *g, int64_t cap, int64_t *okey, int64_t *o0,
                           int64_t *o1, int64_t *o2, int *ovf)
{
    keycnt *order = (keycnt *)malloc((size_t)(g->ng > 0 ? g->ng : 1) * sizeof(keycnt));
    for (int64_t q = 0; q < g->ng; q++) { order[q].key = g->key[q]; order[q].cnt = q; }
    qsort(order, (size_t)g->ng, sizeof(keycnt), cmp_keycnt);
    for (int64_t q = 0; q < g->ng; q++) {
        int64_t s = order[q].cnt;
        for (int a = 0; a < 3; a++) {
            __int128 v = g->s[3 * s + a];
            if (v > (__int128)INT64_MAX || v < (__int128)INT64_MIN) *ovf = 1;
        }
        if (q < cap) {
            okey[q] = order[q].key;
            if (o0) o0[q] = (int64_t)(uint64_t)(unsigned __int128)g->s[3 * s];
            if (o1) o1[q] = (int64_t)(uint64_t)(unsigned __int128)g->s[3 * s + 1];
            if (o2) o2[q] = (int64_t)(uint64_t)(unsigned __int128)g->s[3 * s + 2];
        }
    }
    free(order);
    return g->ng;
}

static void groups_free(groups *g) { hmap_free(&g->h); free(g->key); free(g->s); }

/* Q1: SELECT cat, SUM(qty), COUNT(*) FROM fact JOIN dim ON fk = pk
 *     WHERE day < day_cut GROUP BY cat ORDER BY cat. */
int64_t orc_q1(int64_t nf, const int32_t *fk, const int64_t *qty,
               const int32_t *day, int64_t day_cut, int64_t nd,
               const int32_t *pk, const int32_t *cat, int64_t cap,
               int64_t *o_cat, int64_t *o_sum, int64_t *o_cnt, int *ovf)
{
    dimindex d;
    groups g;
    dimindex_build(&d, nd, pk);
    groups_init(&g, nd > 0 ? nd : 1);
    for (int64_t i = 0; i < nf; i++) {
        if (!((int64_t)day[i] < day_cut)) continue;
        int64_t s = hmap_get(&d.h, fk[i]);
        if (s < 0) continue;
        for (int64_t j = d.head[s]; j != -1; j = d.next[j])
            groups_add(&g, cat[j], qty[i], 1, 0);
    }
    *ovf = 0;
    int64_t ng = groups_emit(&g, cap, o_cat, o_sum, o_cnt, NULL, ovf);
    groups_free(&g); dimindex_free(&d);
    return ng;
}

/* Q2 (skewed star): rows = fact JOIN dim ON fk = pk WHERE day < day_cut;
 *  (a) GROUP BY flag * 2 + (cat mod 2): SUM(qty), SUM(price), COUNT(*)
 *  (b) GROUP BY fk: SUM(qty), COUNT(*).
 * Both outputs ascending by key.  Returns (a)'s group count in *nga and
 * (b)'s in *ngb. */
int orc_q2(int64_t nf, const int32_t *fk, const int64_t *qty,
           const int64_t *price, const int8_t *flag, const int32_t *day,
           int64_t day_cut, int64_t nd, const int32_t *pk, const int32_t *cat,
           int64_t capa, int64_t *a_key, int64_t *a_qty, int64_t *a_price,
           int64_t *a_cnt, int64_t *nga,
           int64_t capb, int64_t *b_key, int64_t *b_qty, int64_t *b_cnt,
           int64_t *ngb, int *ovf)
{
    dimindex d;
    groups ga, gb;
    dimindex_build(&d, nd, pk);
    groups_init(&ga, 64);
    groups_init(&gb, nd > 0 ? nd : 1);
    for (int64_t i = 0; i < nf; i++) {
        if (!((int64_t)day[i] < day_cut)) continue;
        int64_t s = hmap_get(&d.h, fk[i]);
        if (s < 0) continue;
        for (int64_t j = d.head[s]; j != -1; j = d.next[j]) {
            int64_t c = cat[j];
            int64_t cm = ((c % 2) + 2) % 2;
            groups_add(&ga, (int64_t)flag[i] * 2 + cm, qty[i], price[i], 1);
            groups_add(&gb, fk[i], qty[i], 1, 0);
        }
    }
    *ovf = 0;
    *nga = groups_emit(&ga, capa, a_key, a_qty, a_price, a_cnt, ovf);
    *ngb = groups_emit(&gb, capb, b_key, b_qty, b_cnt, NULL, ovf);
    groups_free(&ga); groups_free(&gb); dimindex_free(&d);
    return 0;
}

/* Q3 (star join over three dims, each filtered by attr < attr_cut):
 *   GROUP BY d1.cat * 5 + d2.cat: SUM(qty * price), COUNT(*). */
int64_t orc_q3(int64_t nf, const int32_t *fk1, const int32_t *fk2,
               const int32_t *fk3, const int64_t *qty, const int64_t *price,
               int64_t n1, const int32_t *pk1, const int32_t *cat1, const int32_t *attr1,
               int64_t n2, const int32_t *pk2, const int32_t *cat2, const int32_t *attr2,
               int64_t n3, const int32_t *pk3, const int32_t *attr3,
               int64_t attr_cut, int64_t cap, int64_t *o_key, int64_t *o_sum,
               int64_t *o_cnt, int *ovf)
{
    dimindex d1, d2, d3;
    groups g;
    dimindex_build(&d1, n1, pk1);
    dimindex_build(&d2, n2, pk2);
    dimindex_build(&d3, n3, pk3);
    groups_init(&g, 256);
    for (int64_t i = 0; i < nf; i++) {
        int64_t s3 = hmap_get(&d3.h, fk3[i]);
        if (s3 < 0) continue;
        for (int64_t j3 = d3.head[s3]; j3 != -1; j3 = d3.next[j3]) {
            if (!((int64_t)attr3[j3] < attr_cut)) continue;
            int64_t s2 = hmap_get(&d2.h, fk2[i]);
            if (s2 < 0) continue;
            for (int64_t j2 = d2.head[s2]; j2 != -1; j2 = d2.next[j2]) {
                if (!((int64_t)attr2[j2] < attr_cut)) continue;
                int64_t s1 = hmap_get(&d1.h, fk1[i]);
                if (s1 < 0) continue;
                for (int64_t j1 = d1.head[s1]; j1 != -1; j1 = d1.next[j1]) {
                    if (!((int64_t)attr1[j1] < attr_cut)) continue;
                    groups_add(&g, (int64_t)cat1[j1] * 5 + cat2[j2],
                               (__int128)qty[i] * (__int128)price[i], 1, 0);
                }
            }
        }
    }
    *ovf = 0;
    int64_t ng = groups_emit(&g, cap, o_key, o_sum, o_cnt, NULL, ovf);
    groups_free(&g);
    dimindex_free(&d1); dimindex_free(&d2); dimindex_free(&d3);
    return ng;
}

/* ------------------------------------------------------------------------
 * WHERE + aggregate without materialising the kept rows (the shape of TPC-H
 * Q6, Section 2.3: filters over columns of different types, then one
 * aggregate): over the rows where every predicate holds,
 *   *sum   = SUM(a[i] * b[i])  (b NULL: SUM(a[i]); a NULL: 0), mod 2^64,
 *   *count = COUNT(*).
 * *exact receives 1 when the exact sum (kept in __int128, the products too)
 * stays inside int64, 0 otherwise.
 * ---------------------------------------------------------------------- */
void orc_filter_sum(int64_t n, const void *const *cols, const int *dtypes,
                    int npred, const int *pcol, const int *pop,
                    const int64_t *plit, const void *a, int adt,
                    const void *b, int bdt, int64_t *sum, int64_t *count,
                    int *exact)
{
    __int128 s = 0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; i++) {
        int keep = 1;
        for (int p = 0; p < npred; p++)
            if (!holds(value_at(cols[pcol[p]], dtypes[pcol[p]], i), pop[p], plit[p]))
                keep = 0;
        if (!keep) continue;
        cnt++;
        if (a) {
            __int128 t = value_at(a, adt, i);
            if (b) t *= value_at(b, bdt, i);
            s += t;
        }
    }
    *sum = (int64_t)(uint64_t)(unsigned __int128)s;
    *count = cnt;
    *exact = s >= INT64_MIN && s <= INT64_MAX;
}

/* Q6-shaped query, written directly:
 *   SELECT SUM(price * discount), COUNT(*) FROM items
 *   WHERE ship >= ship_lo AND ship < ship_hi
 *     AND discount >= disc_lo AND discount <= disc_hi AND quantity < qty_cut
 * ship: int64 epoch nanoseconds; discount: int8 hundredths; quantity: int32;
 * price: int64 cents.  The sum is exact (asserted by *exact as above). */
void orc_q6(int64_t n, const int64_t *ship, const int8_t *discount,
            const int32_t *quantity, const int64_t *price, int64_t ship_lo,
            int64_t ship_hi, int64_t disc_lo, int64_t disc_hi, int64_t qty_cut,
            int64_t *sum, int64_t *count, int *exact)
{
    __int128 s = 0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; i++) {
        if (ship[i] < ship_lo || ship[i] >= ship_hi) continue;
        if (discount[i] < disc_lo || discount[i] > disc_hi) continue;
        if (!(quantity[i] < qty_cut)) continue;
        s += (__int128)price[i] * discount[i];
        cnt++;
    }
    *sum = (int64_t)(uint64_t)(unsigned __int128)s;
    *count = cnt;
    *exact = s >= INT64_MIN && s <= INT64_MAX;
}

/* ------------------------------------------------------------------------
 * Strings are the paper's (n x m) tensor of UTF-8 bytes, one row per value,
 * zero-padded to m (Section 2.1).  LIKE 'p%' holds when the row's first plen
 * bytes are p (mode 0); = 'p' when they are and the rest of the row is
 * padding (mode 1).  out[i] is 1 or 0.
 * ---------------------------------------------------------------------- */
void orc_str_match(int64_t n, int m, const uint8_t *chars, const uint8_t *pat,
                   int plen, int mode, int8_t *out)
{
    for (int64_t i = 0; i < n; i++) {
        const uint8_t *row = chars + i * (int64_t)m;
        int ok = plen <= m && memcmp(row, pat, (size_t)plen) == 0;
        if (ok && mode == 1)
            for (int j = plen; j < m; j++)
                if (row[j] != 0) ok = 0;
        out[i] = (int8_t)ok;
    }
}

/* Q14-shaped query, written directly:
 *   SELECT SUM(CASE WHEN type LIKE 'prefix%' THEN price * (100 - discount)
 *              ELSE 0 END), SUM(price * (100 - discount)), COUNT(*)
 *   FROM items JOIN part ON partkey = pk
 *   WHERE ship >= ship_lo AND ship < ship_hi
 * Revenue is in cents x hundredths; sums exact in __int128 (*exact says they
 * fit int64) and wrapped mod 2^64. */
void orc_q14(int64_t ni, const int64_t *ship, const int32_t *partkey,
             const int64_t *price, const int8_t *discount, int64_t ship_lo,
             int64_t ship_hi, int64_t np, const int32_t *pk, int m,
             const uint8_t *types, const uint8_t *prefix, int plen,
             int64_t *promo_rev, int64_t *total_rev, int64_t *count,
             int64_t *promo_count, int *exact)
{
    dimindex d;
    dimindex_build(&d, np, pk);
    __int128 promo = 0, total = 0;
    int64_t cnt = 0, pcnt = 0;
    for (int64_t i = 0; i < ni; i++) {
        if (ship[i] < ship_lo || ship[i] >= ship_hi) continue;
        int64_t s = hmap_get(&d.h, partkey[i]);
        if (s < 0) continue;
        for (int64_t j = d.head[s]; j != -1; j = d.next[j]) {
            __int128 rev = (__int128)price[i] * (100 - (int64_t)discount[i]);
            total += rev;
            cnt++;
            if (plen <= m && memcmp(types + j * (int64_t)m, prefix, (size_t)plen) == 0) {
                promo += rev;
                pcnt++;
            }
        }
    }
    dimindex_free(&d);
    *promo_rev = (int64_t)(uint64_t)(unsigned __int128)promo;
    *total_rev = (int64_t)(uint64_t)(unsigned __int128)total;
    *count = cnt;
    *promo_count = pcnt;
    *exact = total >= INT64_MIN && total <= INT64_MAX && promo >= INT64_MIN && promo <= INT64_MAX;
}

/* ------------------------------------------------------------------------
 * PREDICT inside a query (Section 3.3's prediction query: a model scores each
 * row and a group-by with a CASE compares predictions with ratings).  The
 * model is an MLP with one ReLU hidden layer in fp32:
 *   h[j]  = relu(b1[j] + sum_k W1[j][k] * x[k])     (k ascending)
 *   z[c]  = b2[c] + sum_j W2[c][j] * h[j]            (j ascending)
 *   class = the first c with the largest z[c]
 * Every multiply-add is one fused fmaf, in the order written, and relu(v) is
 * (v > 0 ? v : 0), so a kernel taking the same steps reaches the same class.
 * model = [W1 (H x F, row-major), b1 (H), W2 (C x H), b2 (C)].
 * x[k] is the k-th feature column of row rows[i] (rows NULL: row i),
 * converted to float.
 * ---------------------------------------------------------------------- */
#include <math.h>

static int mlp_class(const float *model, int F, int H, int C, const float *x)
{
    const float *w1 = model, *b1 = w1 + H * F, *w2 = b1 + H, *b2 = w2 + C * H;
    float h[256], best = 0.0f;
    int arg = 0;
    for (int j = 0; j < H; j++) {
        float acc = b1[j];
        for (int k = 0; k < F; k++) acc = fmaf(w1[j * F + k], x[k], acc);
        h[j] = acc > 0.0f ? acc : 0.0f;
    }
    for (int c = 0; c < C; c++) {
        float acc = b2[c];
        for (int j = 0; j < H; j++) acc = fmaf(w2[c * H + j], h[j], acc);
        if (c == 0 || acc > best) { best = acc; arg = c; }
    }
    return arg;
}

void orc_mlp_predict(int64_t n, const void *const *feats, const int *dtypes, int F,
                     const int32_t *rows, const float *model, int H, int C, int8_t *out)
{
    float x[64];
    for (int64_t i = 0; i < n; i++) {
        const int64_t r = rows ? rows[i] : i;
        for (int k = 0; k < F; k++) x[k] = (float)value_at(feats[k], dtypes[k], r);
        out[i] = (int8_t)mlp_class(model, F, H, C, x);
    }
}

/* The prediction query, written directly over the whole table:
 *   SELECT rating, SUM(CASE WHEN PREDICT(model, f) = 1 THEN 1 ELSE 0 END), COUNT(*)
 *   FROM reviews WHERE year >= year_min GROUP BY rating
 * out_pos[r], out_cnt[r] for ratings r in [0, nr). */
void orc_q_predict(int64_t n, const int8_t *rating, const int32_t *year, int64_t year_min,
                   const int32_t *const *feats, int F, const float *model, int H, int C,
                   int nr, int64_t *out_pos, int64_t *out_cnt)
{
    float x[64];
    for (int r = 0; r < nr; r++) out_pos[r] = out_cnt[r] = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!(year[i] >= year_min)) continue;
        for (int k = 0; k < F; k++) x[k] = (float)feats[k][i];
        const int cls = mlp_class(model, F, H, C, x);
        const int r = rating[i];
        if (r < 0 || r >= nr) continue;
        out_cnt[r]++;
        if (cls == 1) out_pos[r]++;
    }
}

/* ------------------------------------------------------------------------
 * The same whole queries on several host threads: the CPU-baseline leg
 * that times the oracle on every core of the host.  Each thread runs the
 * loop body of orc_q1 / orc_q2 / orc_q3 above over its own contiguous share
 * of the fact rows into its own group accumulator; the accumulators are then
 * added group by group (sums of __int128 values, so the merge order changes
 * nothing) and emitted as before.  The parity checker is the single-thread
 * function; these are checked against it.
 * ---------------------------------------------------------------------- */
#include <omp.h>

int orc_max_threads(void) { return omp_get_max_threads(); }

static void groups_merge(groups *dst, const groups *src)
{
    for (int64_t q = 0; q < src->ng; q++)
        groups_add(dst, src->key[q], src->s[3 * q], src->s[3 * q + 1], src->s[3 * q + 2]);
}

int64_t orc_q1_mt(int threads, int64_t nf, const int32_t *fk, const int64_t *qty,
                  const int32_t *day, int64_t day_cut, int64_t nd,
                  const int32_t *pk, const int32_t *cat, int64_t cap,
                  int64_t *o_cat, int64_t *o_sum, int64_t *o_cnt, int *ovf)
{
    dimindex d;
    dimindex_build(&d, nd, pk);
    groups *gt = (groups *)calloc((size_t)threads, sizeof(groups));
#pragma omp parallel num_threads(threads)
    {
        groups *g = &gt[omp_get_thread_num()];
        groups_init(g, 64);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nf; i++) {
            if (!((int64_t)day[i] < day_cut)) continue;
            int64_t s = hmap_get(&d.h, fk[i]);
            if (s < 0) continue;
            for (int64_t j = d.head[s]; j != -1; j = d.next[j])
                groups_add(g, cat[j], qty[i], 1, 0);
        }
    }
    groups all;
    groups_init(&all, 64);
    for (int t = 0; t < threads; t++) {
        if (gt[t].cap) { groups_merge(&all, &gt[t]); groups_free(&gt[t]); }
    }
    free(gt);
    *ovf = 0;
    int64_t ng = groups_emit(&all, cap, o_cat, o_sum, o_cnt, NULL, ovf);
    groups_free(&all); dimindex_free(&d);
    return ng;
}

int orc_q2_mt(int threads, int64_t nf, const int32_t *fk, const int64_t *qty,
              const int64_t *price, const int8_t *flag, const int32_t *day,
              int64_t day_cut, int64_t nd, const int32_t *pk, const int32_t *cat,
              int64_t capa, int64_t *a_key, int64_t *a_qty, int64_t *a_price,
              int64_t *a_cnt, int64_t *nga,
              int64_t capb, int64_t *b_key, int64_t *b_qty, int64_t *b_cnt,
              int64_t *ngb, int *ovf)
{
    dimindex d;
    dimindex_build(&d, nd, pk);
    groups *ga = (groups *)calloc((size_t)threads, sizeof(groups));
    groups *gb = (groups *)calloc((size_t)threads, sizeof(groups));
#pragma omp parallel num_threads(threads)
    {
        const int t = omp_get_thread_num();
        groups_init(&ga[t], 64);
        groups_init(&gb[t], 1 << 16);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nf; i++) {
            if (!((int64_t)day[i] < day_cut)) continue;
            int64_t s = hmap_get(&d.h, fk[i]);
            if (s < 0) continue;
            for (int64_t j = d.head[s]; j != -1; j = d.next[j]) {
                int64_t c = cat[j];
                int64_t cm = ((c % 2) + 2) % 2;
                groups_add(&ga[t], (int64_t)flag[i] * 2 + cm, qty[i], price[i], 1);
                groups_add(&gb[t], fk[i], qty[i], 1, 0);
            }
        }
    }
    groups a, b;
    groups_init(&a, 64);
    groups_init(&b, nd > 0 ? nd : 1);
    for (int t = 0; t < threads; t++) {
        if (ga[t].cap) { groups_merge(&a, &ga[t]); groups_free(&ga[t]); }
        if (gb[t].cap) { groups_merge(&b, &gb[t]); groups_free(&gb[t]); }
    }
    free(ga); free(gb);
    *ovf = 0;
    *nga = groups_emit(&a, capa, a_key, a_qty, a_price, a_cnt, ovf);
    *ngb = groups_emit(&b, capb, b_key, b_qty, b_cnt, NULL, ovf);
    groups_free(&a); groups_free(&b); dimindex_free(&d);
    return 0;
}

int64_t orc_q3_mt(int threads, int64_t nf, const int32_t *fk1, const int32_t *fk2,
                  const int32_t *fk3, const int64_t *qty, const int64_t *price,
                  int64_t n1, const int32_t *pk1, const int32_t *cat1, const int32_t *attr1,
                  int64_t n2, const int32_t *pk2, const int32_t *cat2, const int32_t *attr2,
                  int64_t n3, const int32_t *pk3, const int32_t *attr3,
                  int64_t attr_cut, int64_t cap, int64_t *o_key, int64_t *o_sum,
                  int64_t *o_cnt, int *ovf)
{
    dimindex d1, d2, d3;
    dimindex_build(&d1, n1, pk1);
    dimindex_build(&d2, n2, pk2);
    dimindex_build(&d3, n3, pk3);
    groups *gt = (groups *)calloc((size_t)threads, sizeof(groups));
#pragma omp parallel num_threads(threads)
    {
        groups *g = &gt[omp_get_thread_num()];
        groups_init(g, 256);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nf; i++) {
            int64_t s3 = hmap_get(&d3.h, fk3[i]);
            if (s3 < 0) continue;
            for (int64_t j3 = d3.head[s3]; j3 != -1; j3 = d3.next[j3]) {
                if (!((int64_t)attr3[j3] < attr_cut)) continue;
                int64_t s2 = hmap_get(&d2.h, fk2[i]);
                if (s2 < 0) continue;
                for (int64_t j2 = d2.head[s2]; j2 != -1; j2 = d2.next[j2]) {
                    if (!((int64_t)attr2[j2] < attr_cut)) continue;
                    int64_t s1 = hmap_get(&d1.h, fk1[i]);
                    if (s1 < 0) continue;
                    for (int64_t j1 = d1.head[s1]; j1 != -1; j1 = d1.next[j1]) {
                        if (!((int64_t)attr1[j1] < attr_cut)) continue;
                        groups_add(g, (int64_t)cat1[j1] * 5 + cat2[j2],
                                   (__int128)qty[i] * (__int128)price[i], 1, 0);
                    }
                }
            }
        }
    }
    groups all;
    groups_init(&all, 256);
    for (int t = 0; t < threads; t++) {
        if (gt[t].cap) { groups_merge(&all, &gt[t]); groups_free(&gt[t]); }
    }
    free(gt);
    *ovf = 0;
    int64_t ng = groups_emit(&all, cap, o_key, o_sum, o_cnt, NULL, ovf);
    groups_free(&all);
    dimindex_free(&d1); dimindex_free(&d2); dimindex_free(&d3);
    return ng;
}
