/*
 * Oracle for the hash-partition + hash-join hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU definition of what the GPU library computes.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant with the GPU library, and the GPU library
 * never calls it.
 *
 * What the method computes (arXiv 2101.08878, Section V-B "cuDF Merge" and
 * the caption of the RI2 cuDF figure: every Dask worker shuffles both data
 * frames on the join key -- "Shuffle: True" -- and then merges the frames it
 * received):
 *
 *   1. partition: every row of a table goes to destination
 *      p = fmix64(key) mod P; each destination's rows are packed together.
 *      The paper does not name the hash; this library fixes it to the 64-bit
 *      finalizer of MurmurHash3 (Appleby, public domain), and rows keep their
 *      input order inside a destination (so the result is unique).
 *   2. join: an inner equi-join of the left and right tables on the key, with
 *      multiset semantics (every pair of equal-key rows is one output row).
 *      Output rows are (key, left payload, right payload).
 *
 * Everything is integer: keys are int64 (int32 keys are sign-extended to
 * int64 before hashing and comparing), payloads int64, the hash uint64 with
 * arithmetic mod 2^64, counts and offsets int64.
 *
 * Pins (see tests/test_oracle_pins.py): the SMHasher verification value of
 * MurmurHash3_x64_128 (which uses fmix64 as its finalizer), bijectivity and
 * fmix64(0) = 0; numpy's stable argsort for the partition; nested-loop brute
 * force and pandas.merge for the join; closed-form cardinalities.
 */
#define _POSIX_C_SOURCE 200809L /* pthread barriers under -std=c11 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ---- step 1a: the hash -------------------------------------------------- */

/* MurmurHash3 fmix64: xor-shift by 33, multiply, xor-shift, multiply,
 * xor-shift.  All operations mod 2^64. */
uint64_t oracle_fmix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

/* The destination of one key: fmix64 of the key's two's-complement bits,
 * unsigned 64-bit remainder by P. */
int32_t oracle_partition_of(int64_t key, int32_t P)
{
    return (int32_t)(oracle_fmix64((uint64_t)key) % (uint64_t)P);
}

static int64_t key_at(const void *keys, int32_t key_bytes, int64_t i)
{
    if (key_bytes == 4)
        return (int64_t)((const int32_t *)keys)[i]; /* sign-extend */
    return ((const int64_t *)keys)[i];
}

static void key_put(void *keys, int32_t key_bytes, int64_t i, int64_t k)
{
    if (key_bytes == 4)
        ((int32_t *)keys)[i] = (int32_t)k;
    else
        ((int64_t *)keys)[i] = k;
}

/* ---- step 1b: the partition (stable counting sort) ---------------------- */

/* Counting sort of the rows by destination (textbook, e.g. CLRS 8.2):
 *   count rows per destination; off = exclusive prefix sum of the counts;
 *   walk the rows in input order and place row i at cur[p(i)]++.
 * Destination p ends up in [off[p], off[p+1]) of both output columns, rows in
 * input order.  off has P+1 entries.  Returns 0, or -1 on bad arguments. */
int32_t oracle_hash_partition(const void *keys, int32_t key_bytes, const int64_t *payload,
                              int64_t n, int32_t P, void *keys_out, int64_t *payload_out,
                              int64_t *off)
{
    if (n < 0 || P < 1 || (key_bytes != 4 && key_bytes != 8))
        return -1;
    int64_t *cnt = calloc((size_t)P, sizeof(int64_t));
    int64_t *cur = malloc((size_t)P * sizeof(int64_t));
    if (!cnt || !cur) {
        free(cnt);
        free(cur);
        return -1;
    }
    for (int64_t i = 0; i < n; i++)
        cnt[oracle_partition_of(key_at(keys, key_bytes, i), P)]++;
    off[0] = 0;
    for (int32_t p = 0; p < P; p++)
        off[p + 1] = off[p] + cnt[p];
    memcpy(cur, off, (size_t)P * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        int64_t k = key_at(keys, key_bytes, i);
        int64_t j = cur[oracle_partition_of(k, P)]++;
        key_put(keys_out, key_bytes, j, k);
        payload_out[j] = payload[i];
    }
    free(cnt);
    free(cur);
    return 0;
}

/* ---- step 2: the join (sort-merge) -------------------------------------- */

typedef struct {
    int64_t k, v;
} kv_t;

static int cmp_kv(const void *a, const void *b)
{
    const kv_t *x = a, *y = b;
    if (x->k != y->k)
        return x->k < y->k ? -1 : 1;
    if (x->v != y->v)
        return x->v < y->v ? -1 : 1;
    return 0;
}

typedef struct {
    int64_t l, r, k;
} lrk_t;

static int cmp_lrk(const void *a, const void *b)
{
    const lrk_t *x = a, *y = b;
    if (x->l != y->l)
        return x->l < y->l ? -1 : 1;
    if (x->r != y->r)
        return x->r < y->r ? -1 : 1;
    if (x->k != y->k)
        return x->k < y->k ? -1 : 1;
    return 0;
}

static kv_t *sorted_pairs(const void *keys, int32_t key_bytes, const int64_t *payload, int64_t n)
{
    kv_t *a = malloc((size_t)(n > 0 ? n : 1) * sizeof(kv_t));
    if (!a)
        return NULL;
    for (int64_t i = 0; i < n; i++) {
        a[i].k = key_at(keys, key_bytes, i);
        a[i].v = payload ? payload[i] : i;
    }
    qsort(a, (size_t)n, sizeof(kv_t), cmp_kv);
    return a;
}

/* Inner join of L and R on the key by sort-merge:
 *   sort both sides by (key, payload); walk them together; for every key
 *   present on both sides emit the full cross product of its left run and its
 *   right run as (key, left payload, right payload).
 * If the output fits (|J| <= cap) the rows are written sorted by
 * (left payload, right payload, key) -- the canonical order used to compare
 * against any other implementation, whose row order is free.
 * If the output does not fit, nothing is written.
 * per_part (optional, P entries) receives the output count of every
 * destination p = fmix64(key) mod P.
 * Returns |J|, or -1 on bad arguments / allocation failure. */
int64_t oracle_join(const void *lkeys, const int64_t *lpay, int64_t nl,
                    const void *rkeys, const int64_t *rpay, int64_t nr, int32_t key_bytes,
                    int64_t *out_key, int64_t *out_lpay, int64_t *out_rpay, int64_t cap,
                    int32_t P, int64_t *per_part)
{
    if (nl < 0 || nr < 0 || (key_bytes != 4 && key_bytes != 8) || (per_part && P < 1))
        return -1;
    kv_t *L = sorted_pairs(lkeys, key_bytes, lpay, nl);
    kv_t *R = sorted_pairs(rkeys, key_bytes, rpay, nr);
    if (!L || !R) {
        free(L);
        free(R);
        return -1;
    }
    if (per_part)
        memset(per_part, 0, (size_t)P * sizeof(int64_t));

    /* First walk: the cardinality. */
    int64_t total = 0;
    for (int64_t i = 0, j = 0; i < nl && j < nr;) {
        if (L[i].k < R[j].k) {
            i++;
        } else if (L[i].k > R[j].k) {
            j++;
        } else {
            int64_t k = L[i].k, i2 = i, j2 = j;
            while (i2 < nl && L[i2].k == k)
                i2++;
            while (j2 < nr && R[j2].k == k)
                j2++;
            total += (i2 - i) * (j2 - j);
            if (per_part)
                per_part[oracle_partition_of(k, P)] += (i2 - i) * (j2 - j);
            i = i2;
            j = j2;
        }
    }

    /* Second walk: the rows, if they fit. */
    if (out_key && out_lpay && out_rpay && total <= cap && total > 0) {
        lrk_t *o = malloc((size_t)total * sizeof(lrk_t));
        if (!o) {
            free(L);
            free(R);
            return -1;
        }
        int64_t w = 0;
        for (int64_t i = 0, j = 0; i < nl && j < nr;) {
            if (L[i].k < R[j].k) {
                i++;
            } else if (L[i].k > R[j].k) {
                j++;
            } else {
                int64_t k = L[i].k, i2 = i, j2 = j;
                while (i2 < nl && L[i2].k == k)
                    i2++;
                while (j2 < nr && R[j2].k == k)
                    j2++;
                for (int64_t a = i; a < i2; a++)
                    for (int64_t b = j; b < j2; b++) {
                        o[w].l = L[a].v;
                        o[w].r = R[b].v;
                        o[w].k = k;
                        w++;
                    }
                i = i2;
                j = j2;
            }
        }
        qsort(o, (size_t)total, sizeof(lrk_t), cmp_lrk);
        for (int64_t t = 0; t < total; t++) {
            out_key[t] = o[t].k;
            out_lpay[t] = o[t].l;
            out_rpay[t] = o[t].r;
        }
        free(o);
    }
    free(L);
    free(R);
    return total;
}

/* For every right row j: the number of left rows with the same key,
 * cL(kR[j]) -- the number of output rows that right row produces.
 * Sort the left keys, then two binary searches per right row.
 * Returns 0, or -1 on bad arguments. */
int32_t oracle_match_counts(const void *lkeys, int64_t nl, const void *rkeys, int64_t nr,
                            int32_t key_bytes, int64_t *counts)
{
    if (nl < 0 || nr < 0 || (key_bytes != 4 && key_bytes != 8))
        return -1;
    kv_t *L = sorted_pairs(lkeys, key_bytes, NULL, nl);
    if (!L)
        return -1;
    for (int64_t j = 0; j < nr; j++) {
        int64_t k = key_at(rkeys, key_bytes, j);
        int64_t lo = 0, hi = nl; /* first index with key >= k */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (L[mid].k < k)
                lo = mid + 1;
            else
                hi = mid;
        }
        int64_t a = lo;
        hi = nl; /* first index with key > k */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (L[mid].k <= k)
                lo = mid + 1;
            else
                hi = mid;
        }
        counts[j] = lo - a;
    }
    free(L);
    return 0;
}

/* ---- the same two steps over several host threads (CPU baseline) -------- */

/* What the benchmark times beside the GPU: the partition and the join above,
 * spread over T host threads, with the same result.
 *
 * Partition, per table: the rows are cut into T contiguous blocks; thread b
 * counts its block's rows per destination; the first position of
 * (destination p, block b) is off[p] plus the rows of p in the blocks before
 * b -- the counting sort's prefix taken in (destination, block) order; then
 * thread b places its block's rows in input order.  Every row lands where the
 * one-thread counting sort puts it, so the partitions are identical.
 *
 * Join: destination p of the left table is joined with destination p of the
 * right table (equal keys share a destination) by the sort-merge above, one
 * destination at a time per thread: a walk that counts, a prefix over the
 * destinations, and a walk that writes destination p's rows at
 * [out_off[p], out_off[p+1]) in the walk's order (the canonical order is for
 * comparisons only and is not produced here).  If |J| > cap, only out_off is
 * written.  Returns |J|, or -1 on bad arguments or allocation failure. */

#include <pthread.h>
#include <stdatomic.h>

typedef struct {
    const void *keys;
    const int64_t *pay;
    int64_t n;
    void *keys_out;
    int64_t *pay_out;
    int64_t *off;  /* [P + 1] */
    int64_t *cnt;  /* [T][P]: rows of destination p in block b */
    int64_t *base; /* [T][P]: first position of (p, b) */
} ptab_t;

typedef struct {
    ptab_t tab[2]; /* left, right */
    int32_t key_bytes, P, T;
    kv_t **Ls, **Rs;   /* [P]: destination p's pairs, sorted */
    int64_t *nLs, *nRs;
    int64_t *jcnt;     /* [P]: |J_p| */
    int64_t *out_off;  /* [P + 1] */
    int64_t *out_key, *out_lpay, *out_rpay, cap;
    atomic_int next_sort, next_write, failed;
    pthread_barrier_t bar;
} pmerge_t;

typedef struct {
    pmerge_t *m;
    int32_t b;
} pworker_t;

static void ptab_count(const pmerge_t *m, ptab_t *t, int32_t b)
{
    const int64_t lo = t->n * b / m->T, hi = t->n * (b + 1) / m->T;
    int64_t *c = t->cnt + (int64_t)b * m->P;
    for (int32_t p = 0; p < m->P; p++)
        c[p] = 0;
    for (int64_t i = lo; i < hi; i++)
        c[oracle_partition_of(key_at(t->keys, m->key_bytes, i), m->P)]++;
}

/* One thread: destination offsets and the (destination, block) bases. */
static void ptab_bases(const pmerge_t *m, ptab_t *t)
{
    int64_t run = 0;
    for (int32_t p = 0; p < m->P; p++) {
        t->off[p] = run;
        for (int32_t b = 0; b < m->T; b++) {
            t->base[(int64_t)b * m->P + p] = run;
            run += t->cnt[(int64_t)b * m->P + p];
        }
    }
    t->off[m->P] = run;
}

static void ptab_place(const pmerge_t *m, ptab_t *t, int32_t b)
{
    const int64_t lo = t->n * b / m->T, hi = t->n * (b + 1) / m->T;
    int64_t *cur = t->base + (int64_t)b * m->P;
    for (int64_t i = lo; i < hi; i++) {
        const int64_t k = key_at(t->keys, m->key_bytes, i);
        const int64_t j = cur[oracle_partition_of(k, m->P)]++;
        key_put(t->keys_out, m->key_bytes, j, k);
        t->pay_out[j] = t->pay[i];
    }
}

/* Destination p's (key, payload) pairs of a partitioned table, sorted. */
static kv_t *ptab_pairs(const pmerge_t *m, const ptab_t *t, int32_t p, int64_t *cnt)
{
    const int64_t a = t->off[p], e = t->off[p + 1];
    kv_t *x = malloc((size_t)(e > a ? e - a : 1) * sizeof(kv_t));
    if (!x)
        return NULL;
    for (int64_t i = a; i < e; i++) {
        x[i - a].k = key_at(t->keys_out, m->key_bytes, i);
        x[i - a].v = t->pay_out[i];
    }
    qsort(x, (size_t)(e - a), sizeof(kv_t), cmp_kv);
    *cnt = e - a;
    return x;
}

/* Sort-merge walk of one destination: counts (w == NULL) or writes at w. */
static int64_t pjoin_walk(const kv_t *L, int64_t nl, const kv_t *R, int64_t nr, int64_t *ok,
                          int64_t *ol, int64_t *orr)
{
    int64_t w = 0;
    for (int64_t i = 0, j = 0; i < nl && j < nr;) {
        if (L[i].k < R[j].k) {
            i++;
        } else if (L[i].k > R[j].k) {
            j++;
        } else {
            const int64_t k = L[i].k;
            int64_t i2 = i, j2 = j;
            while (i2 < nl && L[i2].k == k)
                i2++;
            while (j2 < nr && R[j2].k == k)
                j2++;
            if (ok) {
                for (int64_t a = i; a < i2; a++)
                    for (int64_t b = j; b < j2; b++) {
                        ok[w] = k;
                        ol[w] = L[a].v;
                        orr[w] = R[b].v;
                        w++;
                    }
            } else {
                w += (i2 - i) * (j2 - j);
            }
            i = i2;
            j = j2;
        }
    }
    return w;
}

static void *pmerge_worker(void *arg)
{
    const pworker_t *wk = arg;
    pmerge_t *m = wk->m;
    const int32_t b = wk->b;
    ptab_count(m, &m->tab[0], b);
    ptab_count(m, &m->tab[1], b);
    pthread_barrier_wait(&m->bar);
    if (b == 0) {
        ptab_bases(m, &m->tab[0]);
        ptab_bases(m, &m->tab[1]);
    }
    pthread_barrier_wait(&m->bar);
    ptab_place(m, &m->tab[0], b);
    ptab_place(m, &m->tab[1], b);
    pthread_barrier_wait(&m->bar);
    for (int p; (p = atomic_fetch_add(&m->next_sort, 1)) < m->P;) {
        m->Ls[p] = ptab_pairs(m, &m->tab[0], p, &m->nLs[p]);
        m->Rs[p] = ptab_pairs(m, &m->tab[1], p, &m->nRs[p]);
        if (!m->Ls[p] || !m->Rs[p]) {
            atomic_store(&m->failed, 1);
            m->jcnt[p] = 0;
            continue;
        }
        m->jcnt[p] = pjoin_walk(m->Ls[p], m->nLs[p], m->Rs[p], m->nRs[p], NULL, NULL, NULL);
    }
    pthread_barrier_wait(&m->bar);
    if (b == 0) {
        int64_t run = 0;
        for (int32_t p = 0; p < m->P; p++) {
            m->out_off[p] = run;
            run += m->jcnt[p];
        }
        m->out_off[m->P] = run;
    }
    pthread_barrier_wait(&m->bar);
    const int fits = m->out_key && m->out_lpay && m->out_rpay && m->out_off[m->P] <= m->cap &&
                     !atomic_load(&m->failed);
    for (int p; (p = atomic_fetch_add(&m->next_write, 1)) < m->P;) {
        if (fits) {
            const int64_t o = m->out_off[p];
            pjoin_walk(m->Ls[p], m->nLs[p], m->Rs[p], m->nRs[p], m->out_key + o, m->out_lpay + o,
                       m->out_rpay + o);
        }
        free(m->Ls[p]);
        free(m->Rs[p]);
        m->Ls[p] = m->Rs[p] = NULL;
    }
    return NULL;
}

int64_t oracle_merge_threads(const void *lkeys, const int64_t *lpay, int64_t nl,
                             const void *rkeys, const int64_t *rpay, int64_t nr,
                             int32_t key_bytes, int32_t P, int32_t threads, void *lk_out,
                             int64_t *lv_out, int64_t *loff, void *rk_out, int64_t *rv_out,
                             int64_t *roff, int64_t *out_key, int64_t *out_lpay,
                             int64_t *out_rpay, int64_t cap, int64_t *out_off)
{
    if (nl < 0 || nr < 0 || P < 1 || threads < 1 || threads > 1024 ||
        (key_bytes != 4 && key_bytes != 8) || !loff || !roff || !out_off)
        return -1;
    pmerge_t *m = calloc(1, sizeof(pmerge_t));
    pthread_t *th = calloc((size_t)threads, sizeof(pthread_t));
    pworker_t *wk = calloc((size_t)threads, sizeof(pworker_t));
    int64_t *cnt = calloc((size_t)4 * threads * P, sizeof(int64_t));
    int64_t *per = calloc((size_t)3 * P, sizeof(int64_t));
    kv_t **lists = calloc((size_t)2 * P, sizeof(kv_t *));
    int64_t result = -1;
    if (!m || !th || !wk || !cnt || !per || !lists)
        goto done;
    m->key_bytes = key_bytes;
    m->P = P;
    m->T = threads;
    const ptab_t L = {lkeys, lpay, nl, lk_out, lv_out, loff, cnt, cnt + (int64_t)threads * P};
    const ptab_t R = {rkeys, rpay, nr, rk_out, rv_out, roff, cnt + 2 * (int64_t)threads * P,
                      cnt + 3 * (int64_t)threads * P};
    m->tab[0] = L;
    m->tab[1] = R;
    m->Ls = lists;
    m->Rs = lists + P;
    m->nLs = per;
    m->nRs = per + P;
    m->jcnt = per + 2 * (int64_t)P;
    m->out_off = out_off;
    m->out_key = out_key;
    m->out_lpay = out_lpay;
    m->out_rpay = out_rpay;
    m->cap = cap;
    atomic_init(&m->next_sort, 0);
    atomic_init(&m->next_write, 0);
    atomic_init(&m->failed, 0);
    if (pthread_barrier_init(&m->bar, NULL, (unsigned)threads) != 0)
        goto done;
    int32_t started = 0;
    for (; started < threads; started++) {
        wk[started].m = m;
        wk[started].b = started;
        if (pthread_create(&th[started], NULL, pmerge_worker, &wk[started]) != 0)
            break;
    }
    if (started < threads) {
        /* the barrier waits for every thread: without all of them none ends */
        fputs("oracle_merge_threads: pthread_create failed\n", stderr);
        abort();
    }
    for (int32_t t = 0; t < threads; t++)
        pthread_join(th[t], NULL);
    pthread_barrier_destroy(&m->bar);
    result = atomic_load(&m->failed) ? -1 : out_off[P];
done:
    free(m);
    free(th);
    free(wk);
    free(cnt);
    free(per);
    free(lists);
    return result;
}
