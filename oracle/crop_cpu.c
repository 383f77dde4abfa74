/*
 * The paper's own method on the host CPU: a timing baseline for the
 * benchmark, not a checker.  It sits beside the oracle because it is test and
 * benchmark infrastructure; the product library never links it.  A CPU test
 * checks its output against the oracle's.
 *
 * Column-row parallel processing with N owner threads (Section 5, "Parallel
 * processing of entries" with Lemma 1 and its proof; Section 7 for
 * transactions):
 *   - owner t holds the partitions [t P / N, (t+1) P / N), i.e. the hash
 *     interval [q, r) of those partitions (Section 6, Theorem 1);
 *   - every owner reads every transaction, sorts its items by h_b, and for
 *     each item x takes the window of partners y whose h_b lies in
 *     [q - h_a(x), r - h_a(x)) mod 2^32 -- at most two runs of the sorted
 *     order because of the wrap -- keeping the pairs with x < y;
 *   - each owner accumulates its pairs in a private open-addressing table.
 * The result is, per partition, the exact support of every pair, which the
 * caller compares with the oracle.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sm_next(uint64_t *s)
{
    *s += 0x9e3779b97f4a7c15ULL;
    uint64_t z = *s;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint32_t mas(uint64_t a, uint64_t b, uint32_t x)
{
    return (uint32_t)((a * (uint64_t)x + b) >> 32);
}

typedef struct {
    uint64_t *key; /* (x << 32) | y, all ones when free */
    uint32_t *cnt;
    uint64_t mask, used;
    int shift; /* 64 - log2(slots): Fibonacci hashing takes the top bits */
} table_t;

typedef struct {
    const uint32_t *off, *items;
    uint64_t T;
    uint32_t P, p0, p1;
    uint64_t q, r; /* owned hash interval [q, r) */
    uint64_t aa, ba, ab, bb;
    table_t tab;
    uint64_t terms;
    int fail;
} owner_t;

static int tab_init(table_t *t, uint64_t want)
{
    uint64_t n = 1024;
    int lg = 10;
    while (n < 2 * want) {
        n <<= 1;
        ++lg;
    }
    t->shift = 64 - lg;
    t->key = (uint64_t *)malloc(n * sizeof(uint64_t));
    t->cnt = (uint32_t *)calloc(n, sizeof(uint32_t));
    if (!t->key || !t->cnt) return -1;
    memset(t->key, 0xFF, n * sizeof(uint64_t));
    t->mask = n - 1;
    t->used = 0;
    return 0;
}

static int tab_grow(table_t *t)
{
    table_t g;
    if (tab_init(&g, (t->mask + 1)) != 0) return -1;
    for (uint64_t s = 0; s <= t->mask; ++s) {
        if (t->key[s] == ~0ULL) continue;
        uint64_t h = (t->key[s] * 0x9E3779B97F4A7C15ULL) >> g.shift;
        while (g.key[h] != ~0ULL) h = (h + 1) & g.mask;
        g.key[h] = t->key[s];
        g.cnt[h] = t->cnt[s];
        ++g.used;
    }
    free(t->key);
    free(t->cnt);
    *t = g;
    return 0;
}

static inline int tab_add(table_t *t, uint64_t key)
{
    uint64_t h = (key * 0x9E3779B97F4A7C15ULL) >> t->shift;
    for (;;) {
        const uint64_t k = t->key[h];
        if (k == key) {
            ++t->cnt[h];
            return 0;
        }
        if (k == ~0ULL) {
            t->key[h] = key;
            t->cnt[h] = 1;
            if (++t->used * 2 > t->mask + 1) return tab_grow(t);
            return 0;
        }
        h = (h + 1) & t->mask;
    }
}

typedef struct { uint32_t hb, y; } hy_t;

/* insertion sort by h_b (transactions are short) */
static void sort_hy(hy_t *a, uint32_t n)
{
    for (uint32_t i = 1; i < n; ++i) {
        hy_t v = a[i];
        uint32_t j = i;
        while (j > 0 && a[j - 1].hb > v.hb) {
            a[j] = a[j - 1];
            --j;
        }
        a[j] = v;
    }
}

/* first index of sorted a[0..n) with hb >= v */
static inline uint32_t lower(const hy_t *a, uint32_t n, uint64_t v)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)a[mid].hb < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static void *owner_run(void *arg)
{
    owner_t *o = (owner_t *)arg;
    uint32_t cap = 64;
    hy_t *s = (hy_t *)malloc(cap * sizeof(hy_t));
    if (!s) { o->fail = 1; return NULL; }
    const uint64_t len = o->r - o->q; /* 1 .. 2^32 */
    for (uint64_t t = 0; t < o->T; ++t) {
        const uint32_t a0 = o->off[t], n = o->off[t + 1] - a0;
        if (n < 2) continue;
        if (n > cap) {
            cap = n;
            free(s);
            s = (hy_t *)malloc(cap * sizeof(hy_t));
            if (!s) { o->fail = 1; return NULL; }
        }
        for (uint32_t k = 0; k < n; ++k) {
            const uint32_t y = o->items[a0 + k];
            s[k].y = y;
            s[k].hb = mas(o->ab, o->bb, y);
        }
        sort_hy(s, n);
        for (uint32_t k = 0; k < n; ++k) {
            const uint32_t x = o->items[a0 + k];
            const uint32_t ha = mas(o->aa, o->ba, x);
            /* partners y with (ha + hb) mod 2^32 in [q, r): hb in
               [lo, lo + len) mod 2^32 with lo = (q - ha) mod 2^32 */
            const uint64_t lo = (o->q - ha) & 0xFFFFFFFFULL;
            const uint64_t hi = lo + len; /* may pass 2^32: then two runs */
            uint32_t runs[2][2];
            int nr = 0;
            if (hi <= (1ULL << 32)) {
                runs[nr][0] = lower(s, n, lo);
                runs[nr][1] = hi == (1ULL << 32) ? n : lower(s, n, hi);
                ++nr;
            } else {
                runs[nr][0] = lower(s, n, lo);
                runs[nr][1] = n;
                ++nr;
                runs[nr][0] = 0;
                runs[nr][1] = lower(s, n, hi - (1ULL << 32));
                ++nr;
            }
            for (int w = 0; w < nr; ++w)
                for (uint32_t i = runs[w][0]; i < runs[w][1]; ++i) {
                    const uint32_t y = s[i].y;
                    if (y <= x) continue;
                    ++o->terms;
                    if (tab_add(&o->tab, ((uint64_t)x << 32) | y) != 0) {
                        o->fail = 1;
                        free(s);
                        return NULL;
                    }
                }
        }
    }
    free(s);
    return NULL;
}

/*
 * Run the method with n_threads owners over P partitions.  Outputs (may be
 * NULL): part_sizes[P] distinct pairs and part_terms[P] terms per partition,
 * computed from each owner's table (a pair's partition is its hash's
 * interval).  Returns 0, or -1 when memory runs out.
 */
int cpu_crop_tx(const uint32_t *off, uint64_t T, const uint32_t *items, uint32_t P,
                uint64_t seed, uint32_t n_threads, uint64_t *part_sizes, uint64_t *part_terms,
                uint64_t *total_distinct)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > P) n_threads = P;
    uint64_t st = seed;
    const uint64_t aa = sm_next(&st), ba = sm_next(&st), ab = sm_next(&st), bb = sm_next(&st);
    owner_t *o = (owner_t *)calloc(n_threads, sizeof(owner_t));
    pthread_t *th = (pthread_t *)calloc(n_threads, sizeof(pthread_t));
    if (!o || !th) return -1;
    const uint64_t nnz = off[T];
    for (uint32_t t = 0; t < n_threads; ++t) {
        owner_t *w = &o[t];
        w->off = off;
        w->items = items;
        w->T = T;
        w->P = P;
        w->p0 = (uint32_t)(((uint64_t)P * t) / n_threads);
        w->p1 = (uint32_t)(((uint64_t)P * (t + 1)) / n_threads);
        /* partition p owns h with floor(h P / 2^32) = p: [ceil(p 2^32 / P), ...) */
        w->q = (((uint64_t)w->p0 << 32) + P - 1) / P;
        w->r = (((uint64_t)w->p1 << 32) + P - 1) / P;
        w->aa = aa; w->ba = ba; w->ab = ab; w->bb = bb;
        if (tab_init(&w->tab, nnz / n_threads + 1024) != 0) return -1;
    }
    for (uint32_t t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, owner_run, &o[t]);
    for (uint32_t t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    int rc = 0;
    uint64_t distinct = 0;
    if (part_sizes) memset(part_sizes, 0, P * sizeof(uint64_t));
    if (part_terms) memset(part_terms, 0, P * sizeof(uint64_t));
    for (uint32_t t = 0; t < n_threads; ++t) {
        owner_t *w = &o[t];
        if (w->fail) rc = -1;
        distinct += w->tab.used;
        if (part_sizes || part_terms)
            for (uint64_t s = 0; s <= w->tab.mask; ++s) {
                const uint64_t k = w->tab.key[s];
                if (k == ~0ULL) continue;
                const uint32_t h = mas(aa, ba, (uint32_t)(k >> 32)) + mas(ab, bb, (uint32_t)k);
                const uint32_t p = (uint32_t)(((uint64_t)h * P) >> 32);
                if (part_sizes) part_sizes[p] += 1;
                if (part_terms) part_terms[p] += w->tab.cnt[s];
            }
        free(w->tab.key);
        free(w->tab.cnt);
    }
    if (total_distinct) *total_distinct = distinct;
    free(o);
    free(th);
    return rc;
}
