/*
 * CPU oracle for the column-row parallel (CRoP) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the GPU library: the hash
 * specification below is written here a second time, on purpose.
 *
 * Every routine is the plain definition of what it computes, written for a
 * reader to check against the paper by eye: double loops, a library sort,
 * linear scans.  No blocking, no fusion, no reordering beyond the definition.
 *
 * Floating point: products of fp32 inputs are formed in fp64 (exact, since a
 * 24x24-bit significand product fits in 53 bits) and summed in fp64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------
 * Hash specification.
 *
 * Section 5 (proof of Lemma 1): the distribution hash of an entry (i,j) is
 * h(i,j) = (h_a(i) + h_b(j)) mod kappa with h_a, h_b pairwise independent.
 * The paper leaves the family open (its implementation filled tables from a
 * random number generator, Section 7.3).  Reading used here, with
 * kappa = 2^32:
 *   seed -> (alpha_a, beta_a, alpha_b, beta_b) = first four outputs of
 *           SplitMix64 started at state = seed (Steele, Lea, Flood 2014);
 *   h_a(x) = ((alpha_a * x + beta_a) mod 2^64) >> 32, likewise h_b, which is
 *           the multiply-add-shift strongly universal family (Dietzfelbinger
 *           1996) for 32-bit keys;
 *   part(h)      = (h * P) >> 32          (P owners, equal intervals: Thm 1)
 *   bucket(h)    = (h * P * B) >> 32      (P*B summaries; part = bucket / B)
 *   sign(i,j)    = +1 or -1 from the top bit of (g_a(i) + g_b(j)) mod 2^32
 *                  where g_a, g_b use SplitMix64 outputs five to eight.
 * ---------------------------------------------------------------------- */

static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* prm[0..3] = alpha_a, beta_a, alpha_b, beta_b; prm[4..7] the sign hash. */
void orc_hash_params(uint64_t seed, uint64_t prm[8])
{
    uint64_t st = seed;
    for (int k = 0; k < 8; ++k)
        prm[k] = splitmix64_next(&st);
}

void orc_splitmix64(uint64_t seed, uint64_t *out, uint64_t n)
{
    uint64_t st = seed;
    for (uint64_t k = 0; k < n; ++k)
        out[k] = splitmix64_next(&st);
}

static uint32_t mas(uint64_t alpha, uint64_t beta, uint32_t x)
{
    return (uint32_t)((alpha * (uint64_t)x + beta) >> 32);
}

uint32_t orc_ha(const uint64_t prm[8], uint32_t x) { return mas(prm[0], prm[1], x); }
uint32_t orc_hb(const uint64_t prm[8], uint32_t y) { return mas(prm[2], prm[3], y); }

uint32_t orc_h(const uint64_t prm[8], uint32_t x, uint32_t y)
{
    return orc_ha(prm, x) + orc_hb(prm, y); /* mod 2^32 by uint32 wrap */
}

int orc_sign(const uint64_t prm[8], uint32_t x, uint32_t y)
{
    uint32_t g = mas(prm[4], prm[5], x) + mas(prm[6], prm[7], y);
    return (g >> 31) ? -1 : 1;
}

uint32_t orc_part(uint32_t h, uint32_t P)
{
    return (uint32_t)(((uint64_t)h * (uint64_t)P) >> 32);
}

uint32_t orc_bucket(uint32_t h, uint32_t P, uint32_t B)
{
    /* P*B <= 2^32 is required by the caller; the product fits in 64 bits */
    return (uint32_t)(((uint64_t)h * (uint64_t)P * (uint64_t)B) >> 32);
}

/* Element-wise hashes of many ids (for tests). */
void orc_hash_many(uint64_t seed, const uint32_t *x, const uint32_t *y, uint64_t n,
                   uint32_t P, uint32_t *ha, uint32_t *hb, uint32_t *h, uint32_t *part)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    for (uint64_t k = 0; k < n; ++k) {
        if (ha) ha[k] = orc_ha(prm, x[k]);
        if (hb) hb[k] = orc_hb(prm, y[k]);
        uint32_t hh = orc_h(prm, x[k], y[k]);
        if (h) h[k] = hh;
        if (part) part[k] = orc_part(hh, P);
    }
}

/* ------------------------------------------------------------------------
 * Terms.
 *
 * Transactions (Section 7, case study): a transaction is a {0,1} vector v_T
 * and its pairs are the nonzero entries above the diagonal of v_T v_T^T; the
 * entry is keyed (x, y) with x < y and hashed as h_a(x) + h_b(y).
 *
 * Outer products (Section 4, notation): entry (i,j) of the product has
 * weight sum_k a_k(i) b_k(j); each stored pair (a_k(i), b_k(j)) is one term,
 * also when a stored value is 0.0.
 * ---------------------------------------------------------------------- */

uint64_t orc_tx_num_terms(const uint32_t *off, uint64_t T)
{
    uint64_t s = 0;
    for (uint64_t t = 0; t < T; ++t) {
        uint64_t L = (uint64_t)off[t + 1] - off[t];
        s += L ? L * (L - 1) / 2 : 0;
    }
    return s;
}

uint64_t orc_op_num_terms(const uint32_t *a_off, const uint32_t *b_off, uint64_t K)
{
    uint64_t s = 0;
    for (uint64_t k = 0; k < K; ++k)
        s += ((uint64_t)a_off[k + 1] - a_off[k]) * ((uint64_t)b_off[k + 1] - b_off[k]);
    return s;
}

typedef struct { uint32_t part, x, y; } tx_rec;

static int cmp_tx(const void *pa, const void *pb)
{
    const tx_rec *a = (const tx_rec *)pa, *b = (const tx_rec *)pb;
    if (a->part != b->part) return a->part < b->part ? -1 : 1;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    return 0;
}

/*
 * Exact pair supports, grouped by partition (plain definition).
 *
 * Every term (x,y) with hash h in [q, r) is listed; records are sorted by
 * (partition, x, y) with qsort and equal keys are counted.  Output:
 *   part_sizes[P]  distinct keys per partition
 *   part_terms[P]  terms per partition
 *   out_x/out_y/out_cnt  distinct keys in (partition, x, y) order
 * cap must be at least the number of listed terms.  Returns 0 on success,
 * -1 on allocation failure, -2 if cap is too small.
 */
int orc_tx_exact(const uint32_t *off, uint64_t T, const uint32_t *items,
                 uint32_t P, uint64_t seed, uint64_t q, uint64_t r,
                 uint64_t *part_sizes, uint64_t *part_terms,
                 uint32_t *out_x, uint32_t *out_y, uint32_t *out_cnt,
                 uint64_t cap, uint64_t *n_out)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    uint64_t nt = orc_tx_num_terms(off, T);
    tx_rec *rec = (tx_rec *)malloc((nt ? nt : 1) * sizeof(tx_rec));
    if (!rec) return -1;
    uint64_t m = 0;
    for (uint64_t t = 0; t < T; ++t)
        for (uint64_t a = off[t]; a < off[t + 1]; ++a)
            for (uint64_t b = a + 1; b < off[t + 1]; ++b) {
                uint32_t x = items[a] < items[b] ? items[a] : items[b];
                uint32_t y = items[a] < items[b] ? items[b] : items[a];
                uint32_t h = orc_h(prm, x, y);
                if ((uint64_t)h < q || (uint64_t)h >= r) continue;
                rec[m].part = orc_part(h, P);
                rec[m].x = x;
                rec[m].y = y;
                ++m;
            }
    qsort(rec, m, sizeof(tx_rec), cmp_tx);
    for (uint32_t p = 0; p < P; ++p) { part_sizes[p] = 0; part_terms[p] = 0; }
    uint64_t d = 0;
    for (uint64_t k = 0; k < m; ++k) {
        part_terms[rec[k].part] += 1;
        if (k > 0 && cmp_tx(&rec[k], &rec[k - 1]) == 0) {
            out_cnt[d - 1] += 1;
            continue;
        }
        if (d >= cap) { free(rec); return -2; }
        out_x[d] = rec[k].x;
        out_y[d] = rec[k].y;
        out_cnt[d] = 1;
        part_sizes[rec[k].part] += 1;
        ++d;
    }
    *n_out = d;
    free(rec);
    return 0;
}

typedef struct { uint32_t part, i, j; uint32_t k; double v; } op_rec;

static int cmp_op(const void *pa, const void *pb)
{
    const op_rec *a = (const op_rec *)pa, *b = (const op_rec *)pb;
    if (a->part != b->part) return a->part < b->part ? -1 : 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    return 0;
}

/*
 * Exact entry weights of C = sum_k a_k b_k^T, grouped by partition.
 * out_sum = sum_k a_k(i) b_k(j) and out_abs = sum_k |a_k(i) b_k(j)|, both
 * fp64, summed in k order.  Same conventions as orc_tx_exact.
 */
int orc_op_exact(const uint32_t *a_off, const uint32_t *a_idx, const float *a_val,
                 const uint32_t *b_off, const uint32_t *b_idx, const float *b_val,
                 uint64_t K, uint32_t P, uint64_t seed, uint64_t q, uint64_t r,
                 uint64_t *part_sizes, uint64_t *part_terms,
                 uint32_t *out_i, uint32_t *out_j, double *out_sum, double *out_abs,
                 uint32_t *out_nterms, uint64_t cap, uint64_t *n_out)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    uint64_t nt = orc_op_num_terms(a_off, b_off, K);
    op_rec *rec = (op_rec *)malloc((nt ? nt : 1) * sizeof(op_rec));
    if (!rec) return -1;
    uint64_t m = 0;
    for (uint64_t k = 0; k < K; ++k)
        for (uint64_t a = a_off[k]; a < a_off[k + 1]; ++a)
            for (uint64_t b = b_off[k]; b < b_off[k + 1]; ++b) {
                uint32_t h = orc_h(prm, a_idx[a], b_idx[b]);
                if ((uint64_t)h < q || (uint64_t)h >= r) continue;
                rec[m].part = orc_part(h, P);
                rec[m].i = a_idx[a];
                rec[m].j = b_idx[b];
                rec[m].k = (uint32_t)k;
                rec[m].v = (double)a_val[a] * (double)b_val[b];
                ++m;
            }
    qsort(rec, m, sizeof(op_rec), cmp_op);
    for (uint32_t p = 0; p < P; ++p) { part_sizes[p] = 0; part_terms[p] = 0; }
    uint64_t d = 0;
    for (uint64_t k = 0; k < m; ++k) {
        part_terms[rec[k].part] += 1;
        if (k > 0 && rec[k].part == rec[k - 1].part && rec[k].i == rec[k - 1].i &&
            rec[k].j == rec[k - 1].j) {
            out_sum[d - 1] += rec[k].v;
            out_abs[d - 1] += fabs(rec[k].v);
            out_nterms[d - 1] += 1;
            continue;
        }
        if (d >= cap) { free(rec); return -2; }
        out_i[d] = rec[k].i;
        out_j[d] = rec[k].j;
        out_sum[d] = rec[k].v;
        out_abs[d] = fabs(rec[k].v);
        out_nterms[d] = 1;
        part_sizes[rec[k].part] += 1;
        ++d;
    }
    *n_out = d;
    free(rec);
    return 0;
}

/* ------------------------------------------------------------------------
 * Space-Saving, one summary of ell slots per bucket (Section 4, frequent
 * items mining; Figure 1 updates the summary of bucket h(e) with entry e).
 *
 * Weighted update of entry e with weight w > 0 (the weighted form the paper
 * points to for positive updates), with these readings of what the paper
 * leaves open:
 *   - e monitored:            cnt += w
 *   - else a free slot:       the lowest free slot becomes (e, w, 0)
 *   - else:                   the unpinned slot of minimum cnt (lowest slot
 *                             index among equal minima) becomes
 *                             (e, cnt_min + w, cnt_min)
 * Updates are applied in the stream order: transactions in order, pairs of a
 * transaction in (x, y) lexicographic order; outer products in (k, i, j)
 * order.  Pinned slots (learned seeding) hold a given entry from the start
 * with cnt = err = 0 and are never evicted.
 *
 * State arrays are bucket-major, ell slots per bucket:
 *   key_x, key_y  entry of the slot
 *   used          1 if the slot holds an entry
 *   pinned        1 if the slot is pinned
 *   cnt, err      count and overestimation (double; integers in {0,1} mode)
 *   val           signed sum since admission (outer products only)
 * ---------------------------------------------------------------------- */

typedef struct {
    uint32_t ell;
    uint32_t *kx, *ky;
    uint8_t *used, *pinned;
    double *cnt, *err, *val;
} ss_state;

static void ss_update(ss_state *S, uint64_t bucket, uint32_t x, uint32_t y,
                      double w, double v)
{
    uint64_t base = bucket * S->ell;
    for (uint32_t s = 0; s < S->ell; ++s) {
        uint64_t k = base + s;
        if (S->used[k] && S->kx[k] == x && S->ky[k] == y) {
            S->cnt[k] += w;
            if (S->val) S->val[k] += v;
            return;
        }
    }
    for (uint32_t s = 0; s < S->ell; ++s) {
        uint64_t k = base + s;
        if (!S->used[k]) {
            S->used[k] = 1;
            S->kx[k] = x;
            S->ky[k] = y;
            S->cnt[k] = w;
            S->err[k] = 0.0;
            if (S->val) S->val[k] = v;
            return;
        }
    }
    int64_t m = -1;
    for (uint32_t s = 0; s < S->ell; ++s) {
        uint64_t k = base + s;
        if (S->pinned[k]) continue;
        if (m < 0 || S->cnt[k] < S->cnt[(uint64_t)m]) m = (int64_t)k;
    }
    if (m < 0) return; /* every slot pinned: the entry stays unmonitored */
    S->kx[m] = x;
    S->ky[m] = y;
    S->err[m] = S->cnt[m];
    S->cnt[m] = S->cnt[m] + w;
    if (S->val) S->val[m] = v;
}

/*
 * Pin seeds: seeds are taken in the given order; a seed is pinned into the
 * lowest free slot of its bucket while that bucket has fewer than r_max
 * pinned slots, otherwise it is skipped.  Returns the number pinned.
 */
static uint64_t ss_pin(ss_state *S, const uint64_t prm[8], uint32_t P, uint32_t B,
                       const uint32_t *sx, const uint32_t *sy, uint64_t ns, uint32_t r_max)
{
    uint64_t pinned = 0;
    for (uint64_t s = 0; s < ns; ++s) {
        uint64_t bucket = orc_bucket(orc_h(prm, sx[s], sy[s]), P, B);
        uint64_t base = bucket * S->ell;
        uint32_t npin = 0;
        int dup = 0;
        for (uint32_t k = 0; k < S->ell; ++k) {
            if (S->pinned[base + k]) {
                ++npin;
                if (S->kx[base + k] == sx[s] && S->ky[base + k] == sy[s]) dup = 1;
            }
        }
        if (dup || npin >= r_max) continue;
        for (uint32_t k = 0; k < S->ell; ++k) {
            if (!S->used[base + k]) {
                S->used[base + k] = 1;
                S->pinned[base + k] = 1;
                S->kx[base + k] = sx[s];
                S->ky[base + k] = sy[s];
                S->cnt[base + k] = 0.0;
                S->err[base + k] = 0.0;
                if (S->val) S->val[base + k] = 0.0;
                ++pinned;
                break;
            }
        }
    }
    return pinned;
}

static void ss_clear(ss_state *S, uint64_t nslots)
{
    memset(S->used, 0, nslots);
    memset(S->pinned, 0, nslots);
    for (uint64_t k = 0; k < nslots; ++k) {
        S->kx[k] = 0; S->ky[k] = 0; S->cnt[k] = 0.0; S->err[k] = 0.0;
        if (S->val) S->val[k] = 0.0;
    }
}

/*
 * Transactions into P*B Space-Saving summaries of ell slots each, unit
 * weights, canonical stream order.  Optional seeds (sx, sy, ns) are pinned
 * first with at most r_max per bucket.  Output arrays hold P*B*ell slots.
 */
uint64_t orc_tx_spacesaving(const uint32_t *off, uint64_t T, const uint32_t *items,
                            uint64_t seed, uint32_t P, uint32_t B, uint32_t ell,
                            const uint32_t *sx, const uint32_t *sy, uint64_t ns, uint32_t r_max,
                            uint32_t *kx, uint32_t *ky, uint8_t *used, uint8_t *pinned,
                            double *cnt, double *err)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    ss_state S = { ell, kx, ky, used, pinned, cnt, err, NULL };
    uint64_t nslots = (uint64_t)P * B * ell;
    ss_clear(&S, nslots);
    uint64_t npin = ns ? ss_pin(&S, prm, P, B, sx, sy, ns, r_max) : 0;
    for (uint64_t t = 0; t < T; ++t)
        for (uint64_t a = off[t]; a < off[t + 1]; ++a)
            for (uint64_t b = a + 1; b < off[t + 1]; ++b) {
                uint32_t x = items[a] < items[b] ? items[a] : items[b];
                uint32_t y = items[a] < items[b] ? items[b] : items[a];
                uint64_t bucket = orc_bucket(orc_h(prm, x, y), P, B);
                ss_update(&S, bucket, x, y, 1.0, 0.0);
            }
    return npin;
}

/*
 * Outer products into P*B summaries: weight |a_k(i) b_k(j)| (fp64) and the
 * signed sum of the terms since the entry's admission in val.
 */
void orc_op_spacesaving(const uint32_t *a_off, const uint32_t *a_idx, const float *a_val,
                        const uint32_t *b_off, const uint32_t *b_idx, const float *b_val,
                        uint64_t K, uint64_t seed, uint32_t P, uint32_t B, uint32_t ell,
                        uint32_t *kx, uint32_t *ky, uint8_t *used, uint8_t *pinned,
                        double *cnt, double *err, double *val)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    ss_state S = { ell, kx, ky, used, pinned, cnt, err, val };
    ss_clear(&S, (uint64_t)P * B * ell);
    for (uint64_t k = 0; k < K; ++k)
        for (uint64_t a = a_off[k]; a < a_off[k + 1]; ++a)
            for (uint64_t b = b_off[k]; b < b_off[k + 1]; ++b) {
                double v = (double)a_val[a] * (double)b_val[b];
                uint64_t bucket = orc_bucket(orc_h(prm, a_idx[a], b_idx[b]), P, B);
                ss_update(&S, bucket, a_idx[a], b_idx[b], fabs(v), v);
            }
}

/* ------------------------------------------------------------------------
 * Count-Sketch, one estimator per bucket (Section 4 and Figure 1: the
 * estimator of bucket h(e) receives the entry's weight times its sign).
 * cs must hold P*B doubles; it is overwritten.
 * ---------------------------------------------------------------------- */
void orc_tx_countsketch(const uint32_t *off, uint64_t T, const uint32_t *items,
                        uint64_t seed, uint32_t P, uint32_t B, double *cs)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    for (uint64_t k = 0; k < (uint64_t)P * B; ++k) cs[k] = 0.0;
    for (uint64_t t = 0; t < T; ++t)
        for (uint64_t a = off[t]; a < off[t + 1]; ++a)
            for (uint64_t b = a + 1; b < off[t + 1]; ++b) {
                uint32_t x = items[a] < items[b] ? items[a] : items[b];
                uint32_t y = items[a] < items[b] ? items[b] : items[a];
                uint64_t bucket = orc_bucket(orc_h(prm, x, y), P, B);
                cs[bucket] += (double)orc_sign(prm, x, y);
            }
}

void orc_op_countsketch(const uint32_t *a_off, const uint32_t *a_idx, const float *a_val,
                        const uint32_t *b_off, const uint32_t *b_idx, const float *b_val,
                        uint64_t K, uint64_t seed, uint32_t P, uint32_t B, double *cs)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    for (uint64_t k = 0; k < (uint64_t)P * B; ++k) cs[k] = 0.0;
    for (uint64_t k = 0; k < K; ++k)
        for (uint64_t a = a_off[k]; a < a_off[k + 1]; ++a)
            for (uint64_t b = b_off[k]; b < b_off[k + 1]; ++b) {
                double v = (double)a_val[a] * (double)b_val[b];
                uint64_t bucket = orc_bucket(orc_h(prm, a_idx[a], b_idx[b]), P, B);
                cs[bucket] += v * (double)orc_sign(prm, a_idx[a], b_idx[b]);
            }
}

/* Sum of |a_k(i) b_k(j)| per bucket: the magnitude a bucket's fp32 counter
 * is compared against (the plain definition, no signs). */
void orc_op_bucket_abs(const uint32_t *a_off, const uint32_t *a_idx, const float *a_val,
                       const uint32_t *b_off, const uint32_t *b_idx, const float *b_val,
                       uint64_t K, uint64_t seed, uint32_t P, uint32_t B, double *s)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    for (uint64_t k = 0; k < (uint64_t)P * B; ++k) s[k] = 0.0;
    for (uint64_t k = 0; k < K; ++k)
        for (uint64_t a = a_off[k]; a < a_off[k + 1]; ++a)
            for (uint64_t b = b_off[k]; b < b_off[k + 1]; ++b) {
                double v = (double)a_val[a] * (double)b_val[b];
                uint64_t bucket = orc_bucket(orc_h(prm, a_idx[a], b_idx[b]), P, B);
                s[bucket] += fabs(v);
            }
}

/* The Count-Sketch sign of many pairs. */
void orc_sign_many(uint64_t seed, const uint32_t *x, const uint32_t *y, uint64_t n, int8_t *out)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    for (uint64_t k = 0; k < n; ++k) out[k] = (int8_t)orc_sign(prm, x[k], y[k]);
}

/* part and bucket of many hash values (for tests and the Python layer) */
void orc_part_bucket_many(const uint32_t *h, uint64_t n, uint32_t P, uint32_t B,
                          uint32_t *part, uint32_t *bucket)
{
    for (uint64_t k = 0; k < n; ++k) {
        if (part) part[k] = orc_part(h[k], P);
        if (bucket) bucket[k] = orc_bucket(h[k], P, B);
    }
}

/* Terms per partition of a transaction stream (plain loop, no sort). */
void orc_tx_part_terms(const uint32_t *off, uint64_t T, const uint32_t *items,
                       uint32_t P, uint64_t seed, uint64_t *part_terms)
{
    uint64_t prm[8];
    orc_hash_params(seed, prm);
    for (uint32_t p = 0; p < P; ++p) part_terms[p] = 0;
    for (uint64_t t = 0; t < T; ++t)
        for (uint64_t a = off[t]; a < off[t + 1]; ++a)
            for (uint64_t b = a + 1; b < off[t + 1]; ++b) {
                uint32_t x = items[a] < items[b] ? items[a] : items[b];
                uint32_t y = items[a] < items[b] ? items[b] : items[a];
                part_terms[orc_part(orc_h(prm, x, y), P)] += 1;
            }
}
