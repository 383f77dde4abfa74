// Enumeration of the terms of a chunk, shared by the routing kernels and the
// Count-Sketch kernels.
//
// Transactions (Section 7): the terms of a transaction are its pairs x < y.
// Entries of a chunk are staged in LDS with h_b precomputed and ordered by
// their partner count, and every lane loops over the partners of one entry
// (stage_tx / enum_tx).
// Outer products (Section 4): the terms of vector pair k are all
// (a_k(i), b_k(j)); the a-entries are staged and the b-entries read through
// L2, with the same balanced walk over w = |b_k| per a-entry (stage_op /
// walk_op).
#pragma once
#include "crop_device.hpp"
#include "crop_hash.hpp"
#include "crop_internal.hpp"
#include "crop_layout.hpp"

namespace crop {

// ---------------------------------------------------------------- staging

// LDS image of a chunk of transactions.  For entry k (its position inside
// the chunk): xh[k] = (item, h_b(item)); w[k] = its partners, the entries
// after it in its transaction; perm = the entries in order of decreasing w
// (a 64-bucket counting sort).  Each lane owns one entry and loops over its
// w partners; because consecutive lanes take consecutive entries of perm,
// the lanes of a wavefront run loops of nearly equal length and the loop
// body has no divergent branch.
struct TxLds {
    uint2 *xh;
    uint16_t *w;
    uint16_t *perm;
    uint32_t *bucket;  // 64 words
};

template <int BS>
__device__ inline uint32_t stage_tx(const uint32_t *__restrict__ off,
                                    const uint32_t *__restrict__ items, uint32_t r0, uint32_t r1,
                                    const HashParams &hp, const TxLds &L)
{
    const uint32_t p0 = off[r0];
    const uint32_t m = off[r1] - p0;
    for (uint32_t k = threadIdx.x; k < m; k += BS) {
        uint32_t x = items[p0 + k];
        L.xh[k] = make_uint2(x, hash_b(hp, x));
    }
    if (threadIdx.x < 64) L.bucket[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += BS) {
        uint32_t a = off[r] - p0, e = off[r + 1] - p0;
        for (uint32_t k = a; k < e; ++k) {
            uint32_t w = e - k - 1;
            L.w[k] = (uint16_t)w;
            atomicAdd(&L.bucket[63 - min(w, 63u)], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        uint32_t v = L.bucket[threadIdx.x];
        L.bucket[threadIdx.x] = wave_inclusive_scan(v) - v;
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < m; k += BS) {
        uint32_t w = L.w[k];
        L.perm[atomicAdd(&L.bucket[63 - min(w, 63u)], 1u)] = (uint16_t)k;
    }
    __syncthreads();
    return m;
}

// visit(x, y, h) for every pair x < y of the staged chunk.
template <int BS, class Visit>
__device__ inline void enum_tx(uint32_t m, const TxLds &L, const HashParams &hp, Visit visit)
{
    for (uint32_t j = threadIdx.x; j < m; j += BS) {
        const uint32_t k = L.perm[j];
        const uint32_t w = L.w[k];
        if (w == 0) break;  // perm is sorted: every later entry of this thread has w == 0
        const uint32_t x = L.xh[k].x;
        const uint32_t ha = hash_a(hp, x);
        for (uint32_t d = 1; d <= w; ++d) {
            const uint2 yh = L.xh[k + d];
            visit(x, yh.x, ha + yh.y);
        }
    }
}

__device__ inline TxLds tx_lds(uint32_t *smem, uint32_t lead, uint32_t max_items)
{
    const TxLayout t = tx_layout(lead, max_items);
    TxLds L;
    L.xh = reinterpret_cast<uint2 *>(smem + t.xh);
    L.w = reinterpret_cast<uint16_t *>(smem + t.w);
    L.perm = reinterpret_cast<uint16_t *>(smem + t.perm);
    L.bucket = smem + t.bucket;
    return L;
}

template <class KeyT>
__device__ inline KeyT pack_key(uint32_t x, uint32_t y)
{
    if (sizeof(KeyT) == 4) return (KeyT)((x << 16) | y);
    return (KeyT)(((uint64_t)x << 32) | y);
}

// ---- an owner's terms through hash-bucketed windows (Lemma 1)
//
// The owner of the hash interval [q, q + W) needs, for each item x of a
// transaction, the partners y with (h_a(x) + h_b(y)) mod 2^32 in it, i.e.
// with h_b(y) in the window [q - h_a(x), q - h_a(x) + W) mod 2^32: one arc of
// the circular h_b order, two runs of a sorted list where it wraps (Section
// 5, proof of Lemma 1).  Each transaction of the chunk is bucket-sorted by
// the top kb bits of h_b (the hash-and-bucket step of Figure 1; a counting
// sort over (row, bucket)), an entry visits only the buckets its window
// covers, and the exact window test and y > x pick the owner's pairs.
// Requires W <= 2^31, so the two runs of a wrapping window never share a
// bucket.
struct WinLds {
    uint32_t *hist;  // (rows << kb) + 1: exclusive starts, then (after placement) ends
    uint2 *yh;       // (item, h_b) in (row, bucket) order
    uint16_t *row;   // chunk row of each sorted entry
    uint16_t *rin;   // chunk row of each entry in input order
};

__device__ inline WinLds win_lds(uint32_t *smem, uint32_t lead, uint32_t rows, uint32_t kb,
                                 uint32_t max_items)
{
    const WinLayout t = win_layout(lead, rows, kb, max_items);
    WinLds L;
    L.hist = smem + t.hist;
    L.yh = reinterpret_cast<uint2 *>(smem + t.yh);
    L.row = reinterpret_cast<uint16_t *>(smem + t.row);
    L.rin = reinterpret_cast<uint16_t *>(smem + t.rin);
    return L;
}

// Stage rows [r0, r1) bucket-sorted; returns the number of entries.  After
// the call hist[i] holds the end of (row, bucket) slot i, so slot i spans
// [i ? hist[i - 1] : 0, hist[i]).  Each row first marks its entries with
// its index (LDS stores only); then one thread per entry loads its item
// (coalesced), hashes it and counts, and after the scan loads, hashes and
// places it again.
template <int BS>
__device__ inline uint32_t stage_tx_win(const uint32_t *__restrict__ off,
                                        const uint32_t *__restrict__ items, uint32_t r0,
                                        uint32_t r1, uint32_t kb, const HashParams &hp,
                                        const WinLds &L, uint32_t *s_tmp)
{
    const uint32_t p0 = off[r0];
    const uint32_t m = off[r1] - p0;
    const uint32_t nh = (r1 - r0) << kb;
    const uint32_t sh = 32 - kb;
    for (uint32_t i = threadIdx.x; i <= nh; i += BS) L.hist[i] = 0;
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += BS) {
        const uint32_t a = off[r] - p0, e = off[r + 1] - p0;
        for (uint32_t k = a; k < e; ++k) L.rin[k] = (uint16_t)(r - r0);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < m; k += BS) {
        const uint32_t hb = hash_b(hp, items[p0 + k]);
        atomicAdd(&L.hist[((uint32_t)L.rin[k] << kb) + (hb >> sh)], 1u);
    }
    __syncthreads();
    lds_exclusive_scan<BS>(L.hist, nh, s_tmp);
    for (uint32_t k = threadIdx.x; k < m; k += BS) {
        const uint32_t y = items[p0 + k], hb = hash_b(hp, y);
        const uint32_t r = L.rin[k];
        const uint32_t pos = atomicAdd(&L.hist[(r << kb) + (hb >> sh)], 1u);
        L.yh[pos] = make_uint2(y, hb);
        L.row[pos] = (uint16_t)r;
    }
    __syncthreads();
    return m;
}

// visit(x, y, h) for every pair x < y of the staged chunk whose hash lies in
// [q, q + W).
template <int BS, class Visit>
__device__ inline void enum_tx_win(uint32_t m, uint32_t kb, uint32_t q, uint32_t W,
                                   const WinLds &L, const HashParams &hp, Visit visit)
{
    const uint32_t sh = 32 - kb;
    auto start = [&](uint32_t i) { return i ? L.hist[i - 1] : 0u; };
    for (uint32_t j = threadIdx.x; j < m; j += BS) {
        const uint32_t x = L.yh[j].x;
        const uint32_t base = (uint32_t)L.row[j] << kb;
        const uint32_t ha = hash_a(hp, x);
        const uint32_t lo = q - ha;                 // window [lo, lo + W) mod 2^32
        const uint32_t last = lo + (W - 1);
        const uint32_t b0 = lo >> sh, b1 = last >> sh;
        uint32_t a0 = start(base + b0), e0, a1 = 0, e1 = 0;
        if (b1 >= b0 && last >= lo) {
            e0 = start(base + b1 + 1);
        } else {                                    // wraps past 2^32: two runs
            e0 = start(base + (1u << kb));
            a1 = start(base);
            e1 = start(base + b1 + 1);
        }
        for (uint32_t i = a0; i < e0; ++i) {
            const uint2 yh = L.yh[i];
            if (yh.x > x && yh.y - lo < W) visit(x, yh.x, ha + yh.y);
        }
        for (uint32_t i = a1; i < e1; ++i) {
            const uint2 yh = L.yh[i];
            if (yh.x > x && yh.y - lo < W) visit(x, yh.x, ha + yh.y);
        }
    }
}

// ---- outer products

// Stage the a-entries [a_lo, a_hi) of vectors k0..k1-1: s_ai = index,
// s_ha = h_a, s_av = value, s_bs = first b-entry of the vector, s_wp =
// exclusive prefix of |b_k| per a-entry.
template <int BS>
__device__ uint32_t stage_op(const OpChunk ch, const uint32_t *__restrict__ a_off,
                             const uint32_t *__restrict__ a_idx, const float *__restrict__ a_val,
                             const uint32_t *__restrict__ b_off, const HashParams &hp,
                             uint32_t *s_ai, uint32_t *s_ha, float *s_av, uint32_t *s_bs,
                             uint32_t *s_wp, uint32_t *s_tmp, uint32_t *m_out)
{
    const uint32_t m = ch.a_hi - ch.a_lo;
    for (uint32_t k = threadIdx.x; k < m; k += BS) {
        uint32_t i = a_idx[ch.a_lo + k];
        s_ai[k] = i;
        s_ha[k] = hash_a(hp, i);
        s_av[k] = a_val[ch.a_lo + k];
    }
    for (uint32_t v = ch.k0 + threadIdx.x; v < ch.k1; v += BS) {
        uint32_t a = max(a_off[v], ch.a_lo), e = min(a_off[v + 1], ch.a_hi);
        uint32_t bs = b_off[v], nb = b_off[v + 1] - bs;
        for (uint32_t p = a; p < e; ++p) {
            s_bs[p - ch.a_lo] = bs;
            s_wp[p - ch.a_lo] = nb;
        }
    }
    __syncthreads();
    lds_exclusive_scan<BS>(s_wp, m, s_tmp);
    *m_out = m;
    return s_wp[m];
}

template <int BS, class Visit>
__device__ inline void walk_op(uint32_t Tc, uint32_t m, const uint32_t *s_ai, const uint32_t *s_ha,
                               const float *s_av, const uint32_t *s_bs, const uint32_t *s_wp,
                               const uint32_t *__restrict__ b_idx, const float *__restrict__ b_val,
                               const HashParams &hp, Visit visit)
{
    const uint32_t t0 = (uint32_t)(((uint64_t)Tc * threadIdx.x) / BS);
    const uint32_t t1 = (uint32_t)(((uint64_t)Tc * (threadIdx.x + 1)) / BS);
    if (t0 >= t1) return;
    uint32_t lo = 0, hi = m;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (s_wp[mid] <= t0) lo = mid; else hi = mid;
    }
    uint32_t k = lo;
    uint32_t q = s_bs[k] + (t0 - s_wp[k]);
    uint32_t e = s_bs[k] + (s_wp[k + 1] - s_wp[k]);
    uint32_t i = s_ai[k], ha = s_ha[k];
    float av = s_av[k];
    for (uint32_t t = t0; t < t1; ++t) {
        uint32_t j = b_idx[q];
        visit(i, j, ha + hash_b(hp, j), av * b_val[q]);
        if (++q == e && t + 1 < t1) {
            do { ++k; } while (s_wp[k + 1] == s_wp[k]);
            q = s_bs[k];
            e = q + (s_wp[k + 1] - s_wp[k]);
            i = s_ai[k];
            ha = s_ha[k];
            av = s_av[k];
        }
    }
}

struct OpArgs {
    const uint32_t *a_off, *a_idx, *b_off, *b_idx;
    const float *a_val, *b_val;
    const OpChunk *chunks;
};

template <int BS>
__device__ inline uint32_t *op_smem_layout(uint32_t *smem, uint32_t NB, uint32_t max_a,
                                           uint32_t **s_ai, uint32_t **s_ha, float **s_av,
                                           uint32_t **s_bs, uint32_t **s_wp, uint32_t **s_tmp)
{
    uint32_t *hist = smem;
    *s_ai = hist + NB;
    *s_ha = *s_ai + max_a;
    *s_av = reinterpret_cast<float *>(*s_ha + max_a);
    *s_bs = reinterpret_cast<uint32_t *>(*s_av + max_a);
    *s_wp = *s_bs + max_a;
    *s_tmp = *s_wp + max_a + 1;
    return hist;
}

}  // namespace crop
