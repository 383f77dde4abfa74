// Space-Saving summaries per bucket and top-K selection.
//
// Section 4 (frequent items mining) and Figure 1: every entry e of a
// partition updates the Space-Saving summary of its bucket h(e); a summary is
// ell triples (entry, count, overestimation).  Weighted update of entry e
// with weight w > 0:
//   - e monitored:          count += w
//   - else a free slot:     the lowest free slot becomes (e, w, 0)
//   - else:                 the unpinned slot of minimum count (lowest slot
//                           index among equal minima) becomes
//                           (e, count_min + w, count_min)
// Outer products use w = |a_k(i) b_k(j)| and keep the signed sum of the
// entry's terms since its admission.  Pinned slots (learned seeding) hold
// their entry from the start and are never evicted.
//
// GPU organisation.  Routing bins hold whole groups of buckets (bucket =
// (h * P * B) >> 32 and bin = (h * NB) >> 32 with NB dividing P * B, so a
// bucket lies inside one bin).  One workgroup owns a bin at a time: it keeps
// the bin's summaries in LDS, reads the bin's routed terms in micro-batches,
// groups each micro-batch by bucket with a counting sort in LDS, and then one
// lane per bucket applies that bucket's updates in order.  Buckets are
// independent, so the only sequential work is inside a bucket, as in the
// paper's per-bucket summaries.  The order of updates inside a bucket differs
// from the stream order; Space-Saving's bounds (Section 4: overestimation at
// most m/ell, every entry above m/ell monitored) hold for any order.
//
// Top-K: the K monitored entries with the largest (count, then smallest key)
// are found by radix selection over a 96-bit composite (count, ~key) in
// 8-bit digits, then ordered by counting ranks.
#include <algorithm>
#include <type_traits>

#include "crop_device.hpp"
#include "crop_internal.hpp"

namespace crop {

namespace {

constexpr uint8_t kUsed = 1, kPinned = 2;

template <class W> __device__ inline uint32_t wbits(W w);
template <> __device__ inline uint32_t wbits<uint32_t>(uint32_t w) { return w; }
template <> __device__ inline uint32_t wbits<float>(float w) { return __float_as_uint(w); }

template <class KeyT>
__device__ inline uint32_t bucket_of_key(KeyT key, const HashParams &hp, uint64_t PB,
                                         bool narrow)
{
    uint32_t x, y;
    if (narrow) {
        x = (uint32_t)key >> 16;
        y = (uint32_t)key & 0xFFFFu;
    } else {
        x = (uint32_t)((uint64_t)key >> 32);
        y = (uint32_t)key;
    }
    return interval_of(hash_a(hp, x) + hash_b(hp, y), PB);
}

// ---------------------------------------------------------------- state init

__global__ void __launch_bounds__(256)
k_ss_clear(uint64_t n, uint64_t *__restrict__ key, uint32_t *__restrict__ cnt,
           uint32_t *__restrict__ err, float *__restrict__ val, uint8_t *__restrict__ flag)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256) {
        key[i] = 0;
        cnt[i] = 0;
        err[i] = 0;
        val[i] = 0.0f;
        flag[i] = 0;
    }
}

// dup[s] = 1 when seed s repeats an earlier seed.
__global__ void __launch_bounds__(256)
k_seed_dups(const uint32_t *__restrict__ sx, const uint32_t *__restrict__ sy, uint32_t ns,
            uint8_t *__restrict__ dup)
{
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= ns) return;
    const uint32_t x = sx[s], y = sy[s];
    uint8_t d = 0;
    for (uint32_t t = 0; t < s && !d; ++t) d = (sx[t] == x && sy[t] == y) ? 1 : 0;
    dup[s] = d;
}

// Pin seeds: seed s goes to slot r of its bucket when r < r_max, where r is
// the number of earlier non-duplicate seeds of the same bucket (seeds come
// in priority order).  Duplicates are skipped.  One thread per seed, O(ns^2).
__global__ void __launch_bounds__(256)
k_ss_pin(const uint32_t *__restrict__ sx, const uint32_t *__restrict__ sy, uint32_t ns,
         const uint8_t *__restrict__ dup, uint32_t r_max, HashParams hp, uint64_t PB,
         uint32_t ell, uint64_t *__restrict__ key, uint8_t *__restrict__ flag,
         uint32_t *__restrict__ n_pinned)
{
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= ns || dup[s]) return;
    const uint32_t x = sx[s], y = sy[s];
    const uint32_t b = interval_of(hash_a(hp, x) + hash_b(hp, y), PB);
    uint32_t r = 0;
    for (uint32_t t = 0; t < s; ++t)
        if (!dup[t] && interval_of(hash_a(hp, sx[t]) + hash_b(hp, sy[t]), PB) == b) ++r;
    if (r >= r_max) return;
    const uint64_t slot = (uint64_t)b * ell + r;
    key[slot] = ((uint64_t)x << 32) | y;
    flag[slot] = kUsed | kPinned;
    atomicAdd(n_pinned, 1u);
}

__global__ void __launch_bounds__(256) k_zero32(uint32_t *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

// ---------------------------------------------------------------- summaries

template <class KeyT, class W, bool OUTER>
struct SsLds {
    KeyT *k;
    W *c;
    W *e;
    float *v;
    uint8_t *f;
};

// One Space-Saving update of bucket lb (slots [lb*ell, lb*ell+ell)).
template <class KeyT, class W, bool OUTER>
__device__ inline void ss_update(const SsLds<KeyT, W, OUTER> &L, uint32_t base, uint32_t ell,
                                 KeyT key, W w, float v)
{
    int hit = -1, freeslot = -1, mn = -1;
    W cmin = W(0);
    for (uint32_t s = 0; s < ell; ++s) {
        const uint8_t f = L.f[base + s];
        if (f & kUsed) {
            if (L.k[base + s] == key) {
                hit = (int)s;
                break;
            }
            if (!(f & kPinned)) {
                const W c = L.c[base + s];
                if (mn < 0 || c < cmin) {
                    mn = (int)s;
                    cmin = c;
                }
            }
        } else if (freeslot < 0) {
            freeslot = (int)s;
        }
    }
    if (hit >= 0) {
        L.c[base + hit] += w;
        if (OUTER) L.v[base + hit] += v;
    } else if (freeslot >= 0) {
        const uint32_t s = base + freeslot;
        L.k[s] = key;
        L.c[s] = w;
        L.e[s] = W(0);
        if (OUTER) L.v[s] = v;
        L.f[s] = kUsed;
    } else if (mn >= 0) {
        const uint32_t s = base + mn;
        L.k[s] = key;
        L.e[s] = cmin;
        L.c[s] = cmin + w;
        if (OUTER) L.v[s] = v;
    }
    // every slot pinned: the entry stays unmonitored
}

// Persistent workgroups, one routing bin at a time.  Global state is
// bucket-major with ell slots per bucket; counts and overestimations are
// stored as 32-bit words (uint32 for transactions, fp32 bits for outer
// products).
template <int BS, class KeyT, class W, bool OUTER, int MB>
__global__ void __launch_bounds__(BS)
k_ss_bins(const uint32_t *__restrict__ bin_off, const KeyT *__restrict__ keys,
          const float *__restrict__ vals, uint32_t NB, uint32_t nbk, uint32_t ell,
          HashParams hp, uint64_t PB, bool narrow, uint32_t *counter,
          uint64_t *__restrict__ g_key, uint32_t *__restrict__ g_cnt,
          uint32_t *__restrict__ g_err, float *__restrict__ g_val, uint8_t *__restrict__ g_flag)
{
    extern __shared__ uint64_t smem64[];
    const uint32_t nslot = nbk * ell;
    // layout: keys | counts | overestimations | values | staged keys | staged
    // values | bucket starts (nbk + 1) | flags
    KeyT *s_k = reinterpret_cast<KeyT *>(smem64);
    W *s_c = reinterpret_cast<W *>(s_k + nslot);
    W *s_e = s_c + nslot;
    float *s_v = reinterpret_cast<float *>(s_e + nslot);
    KeyT *t_k = reinterpret_cast<KeyT *>(
        reinterpret_cast<uint64_t *>(smem64) +
        ((nslot * sizeof(KeyT) + 2 * nslot * 4 + (OUTER ? nslot * 4 : 0) + 7) / 8));
    float *t_v = reinterpret_cast<float *>(t_k + MB);
    uint32_t *s_pos = reinterpret_cast<uint32_t *>(t_v + (OUTER ? MB : 0));
    uint8_t *s_f = reinterpret_cast<uint8_t *>(s_pos + nbk + 1);
    const SsLds<KeyT, W, OUTER> L{s_k, s_c, s_e, s_v, s_f};
    __shared__ uint32_t s_tmp[BS / kWave + 1];
    __shared__ uint32_t s_bin;

    for (;;) {
        if (threadIdx.x == 0) s_bin = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t b = s_bin;
        if (b >= NB) break;
        const uint64_t g0 = (uint64_t)b * nslot;
        for (uint32_t s = threadIdx.x; s < nslot; s += BS) {
            s_k[s] = (KeyT)g_key[g0 + s];
            s_c[s] = std::is_same<W, float>::value ? (W)__uint_as_float(g_cnt[g0 + s])
                                                   : (W)g_cnt[g0 + s];
            s_e[s] = std::is_same<W, float>::value ? (W)__uint_as_float(g_err[g0 + s])
                                                   : (W)g_err[g0 + s];
            if (OUTER) s_v[s] = g_val[g0 + s];
            s_f[s] = g_flag[g0 + s];
        }
        // seeded slots carry a 64-bit pair key; narrow runs compare packed keys
        if (narrow) {
            for (uint32_t s = threadIdx.x; s < nslot; s += BS) {
                const uint64_t g = g_key[g0 + s];
                s_k[s] = (KeyT)(((uint32_t)(g >> 32) << 16) | (uint32_t)(g & 0xFFFFu));
            }
        }
        __syncthreads();
        const uint32_t k0 = bin_off[b], k1 = bin_off[b + 1];
        const uint64_t bucket0 = (uint64_t)b * nbk;
        for (uint32_t base = k0; base < k1; base += MB) {
            const uint32_t n = min((uint32_t)MB, k1 - base);
            for (uint32_t i = threadIdx.x; i <= nbk; i += BS) s_pos[i] = 0;
            __syncthreads();
            // count per bucket
            for (uint32_t i = threadIdx.x; i < n; i += BS) {
                const uint32_t lb =
                    (uint32_t)(bucket_of_key(keys[base + i], hp, PB, narrow) - bucket0);
                atomicAdd(&s_pos[lb], 1u);
            }
            __syncthreads();
            lds_exclusive_scan<BS>(s_pos, nbk, s_tmp);
            // stage grouped by bucket (s_pos becomes each bucket's end)
            for (uint32_t i = threadIdx.x; i < n; i += BS) {
                const KeyT key = keys[base + i];
                const uint32_t lb = (uint32_t)(bucket_of_key(key, hp, PB, narrow) - bucket0);
                const uint32_t p = atomicAdd(&s_pos[lb], 1u);
                t_k[p] = key;
                if (OUTER) t_v[p] = vals[base + i];
            }
            __syncthreads();
            // one lane per bucket: its run is [end of previous bucket, end)
            for (uint32_t lb = threadIdx.x; lb < nbk; lb += BS) {
                const uint32_t e1 = s_pos[lb];
                const uint32_t e0 = lb ? s_pos[lb - 1] : 0;
                for (uint32_t p = e0; p < e1; ++p) {
                    if (OUTER) {
                        const float v = t_v[p];
                        ss_update<KeyT, W, OUTER>(L, lb * ell, ell, t_k[p], (W)fabsf(v), v);
                    } else {
                        ss_update<KeyT, W, OUTER>(L, lb * ell, ell, t_k[p], (W)1, 0.0f);
                    }
                }
            }
            __syncthreads();
        }
        for (uint32_t s = threadIdx.x; s < nslot; s += BS) {
            uint64_t g;
            if (narrow) {
                const uint32_t kk = (uint32_t)s_k[s];
                g = ((uint64_t)(kk >> 16) << 32) | (kk & 0xFFFFu);
            } else {
                g = (uint64_t)s_k[s];
            }
            g_key[g0 + s] = (s_f[s] & kUsed) ? g : 0;
            g_cnt[g0 + s] = wbits<W>(s_c[s]);
            g_err[g0 + s] = wbits<W>(s_e[s]);
            if (OUTER) g_val[g0 + s] = s_v[s];
            g_flag[g0 + s] = s_f[s];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- top-K

// Composite of a used slot, most significant word first: count (uint32 or
// non-negative fp32 bits, both order-preserving), then the complemented key
// so that smaller keys rank higher.
struct Comp {
    uint32_t w[3];
};

__device__ inline Comp comp_of(const uint64_t *key, const uint32_t *cnt, uint64_t i)
{
    const uint64_t k = key[i];
    return Comp{{cnt[i], ~(uint32_t)(k >> 32), ~(uint32_t)k}};
}

__device__ inline uint32_t digit_of(const Comp &c, uint32_t pass)
{
    return (c.w[pass >> 2] >> (24 - 8 * (pass & 3))) & 0xFFu;
}

// Does c agree with the selected prefix on the digits of passes < pass?
__device__ inline bool prefix_match(const Comp &c, const uint32_t *prefix, uint32_t pass)
{
    for (uint32_t w = 0; w < 3; ++w) {
        const uint32_t bits = pass >= 4 * (w + 1) ? 32u : 8u * (pass - 4 * w);
        if (pass <= 4 * w) break;
        const uint32_t mask = bits == 32 ? 0xFFFFFFFFu : ~(0xFFFFFFFFu >> bits);
        if ((c.w[w] & mask) != (prefix[w] & mask)) return false;
    }
    return true;
}

// Selection state in device memory:
//   st[0..2] prefix words, st[3] remaining rank, st[4] candidate count,
//   st[5] selected count, st[6] used slots, hist[256].
__global__ void __launch_bounds__(256)
k_topk_hist(const uint64_t *__restrict__ key, const uint32_t *__restrict__ cnt,
            const uint8_t *__restrict__ flag, uint64_t n, const uint32_t *__restrict__ cand,
            const uint32_t *__restrict__ st, uint32_t pass, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t m = cand ? st[4] : n;
    for (uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x; t < m;
         t += (uint64_t)gridDim.x * 256) {
        const uint64_t i = cand ? cand[t] : t;
        if (!(flag[i] & kUsed)) continue;
        const Comp c = comp_of(key, cnt, i);
        if (!prefix_match(c, st, pass)) continue;
        atomicAdd(&h[digit_of(c, pass)], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// One wavefront: pick the digit of this pass and clear the histogram.
__global__ void __launch_bounds__(64)
k_topk_pick(uint32_t *__restrict__ st, uint32_t *__restrict__ hist, uint32_t pass, uint32_t K)
{
    if (threadIdx.x != 0) return;
    if (pass == 0) {
        uint32_t used = 0;
        for (int d = 0; d < 256; ++d) used += hist[d];
        st[6] = used;
        st[3] = K < used ? K : used;
    }
    uint32_t rem = st[3];
    uint32_t cum = 0;
    int d = 255;
    if (rem > 0) {
        for (; d > 0; --d) {
            if (cum + hist[d] >= rem) break;
            cum += hist[d];
        }
        st[3] = rem - cum;
    }
    const uint32_t w = pass >> 2, sh = 24 - 8 * (pass & 3);
    st[w] = (st[w] & ~(0xFFu << sh)) | ((uint32_t)d << sh);
    for (int i = 0; i < 256; ++i) hist[i] = 0;
}

__device__ inline bool comp_ge(const Comp &a, const uint32_t *t)
{
    for (int w = 0; w < 3; ++w) {
        if (a.w[w] != t[w]) return a.w[w] > t[w];
    }
    return true;
}

__device__ inline bool comp_gt(const Comp &a, const Comp &b)
{
    for (int w = 0; w < 3; ++w) {
        if (a.w[w] != b.w[w]) return a.w[w] > b.w[w];
    }
    return false;
}

// Keep the slots whose top 16 bits of count reach the selected prefix.
__global__ void __launch_bounds__(256)
k_topk_compact(const uint64_t *__restrict__ key, const uint32_t *__restrict__ cnt,
               const uint8_t *__restrict__ flag, uint64_t n, uint32_t *__restrict__ st,
               uint32_t *__restrict__ cand)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256) {
        if (!(flag[i] & kUsed)) continue;
        if ((cnt[i] >> 16) < (st[0] >> 16)) continue;
        cand[atomicAdd(&st[4], 1u)] = (uint32_t)i;
    }
}

// Collect the selected slots (composite >= threshold): exactly st[3]-ranked.
__global__ void __launch_bounds__(256)
k_topk_collect(const uint64_t *__restrict__ key, const uint32_t *__restrict__ cnt,
               const uint32_t *__restrict__ cand, uint32_t *__restrict__ st,
               uint32_t *__restrict__ sel)
{
    const uint32_t m = st[4];
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < m; t += gridDim.x * 256) {
        const uint32_t i = cand[t];
        if (comp_ge(comp_of(key, cnt, i), st)) sel[atomicAdd(&st[5], 1u)] = i;
    }
}

// rank of every selected slot = number of selected slots ranking above it;
// writes the outputs in rank order.
__global__ void __launch_bounds__(256)
k_topk_rank(const uint64_t *__restrict__ key, const uint32_t *__restrict__ cnt,
            const uint32_t *__restrict__ err, const float *__restrict__ val, bool outer,
            const uint32_t *__restrict__ sel, const uint32_t *__restrict__ st,
            uint32_t *__restrict__ oi, uint32_t *__restrict__ oj, double *__restrict__ ou,
            double *__restrict__ ol, double *__restrict__ ov)
{
    __shared__ Comp tile[256];
    const uint32_t m = st[5];
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    Comp me{{0, 0, 0}};
    if (t < m) me = comp_of(key, cnt, sel[t]);
    uint32_t rank = 0;
    for (uint32_t b = 0; b < m; b += 256) {
        __syncthreads();
        if (b + threadIdx.x < m) tile[threadIdx.x] = comp_of(key, cnt, sel[b + threadIdx.x]);
        __syncthreads();
        const uint32_t lim = min(256u, m - b);
        if (t < m)
            for (uint32_t q = 0; q < lim; ++q) rank += comp_gt(tile[q], me) ? 1u : 0u;
    }
    if (t >= m) return;
    const uint32_t i = sel[t];
    const uint64_t k = key[i];
    oi[rank] = (uint32_t)(k >> 32);
    oj[rank] = (uint32_t)k;
    double c, e;
    if (outer) {
        c = (double)__uint_as_float(cnt[i]);
        e = (double)__uint_as_float(err[i]);
        ov[rank] = (double)val[i];
    } else {
        c = (double)cnt[i];
        e = (double)err[i];
        ov[rank] = c;
    }
    ou[rank] = c;
    ol[rank] = c - e;
}

}  // namespace

// ---------------------------------------------------------------- launchers

static uint32_t grid_for(uint64_t n, uint32_t cap = 4096)
{
    uint64_t g = (n + 255) / 256;
    if (g > cap) g = cap;
    return g ? (uint32_t)g : 1u;
}

hipError_t launch_zero32(uint32_t *p, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero32, dim3(grid_for(n, 1024)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_ss_clear(const SsState &S, hipStream_t s)
{
    hipLaunchKernelGGL(k_ss_clear, dim3(grid_for(S.nslots)), dim3(256), 0, s, S.nslots, S.key,
                       S.cnt, S.err, S.val, S.flag);
    return hipGetLastError();
}

hipError_t launch_ss_pin(const SsState &S, const uint32_t *sx, const uint32_t *sy, uint32_t ns,
                         uint8_t *dup, uint32_t r_max, const HashParams &hp, uint64_t PB,
                         uint32_t ell, uint32_t *n_pinned, hipStream_t s)
{
    if (ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seed_dups, dim3((ns + 255) / 256), dim3(256), 0, s, sx, sy, ns, dup);
    hipLaunchKernelGGL(k_ss_pin, dim3((ns + 255) / 256), dim3(256), 0, s, sx, sy, ns, dup, r_max,
                       hp, PB, ell, S.key, S.flag, n_pinned);
    return hipGetLastError();
}

size_t ss_bins_smem_bytes(uint32_t nbk, uint32_t ell, bool wide_key, bool outer, uint32_t MB)
{
    const size_t nslot = (size_t)nbk * ell;
    const size_t ksz = wide_key ? 8 : 4;
    size_t head = nslot * ksz + 2 * nslot * 4 + (outer ? nslot * 4 : 0);
    head = (head + 7) / 8 * 8;
    return head + MB * ksz + (outer ? MB * 4 : 0) + (nbk + 1) * 4 + nslot + 16;
}

hipError_t launch_ss_bins(const crop_ctx *c, const SsState &S, uint32_t nbk, uint64_t PB,
                          hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint32_t ell = c->ss_ell;
    const bool outer = c->in.mode == Mode::Outer;
    const bool wide = c->in.wide_keys;
    const uint32_t grid = std::min<uint32_t>(pl.NB, 4u * (uint32_t)cus);
    if (outer) {
        constexpr int MB = 1024;
        size_t sm = ss_bins_smem_bytes(nbk, ell, true, true, MB);
        hipLaunchKernelGGL((k_ss_bins<256, uint64_t, float, true, MB>), dim3(grid), dim3(256), sm,
                           s, c->bin_off.as<uint32_t>(), c->keys.as<uint64_t>(),
                           c->vals.as<float>(), pl.NB, nbk, ell, c->hp, PB, false,
                           c->counter.as<uint32_t>(), S.key, S.cnt, S.err, S.val, S.flag);
    } else if (wide) {
        constexpr int MB = 2048;
        size_t sm = ss_bins_smem_bytes(nbk, ell, true, false, MB);
        hipLaunchKernelGGL((k_ss_bins<256, uint64_t, uint32_t, false, MB>), dim3(grid), dim3(256),
                           sm, s, c->bin_off.as<uint32_t>(), c->keys.as<uint64_t>(), nullptr,
                           pl.NB, nbk, ell, c->hp, PB, false, c->counter.as<uint32_t>(), S.key,
                           S.cnt, S.err, S.val, S.flag);
    } else {
        constexpr int MB = 2048;
        size_t sm = ss_bins_smem_bytes(nbk, ell, false, false, MB);
        hipLaunchKernelGGL((k_ss_bins<256, uint32_t, uint32_t, false, MB>), dim3(grid), dim3(256),
                           sm, s, c->bin_off.as<uint32_t>(), c->keys.as<uint32_t>(), nullptr,
                           pl.NB, nbk, ell, c->hp, PB, true, c->counter.as<uint32_t>(), S.key,
                           S.cnt, S.err, S.val, S.flag);
    }
    return hipGetLastError();
}

// Top-K over the summary slots; st (8 words) and hist (256 words) must be
// zero on entry; cand and sel hold up to nslots indices.
hipError_t launch_topk(const SsState &S, uint32_t K, bool outer, uint32_t *st, uint32_t *hist,
                       uint32_t *cand, uint32_t *sel, uint32_t *oi, uint32_t *oj, double *ou,
                       double *ol, double *ov, hipStream_t s)
{
    const uint32_t g = grid_for(S.nslots);
    for (uint32_t pass = 0; pass < 12; ++pass) {
        hipLaunchKernelGGL(k_topk_hist, dim3(g), dim3(256), 0, s, S.key, S.cnt, S.flag, S.nslots,
                           pass < 2 ? nullptr : cand, st, pass, hist);
        hipLaunchKernelGGL(k_topk_pick, dim3(1), dim3(64), 0, s, st, hist, pass, K);
        if (pass == 1)
            hipLaunchKernelGGL(k_topk_compact, dim3(g), dim3(256), 0, s, S.key, S.cnt, S.flag,
                               S.nslots, st, cand);
    }
    hipLaunchKernelGGL(k_topk_collect, dim3(g), dim3(256), 0, s, S.key, S.cnt, cand, st, sel);
    const uint32_t gr = (K + 255) / 256 ? (K + 255) / 256 : 1;
    hipLaunchKernelGGL(k_topk_rank, dim3(gr), dim3(256), 0, s, S.key, S.cnt, S.err, S.val, outer,
                       sel, st, oi, oj, ou, ol, ov);
    return hipGetLastError();
}

}  // namespace crop
