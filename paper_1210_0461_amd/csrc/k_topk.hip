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

// The same pinning for at most kPinLds seeds in one workgroup: the seeds'
// pairs and buckets are staged in LDS, then every seed scans the earlier
// ones there (a duplicate pair first, then the earlier non-duplicate seeds
// of its bucket), all lanes reading the same earlier seed at once and eight
// reads in flight.
constexpr uint32_t kPinLds = 4096;
__global__ void __launch_bounds__(1024)
k_ss_pin_lds(const uint32_t *__restrict__ sx, const uint32_t *__restrict__ sy, uint32_t ns,
             uint32_t r_max, HashParams hp, uint64_t PB, uint32_t ell,
             uint64_t *__restrict__ key, uint8_t *__restrict__ flag, uint32_t *__restrict__ n_pinned)
{
    __shared__ uint64_t s_k[kPinLds];
    __shared__ uint32_t s_b[kPinLds];
    __shared__ uint8_t s_d[kPinLds];
    for (uint32_t i = threadIdx.x; i < ns; i += 1024) {
        const uint32_t x = sx[i], y = sy[i];
        s_k[i] = ((uint64_t)x << 32) | y;
        s_b[i] = interval_of(hash_a(hp, x) + hash_b(hp, y), PB);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < ns; i += 1024) {
        const uint64_t k = s_k[i];
        uint32_t d = 0;
#pragma unroll 8
        for (uint32_t t = 0; t < i; ++t) d |= s_k[t] == k ? 1u : 0u;
        s_d[i] = (uint8_t)d;
    }
    __syncthreads();
    // (every lane of a wavefront runs the same rounds, so the pinned count
    // is summed per wavefront)
    for (uint32_t i0 = 0; i0 < ns; i0 += 1024) {
        const uint32_t i = i0 + threadIdx.x;
        uint32_t pinned = 0;
        if (i < ns && !s_d[i]) {
            const uint32_t b = s_b[i];
            uint32_t r = 0;
#pragma unroll 8
            for (uint32_t t = 0; t < i; ++t) r += (s_b[t] == b && !s_d[t]) ? 1u : 0u;
            if (r < r_max) {
                const uint64_t slot = (uint64_t)b * ell + r;
                key[slot] = s_k[i];
                flag[slot] = kUsed | kPinned;
                pinned = 1;
            }
        }
        const uint32_t tot = wave_count_sum(pinned);
        if (lane_id() == 0 && tot) atomicAdd(n_pinned, tot);
    }
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

// LDS layout of a summaries workgroup (byte offsets), shared by the kernel
// and the host's size computation:
//   state   keys | counts | overestimations | [values] | flags   (nbk * ell)
//   table   keys | weights | [values]                            (2 * MB)
//   staged  keys | weights | [values]                            (MB)
//   bucket positions (nbk + 1)
struct SsLayout {
    uint32_t sk, sc, se, sv, sf, hk, hw, hv, tk, tw, tv, pos, total;
};

__host__ __device__ inline uint32_t align8(uint32_t x) { return (x + 7u) & ~7u; }

__host__ __device__ inline SsLayout ss_layout(uint32_t nbk, uint32_t ell, uint32_t ksz, bool outer,
                                              uint32_t MB)
{
    const uint32_t ns = nbk * ell, hs = 2 * MB;
    SsLayout L;
    uint32_t o = 0;
    L.sk = o; o = align8(o + ns * ksz);
    L.sc = o; o += ns * 4;
    L.se = o; o += ns * 4;
    L.sv = o; o += outer ? ns * 4 : 0;
    L.hk = o = align8(o);
    o = align8(o + hs * ksz);
    L.hw = o; o += hs * 4;
    L.hv = o; o += outer ? hs * 4 : 0;
    L.tk = o = align8(o);
    o = align8(o + MB * ksz);
    L.tw = o; o += MB * 4;
    L.tv = o; o += outer ? MB * 4 : 0;
    L.pos = o; o += (nbk + 1) * 4;
    L.sf = o; o += ns;
    L.total = align8(o);
    return L;
}

// Minimum over each group of G lanes, in every lane of the group: DPP within
// rows of 16 lanes (swap neighbours, swap pairs, rotate the row by 4 and 8),
// then lane shuffles across rows for G = 32 and 64.
template <int G>
__device__ inline uint32_t group_min(uint32_t v)
{
    // old = all ones, the identity of the minimum, lets the compiler fold
    // each move into the min (a lane with no valid source keeps its value)
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0xB1, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x4E, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x124, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x128, 0xF, 0xF, false));
    if (G >= 32) v = min(v, (uint32_t)__shfl_xor((int)v, 16, kWave));
    if (G >= 64) v = min(v, (uint32_t)__shfl_xor((int)v, 32, kWave));
    return v;
}

// The group's bits of a wave ballot, slot j at bit j.
template <int G> struct GroupMask { using T = uint32_t; };
template <> struct GroupMask<64> { using T = uint64_t; };

template <int G>
__device__ inline typename GroupMask<G>::T group_bits(uint64_t b, uint32_t gsh)
{
    if constexpr (G == 64)
        return b;
    else
        return (uint32_t)(b >> gsh) & (uint32_t)((1ull << G) - 1ull);
}

__device__ inline uint32_t lowest_bit(uint32_t m) { return (uint32_t)__builtin_ctz(m); }
__device__ inline uint32_t lowest_bit(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }
__device__ inline uint32_t bit_count(uint32_t m) { return (uint32_t)__popc(m); }
__device__ inline uint32_t bit_count(uint64_t m) { return (uint32_t)__popcll(m); }

template <class KeyT> __device__ inline KeyT empty_key();
template <> __device__ inline uint32_t empty_key<uint32_t>() { return kEmpty32; }
template <> __device__ inline uint64_t empty_key<uint64_t>() { return kEmpty64; }

// Add weight w (and signed value v) of key to the micro-batch table
// (linear probing, at most half full, so a free slot is always reached).
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
// Merge-table weight of an update already applied as a hit (merged weights
// are counts below 2^31 or non-negative fp32 bits, never all ones).
constexpr uint32_t kConsumed = 0xFFFFFFFFu;

// Adds (w, v) to key's entry of the merge table; returns the entry's slot
// when this call inserted the key, else kNoSlot.
template <class KeyT, bool OUTER>
__device__ inline uint32_t table_add(KeyT *hk, uint32_t *hw, float *hv, uint32_t log2hs, KeyT key,
                                     uint32_t w, float v)
{
    const uint32_t mask = (1u << log2hs) - 1;
    uint32_t s = slot_of(key, log2hs);
    for (;;) {
        KeyT cur = hk[s];
        bool inserted = false;
        if (cur == empty_key<KeyT>()) {
            cur = atomicCAS(&hk[s], empty_key<KeyT>(), key);
            if (cur == empty_key<KeyT>()) {
                cur = key;
                inserted = true;
            }
        }
        if (cur == key) {
            if (OUTER) {
                atomicAdd(reinterpret_cast<float *>(&hw[s]), __uint_as_float(w));
                atomicAdd(&hv[s], v);
            } else {
                atomicAdd(&hw[s], w);
            }
            return inserted ? s : kNoSlot;
        }
        s = (s + 1) & mask;
    }
}

// Persistent workgroups take routing bins heaviest first (order[]).  The
// bin's summaries sit in LDS, bucket-major with ell slots per bucket.  The
// bin's routed terms are read in micro-batches of MB:
//   1. equal keys of the micro-batch are merged into one weighted update in
//      an LDS hash table (a wave first merges the copies of its lead key);
//   2. the hits first, in parallel (bins of one bucket, and all bins of
//      transaction counts): every monitored slot takes the merged weight of
//      its key, if the micro-batch has it;
//   3. the remaining updates are grouped by bucket with a counting sort; a
//      bin of one bucket instead keeps them in the order of each key's first
//      copy in the micro-batch, so the bucket sees its entries in stream
//      order (routed keys keep the order of their chunks);
//   4. a group of G lanes (G >= ell) applies one bucket's updates, lane j
//      holding slot j in registers.  Transaction counts (all misses after
//      step 2) take level steps: every slot at the minimum count takes one
//      update at once, which reaches the state of single steps in order.
//      Otherwise single steps:
//        hit    one ballot finds the monitored slot (not needed after 2);
//        free   the lowest free slot (ballot, first set bit);
//        evict  minimum count over the unpinned slots by a G-lane butterfly,
//               the lowest slot among equal minima by a ballot.
// Merging and reordering a bucket's updates keeps Space-Saving's bounds
// (Section 4), which hold for any order of weighted updates.  Counts and
// overestimations are 32-bit words: uint32 for transactions, fp32 bits for
// outer products (non-negative fp32 bits order like the values).
template <int G, class KeyT, bool OUTER, int MB, bool ONE>
__global__ void __launch_bounds__(ONE ? 256 : 512)
k_ss_groups(const uint32_t *__restrict__ bin_off, const uint32_t *__restrict__ order,
            const KeyT *__restrict__ keys, const float *__restrict__ vals, uint32_t NB,
            uint32_t nbk, uint32_t ell, HashParams hp, uint64_t PB, bool narrow,
            uint32_t *counter, uint64_t *__restrict__ g_key, uint32_t *__restrict__ g_cnt,
            uint32_t *__restrict__ g_err, float *__restrict__ g_val, uint8_t *__restrict__ g_flag,
            uint32_t *__restrict__ g_key32, bool fresh)
{
    static_assert(G == 16 || G == 32 || G == 64, "group width");
    static_assert((MB & (MB - 1)) == 0, "micro-batch is a power of two");
    constexpr uint32_t HS = 2 * MB;
    constexpr uint32_t LOG2HS = __builtin_ctz(HS);
    extern __shared__ uint64_t smem64[];
    char *sm = reinterpret_cast<char *>(smem64);
    const SsLayout Lo = ss_layout(nbk, ell, sizeof(KeyT), OUTER, MB);
    KeyT *s_k = reinterpret_cast<KeyT *>(sm + Lo.sk);
    uint32_t *s_c = reinterpret_cast<uint32_t *>(sm + Lo.sc);
    uint32_t *s_e = reinterpret_cast<uint32_t *>(sm + Lo.se);
    float *s_v = reinterpret_cast<float *>(sm + Lo.sv);
    uint8_t *s_f = reinterpret_cast<uint8_t *>(sm + Lo.sf);
    KeyT *h_k = reinterpret_cast<KeyT *>(sm + Lo.hk);
    uint32_t *h_w = reinterpret_cast<uint32_t *>(sm + Lo.hw);
    float *h_v = reinterpret_cast<float *>(sm + Lo.hv);
    KeyT *t_k = reinterpret_cast<KeyT *>(sm + Lo.tk);
    uint32_t *t_w = reinterpret_cast<uint32_t *>(sm + Lo.tw);
    float *t_v = reinterpret_cast<float *>(sm + Lo.tv);
    uint32_t *s_pos = reinterpret_cast<uint32_t *>(sm + Lo.pos);
    __shared__ uint32_t s_tmp[512 / kWave + 1];
    __shared__ uint32_t s_bin, s_cmax;

    // Bins of one bucket run 256 threads (one chain; the merge and grouping
    // phases still use every lane), bins of several buckets 512 (twice the
    // wavefronts per CU for the latency-bound merge, grouping and chains).
    constexpr uint32_t BS = ONE ? 256u : 512u;
    const uint32_t nslot = nbk * ell;
    const uint32_t lane = lane_id();
    const uint32_t j = lane & (G - 1);  // slot held by this lane
    const uint32_t gsh = lane & (uint32_t)(kWave - G);  // first lane of the group
    const uint32_t group = threadIdx.x / G, n_groups = BS / G;
    const bool real = j < ell;

    for (;;) {
        if (threadIdx.x == 0) {
            s_bin = atomicAdd(counter, 1u);
            s_cmax = 0;
        }
        __syncthreads();
        const uint32_t q = s_bin;
        if (q >= NB) break;
        const uint32_t b = order[q];
        const uint64_t g0 = (uint64_t)b * nslot;
        // the bin's state: empty when the run starts from empty summaries
        // (fresh: nothing pinned; every slot of every bin is written back
        // below, so the global state needs no clearing), else as cleared and
        // pinned before the launch
        for (uint32_t s = threadIdx.x; s < nslot; s += BS) {
            if (fresh) {
                s_k[s] = (KeyT)0;
                s_c[s] = 0;
                s_e[s] = 0;
                if (OUTER) s_v[s] = 0.0f;
                s_f[s] = 0;
                continue;
            }
            const uint64_t g = g_key[g0 + s];
            // seeded slots carry a 64-bit pair key; narrow runs compare packed keys
            s_k[s] = narrow ? (KeyT)(((uint32_t)(g >> 32) << 16) | (uint32_t)(g & 0xFFFFu))
                            : (KeyT)g;
            const uint32_t cnt = g_cnt[g0 + s];
            s_c[s] = cnt;
            if (!OUTER && cnt) atomicMax(&s_cmax, cnt);
            s_e[s] = g_err[g0 + s];
            if (OUTER) s_v[s] = g_val[g0 + s];
            s_f[s] = g_flag[g0 + s];
        }
        const uint32_t k0 = bin_off[b], k1 = bin_off[b + 1];
        const uint64_t bucket0 = (uint64_t)b * nbk;
        // The keys (and values) of a micro-batch, MB / BS per thread, are
        // loaded while the previous micro-batch is applied, so their HBM
        // latency overlaps the serial work.
        constexpr uint32_t PT = MB / BS;
        static_assert(PT * BS == MB, "micro-batch is a multiple of the block");
        KeyT kk[PT];
        float vv[PT];
        auto load_batch = [&](uint32_t b0) {
            const uint32_t m = b0 < k1 ? min((uint32_t)MB, k1 - b0) : 0u;
#pragma unroll
            for (uint32_t q = 0; q < PT; ++q) {
                const uint32_t i = threadIdx.x + q * BS;
                kk[q] = i < m ? keys[b0 + i] : empty_key<KeyT>();
                vv[q] = (OUTER && i < m) ? vals[b0 + i] : 0.0f;
            }
        };
        load_batch(k0);
        for (uint32_t base = k0; base < k1;) {
            const uint32_t n = min((uint32_t)MB, k1 - base);
            const uint32_t next = base + n;  // <= k1: no wrap-around
            for (uint32_t i = threadIdx.x; i < HS; i += BS) {
                h_k[i] = empty_key<KeyT>();
                h_w[i] = 0u;
                if (OUTER) h_v[i] = 0.0f;
            }
            for (uint32_t i = threadIdx.x; i <= nbk; i += BS) s_pos[i] = 0;
            // one bucket: t_w[i] = merge-table slot of the key first seen at i
            if (ONE)
                for (uint32_t i = threadIdx.x; i < MB; i += BS) t_w[i] = kNoSlot;
            __syncthreads();
            // 1. merge equal keys (kk, vv hold this micro-batch)
#pragma unroll
            for (uint32_t q = 0; q < PT; ++q) {
                if (q * BS >= n) break;  // uniform
                const uint32_t i = threadIdx.x + q * BS;
                const bool valid = i < n;
                const KeyT key = kk[q];
                uint32_t first = kNoSlot;
                if (OUTER) {
                    if (valid) {
                        const float v = vv[q];
                        first = table_add<KeyT, true>(h_k, h_w, h_v, LOG2HS, key,
                                                      __float_as_uint(fabsf(v)), v);
                    }
                } else {
                    const uint64_t vm = __ballot(valid);
                    if (!vm) continue;
                    const uint32_t src = (uint32_t)(__ffsll((long long)vm) - 1);
                    KeyT lead;
                    if constexpr (sizeof(KeyT) == 4)
                        lead = (KeyT)lane_value((uint32_t)key, src);
                    else
                        lead = (KeyT)(((uint64_t)lane_value((uint32_t)((uint64_t)key >> 32), src)
                                       << 32) |
                                      lane_value((uint32_t)key, src));
                    const bool same = valid && key == lead;
                    const uint64_t m = __ballot(same);
                    if (same) {
                        if (lane == (uint32_t)__ffsll((long long)m) - 1)
                            first = table_add<KeyT, false>(h_k, h_w, h_v, LOG2HS, key,
                                                           (uint32_t)__popcll(m), 0.0f);
                    } else if (valid) {
                        first = table_add<KeyT, false>(h_k, h_w, h_v, LOG2HS, key, 1u, 0.0f);
                    }
                }
                // the inserting copy is one of the key's first copies: rounds
                // of 256 positions run in order, a wave's lowest lane inserts
                // for its copies (only waves of one round can race)
                if (ONE && first != kNoSlot) t_w[i] = first;
            }
            load_batch(next);  // the next micro-batch, used after step 4
            __syncthreads();
            // 2. the hits in one parallel step (bins of one bucket, and bins
            // of transaction counts): every monitored slot looks its key up
            // in the merge table and takes the merged weight, and the entry
            // is marked consumed (keys are only read here, so probe chains
            // stay intact).  A micro-batch holds each key once, so a key that
            // is not monitored now cannot become monitored before its own
            // update: every update left for step 4 is a miss.  Any order of
            // the updates keeps the Section 4 bounds.  (Outer-product bins of
            // many buckets keep the hit test in step 4.)
            for (uint32_t q = threadIdx.x; (ONE || !OUTER) && q < nslot; q += BS) {
                if (!(s_f[q] & kUsed)) continue;
                const KeyT key = s_k[q];
                uint32_t sl = slot_of(key, LOG2HS);
                for (;;) {
                    const KeyT cur = h_k[sl];
                    if (cur == key) {
                        const uint32_t w = h_w[sl];
                        if (OUTER) {
                            s_c[q] = __float_as_uint(__uint_as_float(s_c[q]) + __uint_as_float(w));
                            s_v[q] += h_v[sl];
                        } else {
                            s_c[q] += w;
                        }
                        h_w[sl] = kConsumed;
                        break;
                    }
                    if (cur == empty_key<KeyT>()) break;
                    sl = (sl + 1) & (HS - 1);
                }
            }
            __syncthreads();
            // 3. group the remaining (missed) updates by bucket
            if constexpr (ONE) {
                // order of first copies: compact t_w's slots in position
                // order (every thread reads its positions before the scan's
                // barriers and writes at or below them afterwards; the
                // workgroup has 256 threads, see ss_block_threads)
                constexpr uint32_t PER = MB / 256;
                uint32_t sl[PER], cnt = 0;
#pragma unroll
                for (uint32_t q = 0; q < PER; ++q) {
                    sl[q] = t_w[threadIdx.x * PER + q];
                    if (sl[q] != kNoSlot && h_w[sl[q]] == kConsumed) sl[q] = kNoSlot;
                    cnt += sl[q] != kNoSlot ? 1u : 0u;
                }
                uint32_t total;
                uint32_t p = block_exclusive_scan<256>(cnt, s_tmp, &total);
#pragma unroll
                for (uint32_t q = 0; q < PER; ++q) {
                    if (sl[q] == kNoSlot) continue;
                    t_k[p] = h_k[sl[q]];
                    t_w[p] = h_w[sl[q]];
                    if (OUTER) t_v[p] = h_v[sl[q]];
                    ++p;
                }
                if (threadIdx.x == 0) s_pos[0] = total;  // the bucket's end
            } else {
                // (entries consumed as hits in step 2 are left out)
                for (uint32_t i = threadIdx.x; i < HS; i += BS) {
                    const KeyT key = h_k[i];
                    if (key == empty_key<KeyT>() || h_w[i] == kConsumed) continue;
                    atomicAdd(&s_pos[(uint32_t)(bucket_of_key(key, hp, PB, narrow) - bucket0)],
                              1u);
                }
                __syncthreads();
                lds_exclusive_scan_rt(s_pos, nbk, s_tmp);
                for (uint32_t i = threadIdx.x; i < HS; i += BS) {
                    const KeyT key = h_k[i];
                    if (key == empty_key<KeyT>() || h_w[i] == kConsumed) continue;
                    const uint32_t lb = (uint32_t)(bucket_of_key(key, hp, PB, narrow) - bucket0);
                    const uint32_t p = atomicAdd(&s_pos[lb], 1u);  // becomes the bucket's end
                    t_k[p] = key;
                    t_w[p] = h_w[i];
                    if (OUTER) t_v[p] = h_v[i];
                }
            }
            __syncthreads();
            // 4. one group per bucket applies its updates in order; after
            // step 2 (one-bucket bins) they are all misses
            // A bin of one bucket has a single chain of updates; workgroups
            // run it on different wavefronts (blockIdx mod 4) so that the
            // chains of the workgroups sharing a CU spread over its SIMDs.
            const uint32_t g_one = ONE ? (blockIdx.x & 3u) * (uint32_t)(kWave / G) : 0u;
            for (uint32_t lb = group - g_one; lb < nbk; lb += n_groups) {
                uint32_t e1 = s_pos[lb];
                uint32_t e0 = lb ? s_pos[lb - 1] : 0;
                if constexpr (ONE) {
                    // a bin of one bucket has one active group, lanes [0, G)
                    // of one wavefront: its bounds are wave-uniform
                    e1 = __builtin_amdgcn_readfirstlane(e1);
                    e0 = __builtin_amdgcn_readfirstlane(e0);
                }
                if (e0 == e1) continue;  // uniform over the group
                const uint32_t sidx = lb * ell + j;
                KeyT k = real ? s_k[sidx] : (KeyT)0;
                uint32_t c = real ? s_c[sidx] : 0u;
                uint32_t e = real ? s_e[sidx] : 0u;
                float v = (OUTER && real) ? s_v[sidx] : 0.0f;
                uint8_t f = real ? s_f[sidx] : (uint8_t)0;
                auto step = [&](const KeyT key, const uint32_t w, const float val) {
                    const bool used = (f & kUsed) != 0;
                    bool missed = true;  // uniform over the group
                    if constexpr (!ONE) {
                        const bool hit = real && used && k == key;
                        const auto hg = group_bits<G>(__builtin_amdgcn_ballot_w64(hit), gsh);
                        // hit: the monitored slot takes the weight
                        if (hit) {
                            if (OUTER) {
                                c = __float_as_uint(__uint_as_float(c) + __uint_as_float(w));
                                v += val;
                            } else {
                                c += w;
                            }
                        }
                        missed = !hg;
                    }
                    const auto fg = group_bits<G>(__builtin_amdgcn_ballot_w64(real && !used), gsh);
                    // free: the lowest free slot takes the entry
                    if (missed && fg && j == lowest_bit(fg)) {
                        k = key;
                        c = w;
                        e = 0u;
                        v = val;
                        f = kUsed;
                    }
                    // evict: the lowest unpinned slot of minimum count
                    const bool need = missed && !fg;  // uniform over the group
                    if (__builtin_amdgcn_ballot_w64(need)) {
                        const bool cand = need && real && !(f & kPinned);
                        const uint32_t mine = cand ? c : 0xFFFFFFFFu;
                        const uint32_t mn = group_min<G>(mine);
                        const auto mg =
                            group_bits<G>(__builtin_amdgcn_ballot_w64(cand && mine == mn), gsh);
                        if (mg && j == lowest_bit(mg)) {
                            e = c;
                            c = OUTER ? __float_as_uint(__uint_as_float(c) + __uint_as_float(w))
                                      : c + w;
                            k = key;
                            v = val;
                        }
                    }
                };
                // Transaction counts take level steps (below) while every
                // count of the bin stays below 2^(30 - log2 G) - 1 (a count
                // is at most the bin's largest initial count plus its
                // k1 - k0 terms of unit weight); otherwise, and for outer
                // products, single steps.
                constexpr uint32_t LOGG = G == 16 ? 4u : G == 32 ? 5u : 6u;
                constexpr uint32_t kPackLim = 1u << (30 - LOGG);
                const uint32_t cmax0 = __builtin_amdgcn_readfirstlane(s_cmax);  // uniform
                const bool pack = !OUTER && (uint64_t)cmax0 + (k1 - k0) < kPackLim - 1;
                const uint32_t notreal = real ? 0u : 0xFFFFFFFFu;
                // Level steps (transactions): with ties broken by the
                // lowest slot, the single steps take the slots at the
                // minimum level (free slots below every count, then
                // count c at level c + 1) one by one in slot order, and
                // each taken slot rises by its weight (at least one)
                // above that level.  One step therefore applies the
                // next updates to all slots at the minimum level at
                // once, the r-th slot in slot order taking the r-th
                // update, read from the update list in LDS; the state is
                // the one the single steps reach.
                // (the group's ballot bits start at lane gsh; a bin of one
                // bucket has lanes [0, G): no shift, and its bits stay
                // scalar)
                using M = typename GroupMask<G>::T;
                const uint32_t sh = ONE ? 0u : gsh;
                auto chain_level = [&]() {
                    // pinned slots and padding never take an update; with
                    // every slot of the bucket pinned all updates drop
                    const uint32_t fixed = ((f & kPinned) ? 0xFFFFFFFFu : 0u) | notreal;
                    if (group_bits<G>(__builtin_amdgcn_ballot_w64(fixed == 0u), sh) == 0)
                        return;
                    const M below = ((M)1 << j) - (M)1;
                    for (uint32_t pos = e0; pos < e1;) {
                        // level offer: 0 free, c + 1 used (counts stay
                        // below 2^26), all ones if fixed
                        const uint32_t lvl = ((f & kUsed) ? c + 1u : 0u) | fixed;
                        const uint32_t mn = group_min<G>(lvl);
                        const M at = group_bits<G>(__builtin_amdgcn_ballot_w64(lvl == mn), sh);
                        const uint32_t take = min(bit_count(at), e1 - pos);
                        const uint32_t rank = bit_count(at & below);
                        if (lvl == mn && rank < take) {
                            const KeyT nk = t_k[pos + rank];
                            const uint32_t nw = t_w[pos + rank];
                            e = mn ? c : 0u;
                            c = mn ? c + nw : nw;
                            k = nk;
                            f |= kUsed;
                        }
                        pos += take;
                    }
                };
                if constexpr (ONE) {
                    // G updates per LDS load: lane j holds update p0 + j and
                    // each update is broadcast from its lane in turn, so the
                    // serial chain waits on LDS once per G updates
                    // (the trip count is read into a scalar register and the
                    // two update forms get loops of their own, so the loop
                    // control stays scalar)
                    auto chain = [&](auto apply) {
                        for (uint32_t p0 = e0; p0 < e1; p0 += G) {
                            const uint32_t q = p0 + j;
                            const KeyT bk = q < e1 ? t_k[q] : (KeyT)0;
                            const uint32_t bw = q < e1 ? t_w[q] : 0u;
                            const float bv = (OUTER && q < e1) ? t_v[q] : 0.0f;
                            const uint32_t cnt = (uint32_t)__builtin_amdgcn_readfirstlane(
                                (int)min((uint32_t)G, e1 - p0));
                            for (uint32_t i = 0; i < cnt; ++i) {
                                KeyT key;
                                if constexpr (sizeof(KeyT) == 8) {
                                    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(
                                        (int)(uint32_t)bk, (int)i);
                                    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(
                                        (int)(uint32_t)((uint64_t)bk >> 32), (int)i);
                                    key = (KeyT)(((uint64_t)hi << 32) | lo);
                                } else {
                                    key = (KeyT)(uint32_t)__builtin_amdgcn_readlane((int)bk,
                                                                                    (int)i);
                                }
                                const uint32_t w =
                                    (uint32_t)__builtin_amdgcn_readlane((int)bw, (int)i);
                                float val = 0.0f;
                                if (OUTER)
                                    val = __int_as_float(
                                        __builtin_amdgcn_readlane(__float_as_int(bv), (int)i));
                                apply(key, w, val);
                            }
                        }
                    };
                    if constexpr (!OUTER) {
                        if (pack)
                            chain_level();
                        else
                            chain([&](KeyT key, uint32_t w, float val) { step(key, w, val); });
                    } else {
                        chain([&](KeyT key, uint32_t w, float val) { step(key, w, val); });
                    }
                } else {
                    auto chain = [&](auto apply) {
                        KeyT nk = t_k[e0];
                        uint32_t nw = t_w[e0];
                        float nv = OUTER ? t_v[e0] : 0.0f;
                        for (uint32_t p = e0; p < e1; ++p) {
                            const KeyT key = nk;
                            const uint32_t w = nw;
                            const float val = nv;
                            if (p + 1 < e1) {  // prefetch the next update
                                nk = t_k[p + 1];
                                nw = t_w[p + 1];
                                if (OUTER) nv = t_v[p + 1];
                            }
                            apply(key, w, val);
                        }
                    };
                    if constexpr (!OUTER) {
                        // transactions: the hits were taken in step 2
                        if (pack)
                            chain_level();
                        else
                            chain([&](KeyT key, uint32_t w, float val) { step(key, w, val); });
                    } else {
                        chain([&](KeyT key, uint32_t w, float val) { step(key, w, val); });
                    }
                }
                if (real) {
                    s_k[sidx] = k;
                    s_c[sidx] = c;
                    s_e[sidx] = e;
                    if (OUTER) s_v[sidx] = v;
                    s_f[sidx] = f;
                }
            }
            __syncthreads();
            base = next;
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
            if constexpr (sizeof(KeyT) == 4)
                if (g_key32) g_key32[g0 + s] = (s_f[s] & kUsed) ? (uint32_t)s_k[s] : 0u;
            g_cnt[g0 + s] = s_c[s];
            g_err[g0 + s] = s_e[s];
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

// Counts are shifted left by the leading zeros of the largest count (st[7]),
// so the first radix digits separate the slots.
__device__ inline uint32_t count_shift(const uint32_t *st)
{
    return st[7] ? (uint32_t)__clz(st[7]) : 0u;
}

// Lower bound of a summary slot: count - overestimation (fp32 difference for
// outer products, never negative), as an order-preserving 32-bit word.
__device__ inline uint32_t lower_of(uint32_t c, uint32_t e, bool fp)
{
    if (!fp) return c - e;
    return __float_as_uint(fmaxf(__uint_as_float(c) - __uint_as_float(e), 0.0f));
}

// The ranked value of a slot as an order-preserving 32-bit word: the count
// (upper bound) or, when ranking by guaranteed count, the lower bound.  With
// err_is_lower the err array holds the lower bound itself (combined entries
// of an amplified run).
struct RankBy {
    const uint32_t *cnt, *err;
    bool lower, fp, err_is_lower;
    __device__ uint32_t operator()(uint64_t i) const
    {
        const uint32_t c = cnt[i];
        if (!lower) return c;
        if (err_is_lower) return err[i];
        return lower_of(c, err[i], fp);
    }
};

__device__ inline Comp comp_of(const uint64_t *key, const RankBy &rv, uint64_t i, uint32_t sh)
{
    const uint64_t k = key[i];
    return Comp{{rv(i) << sh, ~(uint32_t)(k >> 32), ~(uint32_t)k}};
}

__global__ void __launch_bounds__(256)
k_topk_max(RankBy rv, const uint8_t *__restrict__ flag, uint64_t n, uint32_t *__restrict__ st)
{
    __shared__ uint32_t s_mx[256 / kWave];
    uint32_t mx = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256)
        if (flag[i] & kUsed) mx = max(mx, rv(i));
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, kWave));
    if (lane_id() == 0) s_mx[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / kWave; ++w) mx = max(mx, s_mx[w]);
        if (mx) atomicMax(&st[7], mx);  // one atomic per workgroup
    }
}

// Append the lanes with `keep` to list[*count], one atomic per wavefront.
__device__ inline void wave_append(bool keep, uint32_t value, uint32_t *count, uint32_t *list)
{
    const uint64_t m = __ballot(keep);
    if (!m) return;
    const int first = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane_id() == (uint32_t)first) base = atomicAdd(count, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, first, kWave);
    if (keep) list[base + (uint32_t)__popcll(m & ((1ull << lane_id()) - 1))] = value;
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
//   st[5] selected count, st[6] used slots, st[7] largest count, hist[256].
//
// Histogram of one of the first four digits (the ranked value's bytes) over
// every used slot that matches the prefix so far; the slot's key (8 of its
// 17 bytes) is not read.
__global__ void __launch_bounds__(256)
k_topk_hist(RankBy rv, const uint8_t *__restrict__ flag, uint64_t n,
            const uint32_t *__restrict__ st, uint32_t pass, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t sh = count_shift(st);
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256) {
        if (!(flag[i] & kUsed)) continue;
        const Comp c{{rv(i) << sh, 0u, 0u}};
        if (!prefix_match(c, st, pass)) continue;
        atomicAdd(&h[digit_of(c, pass)], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// One wavefront: pick the digit of this pass and clear the histogram.
// Walking the digits from 255 down, the pick is the first digit d >= 1 at
// which the running count reaches the remaining rank (else 0); the new
// remaining rank excludes the digits above d.  Lane L holds digits
// 255 - 4L .. 252 - 4L, so a scan over lanes gives every running count.
// (one full wavefront, lane = its lane; st and hist in global memory or LDS)
__device__ inline void topk_pick_wave(uint32_t *st, uint32_t *hist, uint32_t pass, uint32_t K,
                                      uint32_t lane)
{
    uint32_t h[4], local = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = hist[255 - (4 * lane + q)];
        local += h[q];
    }
    const uint32_t incl = wave_inclusive_scan(local);
    uint32_t rem;
    if (pass == 0) {
        const uint32_t used = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
        rem = K < used ? K : used;
        if (lane == 0) st[6] = used;
    } else {
        rem = st[3];
    }
    uint32_t before[4], run = incl - local;
    int myq = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        before[q] = run;
        const uint32_t d = 255 - (4 * lane + q);
        if (myq < 0 && d >= 1 && run + h[q] >= rem) myq = q;
        run += h[q];
    }
    uint32_t d = 255, new_rem = rem;
    if (rem > 0) {
        const uint64_t m = __ballot(myq >= 0);
        uint32_t b = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (myq == q) b = before[q];
        if (m) {
            const int L = __ffsll((long long)m) - 1;
            const int qL = __shfl(myq, L, kWave);
            d = 255 - (4 * (uint32_t)L + (uint32_t)qL);
            new_rem = rem - (uint32_t)__shfl((int)b, L, kWave);
        } else {
            d = 0;  // digit 0: lane 63, slot 3
            new_rem = rem - (uint32_t)__shfl((int)before[3], kWave - 1, kWave);
        }
    }
    if (lane == 0) {
        st[3] = new_rem;
        const uint32_t w = pass >> 2, sh = 24 - 8 * (pass & 3);
        st[w] = (st[w] & ~(0xFFu << sh)) | (d << sh);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) hist[4 * lane + q] = 0;
}

__global__ void __launch_bounds__(64)
k_topk_pick(uint32_t *__restrict__ st, uint32_t *__restrict__ hist, uint32_t pass, uint32_t K)
{
    topk_pick_wave(st, hist, pass, K, threadIdx.x);
}

// Passes 2 .. 11 over the compacted candidates in one workgroup: the
// histogram and the selection state in LDS, each pass a histogram of the
// candidates that match the prefix so far and a pick by the first
// wavefront (the same steps as k_topk_hist and k_topk_pick, without a launch
// per pass).  After a pass over the global list, the candidates that still
// match the prefix are copied into an LDS list; once they fit (at most
// kFinishList), later passes read only that list.  The global list is left
// as it is (k_topk_collect reads it), and the state goes back to st at the
// end.
constexpr uint32_t kFinishList = 8192;
__global__ void __launch_bounds__(1024)
k_topk_finish(const uint64_t *__restrict__ key, RankBy rv, const uint8_t *__restrict__ flag,
              const uint32_t *__restrict__ cand, uint32_t *__restrict__ st, uint32_t K)
{
    __shared__ uint32_t h[256], s_st[8], s_list[kFinishList], s_n;
    if (threadIdx.x < 8) s_st[threadIdx.x] = st[threadIdx.x];
    __syncthreads();
    const uint32_t m = s_st[4];
    const uint32_t sh = count_shift(s_st);
    bool local = false;  // workgroup-uniform: the LDS list holds the candidates
    uint32_t n = m;
    for (uint32_t pass = 2; pass < 12; ++pass) {
        if (threadIdx.x < 256) h[threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < n; t += 1024) {
            const uint32_t i = local ? s_list[t] : cand[t];
            if (!(flag[i] & kUsed)) continue;
            const Comp c = comp_of(key, rv, i, sh);
            if (!prefix_match(c, s_st, pass)) continue;
            atomicAdd(&h[digit_of(c, pass)], 1u);
        }
        __syncthreads();
        if (threadIdx.x < kWave) topk_pick_wave(s_st, h, pass, K, threadIdx.x);
        __syncthreads();
        if (!local && pass + 1 < 12) {
            if (threadIdx.x == 0) s_n = 0;
            __syncthreads();
            for (uint32_t t = threadIdx.x; t < m; t += 1024) {
                const uint32_t i = cand[t];
                if (!(flag[i] & kUsed)) continue;
                if (!prefix_match(comp_of(key, rv, i, sh), s_st, pass + 1)) continue;
                const uint32_t j = atomicAdd(&s_n, 1u);
                if (j < kFinishList) s_list[j] = i;
            }
            __syncthreads();
            if (s_n <= kFinishList) {
                local = true;
                n = s_n;
            }
            __syncthreads();  // s_n is read by every thread before any reset
        }
    }
    if (threadIdx.x < 8) st[threadIdx.x] = s_st[threadIdx.x];
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
k_topk_compact(RankBy rv, const uint8_t *__restrict__ flag, uint64_t n,
               uint32_t *__restrict__ st, uint32_t *__restrict__ cand)
{
    const uint32_t sh = count_shift(st);
    const uint32_t lim = st[0] >> 16;
    // whole wavefronts iterate together so the append can use ballots
    const uint64_t n_all = (n + kWave - 1) / kWave * kWave;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n_all;
         i += (uint64_t)gridDim.x * 256) {
        const bool keep = i < n && (flag[i] & kUsed) && ((rv(i) << sh) >> 16) >= lim;
        wave_append(keep, (uint32_t)i, &st[4], cand);
    }
}

// Collect the selected slots (composite >= threshold): exactly st[3]-ranked.
__global__ void __launch_bounds__(256)
k_topk_collect(const uint64_t *__restrict__ key, RankBy rv,
               const uint32_t *__restrict__ cand, uint32_t *__restrict__ st,
               uint32_t *__restrict__ sel)
{
    const uint32_t m = st[4];
    const uint32_t sh = count_shift(st);
    const uint32_t m_all = (m + kWave - 1) / kWave * kWave;
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < m_all; t += gridDim.x * 256) {
        const uint32_t i = t < m ? cand[t] : 0u;
        wave_append(t < m && comp_ge(comp_of(key, rv, i, sh), st), i, &st[5], sel);
    }
}

// Rank of every selected slot = number of selected slots ranking above it,
// counted tile against tile: block (bi, bj) compares the 256 selected slots
// of tile bi with the 256 of tile bj and adds its counts to rank[] (zero on
// entry), so the m^2 comparisons spread over the whole GPU.
__global__ void __launch_bounds__(256)
k_topk_rank_tiles(const uint64_t *__restrict__ key, RankBy rv, const uint32_t *__restrict__ sel,
                  const uint32_t *__restrict__ st, uint32_t *__restrict__ rank)
{
    __shared__ Comp tile[256];
    const uint32_t m = st[5];
    const uint32_t i0 = blockIdx.x * 256;
    if (i0 >= m) return;  // uniform over the block
    const uint32_t sh = count_shift(st);
    const uint32_t t = i0 + threadIdx.x;
    const Comp me = t < m ? comp_of(key, rv, sel[t], sh) : Comp{{0, 0, 0}};
    // tiles bj = blockIdx.y, blockIdx.y + gridDim.y, ... (the grid's y size
    // is capped, so a large K still launches)
    for (uint32_t j0 = blockIdx.y * 256; j0 < m; j0 += gridDim.y * 256) {
        __syncthreads();
        if (j0 + threadIdx.x < m) tile[threadIdx.x] = comp_of(key, rv, sel[j0 + threadIdx.x], sh);
        __syncthreads();
        if (t < m) {
            const uint32_t lim = min(256u, m - j0);
            uint32_t r = 0;
            for (uint32_t q = 0; q < lim; ++q) r += comp_gt(tile[q], me) ? 1u : 0u;
            if (r) atomicAdd(&rank[t], r);
        }
    }
}

// Write every selected slot at its rank.
__global__ void __launch_bounds__(256)
k_topk_emit(const uint64_t *__restrict__ key, RankBy rv, const uint32_t *__restrict__ cnt,
            const uint32_t *__restrict__ err, const float *__restrict__ val, bool outer,
            const uint8_t *__restrict__ votes, const uint32_t *__restrict__ sel,
            const uint32_t *__restrict__ st, const uint32_t *__restrict__ rank,
            uint32_t *__restrict__ oi, uint32_t *__restrict__ oj, double *__restrict__ ou,
            double *__restrict__ ol, double *__restrict__ ov, uint32_t *__restrict__ ovotes)
{
    const uint32_t m = st[5];
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= m) return;
    const uint32_t r = rank[t];
    const uint32_t i = sel[t];
    const uint64_t k = key[i];
    oi[r] = (uint32_t)(k >> 32);
    oj[r] = (uint32_t)k;
    double c, e;
    if (outer) {
        c = (double)__uint_as_float(cnt[i]);
        e = (double)__uint_as_float(err[i]);
        ov[r] = (double)val[i];
    } else {
        c = (double)cnt[i];
        e = (double)err[i];
        ov[r] = c;
    }
    ou[r] = c;
    ol[r] = rv.err_is_lower ? e : c - e;
    ovotes[r] = votes ? votes[i] : 1u;
}

// Majority reporting over t independent instances (Section 6, proof of
// Theorem 2): an entry counts as reported by instance j when j's summaries
// monitor it, i.e. it sits in one of the ell slots of its bucket under j's
// hash functions.  Every monitored slot looks its entry up in the other
// instances' buckets; the lowest instance that monitors the entry owns it,
// so each entry is combined once.  Entries with at least min_votes votes get
// the intersection of the reporting instances' bounds (every instance's
// [lower, upper] holds the true weight, Section 4), so upper = the least
// count and lower = the largest lower bound; outer products also get the
// median of the reporting instances' signed sums (mean of the two middle
// values for an even number of votes).
template <bool OUTER>
__global__ void __launch_bounds__(256)
k_amp_combine(CsParams ip, uint32_t ell, uint64_t ns, uint32_t min_votes,
              const uint64_t *__restrict__ key, const uint32_t *__restrict__ key32,
              const uint32_t *__restrict__ cnt,
              const uint32_t *__restrict__ err, const float *__restrict__ val,
              const uint8_t *__restrict__ flag, uint32_t *__restrict__ up,
              uint32_t *__restrict__ lo, float *__restrict__ mv, uint8_t *__restrict__ oflag,
              uint8_t *__restrict__ votes)
{
    const uint64_t total = ns * ip.t;
    for (uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x; g < total;
         g += (uint64_t)gridDim.x * 256) {
        oflag[g] = 0;
        if (!(flag[g] & kUsed)) continue;
        const uint32_t inst = (uint32_t)(g / ns);
        uint32_t x, y;
        if (key32) {
            const uint32_t p32 = key32[g];
            x = p32 >> 16;
            y = p32 & 0xFFFFu;
        } else {
            const uint64_t k64 = key[g];
            x = (uint32_t)(k64 >> 32);
            y = (uint32_t)k64;
        }
        const uint64_t k = ((uint64_t)x << 32) | y;
        uint32_t v = 0, u = 0xFFFFFFFFu, l = 0;
        float sv[kCsMaxInstances];
        bool own = true;
        for (uint32_t j = 0; j < ip.t && own; ++j) {
            uint64_t q = g;
            if (j != inst) {
                const uint64_t b = interval_of(hash_a(ip.hp[j], x) + hash_b(ip.hp[j], y), ip.PB);
                const uint64_t base = (uint64_t)j * ns + b * ell;
                q = ~0ull;
                // keys first: a free slot's key is 0, so its flag is read only
                // when the entry's own key is 0 (outer products' (0, 0)).  The
                // keys are loaded eight at a time before any is compared, so
                // the loads of a bucket overlap; narrow runs compare the
                // packed 32-bit copies (half the bytes per bucket).
                if (key32 && (ell & 3u) == 0) {
                    // 16-byte loads: one request per four keys (base and r0
                    // are multiples of four when ell is)
                    const uint32_t k32 = (x << 16) | y;
                    for (uint32_t r0 = 0; r0 < ell && q == ~0ull; r0 += 8) {
                        uint4 kb[2];
                        kb[0] = *reinterpret_cast<const uint4 *>(key32 + base + r0);
                        kb[1] = r0 + 4 < ell
                                    ? *reinterpret_cast<const uint4 *>(key32 + base + r0 + 4)
                                    : make_uint4(~k32, ~k32, ~k32, ~k32);
                        const uint32_t kw[8] = {kb[0].x, kb[0].y, kb[0].z, kb[0].w,
                                                kb[1].x, kb[1].y, kb[1].z, kb[1].w};
#pragma unroll
                        for (uint32_t t = 0; t < 8; ++t)
                            if (q == ~0ull && kw[t] == k32 && (flag[base + r0 + t] & kUsed))
                                q = base + r0 + t;
                    }
                } else if (key32) {
                    const uint32_t k32 = (x << 16) | y;
                    for (uint32_t r0 = 0; r0 < ell && q == ~0ull; r0 += 8) {
                        uint32_t kb[8];
#pragma unroll
                        for (uint32_t t = 0; t < 8; ++t)
                            kb[t] = r0 + t < ell ? key32[base + r0 + t] : ~k32;
#pragma unroll
                        for (uint32_t t = 0; t < 8; ++t)
                            if (q == ~0ull && kb[t] == k32 && (flag[base + r0 + t] & kUsed))
                                q = base + r0 + t;
                    }
                } else {
                    for (uint32_t r0 = 0; r0 < ell && q == ~0ull; r0 += 8) {
                        uint64_t kb[8];
#pragma unroll
                        for (uint32_t t = 0; t < 8; ++t)
                            kb[t] = r0 + t < ell ? key[base + r0 + t] : ~k;
#pragma unroll
                        for (uint32_t t = 0; t < 8; ++t)
                            if (q == ~0ull && kb[t] == k && (flag[base + r0 + t] & kUsed))
                                q = base + r0 + t;
                    }
                }
                if (q == ~0ull) continue;
                if (j < inst) {
                    own = false;
                    break;
                }
            }
            const uint32_t c = cnt[q];
            u = min(u, c);
            l = max(l, lower_of(c, err[q], OUTER));
            if (OUTER) {
                // insertion into the sorted prefix sv[0..v)
                const float w = val[q];
                uint32_t p = v;
                while (p > 0 && sv[p - 1] > w) {
                    sv[p] = sv[p - 1];
                    --p;
                }
                sv[p] = w;
            }
            ++v;
        }
        if (!own || v < min_votes) continue;
        up[g] = u;
        lo[g] = l;
        if (OUTER) {
            const uint32_t h = v / 2;
            mv[g] = (v & 1u) ? sv[h] : 0.5f * (sv[h - 1] + sv[h]);
        } else {
            mv[g] = 0.0f;
        }
        votes[g] = (uint8_t)v;
        oflag[g] = kUsed;
    }
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
    if (ns <= kPinLds) {
        hipLaunchKernelGGL(k_ss_pin_lds, dim3(1), dim3(1024), 0, s, sx, sy, ns, r_max, hp, PB,
                           ell, S.key, S.flag, n_pinned);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_seed_dups, dim3((ns + 255) / 256), dim3(256), 0, s, sx, sy, ns, dup);
    hipLaunchKernelGGL(k_ss_pin, dim3((ns + 255) / 256), dim3(256), 0, s, sx, sy, ns, dup, r_max,
                       hp, PB, ell, S.key, S.flag, n_pinned);
    return hipGetLastError();
}

size_t ss_bins_smem_bytes(uint32_t nbk, uint32_t ell, bool wide_key, bool outer, uint32_t MB)
{
    return ss_layout(nbk, ell, wide_key ? 8 : 4, outer, MB).total;
}

uint32_t ss_group_width(uint32_t ell) { return ell <= 16 ? 16u : ell <= 32 ? 32u : 64u; }

// Workgroup size of the summary kernel, whatever the group width: 256
// threads for bins of one bucket (the merge and grouping phases use every
// lane while one group runs the chain; measured faster than workgroups sized
// to the bin's groups and than 512 threads), 512 for bins of several
// buckets (twice the wavefronts per CU for the latency-bound phases).
uint32_t ss_block_threads(uint32_t nbk, uint32_t ell)
{
    (void)ell;
    return nbk == 1 ? 256u : 512u;  // as k_ss_groups' BS for ONE and not ONE
}

// One launch of the summary kernel: bins of one bucket take the ONE variant.
template <int G, class KeyT, bool OUTER, int MB>
static void launch_ss_k(const crop_ctx *c, const SsState &S, uint32_t nbk, uint64_t PB,
                        uint32_t grid, uint32_t bs, bool narrow, const KeyT *keys,
                        const float *vals, bool fresh, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    const uint32_t ell = c->ss_ell;
    const size_t sm = ss_bins_smem_bytes(nbk, ell, sizeof(KeyT) == 8, OUTER, MB);
    if (nbk == 1)
        hipLaunchKernelGGL((k_ss_groups<G, KeyT, OUTER, MB, true>), dim3(grid), dim3(bs), sm, s,
                           c->bin_off.as<uint32_t>(), c->bin_order.as<uint32_t>(), keys, vals,
                           pl.NB, nbk, ell, c->hp, PB, narrow, c->counter.as<uint32_t>(), S.key,
                           S.cnt, S.err, S.val, S.flag, S.key32, fresh);
    else
        hipLaunchKernelGGL((k_ss_groups<G, KeyT, OUTER, MB, false>), dim3(grid), dim3(bs), sm, s,
                           c->bin_off.as<uint32_t>(), c->bin_order.as<uint32_t>(), keys, vals,
                           pl.NB, nbk, ell, c->hp, PB, narrow, c->counter.as<uint32_t>(), S.key,
                           S.cnt, S.err, S.val, S.flag, S.key32, fresh);
}

template <int G>
static void launch_ss_g(const crop_ctx *c, const SsState &S, uint32_t nbk, uint64_t PB,
                        uint32_t grid, uint32_t bs, bool fresh, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    if (c->in.mode == Mode::Outer)
        launch_ss_k<G, uint64_t, true, kSsBatchOuter>(c, S, nbk, PB, grid, bs, false,
                                                       c->keys.as<uint64_t>(),
                                                       c->vals.as<float>(), fresh, s);
    else if (c->in.wide_keys)
        launch_ss_k<G, uint64_t, false, kSsBatchWide>(c, S, nbk, PB, grid, bs, false,
                                                       c->keys.as<uint64_t>(), nullptr, fresh,
                                                       s);
    else if (pl.ss_mb == kSsBatchTxLarge)
        launch_ss_k<G, uint32_t, false, kSsBatchTxLarge>(c, S, nbk, PB, grid, bs, true,
                                                          c->keys.as<uint32_t>(), nullptr, fresh,
                                                          s);
    else
        launch_ss_k<G, uint32_t, false, kSsBatchTx>(c, S, nbk, PB, grid, bs, true,
                                                     c->keys.as<uint32_t>(), nullptr, fresh,
                                                     s);
}

hipError_t launch_ss_bins(const crop_ctx *c, const SsState &S, uint32_t nbk, uint64_t PB,
                          hipStream_t s, bool fresh)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint32_t ell = c->ss_ell;
    const uint32_t bs = ss_block_threads(nbk, ell);
    const uint32_t grid = std::min<uint32_t>(c->plan.NB, 4 * (uint32_t)cus);
    switch (ss_group_width(ell)) {
    case 16: launch_ss_g<16>(c, S, nbk, PB, grid, bs, fresh, s); break;
    case 32: launch_ss_g<32>(c, S, nbk, PB, grid, bs, fresh, s); break;
    default: launch_ss_g<64>(c, S, nbk, PB, grid, bs, fresh, s); break;
    }
    return hipGetLastError();
}

// Top-K over the summary slots; st (8 words) and hist (256 words) must be
// zero on entry; cand and sel hold up to nslots indices.
hipError_t launch_topk(const SsState &S, uint32_t K, bool outer, bool by_lower, bool err_is_lower,
                       const uint8_t *votes, uint32_t *st, uint32_t *hist, uint32_t *cand,
                       uint32_t *sel, uint32_t *rank, uint32_t *oi, uint32_t *oj, double *ou,
                       double *ol, double *ov, uint32_t *ovotes, hipStream_t s)
{
    const uint32_t g = grid_for(S.nslots);
    const RankBy rv{S.cnt, S.err, by_lower, outer, err_is_lower};
    hipLaunchKernelGGL(k_topk_max, dim3(grid_for(S.nslots, 1024)), dim3(256), 0, s, rv, S.flag,
                       S.nslots, st);
    // the first two digits over every slot, then the rest over the
    // candidates that share them, in one workgroup
    for (uint32_t pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_topk_hist, dim3(g), dim3(256), 0, s, rv, S.flag, S.nslots, st, pass,
                           hist);
        hipLaunchKernelGGL(k_topk_pick, dim3(1), dim3(64), 0, s, st, hist, pass, K);
    }
    hipLaunchKernelGGL(k_topk_compact, dim3(g), dim3(256), 0, s, rv, S.flag, S.nslots, st, cand);
    hipLaunchKernelGGL(k_topk_finish, dim3(1), dim3(1024), 0, s, S.key, rv, S.flag, cand, st, K);
    hipLaunchKernelGGL(k_topk_collect, dim3(g), dim3(256), 0, s, S.key, rv, cand, st, sel);
    const uint32_t gr = (K + 255) / 256 ? (K + 255) / 256 : 1;
    hipLaunchKernelGGL(k_zero32, dim3(grid_for(K, 1024)), dim3(256), 0, s, rank, K);
    hipLaunchKernelGGL(k_topk_rank_tiles, dim3(gr, std::min<uint32_t>(gr, 1024)), dim3(256), 0, s,
                       S.key, rv, sel, st, rank);
    hipLaunchKernelGGL(k_topk_emit, dim3(gr), dim3(256), 0, s, S.key, rv, S.cnt, S.err, S.val,
                       outer, votes, sel, st, rank, oi, oj, ou, ol, ov, ovotes);
    return hipGetLastError();
}

// Combined entries of t instances' summaries S (instance i at slots
// [i * nslots, (i + 1) * nslots)) into A (same indexing, keys shared with S).
hipError_t launch_amp_combine(const CsParams &ip, const SsState &S, uint32_t ell, uint64_t nslots,
                              uint32_t min_votes, bool outer, bool narrow, const SsState &A,
                              uint8_t *votes, hipStream_t s)
{
    const uint32_t *k32 = narrow ? S.key32 : nullptr;
    const uint32_t g = grid_for(nslots * ip.t, 8192);
    if (outer)
        hipLaunchKernelGGL(k_amp_combine<true>, dim3(g), dim3(256), 0, s, ip, ell, nslots,
                           min_votes, S.key, k32, S.cnt, S.err, S.val, S.flag, A.cnt, A.err,
                           A.val, A.flag, votes);
    else
        hipLaunchKernelGGL(k_amp_combine<false>, dim3(g), dim3(256), 0, s, ip, ell, nslots,
                           min_votes, S.key, k32, S.cnt, S.err, S.val, S.flag, A.cnt, A.err,
                           A.val, A.flag, votes);
    return hipGetLastError();
}

}  // namespace crop
