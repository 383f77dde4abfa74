// Exact accumulation of each routing bin in an LDS open-addressing table.
//
// A partition's exact result is the weight of every entry it owns
// (Section 4: sum_k a_k(i) b_k(j); Section 7: pair supports).  The paper
// sets its shared-nothing owners against one big table that all processors
// update at random (Section 7.3, throughput discussion): here every routing
// bin belongs to one workgroup, whose table lives in that CU's LDS, so all
// random updates are on-chip and no two workgroups share an entry.
//
// Persistent workgroups pull bins from a counter.  A bin's keys are read
// once, coalesced, and inserted with linear probing: compare-and-swap claims
// an empty slot, an atomic add accumulates.  Packed 32-bit keys use 64-bit
// slots (key and count in one word, k_aggregate_flat); 64-bit keys and fp32
// sums use separate key and weight arrays, and each wavefront first merges
// repeated copies of its lead key (k_aggregate).  When the table passes its
// fill limit the workgroup stops inserting and entries that are not present
// are spilled to HBM with their weight; once the key set is frozen (at a
// barrier) the table is written out and the spilled entries are accumulated
// in further rounds.  The table's entries and a later round's entries are
// disjoint, so every key is written exactly once.  Output: distinct keys in
// place of the bin's routed keys, weights in a parallel array, and the bin's
// entry count.
#include <type_traits>

#include "crop_device.hpp"
#include "crop_internal.hpp"
#include "crop_runs.hpp"

namespace crop {

namespace {

template <class KeyT> struct Empty;
template <> struct Empty<uint64_t> { static constexpr uint64_t v = kEmpty64; };

template <class KeyT>
__device__ inline KeyT shfl_key(KeyT k, int src)
{
    if (sizeof(KeyT) == 4) return (KeyT)lane_value((uint32_t)k, (uint32_t)src);
    uint32_t lo = lane_value((uint32_t)k, (uint32_t)src);
    uint32_t hi = lane_value((uint32_t)((uint64_t)k >> 32), (uint32_t)src);
    return (KeyT)(((uint64_t)hi << 32) | lo);
}

// Merge lanes of the wavefront that hold the same key as the first open
// lane (two rounds): the lowest such lane takes the total unit weight, the
// others drop out.  Lanes with w == 0 do not take part.
template <class KeyT>
__device__ inline void wave_merge_unit(KeyT key, uint32_t &w)
{
    bool open = w != 0;
    const uint32_t lane = lane_id();
#pragma unroll
    for (int round = 0; round < 2; ++round) {
        uint64_t act = __ballot(open);
        if (act == 0) break;
        int leader = __ffsll((long long)act) - 1;
        KeyT lk = shfl_key(key, leader);
        bool eq = open && key == lk;
        uint64_t m = __ballot(eq);
        if (eq) {
            open = false;
            w = (lane == (uint32_t)leader) ? (uint32_t)__popcll(m) : 0u;
        }
    }
}

// One round of wave_merge_unit for 32-bit keys: lanes holding the first open
// lane's key hand their weight to the lowest of them.
__device__ inline void wave_merge_lead(uint32_t key, uint32_t &w)
{
    const bool open = w != 0;
    const uint64_t act = __ballot(open);
    if (act == 0) return;
    const int leader = __ffsll((long long)act) - 1;
    const uint32_t lk = lane_value(key, (uint32_t)leader);
    const bool eq = open && key == lk;
    const uint64_t m = __ballot(eq);
    if (eq) w = (lane_id() == (uint32_t)leader) ? (uint32_t)__popcll(m) : 0u;
}

template <class KeyT, class W>
struct Table {
    KeyT *k;
    W *w;
    uint32_t mask, log2;
};

__device__ inline void add_weight(uint32_t *p, uint32_t w) { atomicAdd(p, w); }
__device__ inline void add_weight(float *p, float w) { atomicAdd(p, w); }

// Returns false when the key is absent and may not be inserted.
template <class KeyT, class W>
__device__ inline bool table_add(const Table<KeyT, W> &t, KeyT key, W w, bool may_insert,
                                 uint32_t *s_occ)
{
    uint32_t s = slot_of(key, t.log2);
    for (;;) {
        KeyT cur = t.k[s];
        if (cur == key) {
            add_weight(&t.w[s], w);
            return true;
        }
        if (cur == Empty<KeyT>::v) {
            if (!may_insert) return false;
            KeyT old = atomicCAS(&t.k[s], Empty<KeyT>::v, key);
            if (old == Empty<KeyT>::v) {
                atomicAdd(s_occ, 1u);
                add_weight(&t.w[s], w);
                return true;
            }
            if (old == key) {
                add_weight(&t.w[s], w);
                return true;
            }
        }
        s = (s + 1) & t.mask;
    }
}

template <class KeyT, class W>
struct Spilled {
    KeyT key;
    W w;
};

// Write the table's entries to keys_out/w_out starting at *s_nout.
template <int BS, class KeyT, class W>
__device__ inline void table_dump(const Table<KeyT, W> &t, uint32_t S, KeyT *keys_out, W *w_out,
                                  uint32_t *s_nout)
{
    const uint32_t lane = lane_id();
    for (uint32_t s0 = 0; s0 < S; s0 += BS) {
        uint32_t s = s0 + threadIdx.x;
        bool has = s < S && t.k[s] != Empty<KeyT>::v;
        uint64_t m = __ballot(has);
        uint32_t n = (uint32_t)__popcll(m);
        uint32_t base = 0;
        if (n) {
            if (lane == (uint32_t)(__ffsll((long long)m) - 1)) base = atomicAdd(s_nout, n);
            base = lane_value(base, (uint32_t)(__ffsll((long long)m) - 1));
        }
        if (has) {
            uint32_t r = (uint32_t)__popcll(m & ((1ull << lane) - 1));
            keys_out[base + r] = t.k[s];
            w_out[base + r] = t.w[s];
        }
    }
}

template <int BS, class KeyT, class W>
__device__ inline void table_clear(const Table<KeyT, W> &t, uint32_t S)
{
    for (uint32_t s = threadIdx.x; s < S; s += BS) {
        t.k[s] = Empty<KeyT>::v;
        t.w[s] = (W)0;
    }
}

// One persistent workgroup per CU.  Input: keys[bin_off[b] .. bin_off[b+1])
// (one term each) and, for weighted input (sums), vals.  Output in place of
// the keys: distinct keys and their weights in w_out, count in bin_size[b].
template <int BS, class KeyT, class W, int LOG2S>
__global__ void __launch_bounds__(BS)
k_aggregate(const uint32_t *__restrict__ bin_off, KeyT *__restrict__ keys,
            const float *__restrict__ vals, W *__restrict__ w_out, uint32_t *__restrict__ bin_size,
            Spilled<KeyT, W> *__restrict__ spill, uint32_t NB, uint32_t *counter,
            uint32_t cap_soft)
{
    constexpr uint32_t S = 1u << LOG2S;
    constexpr int U = 4;  // keys per thread per batch
    __shared__ KeyT s_k[S];
    __shared__ W s_w[S];
    __shared__ uint32_t s_occ, s_nout, s_nspill, s_bin;
    __shared__ int s_insert;
    const Table<KeyT, W> t{s_k, s_w, S - 1, LOG2S};

    for (;;) {
        if (threadIdx.x == 0) s_bin = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t b = s_bin;
        if (b >= NB) break;
        const uint32_t k0 = bin_off[b], k1 = bin_off[b + 1];
        table_clear<BS>(t, S);
        if (threadIdx.x == 0) {
            s_occ = 0;
            s_nout = 0;
            s_nspill = 0;
            s_insert = 1;
        }
        __syncthreads();

        // first round: the routed terms
        for (uint32_t base = k0; base < k1; base += BS * U) {
            KeyT kk[U];
            W ww[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                uint32_t i = base + u * BS + threadIdx.x;
                bool valid = i < k1;
                kk[u] = valid ? keys[i] : Empty<KeyT>::v;
                if constexpr (std::is_same<W, uint32_t>::value) {
                    uint32_t w1 = valid ? 1u : 0u;
                    wave_merge_unit(kk[u], w1);
                    ww[u] = (W)w1;
                } else {
                    ww[u] = valid ? (W)vals[i] : (W)0;
                    if (!valid) kk[u] = Empty<KeyT>::v;
                }
            }
            const bool ins = s_insert != 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                bool live = kk[u] != Empty<KeyT>::v;
                if constexpr (std::is_same<W, uint32_t>::value) live = live && ww[u] != 0;
                if (live && !table_add(t, kk[u], ww[u], ins, &s_occ)) {
                    uint32_t p = atomicAdd(&s_nspill, 1u);
                    spill[k0 + p] = Spilled<KeyT, W>{kk[u], ww[u]};
                }
            }
            __syncthreads();
            if (threadIdx.x == 0 && s_occ > cap_soft) s_insert = 0;
            __syncthreads();
        }
        table_dump<BS>(t, S, keys + k0, w_out + k0, &s_nout);
        __syncthreads();

        // later rounds: spilled entries (in place in the spill segment)
        while (s_nspill != 0) {
            const uint32_t n = s_nspill;
            __syncthreads();
            table_clear<BS>(t, S);
            if (threadIdx.x == 0) {
                s_occ = 0;
                s_nspill = 0;
                s_insert = 1;
            }
            __syncthreads();
            for (uint32_t base = 0; base < n; base += BS) {
                uint32_t i = base + threadIdx.x;
                Spilled<KeyT, W> e{Empty<KeyT>::v, (W)0};
                if (i < n) e = spill[k0 + i];
                const bool ins = s_insert != 0;
                __syncthreads();  // every entry of this batch is read before any rewrite
                if (i < n && !table_add(t, e.key, e.w, ins, &s_occ)) {
                    uint32_t p = atomicAdd(&s_nspill, 1u);
                    spill[k0 + p] = e;
                }
                __syncthreads();
                if (threadIdx.x == 0 && s_occ > cap_soft) s_insert = 0;
                __syncthreads();
            }
            table_dump<BS>(t, S, keys + k0, w_out + k0, &s_nout);
            __syncthreads();
        }
        if (threadIdx.x == 0) bin_size[b] = s_nout;
        __syncthreads();
    }
}

// ---- packed table for 32-bit keys with 32-bit counts (transaction pairs)
//
// One 64-bit LDS word per slot: key in the low half (kEmpty32 when free),
// count in the high half.  A hit is one 64-bit atomic add of (w << 32); an
// insertion is one compare-and-swap of the whole word, so key and count
// appear together.

constexpr uint64_t kFreeSlot = 0x00000000FFFFFFFFull;

// The count half of a packed slot (little-endian: the high word).  Adding
// to it with a 32-bit atomic leaves the key half untouched.
__device__ inline uint32_t *count_word(uint64_t *slot)
{
    return reinterpret_cast<uint32_t *>(slot) + 1;
}

enum { kDone = 0, kInserted = 1, kAbsent = 2 };

template <uint32_t MASK, uint32_t LOG2S>
__device__ inline int packed_add(uint64_t *tab, uint32_t key, uint32_t w, bool may_insert)
{
    uint32_t s = slot_of(key, LOG2S);
    uint64_t v = tab[s];
    for (;;) {
        const uint32_t k = (uint32_t)v;
        if (k == key) {
            atomicAdd(count_word(&tab[s]), w);
            return kDone;
        }
        if (k == kEmpty32) {
            if (!may_insert) return kAbsent;
            const uint64_t old = atomicCAS((unsigned long long *)&tab[s], (unsigned long long)v,
                                           ((unsigned long long)w << 32) | key);
            if (old == v) return kInserted;
            v = old;  // taken meanwhile: look at the new occupant of the same slot
            continue;
        }
        s = (s + 1) & MASK;
        v = tab[s];
    }
}

template <int BS, int LOG2S>
__device__ inline void packed_dump(const uint64_t *tab, uint32_t *keys_out, uint32_t *w_out,
                                   uint32_t *s_nout)
{
    constexpr uint32_t S = 1u << LOG2S;
    const uint32_t lane = lane_id();
    for (uint32_t s0 = 0; s0 < S; s0 += BS) {
        const uint64_t v = tab[s0 + threadIdx.x];
        const bool has = (uint32_t)v != kEmpty32;
        const uint64_t m = __ballot(has);
        const uint32_t n = (uint32_t)__popcll(m);
        uint32_t base = 0;
        if (n) {
            const int first = __ffsll((long long)m) - 1;
            if (lane == (uint32_t)first) base = atomicAdd(s_nout, n);
            base = lane_value(base, (uint32_t)first);
        }
        if (has) {
            const uint32_t r = (uint32_t)__popcll(m & ((1ull << lane) - 1));
            keys_out[base + r] = (uint32_t)v;
            w_out[base + r] = (uint32_t)(v >> 32);
        }
    }
}

// After the table's key set is frozen: spilled entries whose key is in the
// table add their weight there; the others stay in the spill list, which is
// compacted in place (a batch is read before any entry is rewritten, and
// the kept entries never outnumber the entries read).  Afterwards the spill
// list and the table hold disjoint keys.
template <int BS, int LOG2S>
__device__ void packed_absorb_spill(uint64_t *tab, Spilled<uint32_t, uint32_t> *spill,
                                    uint32_t k0, uint32_t *s_nspill_p)
{
    constexpr uint32_t MASK = (1u << LOG2S) - 1;
    uint32_t &s_nspill = *s_nspill_p;
    const uint32_t n = s_nspill;
    __syncthreads();
    if (threadIdx.x == 0) s_nspill = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += BS) {
        const uint32_t i = base + threadIdx.x;
        Spilled<uint32_t, uint32_t> e{kEmpty32, 0u};
        if (i < n) e = spill[k0 + i];
        __syncthreads();
        if (i < n && packed_add<MASK, LOG2S>(tab, e.key, e.w, false) == kAbsent)
            spill[k0 + atomicAdd(&s_nspill, 1u)] = e;
        __syncthreads();
    }
}

// Further rounds over a bin's spilled (key, weight) pairs until none is
// left: each round fills the emptied table up to cap_soft and dumps it.
template <int BS, int LOG2S>
__device__ void packed_spill_rounds(uint64_t *tab, Spilled<uint32_t, uint32_t> *spill,
                                    uint32_t k0, uint32_t *keys, uint32_t *w_out,
                                    uint32_t cap_soft, uint32_t *s_occ_p, uint32_t *s_nout,
                                    uint32_t *s_nspill_p, int *s_insert_p)
{
    constexpr uint32_t S = 1u << LOG2S;
    constexpr uint32_t MASK = S - 1;
    uint32_t &s_occ = *s_occ_p;
    uint32_t &s_nspill = *s_nspill_p;
    int &s_insert = *s_insert_p;
    while (s_nspill != 0) {
        const uint32_t n = s_nspill;
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < S; s += BS) tab[s] = kFreeSlot;
        if (threadIdx.x == 0) {
            s_occ = 0;
            s_nspill = 0;
            s_insert = 1;
        }
        __syncthreads();
        for (uint32_t base = 0; base < n; base += BS) {
            const uint32_t i = base + threadIdx.x;
            Spilled<uint32_t, uint32_t> e{kEmpty32, 0u};
            if (i < n) e = spill[k0 + i];
            const bool ins = s_insert != 0;
            __syncthreads();  // the batch is read before any entry is rewritten
            uint32_t n_new = 0;
            if (i < n) {
                const int r = packed_add<MASK, LOG2S>(tab, e.key, e.w, ins);
                if (r == kInserted) {
                    n_new = 1;
                } else if (r == kAbsent) {
                    const uint32_t p = atomicAdd(&s_nspill, 1u);
                    spill[k0 + p] = e;
                }
            }
            if (n_new) atomicAdd(&s_occ, 1u);
            __syncthreads();
            if (threadIdx.x == 0 && s_occ > cap_soft) s_insert = 0;
            __syncthreads();
        }
        packed_dump<BS, LOG2S>(tab, keys + k0, w_out + k0, s_nout);
        __syncthreads();
    }
}

// One wavefront batch of the packed table: U keys per lane with weights
// wt[u] (0: no key).  Copies of the wavefront's lead key merge into its
// lowest lane first.  Every key then looks at its home slot only: a hit
// adds its weight (no wait), a free home is claimed with a compare-and-swap
// (issued for all keys before any result is looked at).  A key whose home
// holds another key -- for good: slots are never freed -- goes to the
// wavefront's queue q (2 x 64 entries, qn of them in use), which is drained
// a full wavefront at a time by linear probing from home + 1, so the probe
// loops run with every lane busy; flush drains what is left (the
// wavefront's last batch of the bin).  With ins false a key that is not
// present is spilled instead (k0: the bin's spill segment).  Returns the
// keys this lane inserted.
template <int U, int LOG2S>
__device__ inline uint32_t packed_insert_batch(uint64_t *tab, const uint32_t (&cur)[U],
                                               uint32_t (&wt)[U], bool ins,
                                               Spilled<uint32_t, uint32_t> *spill, uint32_t k0,
                                               uint32_t *s_nspill, uint2 *q, uint32_t &qn,
                                               bool flush)
{
    constexpr uint32_t MASK = (1u << LOG2S) - 1;
    const uint32_t lane = lane_id();
    uint32_t n_new = 0, hs[U];
    uint64_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        wave_merge_lead(cur[u], wt[u]);
        hs[u] = slot_of(cur[u], LOG2S);
        v[u] = tab[hs[u]];
    }
    uint32_t slow = 0, cas = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (!wt[u]) continue;
        const uint32_t k = (uint32_t)v[u];
        if (k == cur[u]) {
            atomicAdd(count_word(&tab[hs[u]]), wt[u]);
        } else if (k == kEmpty32) {
            // absent: no key of this probe sequence lies past a free slot
            if (ins)
                cas |= 1u << u;
            else
                spill[k0 + atomicAdd(s_nspill, 1u)] = Spilled<uint32_t, uint32_t>{cur[u], wt[u]};
        } else {
            slow |= 1u << u;
        }
    }
    uint64_t old[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        if ((cas >> u) & 1u)
            old[u] = atomicCAS((unsigned long long *)&tab[hs[u]], (unsigned long long)kFreeSlot,
                               ((unsigned long long)wt[u] << 32) | cur[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (!((cas >> u) & 1u)) continue;
        if (old[u] == kFreeSlot)
            ++n_new;
        else if ((uint32_t)old[u] == cur[u])
            atomicAdd(count_word(&tab[hs[u]]), wt[u]);
        else
            slow |= 1u << u;  // another key took the home slot
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool sl = (slow >> u) & 1u;
        const uint64_t m = __ballot(sl);
        if (sl) q[qn + __popcll(m & ((1ull << lane) - 1))] = make_uint2(cur[u], wt[u]);
        qn += (uint32_t)__popcll(m);
        // drain: the queue holds fewer than 64 keys between drains, so at
        // most 2 x 64 after an enqueue
        while (qn >= (uint32_t)kWave || (u == U - 1 && flush && qn)) {
            const uint32_t take = qn < (uint32_t)kWave ? qn : (uint32_t)kWave;
            const uint32_t base = qn - take;
            bool live = lane < take;
            const uint2 e = live ? q[base + lane] : make_uint2(kEmpty32, 0u);
            qn = base;
            uint32_t at = (slot_of(e.x, LOG2S) + 1) & MASK;
            uint64_t val = live ? tab[at] : 0;
            while (live) {
                const uint32_t k = (uint32_t)val;
                if (k == e.x) {
                    atomicAdd(count_word(&tab[at]), e.y);
                    live = false;
                } else if (k == kEmpty32) {
                    if (!ins) {
                        spill[k0 + atomicAdd(s_nspill, 1u)] = Spilled<uint32_t, uint32_t>{e.x, e.y};
                        live = false;
                    } else {
                        const uint64_t o = atomicCAS((unsigned long long *)&tab[at],
                                                     (unsigned long long)kFreeSlot,
                                                     ((unsigned long long)e.y << 32) | e.x);
                        if (o == kFreeSlot) {
                            ++n_new;
                            live = false;
                        } else {
                            val = o;  // taken meanwhile: look at the new occupant
                        }
                    }
                } else {
                    at = (at + 1) & MASK;
                    val = tab[at];
                }
            }
        }
    }
    return n_new;
}

// Flat variant of the packed aggregation: every wavefront walks its own
// batches of the bin (64 U keys: U per lane, two batches loaded ahead, in
// three register sets used in turn) and runs them through
// packed_insert_batch.  There is no barrier between
// batches: a wavefront decides whether it may insert from the workgroup's
// insert counter, read before each batch and raised by the batch's inserts
// right after it.  A wavefront has at most one batch whose inserts are not
// yet counted, and a batch inserts at most its own 64 U keys plus the fewer
// than 64 it found queued, so when the last batch allowed to insert read at
// most cap_soft, the table never holds more than cap_soft + BS (U + 1) keys.
template <int BS, int LOG2S, int U>
__global__ void __launch_bounds__(BS)
k_aggregate_flat(const uint32_t *__restrict__ bin_off, uint32_t *__restrict__ keys,
                 uint32_t *__restrict__ w_out, uint32_t *__restrict__ bin_size,
                 Spilled<uint32_t, uint32_t> *__restrict__ spill, uint32_t NB,
                 uint32_t *counter, uint32_t cap_soft, const uint32_t *__restrict__ order)
{
    constexpr uint32_t S = 1u << LOG2S;
    constexpr uint32_t NW = BS / kWave;       // wavefronts
    constexpr uint32_t WB = kWave * U;        // keys of one wavefront batch
    static_assert(S % BS == 0, "table size must be a multiple of the block size");
    static_assert(S > BS * U, "a batch must fit in the table");
    __shared__ uint64_t tab[S];
    __shared__ uint2 s_q[NW][2 * kWave];  // each wavefront's queue of keys to probe
    __shared__ uint32_t s_occ, s_nout, s_nspill, s_bin;
    __shared__ int s_insert;
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x / kWave;

    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t i = atomicAdd(counter, 1u);
            s_bin = i < NB ? order[i] : NB;
        }
        __syncthreads();
        const uint32_t b = s_bin;
        if (b >= NB) break;
        const uint32_t k0 = bin_off[b], k1 = bin_off[b + 1];
        for (uint32_t s = threadIdx.x; s < S; s += BS) tab[s] = kFreeSlot;
        if (threadIdx.x == 0) {
            s_occ = 0;
            s_nout = 0;
            s_nspill = 0;
        }
        const uint32_t last = k1 - 1;  // read only when the bin is not empty
        uint32_t base = k0 + wave * WB;
        // the batch at bb (positions past the bin read its last key)
        auto load = [&](uint32_t (&k)[U], uint32_t bb) {
#pragma unroll
            for (int u = 0; u < U; ++u) k[u] = keys[min(bb + u * kWave + lane, last)];
        };
        uint32_t qn = 0;
        auto insert = [&](const uint32_t (&k)[U], uint32_t bb) {
            const bool ins =
                __hip_atomic_load(&s_occ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <=
                cap_soft;
            // copies of each wavefront's lead key merge into its lowest lane
            // (a hot pair fills most of its bin; one atomic instead of many)
            uint32_t cur[U], wt[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cur[u] = k[u];
                wt[u] = bb + u * kWave + lane < k1 ? 1u : 0u;
            }
            const uint32_t n_new = packed_insert_batch<U, LOG2S>(
                tab, cur, wt, ins, spill, k0, &s_nspill, s_q[wave], qn, bb + NW * WB >= k1);
            const uint32_t tot = wave_count_sum(n_new);
            if (lane == 0 && tot) atomicAdd(&s_occ, tot);
        };
        // three batches in rotation by name (register copies would wait for
        // the loads being copied): batch i + 2 is loaded while batch i is
        // inserted
        uint32_t kA[U], kB[U], kC[U];
        if (base < k1) {
            load(kA, base);
            load(kB, base + NW * WB);
        }
        __syncthreads();
        for (;;) {
            if (base >= k1) break;
            load(kC, base + 2 * NW * WB);
            insert(kA, base);
            base += NW * WB;
            if (base >= k1) break;
            load(kA, base + 2 * NW * WB);
            insert(kB, base);
            base += NW * WB;
            if (base >= k1) break;
            load(kB, base + 2 * NW * WB);
            insert(kC, base);
            base += NW * WB;
        }
        __syncthreads();  // keys of the bin are consumed; the spill list is complete
        // a wavefront may have spilled a key that a slower one inserted
        packed_absorb_spill<BS, LOG2S>(tab, spill, k0, &s_nspill);
        packed_dump<BS, LOG2S>(tab, keys + k0, w_out + k0, &s_nout);
        __syncthreads();
        packed_spill_rounds<BS, LOG2S>(tab, spill, k0, keys, w_out, cap_soft, &s_occ, &s_nout,
                                       &s_nspill, &s_insert);
        if (threadIdx.x == 0) bin_size[b] = s_nout;
        __syncthreads();
    }
}

// The packed aggregation fed straight from the region route: bin b's keys
// are one run in each sub-batch region (its bin starts in the transposed
// header), read where the route wrote them instead of from a bin-contiguous
// copy.  Wavefront w takes the sub-batches [w n_sub / NW, (w + 1) n_sub /
// NW), 64 at a time: one lane per sub-batch reads the run of bin b (the
// header words of the next 64 already loaded), the non-empty runs are
// listed in the wavefront's own LDS (routed position, keys before), and
// sb_span maps 64 consecutive positions of the list to routed positions.  U
// such spans make a batch for packed_insert_batch, two batches loaded
// ahead, as in k_aggregate_flat; the output (distinct keys and counts from
// bin_off[b], the spill segment there) is the same.
template <int BS, int LOG2S, int U>
__global__ void __launch_bounds__(BS)
k_aggregate_regions(const uint16_t *__restrict__ hdrT, const SbSeg *__restrict__ segs,
                    const uint32_t *__restrict__ bin_seg,
                    const uint32_t *__restrict__ sb_base, const uint32_t *__restrict__ routed,
                    const uint32_t *__restrict__ bin_off, uint32_t *__restrict__ keys,
                    uint32_t *__restrict__ w_out, uint32_t *__restrict__ bin_size,
                    Spilled<uint32_t, uint32_t> *__restrict__ spill, uint32_t NB,
                    uint32_t *counter, uint32_t cap_soft, const uint32_t *__restrict__ order)
{
    constexpr uint32_t S = 1u << LOG2S;
    constexpr uint32_t NW = BS / kWave;
    static_assert(S % BS == 0, "table size must be a multiple of the block size");
    static_assert(S > BS * U, "a batch must fit in the table");
    __shared__ uint64_t tab[S];
    __shared__ uint2 s_q[NW][2 * kWave];  // each wavefront's queue of keys to probe
    __shared__ uint32_t s_rb[NW][kWave], s_rp[NW][kWave + 1], s_flag[NW][kWave];
    __shared__ uint32_t s_occ, s_nout, s_nspill, s_bin;
    __shared__ int s_insert;
    const uint32_t lane = lane_id();
    // (wavefront-uniform, so the wavefront's LDS arrays get scalar bases)
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    uint32_t *rb = s_rb[wave], *rp = s_rp[wave], *wflag = s_flag[wave];
    wflag[lane] = 0;
    uint32_t tag = 0;  // the span tags only grow, so old flags never match

    // Bins are dealt per XCD: the workgroups of XCD x (block % 8) take the
    // x-th eighth of the bins, heaviest first, then in index order
    // (counter[x]; order[] is ordered per eighth), so the bins in flight on
    // one XCD are neighbours whose runs share lines in its L2.  A workgroup
    // whose eighth is dealt out takes bins of the next eighths.
    const uint32_t home = blockIdx.x % kNumXcd;
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t bin = NB;
            for (uint32_t k = 0; k < (uint32_t)kNumXcd && bin == NB; ++k) {
                const uint32_t x = (home + k) % kNumXcd;
                const uint32_t lo = (uint32_t)((uint64_t)NB * x / kNumXcd);
                const uint32_t hi = (uint32_t)((uint64_t)NB * (x + 1) / kNumXcd);
                // an eighth already dealt out is not counted further
                if (__hip_atomic_load(&counter[x], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT) >= hi - lo)
                    continue;
                const uint32_t i = atomicAdd(&counter[x], 1u);
                if (lo + i < hi) bin = order[lo + i];
            }
            s_bin = bin;
        }
        __syncthreads();
        const uint32_t b = s_bin;
        if (b >= NB) break;
        const uint32_t k0 = bin_off[b];
        for (uint32_t s = threadIdx.x; s < S; s += BS) tab[s] = kFreeSlot;
        if (threadIdx.x == 0) {
            s_occ = 0;
            s_nout = 0;
            s_nspill = 0;
        }
        // the bin's segment (its sub-batches and transposed header rows),
        // this wavefront's share of the sub-batches, and the header words of
        // the next 64
        const SbSeg &sg = segs[bin_seg ? bin_seg[b] : 0u];
        const uint32_t n_sub = sg.n_sub, sub0 = sg.sub0;
        uint32_t g = (uint32_t)(((uint64_t)n_sub * wave) / NW);
        const uint32_t g_end = (uint32_t)(((uint64_t)n_sub * (wave + 1)) / NW);
        const uint16_t *h0 = hdrT + sg.hdrT0 + (size_t)(b - sg.bin0) * sg.hts, *h1 = h0 + sg.hts;
        uint32_t na = 0, ne = 0, nbase = 0;
        auto load_rows = [&]() {
            const uint32_t sb = g + lane;
            na = ne = nbase = 0;
            if (sb < g_end) {
                na = h0[sb];
                ne = h1[sb];
                nbase = sb_base[sub0 + sb];
            }
        };
        load_rows();
        // the listed runs: count, keys, next position and the run holding it
        uint32_t nr = 0, tk = 0, c = 0, r0 = 0;
        // Positions c .. c + 63 of the listed runs (a new list once they are
        // used up): the load of each lane's key (ok: the lane has one);
        // false when the wavefront's keys are done (wavefront-uniform).
        auto span = [&](uint32_t &key, bool &ok) {
            while (c >= tk && g < g_end) {
                const uint32_t len = ne - na;
                const uint32_t incl = wave_inclusive_scan(len);
                const uint64_t nz = __ballot(len != 0u);
                // the last list's reads are complete before it is rewritten
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                if (len) {
                    const uint32_t ri = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(nz >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)nz, 0u));
                    rb[ri] = nbase + na;
                    rp[ri] = incl - len;
                }
                nr = (uint32_t)__popcll(nz);
                tk = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
                if (lane == 0) rp[nr] = tk;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                c = 0;
                r0 = 0;
                g += kWave;
                load_rows();
            }
            // the load is issued on every path (lanes without a key read
            // word 0), so every batch issues the same loads and the waits
            // for a batch count only the loads issued after it
            const bool more = c < tk;
            uint32_t src = 0;
            ok = false;
            if (more) {
                src = sb_span(c, r0, nr, rb, rp, wflag, ++tag);
                ok = c + lane < tk;
                c += kWave;
            }
            key = routed[ok ? src : 0u];
            return more;
        };
        // U spans: the raw loads in k (not read until the batch is inserted)
        // and a bit per span of the lanes that hold a key
        auto batch = [&](uint32_t (&k)[U], uint32_t &m) {
            bool any = false;
            m = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                bool ok;
                any = span(k[u], ok) || any;
                m |= ok ? 1u << u : 0u;
            }
            return any;
        };
        uint32_t qn = 0;
        auto insert = [&](const uint32_t (&k)[U], uint32_t m, bool last) {
            const bool ins = __hip_atomic_load(&s_occ, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP) <= cap_soft;
            uint32_t cur[U], wt[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = (m >> u) & 1u;
                cur[u] = ok ? k[u] : kEmpty32;
                wt[u] = ok ? 1u : 0u;
            }
            // the last batch of the wavefront drains its queue
            const uint32_t n_new = packed_insert_batch<U, LOG2S>(
                tab, cur, wt, ins, spill, k0, &s_nspill, s_q[wave], qn, last);
            const uint32_t tot = wave_count_sum(n_new);
            if (lane == 0 && tot) atomicAdd(&s_occ, tot);
        };
        __syncthreads();  // the table is clear
        // Three batches in rotation by name (no register copies, which
        // would wait for the loads being copied): batch i + 2 is loaded
        // while batch i is inserted.  A batch without keys ends the
        // wavefront's share (wavefront-uniform).
        uint32_t kA[U], kB[U], kC[U], mA, mB, mC;
        bool aA = batch(kA, mA), aB = batch(kB, mB), aC;
        for (;;) {
            aC = batch(kC, mC);
            if (!aA) break;
            insert(kA, mA, !aB);
            aA = batch(kA, mA);
            if (!aB) break;
            insert(kB, mB, !aC);
            aB = batch(kB, mB);
            if (!aC) break;
            insert(kC, mC, !aA);
        }
        __syncthreads();  // keys of the bin are consumed; the spill list is complete
        packed_absorb_spill<BS, LOG2S>(tab, spill, k0, &s_nspill);
        packed_dump<BS, LOG2S>(tab, keys + k0, w_out + k0, &s_nout);
        __syncthreads();
        packed_spill_rounds<BS, LOG2S>(tab, spill, k0, keys, w_out, cap_soft, &s_occ, &s_nout,
                                       &s_nspill, &s_insert);
        if (threadIdx.x == 0) bin_size[b] = s_nout;
        __syncthreads();
    }
}

}  // namespace

static uint32_t persistent_grid(uint32_t NB)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    uint32_t g = (uint32_t)cus;
    return NB < g ? NB : g;
}

// Keys per thread and batch of the flat aggregation.  A batch starts
// inserting only while the table holds at most kPackedCapSoft keys, so it
// never holds more than kPackedCapSoft + 1024 * (kFlatU + 1): that must
// leave free slots, or a probe could run forever.
constexpr int kFlatU = 4;
constexpr uint32_t kPackedCapSoft = (1u << 14) - 1024 * (kFlatU + 1) - 1024;
static_assert(kPackedCapSoft + 1024 * (kFlatU + 1) < (1u << 14),
              "packed table must keep free slots");

hipError_t launch_aggregate_regions(const crop_ctx *c, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    const SbPlan &sp = c->sb;
    if (pl.NB == 0) return hipSuccess;
    if (c->in.wide_keys) return hipErrorInvalidValue;  // 64-bit keys stay on the chunk route
    hipLaunchKernelGGL((k_aggregate_regions<1024, 14, kFlatU>), dim3(persistent_grid(pl.NB)),
                       dim3(1024), 0, s, c->sb_hdrT.as<uint16_t>(), c->sb_seg.as<SbSeg>(),
                       sp.segs.size() > 1 ? c->sb_binseg.as<uint32_t>() : nullptr,
                       c->sb_term.as<uint32_t>(), c->routed.as<uint32_t>(),
                       c->bin_off.as<uint32_t>(), c->keys.as<uint32_t>(),
                       c->out_cnt.as<uint32_t>(), c->bin_size.as<uint32_t>(),
                       c->spill.as<Spilled<uint32_t, uint32_t>>(), pl.NB,
                       c->counter.as<uint32_t>(), kPackedCapSoft, c->bin_order.as<uint32_t>());
    return hipGetLastError();
}

hipError_t launch_aggregate_counts(const crop_ctx *c, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    uint32_t grid = persistent_grid(pl.NB);
    if (!c->in.wide_keys) {
        constexpr int L = 14;
        hipLaunchKernelGGL((k_aggregate_flat<1024, L, kFlatU>), dim3(grid), dim3(1024), 0, s,
                           c->bin_off.as<uint32_t>(), c->keys.as<uint32_t>(),
                           c->out_cnt.as<uint32_t>(), c->bin_size.as<uint32_t>(),
                           c->spill.as<Spilled<uint32_t, uint32_t>>(), pl.NB,
                           c->counter.as<uint32_t>(), kPackedCapSoft, c->bin_order.as<uint32_t>());
    } else {
        constexpr int L = 13;
        hipLaunchKernelGGL((k_aggregate<512, uint64_t, uint32_t, L>), dim3(grid), dim3(512), 0, s,
                           c->bin_off.as<uint32_t>(), c->keys.as<uint64_t>(), nullptr,
                           c->out_cnt.as<uint32_t>(), c->bin_size.as<uint32_t>(),
                           c->spill.as<Spilled<uint64_t, uint32_t>>(), pl.NB,
                           c->counter.as<uint32_t>(), (1u << L) * 5 / 8);
    }
    return hipGetLastError();
}

hipError_t launch_aggregate_sums(const crop_ctx *c, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    uint32_t grid = persistent_grid(pl.NB);
    constexpr int L = 13;
    hipLaunchKernelGGL((k_aggregate<512, uint64_t, float, L>), dim3(grid), dim3(512), 0, s,
                       c->bin_off.as<uint32_t>(), c->keys.as<uint64_t>(),
                       c->vals.as<float>(), c->vals.as<float>(), c->bin_size.as<uint32_t>(),
                       c->spill.as<Spilled<uint64_t, float>>(), pl.NB, c->counter.as<uint32_t>(),
                       (1u << L) * 5 / 8);
    return hipGetLastError();
}

size_t spill_entry_bytes(bool wide, bool sums)
{
    if (sums) return sizeof(Spilled<uint64_t, float>);
    return wide ? sizeof(Spilled<uint64_t, uint32_t>) : sizeof(Spilled<uint32_t, uint32_t>);
}

}  // namespace crop
