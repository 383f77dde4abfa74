// Term enumeration and routing: every nonzero term of the stream is mapped
// to its routing bin by the consistent hash and written, bin by bin, into
// one array of packed keys.
//
// Routing bins are equal intervals of the 2^32 hash space, bin =
// (h * NB) >> 32 with NB = P * S; bin / S is the term's partition, the
// owner interval of Section 6, Theorem 1 (nested-floor identity).  Each
// bin is later accumulated by one workgroup in LDS.
//
// The pass is split the way a counting sort is: a count kernel builds a
// [chunk x bin] matrix of term counts, a scan turns it into write offsets
// (bin-major, so every bin is one contiguous segment), and a scatter kernel
// enumerates again and writes each key at its offset.  Enumerating twice is
// cheaper than moving the terms twice: a term is a few ALU operations on
// staged LDS data, while its key costs HBM traffic.
//
// The enumeration inside a chunk is in crop_enum.hpp.
#include <algorithm>

#include "crop_device.hpp"
#include "crop_enum.hpp"
#include "crop_internal.hpp"

namespace crop {

namespace {

// Threads of a workgroup of the unstaged scatter and of the count pass
// (measured on the 1M-transaction stream: scatter 1024 > 512 > 256; count
// 512 beats 256 by 18 % and 1024 by 33 %).
constexpr int kScatterBS = 1024;
constexpr int kCountBS = 512;

// Row groups of the count-matrix scan: at most this many (k_colprefix keeps
// one partial per group in registers).
constexpr uint32_t kMaxScanGroups = 64;

// ---------------------------------------------------------------- chunks

// One chunk of transactions as the count and scatter kernels see it: rows
// [r0, r1), the NB routing bins of its stream, its row of the count matrix
// (counts, later write cursors) and the next row (or the stream's bin ends
// for its last chunk), which bounds its run in each bin.
struct ChunkView {
    uint32_t r0, r1, NB;
    BinMap bm;
    uint32_t *row;
    const uint32_t *nxt;
};

// A single stream: chunk c holds rows [c R, c R + R).
struct SingleChunks {
    uint32_t T, R, NB, n_chunks;
    BinMap bm;
    uint32_t *cnt;
    const uint32_t *bin_off;
    __device__ ChunkView view(uint32_t c) const
    {
        ChunkView v;
        v.r0 = c * R;
        v.r1 = min(v.r0 + R, T);
        v.NB = NB;
        v.bm = bm;
        v.row = cnt + (size_t)c * NB;
        v.nxt = c + 1 < n_chunks ? v.row + NB : bin_off + 1;
        return v;
    }
};

// A batch of streams concatenated row-wise: chunk c holds rows
// [crow[c], crow[c+1]) of stream cstream[c]; no chunk crosses a stream.
struct BatchChunks {
    const uint32_t *crow;
    const uint32_t *cstream;
    const BatchStreamDev *st;
    uint32_t *cnt;
    const uint32_t *bin_off;
    __device__ ChunkView view(uint32_t c) const
    {
        const BatchStreamDev S = st[cstream[c]];
        ChunkView v;
        v.r0 = crow[c];
        v.r1 = crow[c + 1];
        v.NB = S.NB;
        v.bm = BinMap{S.NB, 0, S.NB, 0};
        v.row = cnt + S.cnt_base + (size_t)(c - S.chunk0) * S.NB;
        v.nxt = c + 1 < S.chunk0 + S.n_chunks ? v.row + S.NB : bin_off + S.bin_base + 1;
        return v;
    }
};

// ---------------------------------------------------------------- kernels

// NBmax sizes the LDS layout; each chunk uses the NB of its stream.
template <int BS, class Chunks>
__global__ void __launch_bounds__(BS)
k_tx_count(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items, HashParams hp,
           uint32_t NBmax, uint32_t max_items, Chunks ch)
{
    extern __shared__ uint32_t smem[];
    uint32_t *hist = smem;
    const TxLds L = tx_lds(smem, NBmax, max_items);
    const uint32_t chunk = xcd_contiguous(blockIdx.x, gridDim.x);
    const ChunkView cv = ch.view(chunk);
    const uint32_t NB = cv.NB;
    for (uint32_t b = threadIdx.x; b < NB; b += BS) hist[b] = 0;
    const uint32_t m = stage_tx<BS>(off, items, cv.r0, cv.r1, hp, L);
    enum_tx<BS>(m, L, hp, [&](uint32_t, uint32_t, uint32_t h) {
        const uint32_t bin = cv.bm.local(h);
        if (bin < NB) atomicAdd(&hist[bin], 1u);
    });
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < NB; b += BS) cv.row[b] = hist[b];
}

// Staged scatter (cap > 0; without staging k_tx_scatter_direct runs).
// Every term takes a slot of its bin's run in this chunk with an LDS atomic
// on the bin's local cursor; the chunk's terms of a window of bins are put
// in LDS sorted by bin first and written out run by run, so consecutive
// lanes store consecutive addresses.  A window holds at most cap terms, a
// bin with more terms than that in one chunk is written directly, and
// windows are set by bin, a property of the term itself, so each term lands
// in exactly one window.
template <int BS, class KeyT, class Chunks>
__global__ void __launch_bounds__(BS)
k_tx_scatter(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items, HashParams hp,
             uint32_t NBmax, uint32_t max_items, Chunks ch, KeyT *__restrict__ keys,
             uint32_t cap)
{
    extern __shared__ uint32_t smem[];
    uint32_t *lstart = smem;                  // NB + 1: local start of each bin's run
    uint32_t *lcur = smem + NBmax + 1;        // NB: local cursor
    uint32_t *delta = smem + 2 * NBmax + 1;   // NB: global start - local start
    const uint32_t lead = 3 * NBmax + 1;
    const TxLds L = tx_lds(smem, lead, max_items);
    KeyT *stage =
        reinterpret_cast<KeyT *>(smem + ((tx_lds_words(lead, max_items) + 1) & ~(size_t)1));
    __shared__ uint32_t s_tmp[BS / kWave + 1];
    __shared__ uint32_t s_b1, s_direct;

    const uint32_t chunk = xcd_contiguous(blockIdx.x, gridDim.x);
    const ChunkView cv = ch.view(chunk);
    const uint32_t NB = cv.NB;
    const uint32_t *row = cv.row;
    const uint32_t *nxt = cv.nxt;
    for (uint32_t b = threadIdx.x; b < NB; b += BS) lstart[b] = nxt[b] - row[b];
    __syncthreads();
    lds_exclusive_scan<BS>(lstart, NB, s_tmp);
    const uint32_t Tc = lstart[NB];
    for (uint32_t b = threadIdx.x; b < NB; b += BS) {
        lcur[b] = lstart[b];
        delta[b] = row[b] - lstart[b];
    }
    const uint32_t m = stage_tx<BS>(off, items, cv.r0, cv.r1, hp, L);
    if (Tc == 0) return;

    for (uint32_t b0 = 0; b0 < NB;) {
        if (threadIdx.x == 0) {
            // last b1 in [b0, NB] with lstart[b1] - lstart[b0] <= cap (lstart is
            // non-decreasing); an empty window means bin b0 alone exceeds cap
            const uint32_t lim = lstart[b0] + cap;
            uint32_t lo = b0, hi = NB + 1;  // lstart[lo] <= lim < lstart[hi] (hi = NB+1: +inf)
            while (hi - lo > 1) {
                uint32_t mid = (lo + hi) >> 1;
                if (lstart[mid] <= lim) lo = mid; else hi = mid;
            }
            s_direct = lo == b0 ? 1u : 0u;
            s_b1 = lo == b0 ? b0 + 1 : lo;
        }
        __syncthreads();
        const uint32_t b1 = s_b1;
        const bool direct = s_direct != 0;
        const uint32_t s0 = lstart[b0];
        const bool whole = b0 == 0 && b1 == NB;
        enum_tx<BS>(m, L, hp, [&](uint32_t x, uint32_t y, uint32_t h) {
            const uint32_t bin = cv.bm.local(h);
            if (bin >= NB || (!whole && (bin < b0 || bin >= b1))) return;
            const uint32_t p = atomicAdd(&lcur[bin], 1u);
            const KeyT key = pack_key<KeyT>(x, y);
            if (direct)
                keys[p + delta[bin]] = key;
            else
                stage[p - s0] = key;
        });
        __syncthreads();
        if (!direct) {
            const uint32_t n = lstart[b1] - s0;
            for (uint32_t i = threadIdx.x; i < n; i += BS) {
                const KeyT key = stage[i];
                keys[i + s0 + delta[cv.bm.local(hash_of_key(key, hp))]] = key;
            }
        }
        __syncthreads();
        b0 = b1;
    }
}

// Scatter without staging: the chunk's bin cursors start at its global
// write positions (its row of the scanned count matrix), so a term's LDS
// atomic returns its slot in HBM and the key is stored there.  LDS: the
// cursors and the chunk image only.
template <int BS, class KeyT, class Chunks>
__global__ void __launch_bounds__(BS)
k_tx_scatter_direct(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items,
                    HashParams hp, uint32_t NBmax, uint32_t max_items, Chunks ch,
                    KeyT *__restrict__ keys)
{
    extern __shared__ uint32_t smem[];
    uint32_t *lcur = smem;  // NB: global write cursor of each bin
    const TxLds L = tx_lds(smem, NBmax, max_items);
    const uint32_t chunk = xcd_contiguous(blockIdx.x, gridDim.x);
    const ChunkView cv = ch.view(chunk);
    const uint32_t NB = cv.NB;
    for (uint32_t b = threadIdx.x; b < NB; b += BS) lcur[b] = cv.row[b];
    const uint32_t m = stage_tx<BS>(off, items, cv.r0, cv.r1, hp, L);  // ends with a barrier
    enum_tx<BS>(m, L, hp, [&](uint32_t x, uint32_t y, uint32_t h) {
        const uint32_t bin = cv.bm.local(h);
        if (bin < NB) keys[atomicAdd(&lcur[bin], 1u)] = pack_key<KeyT>(x, y);
    });
}

// ---- an owner's share: windowed enumeration (one chunk per workgroup)
//
// The count and scatter of a run that owns the hash interval [q, q + W)
// with W <= 2^31: each chunk is bucket-sorted by h_b and every entry walks
// only its window (enum_tx_win), so the enumeration costs the owner's terms
// plus the window searches instead of every term of the stream.

template <int BS>
__global__ void __launch_bounds__(BS)
k_tx_count_win(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items, HashParams hp,
               uint32_t NB, BinMap bm, uint32_t max_items, uint32_t T, uint32_t R, uint32_t kb,
               uint32_t q, uint32_t W, uint32_t *__restrict__ cnt)
{
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_tmp[BS / kWave + 1];
    uint32_t *hist = smem;
    const WinLds L = win_lds(smem, NB, R, kb, max_items);
    const uint32_t chunk = xcd_contiguous(blockIdx.x, gridDim.x);
    const uint32_t r0 = chunk * R, r1 = min(r0 + R, T);
    for (uint32_t b = threadIdx.x; b < NB; b += BS) hist[b] = 0;
    const uint32_t m = stage_tx_win<BS>(off, items, r0, r1, kb, hp, L, s_tmp);
    enum_tx_win<BS>(m, kb, q, W, L, hp, [&](uint32_t, uint32_t, uint32_t h) {
        const uint32_t bin = bm.local(h);
        if (bin < NB) atomicAdd(&hist[bin], 1u);
    });
    __syncthreads();
    uint32_t *row = cnt + (size_t)chunk * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += BS) row[b] = hist[b];
}

template <int BS, class KeyT>
__global__ void __launch_bounds__(BS)
k_tx_scatter_win(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items,
                 HashParams hp, uint32_t NB, BinMap bm, uint32_t max_items, uint32_t T,
                 uint32_t R, uint32_t kb, uint32_t q, uint32_t W,
                 const uint32_t *__restrict__ cur, KeyT *__restrict__ keys)
{
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_tmp[BS / kWave + 1];
    uint32_t *lcur = smem;
    const WinLds L = win_lds(smem, NB, R, kb, max_items);
    const uint32_t chunk = xcd_contiguous(blockIdx.x, gridDim.x);
    const uint32_t r0 = chunk * R, r1 = min(r0 + R, T);
    const uint32_t *row = cur + (size_t)chunk * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += BS) lcur[b] = row[b];
    const uint32_t m = stage_tx_win<BS>(off, items, r0, r1, kb, hp, L, s_tmp);
    enum_tx_win<BS>(m, kb, q, W, L, hp, [&](uint32_t x, uint32_t y, uint32_t h) {
        const uint32_t bin = bm.local(h);
        if (bin < NB) keys[atomicAdd(&lcur[bin], 1u)] = pack_key<KeyT>(x, y);
    });
}

// ---- chunk ranges: one workgroup per contiguous range of chunks

// The range of chunks of workgroup w when n_chunks chunks are split over
// n_wg workgroups.
__device__ inline void chunk_range(uint32_t w, uint32_t n_wg, uint32_t n_chunks, uint32_t *c0,
                                   uint32_t *c1)
{
    *c0 = (uint32_t)(((uint64_t)n_chunks * w) / n_wg);
    *c1 = (uint32_t)(((uint64_t)n_chunks * (w + 1)) / n_wg);
}

// Count over a range of chunks: one histogram row per workgroup, so the
// count matrix is [n_wg x NB] rather than [chunk x NB].
template <int BS>
__global__ void __launch_bounds__(BS)
k_tx_count_ranges(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items,
                  HashParams hp, uint32_t NB, BinMap bm, uint32_t max_items, uint32_t T,
                  uint32_t R, uint32_t n_chunks, uint32_t *__restrict__ cnt)
{
    extern __shared__ uint32_t smem[];
    uint32_t *hist = smem;
    const TxLds L = tx_lds(smem, NB, max_items);
    const uint32_t w = xcd_contiguous(blockIdx.x, gridDim.x);
    uint32_t c0, c1;
    chunk_range(w, gridDim.x, n_chunks, &c0, &c1);
    for (uint32_t b = threadIdx.x; b < NB; b += BS) hist[b] = 0;
    for (uint32_t c = c0; c < c1; ++c) {
        __syncthreads();  // the previous chunk's image is no longer read
        const uint32_t r0 = c * R, r1 = min(r0 + R, T);
        const uint32_t m = stage_tx<BS>(off, items, r0, r1, hp, L);
        enum_tx<BS>(m, L, hp, [&](uint32_t, uint32_t, uint32_t h) {
            const uint32_t bin = bm.local(h);
            if (bin < NB) atomicAdd(&hist[bin], 1u);
        });
    }
    __syncthreads();
    uint32_t *row = cnt + (size_t)w * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += BS) row[b] = hist[b];
}

// Scatter over the same ranges.  The workgroup keeps its write cursor of
// every bin in LDS (started from its row of the scanned count matrix) and,
// chunk by chunk, counts the chunk's terms per bin, places them in LDS
// grouped by bin and writes the runs at the cursors.  Chunk ranges and their
// order are those of k_tx_count_ranges, so every workgroup writes exactly
// the slots its count reserved.
template <int BS, class KeyT>
__global__ void __launch_bounds__(BS)
k_tx_scatter_ranges(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items,
                    HashParams hp, uint32_t NB, BinMap bm, uint32_t max_items, uint32_t T,
                    uint32_t R, uint32_t n_chunks, const uint32_t *__restrict__ cur,
                    KeyT *__restrict__ keys, uint32_t cap)
{
    extern __shared__ uint32_t smem[];
    uint32_t *gcur = smem;                 // NB: global cursor of each bin
    uint32_t *lstart = smem + NB;          // NB + 1: local start of each bin's run
    uint32_t *lpos = smem + 2 * NB + 1;    // NB: local cursor
    const uint32_t lead = 3 * NB + 1;
    const TxLds L = tx_lds(smem, lead, max_items);
    KeyT *stage =
        reinterpret_cast<KeyT *>(smem + ((tx_lds_words(lead, max_items) + 1) & ~(size_t)1));
    __shared__ uint32_t s_tmp[BS / kWave + 1];
    __shared__ uint32_t s_b1, s_direct;

    const uint32_t w = xcd_contiguous(blockIdx.x, gridDim.x);
    uint32_t c0, c1;
    chunk_range(w, gridDim.x, n_chunks, &c0, &c1);
    for (uint32_t b = threadIdx.x; b < NB; b += BS) gcur[b] = cur[(size_t)w * NB + b];
    for (uint32_t c = c0; c < c1; ++c) {
        __syncthreads();  // previous chunk: runs written, cursors advanced
        for (uint32_t b = threadIdx.x; b < NB; b += BS) lstart[b] = 0;
        const uint32_t r0 = c * R, r1 = min(r0 + R, T);
        const uint32_t m = stage_tx<BS>(off, items, r0, r1, hp, L);  // ends with a barrier
        enum_tx<BS>(m, L, hp, [&](uint32_t, uint32_t, uint32_t h) {
            const uint32_t bin = bm.local(h);
            if (bin < NB) atomicAdd(&lstart[bin], 1u);
        });
        __syncthreads();
        lds_exclusive_scan<BS>(lstart, NB, s_tmp);
        const uint32_t Tc = lstart[NB];
        for (uint32_t b = threadIdx.x; b < NB; b += BS) lpos[b] = lstart[b];
        __syncthreads();
        for (uint32_t b0 = 0; b0 < NB && Tc;) {
            if (threadIdx.x == 0 && cap == 0) {
                s_direct = 1u;
                s_b1 = NB;
            } else if (threadIdx.x == 0) {
                // last b1 in [b0, NB] with lstart[b1] - lstart[b0] <= cap; an
                // empty window means bin b0 alone exceeds cap
                const uint32_t lim = lstart[b0] + cap;
                uint32_t lo = b0, hi = NB + 1;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (lstart[mid] <= lim) lo = mid; else hi = mid;
                }
                s_direct = lo == b0 ? 1u : 0u;
                s_b1 = lo == b0 ? b0 + 1 : lo;
            }
            __syncthreads();
            const uint32_t b1 = s_b1;
            const bool direct = s_direct != 0;
            const uint32_t s0 = lstart[b0];
            const bool whole = b0 == 0 && b1 == NB;
            enum_tx<BS>(m, L, hp, [&](uint32_t x, uint32_t y, uint32_t h) {
                const uint32_t bin = bm.local(h);
                if (bin >= NB || (!whole && (bin < b0 || bin >= b1))) return;
                const uint32_t p = atomicAdd(&lpos[bin], 1u);
                const KeyT key = pack_key<KeyT>(x, y);
                if (direct)
                    keys[gcur[bin] + (p - lstart[bin])] = key;
                else
                    stage[p - s0] = key;
            });
            __syncthreads();
            if (!direct) {
                const uint32_t n = lstart[b1] - s0;
                for (uint32_t i = threadIdx.x; i < n; i += BS) {
                    const KeyT key = stage[i];
                    const uint32_t bin = bm.local(hash_of_key(key, hp));
                    keys[gcur[bin] + (i + s0 - lstart[bin])] = key;
                }
            }
            __syncthreads();
            b0 = b1;
        }
        for (uint32_t b = threadIdx.x; b < NB; b += BS) gcur[b] += lstart[b + 1] - lstart[b];
    }
}

template <int BS>
__global__ void __launch_bounds__(BS)
k_op_count(OpArgs a, HashParams hp, uint32_t NB, BinMap bm, uint32_t max_a,
           uint32_t *__restrict__ cnt)
{
    extern __shared__ uint32_t smem[];
    uint32_t *s_ai, *s_ha, *s_bs, *s_wp, *s_tmp;
    float *s_av;
    uint32_t *hist = op_smem_layout<BS>(smem, NB, max_a, &s_ai, &s_ha, &s_av, &s_bs, &s_wp, &s_tmp);
    const uint32_t chunk = xcd_contiguous(blockIdx.x, gridDim.x);
    for (uint32_t b = threadIdx.x; b < NB; b += BS) hist[b] = 0;
    uint32_t m;
    const uint32_t Tc = stage_op<BS>(a.chunks[chunk], a.a_off, a.a_idx, a.a_val, a.b_off, hp, s_ai,
                                     s_ha, s_av, s_bs, s_wp, s_tmp, &m);
    walk_op<BS>(Tc, m, s_ai, s_ha, s_av, s_bs, s_wp, a.b_idx, a.b_val, hp,
                [&](uint32_t, uint32_t, uint32_t h, float) {
                    const uint32_t bin = bm.local(h);
                    if (bin < NB) atomicAdd(&hist[bin], 1u);
                });
    __syncthreads();
    uint32_t *row = cnt + (size_t)chunk * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += BS) row[b] = hist[b];
}

template <int BS>
__global__ void __launch_bounds__(BS)
k_op_scatter(OpArgs a, HashParams hp, uint32_t NB, BinMap bm, uint32_t max_a,
             const uint32_t *__restrict__ cur, uint64_t *__restrict__ keys,
             float *__restrict__ vals)
{
    extern __shared__ uint32_t smem[];
    uint32_t *s_ai, *s_ha, *s_bs, *s_wp, *s_tmp;
    float *s_av;
    uint32_t *pos = op_smem_layout<BS>(smem, NB, max_a, &s_ai, &s_ha, &s_av, &s_bs, &s_wp, &s_tmp);
    const uint32_t chunk = xcd_contiguous(blockIdx.x, gridDim.x);
    const uint32_t *row = cur + (size_t)chunk * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += BS) pos[b] = row[b];
    uint32_t m;
    const uint32_t Tc = stage_op<BS>(a.chunks[chunk], a.a_off, a.a_idx, a.a_val, a.b_off, hp, s_ai,
                                     s_ha, s_av, s_bs, s_wp, s_tmp, &m);
    walk_op<BS>(Tc, m, s_ai, s_ha, s_av, s_bs, s_wp, a.b_idx, a.b_val, hp,
                [&](uint32_t i, uint32_t j, uint32_t h, float v) {
                    const uint32_t bin = bm.local(h);
                    if (bin >= NB) return;
                    const uint32_t p = atomicAdd(&pos[bin], 1u);
                    keys[p] = ((uint64_t)i << 32) | j;
                    vals[p] = v;
                });
}

// ---------------------------------------------------------------- scan

// part[g][b] = sum of cnt[c][b] over the rows c of group g.
__global__ void __launch_bounds__(256)
k_colsum(const uint32_t *__restrict__ cnt, uint32_t n, uint32_t NB, uint32_t rows_per_g,
         uint32_t *__restrict__ part)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= NB) return;
    const uint32_t g = blockIdx.y;
    const uint32_t c0 = g * rows_per_g, c1 = min(n, c0 + rows_per_g);
    uint32_t s = 0;
#pragma unroll 8
    for (uint32_t c = c0; c < c1; ++c) s += cnt[(size_t)c * NB + b];
    part[(size_t)g * NB + b] = s;
}

// Per bin b: part[g][b] <- exclusive prefix over the groups g; tot[b] <- sum.
__global__ void __launch_bounds__(256)
k_colprefix(uint32_t *__restrict__ part, uint32_t NB, uint32_t G, uint32_t *__restrict__ tot)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= NB) return;
    // G <= kMaxScanGroups: every group's partial is loaded before any is
    // rewritten, so the loads are in flight together
    uint32_t v[kMaxScanGroups];
#pragma unroll
    for (uint32_t g = 0; g < kMaxScanGroups; ++g) v[g] = g < G ? part[(size_t)g * NB + b] : 0u;
    uint32_t run = 0;
#pragma unroll
    for (uint32_t g = 0; g < kMaxScanGroups; ++g) {
        if (g < G) part[(size_t)g * NB + b] = run;
        run += v[g];
    }
    tot[b] = run;
}

// One workgroup: bin_off[b] <- exclusive prefix over b of the bin totals
// (given in bin_off itself); bin_off[NB] <- total; resets the work counters.
__global__ void __launch_bounds__(1024)
k_colbase(uint32_t NB, uint32_t *__restrict__ bin_off, uint32_t *__restrict__ counter)
{
    __shared__ uint32_t s_tmp[1024 / kWave + 1];
    const uint32_t per = (NB + 1023) / 1024;
    const uint32_t b0 = threadIdx.x * per, b1 = min(NB, b0 + per);
    uint32_t sum = 0;
    for (uint32_t b = b0; b < b1; ++b) sum += bin_off[b];
    uint32_t total;
    uint32_t run = block_exclusive_scan<1024>(sum, s_tmp, &total);
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t t = bin_off[b];
        bin_off[b] = run;
        run += t;
    }
    if (threadIdx.x == 0) {
        bin_off[NB] = total;
        counter[0] = 0;
        counter[1] = 0;
    }
}

// One workgroup per segment of the bins (segment g: bins [g NB / n_seg,
// (g + 1) NB / n_seg)): order[] lists, in place of the segment, its bins
// with more than twice the mean term count first (in index order), then
// the others, so that the persistent aggregation workgroups start the
// longest bins first.  The first workgroup also clears the n_zero words at
// zero (the aggregation's bin counters), which saves a launch.
__global__ void __launch_bounds__(1024)
k_bin_order(uint32_t NB, const uint32_t *__restrict__ bin_off, uint32_t *__restrict__ order,
            uint32_t *__restrict__ zero, uint32_t n_zero)
{
    __shared__ uint32_t s_tmp[1024 / kWave + 1];
    if (blockIdx.x == 0 && threadIdx.x < n_zero) zero[threadIdx.x] = 0;
    __shared__ uint32_t s_nheavy;
    const uint64_t thresh = 2ull * bin_off[NB] / (NB ? NB : 1);
    const uint32_t lo = (uint32_t)((uint64_t)NB * blockIdx.x / gridDim.x);
    const uint32_t hi = (uint32_t)((uint64_t)NB * (blockIdx.x + 1) / gridDim.x);
    const uint32_t per = (hi - lo + 1023) / 1024;
    const uint32_t b0 = min(hi, lo + threadIdx.x * per), b1 = min(hi, b0 + per);
    uint32_t nh = 0;
    for (uint32_t b = b0; b < b1; ++b) nh += (bin_off[b + 1] - bin_off[b]) > thresh;
    uint32_t total;
    uint32_t h = block_exclusive_scan<1024>(nh, s_tmp, &total);
    if (threadIdx.x == 0) s_nheavy = total;
    __syncthreads();
    // light bins of the segment before b0 = (b0 - lo) - heavy bins before b0
    uint32_t l = lo + s_nheavy + (b0 - lo) - h;
    h += lo;
    for (uint32_t b = b0; b < b1; ++b) {
        if ((bin_off[b + 1] - bin_off[b]) > thresh)
            order[h++] = b;
        else
            order[l++] = b;
    }
}

// cnt[c][b] <- bin_off[b] + part[g][b] + sum of cnt[c'][b] for earlier c' in g.
__global__ void __launch_bounds__(256)
k_colapply(uint32_t *__restrict__ cnt, uint32_t n, uint32_t NB, uint32_t rows_per_g,
           const uint32_t *__restrict__ part, const uint32_t *__restrict__ bin_off)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= NB) return;
    const uint32_t g = blockIdx.y;
    const uint32_t c0 = g * rows_per_g, c1 = min(n, c0 + rows_per_g);
    uint32_t run = bin_off[b] + part[(size_t)g * NB + b];
#pragma unroll 8
    for (uint32_t c = c0; c < c1; ++c) {
        uint32_t v = cnt[(size_t)c * NB + b];
        cnt[(size_t)c * NB + b] = run;
        run += v;
    }
}

// ---- batches: the count matrix of stream s is [its chunks x its NB bins] at
// cnt_base; global bin g = bin_base + local bin.

// Per global bin: the stream's column of counts -> exclusive prefix over its
// chunks, in place; tot[g] <- the column total.
__global__ void __launch_bounds__(256)
k_bcolscan(BatchDev b, uint32_t *__restrict__ cnt, uint32_t *__restrict__ tot)
{
    const uint32_t g = blockIdx.x * 256 + threadIdx.x;
    if (g >= b.NBtot) return;
    const BatchStreamDev S = b.streams[b.bin_stream[g]];
    const uint32_t lb = g - S.bin_base;
    uint32_t *col = cnt + S.cnt_base + lb;
    uint32_t run = 0;
#pragma unroll 8
    for (uint32_t c = 0; c < S.n_chunks; ++c) {
        const uint32_t v = col[(size_t)c * S.NB];
        col[(size_t)c * S.NB] = run;
        run += v;
    }
    tot[g] = run;
}

// Device-wide exclusive scan in three launches over tiles of kScanTile.
constexpr uint32_t kScanTile = 4096;

__global__ void __launch_bounds__(1024)
k_scan_tiles(const uint32_t *__restrict__ in, uint32_t n, uint32_t *__restrict__ tile_sum)
{
    __shared__ uint32_t s_tmp[1024 / kWave + 1];
    const uint32_t base = blockIdx.x * kScanTile;
    uint32_t sum = 0;
    for (uint32_t k = 0; k < kScanTile / 1024; ++k) {
        const uint32_t i = base + threadIdx.x * (kScanTile / 1024) + k;
        if (i < n) sum += in[i];
    }
    uint32_t total;
    (void)block_exclusive_scan<1024>(sum, s_tmp, &total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One workgroup: exclusive prefix of the tile sums; out[n] <- the total;
// resets the persistent kernels' work counters.
__global__ void __launch_bounds__(1024)
k_scan_top(uint32_t *__restrict__ tile_sum, uint32_t n_tiles, uint32_t *__restrict__ out,
           uint32_t n, uint32_t *__restrict__ counter)
{
    __shared__ uint32_t s_tmp[1024 / kWave + 1];
    const uint32_t per = (n_tiles + 1023) / 1024;
    const uint32_t t0 = threadIdx.x * per, t1 = min(n_tiles, t0 + per);
    uint32_t sum = 0;
    for (uint32_t t = t0; t < t1; ++t) sum += tile_sum[t];
    uint32_t total;
    uint32_t run = block_exclusive_scan<1024>(sum, s_tmp, &total);
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t v = tile_sum[t];
        tile_sum[t] = run;
        run += v;
    }
    if (threadIdx.x == 0) {
        out[n] = total;
        counter[0] = 0;
        counter[1] = 0;
    }
}

__global__ void __launch_bounds__(1024)
k_scan_apply(const uint32_t *__restrict__ in, uint32_t n, const uint32_t *__restrict__ tile_sum,
             uint32_t *__restrict__ out)
{
    __shared__ uint32_t s_tmp[1024 / kWave + 1];
    constexpr uint32_t E = kScanTile / 1024;
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * E;
    uint32_t v[E];
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < E; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        sum += v[k];
    }
    uint32_t total;
    uint32_t run = tile_sum[blockIdx.x] + block_exclusive_scan<1024>(sum, s_tmp, &total);
#pragma unroll
    for (uint32_t k = 0; k < E; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

// Per global bin: add the bin's start to its column of chunk prefixes.
__global__ void __launch_bounds__(256)
k_bapply(BatchDev b, uint32_t *__restrict__ cnt, const uint32_t *__restrict__ bin_off)
{
    const uint32_t g = blockIdx.x * 256 + threadIdx.x;
    if (g >= b.NBtot) return;
    const BatchStreamDev S = b.streams[b.bin_stream[g]];
    uint32_t *col = cnt + S.cnt_base + (g - S.bin_base);
    const uint32_t base = bin_off[g];
#pragma unroll 8
    for (uint32_t c = 0; c < S.n_chunks; ++c) col[(size_t)c * S.NB] += base;
}

// ---------------------------------------------------------------- validation

// bad <- min over offending vectors v of v (vector v is [v_off[v], v_off[v+1])).
__global__ void __launch_bounds__(256)
k_validate_csr(const uint32_t *__restrict__ v_off, uint64_t K, const uint32_t *__restrict__ idx,
               uint64_t nnz, uint32_t n, unsigned long long *bad)
{
    for (uint64_t v = (uint64_t)blockIdx.x * 256 + threadIdx.x; v < K;
         v += (uint64_t)gridDim.x * 256) {
        uint32_t a = v_off[v], e = v_off[v + 1];
        bool ok = a <= e && e <= nnz;
        if (ok) {
            for (uint32_t k = a; k < e; ++k) {
                uint32_t x = idx[k];
                if (x >= n || (k > a && x <= idx[k - 1])) {
                    ok = false;
                    break;
                }
            }
        }
        if (!ok) atomicMin(bad, (unsigned long long)v);
    }
}

// bad <- min over q of q where pair (qx[q], qy[q]) breaks x < y < n.
__global__ void __launch_bounds__(256)
k_check_pairs(const uint32_t *__restrict__ qx, const uint32_t *__restrict__ qy, uint64_t n,
              uint32_t n_items, unsigned long long *bad)
{
    for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; q < n;
         q += (uint64_t)gridDim.x * 256) {
        const uint32_t x = qx[q], y = qy[q];
        if (!(x < y && y < n_items)) atomicMin(bad, (unsigned long long)q);
    }
}

// Consistent hash of query pairs: h[q] = h_a(qx[q]) + h_b(qy[q]) mod 2^32 and
// part[q] = (h[q] P) >> 32 (either output may be null).
__global__ void __launch_bounds__(256)
k_hash_pairs(const uint32_t *__restrict__ qx, const uint32_t *__restrict__ qy, uint64_t n,
             HashParams hp, uint32_t P, uint32_t *__restrict__ h, uint32_t *__restrict__ part)
{
    for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; q < n;
         q += (uint64_t)gridDim.x * 256) {
        const uint32_t v = hash_a(hp, qx[q]) + hash_b(hp, qy[q]);
        if (h) h[q] = v;
        if (part) part[q] = interval_of(v, P);
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers

size_t tx_count_smem_bytes(uint32_t NB, uint32_t max_items)
{
    return 4 * tx_lds_words(NB, max_items);
}

size_t tx_scatter_smem_bytes(uint32_t NB, uint32_t max_items, uint32_t cap, bool wide)
{
    size_t w = (tx_lds_words(3 * NB + 1, max_items) + 1) & ~(size_t)1;
    return 4 * w + (size_t)cap * (wide ? 8 : 4);
}

// Every chunk image the transaction kernels place in LDS (count, direct and
// staged scatter) is aligned, disjoint and inside the dynamic LDS of its
// launch, and that LDS fits a CU.
bool tx_launch_layouts_ok(uint32_t NB, uint32_t max_items, uint32_t cap, bool wide)
{
    const size_t count = tx_count_smem_bytes(NB, max_items);
    const size_t direct = 4 * tx_lds_words(NB, max_items);
    const size_t staged = tx_scatter_smem_bytes(NB, max_items, cap, wide);
    if (!tx_layout_ok(NB, max_items, count) || !tx_layout_ok(NB, max_items, direct) ||
        !tx_layout_ok(3 * NB + 1, max_items, staged))
        return false;
    const size_t cu = 160 * 1024;
    return count <= cu && direct <= cu && (cap == 0 || staged <= cu);
}

static size_t op_smem_bytes(uint32_t NB, uint32_t max_a, uint32_t BS)
{
    return sizeof(uint32_t) * ((size_t)NB + 5 * (size_t)max_a + 1 + BS / kWave + 1);
}

BinMap bin_map(const RoutePlan &pl) { return BinMap{pl.M, pl.u0, pl.nu, pl.g}; }

static SingleChunks single_chunks(const crop_ctx *c, uint32_t *cnt)
{
    const RoutePlan &pl = c->plan;
    return SingleChunks{(uint32_t)c->in.T, pl.R, pl.NB, pl.n_chunks, bin_map(pl), cnt,
                        c->bin_off.as<uint32_t>()};
}

hipError_t launch_tx_count(const crop_ctx *c, uint32_t *cnt, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    size_t sm = tx_count_smem_bytes(pl.NB, pl.max_items);
    hipLaunchKernelGGL((k_tx_count<kCountBS, SingleChunks>), dim3(pl.n_chunks), dim3(kCountBS),
                       sm, s, c->in.off, c->in.items, c->hp, pl.NB, pl.max_items,
                       single_chunks(c, cnt));
    return hipGetLastError();
}

hipError_t launch_tx_scatter(const crop_ctx *c, const uint32_t *cur, void *keys, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    const bool wide = c->in.wide_keys;
    size_t sm = tx_scatter_smem_bytes(pl.NB, pl.max_items, pl.stage_cap, wide);
    const SingleChunks ch = single_chunks(c, const_cast<uint32_t *>(cur));
    if (pl.stage_cap == 0) {
        sm = 4 * tx_lds_words(pl.NB, pl.max_items);
        if (wide)
            hipLaunchKernelGGL((k_tx_scatter_direct<kScatterBS, uint64_t, SingleChunks>),
                               dim3(pl.n_chunks), dim3(kScatterBS), sm, s, c->in.off, c->in.items,
                               c->hp, pl.NB, pl.max_items, ch, static_cast<uint64_t *>(keys));
        else
            hipLaunchKernelGGL((k_tx_scatter_direct<kScatterBS, uint32_t, SingleChunks>),
                               dim3(pl.n_chunks), dim3(kScatterBS), sm, s, c->in.off, c->in.items,
                               c->hp, pl.NB, pl.max_items, ch, static_cast<uint32_t *>(keys));
        return hipGetLastError();
    }
    if (wide)
        hipLaunchKernelGGL((k_tx_scatter<1024, uint64_t, SingleChunks>), dim3(pl.n_chunks),
                           dim3(1024), sm, s, c->in.off, c->in.items, c->hp, pl.NB, pl.max_items,
                           ch, static_cast<uint64_t *>(keys), pl.stage_cap);
    else
        hipLaunchKernelGGL((k_tx_scatter<1024, uint32_t, SingleChunks>), dim3(pl.n_chunks),
                           dim3(1024), sm, s, c->in.off, c->in.items, c->hp, pl.NB, pl.max_items,
                           ch, static_cast<uint32_t *>(keys), pl.stage_cap);
    return hipGetLastError();
}

size_t tx_win_smem_bytes(uint32_t NB, uint32_t R, uint32_t kb, uint32_t max_items)
{
    return 4 * win_layout(NB, R, kb, max_items).end;
}

bool tx_win_layout_ok(uint32_t NB, uint32_t R, uint32_t kb, uint32_t max_items)
{
    const size_t sm = tx_win_smem_bytes(NB, R, kb, max_items);
    return sm <= 160 * 1024 && win_layout_ok(NB, R, kb, max_items, sm);
}

hipError_t launch_tx_count_win(const crop_ctx *c, uint32_t *cnt, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    const size_t sm = tx_win_smem_bytes(pl.NB, pl.R, pl.win_kb, pl.max_items);
    hipLaunchKernelGGL(k_tx_count_win<kCountBS>, dim3(pl.n_chunks), dim3(kCountBS), sm, s,
                       c->in.off, c->in.items, c->hp, pl.NB, bin_map(pl), pl.max_items,
                       (uint32_t)c->in.T, pl.R, pl.win_kb, pl.win_q, pl.win_W, cnt);
    return hipGetLastError();
}

hipError_t launch_tx_scatter_win(const crop_ctx *c, const uint32_t *cur, void *keys,
                                 hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    const size_t sm = tx_win_smem_bytes(pl.NB, pl.R, pl.win_kb, pl.max_items);
    if (c->in.wide_keys)
        hipLaunchKernelGGL((k_tx_scatter_win<kScatterBS, uint64_t>), dim3(pl.n_chunks),
                           dim3(kScatterBS), sm, s, c->in.off, c->in.items, c->hp, pl.NB,
                           bin_map(pl), pl.max_items, (uint32_t)c->in.T, pl.R, pl.win_kb,
                           pl.win_q, pl.win_W, cur, static_cast<uint64_t *>(keys));
    else
        hipLaunchKernelGGL((k_tx_scatter_win<kScatterBS, uint32_t>), dim3(pl.n_chunks),
                           dim3(kScatterBS), sm, s, c->in.off, c->in.items, c->hp, pl.NB,
                           bin_map(pl), pl.max_items, (uint32_t)c->in.T, pl.R, pl.win_kb,
                           pl.win_q, pl.win_W, cur, static_cast<uint32_t *>(keys));
    return hipGetLastError();
}

hipError_t launch_tx_count_ranges(const crop_ctx *c, uint32_t *cnt, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    size_t sm = tx_count_smem_bytes(pl.NB, pl.max_items);
    hipLaunchKernelGGL(k_tx_count_ranges<1024>, dim3(pl.n_wg), dim3(1024), sm, s, c->in.off,
                       c->in.items, c->hp, pl.NB, bin_map(pl), pl.max_items, (uint32_t)c->in.T,
                       pl.R, pl.n_chunks, cnt);
    return hipGetLastError();
}

hipError_t launch_tx_scatter_ranges(const crop_ctx *c, const uint32_t *cur, void *keys,
                                    hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    const bool wide = c->in.wide_keys;
    size_t sm = tx_scatter_smem_bytes(pl.NB, pl.max_items, pl.stage_cap, wide);
    if (wide)
        hipLaunchKernelGGL((k_tx_scatter_ranges<1024, uint64_t>), dim3(pl.n_wg), dim3(1024), sm,
                           s, c->in.off, c->in.items, c->hp, pl.NB, bin_map(pl), pl.max_items,
                           (uint32_t)c->in.T, pl.R, pl.n_chunks, cur,
                           static_cast<uint64_t *>(keys), pl.stage_cap);
    else
        hipLaunchKernelGGL((k_tx_scatter_ranges<1024, uint32_t>), dim3(pl.n_wg), dim3(1024), sm,
                           s, c->in.off, c->in.items, c->hp, pl.NB, bin_map(pl), pl.max_items,
                           (uint32_t)c->in.T, pl.R, pl.n_chunks, cur,
                           static_cast<uint32_t *>(keys), pl.stage_cap);
    return hipGetLastError();
}

hipError_t launch_batch_count(const uint32_t *off, const uint32_t *items, const HashParams &hp,
                              const BatchDev &b, uint32_t *cnt, const uint32_t *bin_off,
                              hipStream_t s)
{
    if (!b.n_chunks) return hipSuccess;
    size_t sm = tx_count_smem_bytes(b.NBmax, b.max_items);
    const BatchChunks ch{b.crow, b.cstream, b.streams, cnt, bin_off};
    hipLaunchKernelGGL((k_tx_count<kCountBS, BatchChunks>), dim3(b.n_chunks), dim3(kCountBS), sm,
                       s, off, items, hp, b.NBmax, b.max_items, ch);
    return hipGetLastError();
}

hipError_t launch_batch_scatter(const uint32_t *off, const uint32_t *items, const HashParams &hp,
                                const BatchDev &b, uint32_t *cur, const uint32_t *bin_off,
                                void *keys, bool wide, hipStream_t s)
{
    if (!b.n_chunks) return hipSuccess;
    size_t sm = tx_scatter_smem_bytes(b.NBmax, b.max_items, b.stage_cap, wide);
    const BatchChunks ch{b.crow, b.cstream, b.streams, cur, bin_off};
    if (b.stage_cap == 0) {
        sm = 4 * tx_lds_words(b.NBmax, b.max_items);
        if (wide)
            hipLaunchKernelGGL((k_tx_scatter_direct<kScatterBS, uint64_t, BatchChunks>),
                               dim3(b.n_chunks), dim3(kScatterBS), sm, s, off, items, hp, b.NBmax,
                               b.max_items, ch, static_cast<uint64_t *>(keys));
        else
            hipLaunchKernelGGL((k_tx_scatter_direct<kScatterBS, uint32_t, BatchChunks>),
                               dim3(b.n_chunks), dim3(kScatterBS), sm, s, off, items, hp, b.NBmax,
                               b.max_items, ch, static_cast<uint32_t *>(keys));
        return hipGetLastError();
    }
    if (wide)
        hipLaunchKernelGGL((k_tx_scatter<1024, uint64_t, BatchChunks>), dim3(b.n_chunks),
                           dim3(1024), sm, s, off, items, hp, b.NBmax, b.max_items, ch,
                           static_cast<uint64_t *>(keys), b.stage_cap);
    else
        hipLaunchKernelGGL((k_tx_scatter<1024, uint32_t, BatchChunks>), dim3(b.n_chunks),
                           dim3(1024), sm, s, off, items, hp, b.NBmax, b.max_items, ch,
                           static_cast<uint32_t *>(keys), b.stage_cap);
    return hipGetLastError();
}

static OpArgs op_args(const crop_ctx *c)
{
    OpArgs a;
    a.a_off = c->in.a_off;
    a.a_idx = c->in.a_idx;
    a.a_val = c->in.a_val;
    a.b_off = c->in.b_off;
    a.b_idx = c->in.b_idx;
    a.b_val = c->in.b_val;
    a.chunks = c->in.d_op_chunks.as<OpChunk>();
    return a;
}

hipError_t launch_op_count(const crop_ctx *c, uint32_t *cnt, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    size_t sm = op_smem_bytes(pl.NB, pl.max_items, 256);
    hipLaunchKernelGGL(k_op_count<256>, dim3(pl.n_chunks), dim3(256), sm, s, op_args(c), c->hp,
                       pl.NB, bin_map(pl), pl.max_items, cnt);
    return hipGetLastError();
}

hipError_t launch_op_scatter(const crop_ctx *c, const uint32_t *cur, void *keys, float *vals,
                             hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    size_t sm = op_smem_bytes(pl.NB, pl.max_items, 256);
    hipLaunchKernelGGL(k_op_scatter<256>, dim3(pl.n_chunks), dim3(256), sm, s, op_args(c), c->hp,
                       pl.NB, bin_map(pl), pl.max_items, cur, static_cast<uint64_t *>(keys), vals);
    return hipGetLastError();
}

hipError_t launch_bin_order(uint32_t NB, const uint32_t *bin_off, uint32_t *order, hipStream_t s,
                            uint32_t n_seg, uint32_t *zero, uint32_t n_zero)
{
    if (n_zero > 1024 || (n_zero && !zero)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bin_order, dim3(n_seg), dim3(1024), 0, s, NB, bin_off, order, zero,
                       n_zero);
    return hipGetLastError();
}

hipError_t launch_scan_counts(uint32_t *cnt, uint32_t n_chunks, uint32_t NB, uint32_t G,
                              uint32_t *part, uint32_t *bin_off, uint32_t *counter,
                              hipStream_t s)
{
    if (G < 1 || G > kMaxScanGroups) return hipErrorInvalidValue;
    const uint32_t rows_per_g = (n_chunks + G - 1) / G;
    dim3 grid((NB + 255) / 256, G);
    hipLaunchKernelGGL(k_colsum, grid, dim3(256), 0, s, cnt, n_chunks, NB, rows_per_g, part);
    hipLaunchKernelGGL(k_colprefix, dim3((NB + 255) / 256), dim3(256), 0, s, part, NB, G, bin_off);
    hipLaunchKernelGGL(k_colbase, dim3(1), dim3(1024), 0, s, NB, bin_off, counter);
    hipLaunchKernelGGL(k_colapply, grid, dim3(256), 0, s, cnt, n_chunks, NB, rows_per_g, part,
                       bin_off);
    return hipGetLastError();
}

uint32_t batch_scan_tiles(uint32_t NBtot) { return (NBtot + kScanTile - 1) / kScanTile; }

// tot: NBtot words; tiles: batch_scan_tiles(NBtot) words.
hipError_t launch_batch_scan(const BatchDev &b, uint32_t *cnt, uint32_t *tot, uint32_t *tiles,
                             uint32_t *bin_off, uint32_t *counter, hipStream_t s)
{
    const uint32_t g = (b.NBtot + 255) / 256;
    const uint32_t nt = batch_scan_tiles(b.NBtot);
    hipLaunchKernelGGL(k_bcolscan, dim3(g), dim3(256), 0, s, b, cnt, tot);
    hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(1024), 0, s, tot, b.NBtot, tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tiles, nt, bin_off, b.NBtot,
                       counter);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(1024), 0, s, tot, b.NBtot, tiles, bin_off);
    hipLaunchKernelGGL(k_bapply, dim3(g), dim3(256), 0, s, b, cnt, bin_off);
    return hipGetLastError();
}

hipError_t launch_validate_tx(const uint32_t *off, uint64_t T, const uint32_t *items,
                              uint64_t nnz, uint32_t n_items, unsigned long long *bad,
                              hipStream_t s)
{
    uint64_t blocks = (T + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_validate_csr, dim3((uint32_t)blocks), dim3(256), 0, s, off, T, items,
                       nnz, n_items, bad);
    return hipGetLastError();
}

hipError_t launch_check_pairs(const uint32_t *qx, const uint32_t *qy, uint64_t n,
                              uint32_t n_items, unsigned long long *bad, hipStream_t s)
{
    if (!n) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_check_pairs, dim3((uint32_t)blocks), dim3(256), 0, s, qx, qy, n, n_items,
                       bad);
    return hipGetLastError();
}

hipError_t launch_hash_pairs(const uint32_t *qx, const uint32_t *qy, uint64_t n,
                             const HashParams &hp, uint32_t P, uint32_t *h, uint32_t *part,
                             hipStream_t s)
{
    if (!n) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_hash_pairs, dim3((uint32_t)blocks), dim3(256), 0, s, qx, qy, n, hp, P,
                       h, part);
    return hipGetLastError();
}

hipError_t launch_validate_outer(const uint32_t *v_off, uint64_t K, const uint32_t *idx,
                                 uint64_t nnz, uint32_t n, unsigned long long *bad,
                                 hipStream_t s)
{
    return launch_validate_tx(v_off, K, idx, nnz, n, bad, s);
}

}  // namespace crop
