// Device-side building blocks shared by the CRoP kernels (wave64, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crop {

constexpr int kWave = 64;
constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;
constexpr uint64_t kEmpty64 = 0xFFFFFFFFFFFFFFFFull;
constexpr int kNumXcd = 8;  // MI355X: 256 CUs in 8 XCDs, one L2 each

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b % 8).  Remap so that each XCD receives a contiguous range of logical
// work items: consecutive items then share that XCD's L2.
__device__ inline uint32_t xcd_contiguous(uint32_t b, uint32_t n)
{
    const uint32_t x = b % kNumXcd, j = b / kNumXcd;
    const uint32_t q = n / kNumXcd, r = n % kNumXcd;
    return x * q + (x < r ? x : r) + j;
}

__device__ inline uint32_t lane_id() { return __lane_id(); }

// Inclusive scan of v across the 64 lanes of a wave (every lane active),
// in DPP moves: shifts by 1, 2, 4 and 8 lanes inside each row of 16 (lanes
// shifted in from outside the row read 0), then the last lane of row 0 is
// added to row 1 and of row 2 to row 3 (row_bcast:15), then the last lane
// of row 1 to rows 2 and 3 (row_bcast:31).  No LDS round trip.
__device__ inline uint32_t wave_inclusive_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// Sum over the wave of per-lane counts, wave-uniform: one ballot per bit of
// the counts (no LDS round trip), as many as the largest count needs.
__device__ inline uint32_t wave_count_sum(uint32_t v)
{
    uint32_t tot = 0;
    for (uint32_t bit = 0; bit < 32; ++bit) {
        tot += (uint32_t)__popcll(__ballot((v >> bit) & 1u)) << bit;
        if (__ballot((v >> bit) > 1u) == 0) break;
    }
    return tot;
}

// v of lane `src`, a wave-uniform lane index (one readlane, no LDS).
__device__ inline uint32_t lane_value(uint32_t v, uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)src);
}

// Exclusive scan over the block; returns this thread's prefix and the
// block total in *total.  s_tmp needs BS/64 + 1 words.  Contains barriers:
// every thread of the block must call it.
template <int BS>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp, uint32_t *total)
{
    constexpr int NW = BS / kWave;
    const uint32_t lane = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) s_tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int k = 0; k < NW; ++k) {
            uint32_t t = s_tmp[k];
            s_tmp[k] = run;
            run += t;
        }
        s_tmp[NW] = run;
    }
    __syncthreads();
    uint32_t res = s_tmp[w] + inc - v;
    *total = s_tmp[NW];
    __syncthreads();
    return res;
}

// In-place exclusive scan of an LDS array a[0..m); writes the total to a[m].
// Each thread scans a contiguous segment.  Contains barriers.
template <int BS>
__device__ inline void lds_exclusive_scan(uint32_t *a, uint32_t m, uint32_t *s_tmp)
{
    const uint32_t per = (m + BS - 1) / BS;
    const uint32_t beg = threadIdx.x * per;
    const uint32_t end = beg + per < m ? beg + per : m;
    uint32_t sum = 0;
    for (uint32_t k = beg; k < end; ++k) sum += a[k];
    uint32_t total;
    uint32_t run = block_exclusive_scan<BS>(sum, s_tmp, &total);
    for (uint32_t k = beg; k < end; ++k) {
        uint32_t t = a[k];
        a[k] = run;
        run += t;
    }
    if (threadIdx.x == 0) a[m] = total;
    __syncthreads();
}

// In-place exclusive scan of a[0..m) in LDS for a workgroup of any size
// that is a multiple of 64 (at most 1024); writes the total to a[m].
// s_tmp needs blockDim.x / 64 + 1 words.  Contains barriers.
__device__ inline void lds_exclusive_scan_rt(uint32_t *a, uint32_t m, uint32_t *s_tmp)
{
    const uint32_t BS = blockDim.x, NW = BS / kWave;
    const uint32_t per = (m + BS - 1) / BS;
    const uint32_t beg = threadIdx.x * per;
    const uint32_t end = beg + per < m ? beg + per : m;
    uint32_t sum = 0;
    for (uint32_t k = beg; k < end; ++k) sum += a[k];
    const uint32_t inc = wave_inclusive_scan(sum);
    const uint32_t w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) s_tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t k = 0; k < NW; ++k) {
            const uint32_t t = s_tmp[k];
            s_tmp[k] = run;
            run += t;
        }
        s_tmp[NW] = run;
    }
    __syncthreads();
    uint32_t run = s_tmp[w] + inc - sum;
    for (uint32_t k = beg; k < end; ++k) {
        const uint32_t t = a[k];
        a[k] = run;
        run += t;
    }
    if (threadIdx.x == 0) a[m] = s_tmp[NW];
    __syncthreads();
}

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load, which would drain a register prefetch.
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Fibonacci hashing of a key to a table slot (Knuth, TAOCP vol. 3, 6.4).
__device__ inline uint32_t slot_of(uint32_t key, uint32_t log2_slots)
{
    return (key * 0x9E3779B1u) >> (32 - log2_slots);
}

__device__ inline uint32_t slot_of(uint64_t key, uint32_t log2_slots)
{
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - log2_slots));
}

}  // namespace crop
