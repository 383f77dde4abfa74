// Consistent distribution hash of the column-row method, device side.
//
// Section 5 (Lemma 1 and its proof): entry (i,j) goes to bucket
// h(i,j) = (h_a(i) + h_b(j)) mod kappa, with h_a and h_b pairwise
// independent; that additive form is what lets an owner of a hash interval
// find its own entries.  kappa = 2^32 here.  The family (the paper leaves it
// open) is multiply-add-shift, h(x) = ((alpha * x + beta) mod 2^64) >> 32,
// strongly universal for 32-bit keys (Dietzfelbinger 1996), with the four
// 64-bit parameters drawn from SplitMix64 (Steele, Lea, Flood 2014) started
// at the user's seed.  Owners take equal intervals of the hash space
// (Section 6, Theorem 1): part = (h * P) >> 32, and the summaries inside an
// owner take finer equal intervals: bucket = (h * P * B) >> 32.
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

namespace crop {

struct HashParams {
    uint64_t alpha_a, beta_a, alpha_b, beta_b;   // distribution hash h_a, h_b
    uint64_t alpha_s, beta_s, alpha_t, beta_t;   // sign hash s (Count-Sketch)
};

// SplitMix64 step (Steele, Lea, Flood 2014).
inline uint64_t splitmix64_step(uint64_t &state)
{
    state += 0x9e3779b97f4a7c15ULL;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

inline HashParams make_hash_params(uint64_t seed)
{
    uint64_t st = seed;
    HashParams p;
    p.alpha_a = splitmix64_step(st);
    p.beta_a = splitmix64_step(st);
    p.alpha_b = splitmix64_step(st);
    p.beta_b = splitmix64_step(st);
    p.alpha_s = splitmix64_step(st);
    p.beta_s = splitmix64_step(st);
    p.alpha_t = splitmix64_step(st);
    p.beta_t = splitmix64_step(st);
    return p;
}

__host__ __device__ inline uint32_t mul_add_shift(uint64_t alpha, uint64_t beta, uint32_t x)
{
    return (uint32_t)((alpha * (uint64_t)x + beta) >> 32);
}

__host__ __device__ inline uint32_t hash_a(const HashParams &p, uint32_t x)
{
    return mul_add_shift(p.alpha_a, p.beta_a, x);
}

__host__ __device__ inline uint32_t hash_b(const HashParams &p, uint32_t y)
{
    return mul_add_shift(p.alpha_b, p.beta_b, y);
}

// Interval index of hash value h among n <= 2^32 equal intervals of [0, 2^32).
__host__ __device__ inline uint32_t interval_of(uint32_t h, uint64_t n)
{
    return (uint32_t)(((uint64_t)h * n) >> 32);
}

// +1 / -1 sign of an entry for Count-Sketch: top bit of g_a(i) + g_b(j).
__host__ __device__ inline int sign_of(const HashParams &p, uint32_t i, uint32_t j)
{
    uint32_t g = mul_add_shift(p.alpha_s, p.beta_s, i) + mul_add_shift(p.alpha_t, p.beta_t, j);
    return (g >> 31) ? -1 : 1;
}

// Routing bins of a run.  A hash value h maps to u = floor(h M / 2^32)
// (M = partitions x bins per partition, or partitions alone when a bin groups
// 2^g of them); the run keeps u in [u0, u0 + nu) -- its owned partitions --
// and local() is the kept bin (u >> g) - (u0 >> g), or kNoBin for a term
// outside the kept range.  Partition p = floor(h P / 2^32) nests in its bins
// because every bin boundary is a partition boundary (nested floors).
constexpr uint32_t kNoBin = 0xFFFFFFFFu;

struct BinMap {
    uint64_t M;
    uint32_t u0, nu, g;
    __host__ __device__ uint32_t local(uint32_t h) const
    {
        const uint32_t u = interval_of(h, M);
        return u - u0 < nu ? (u >> g) - (u0 >> g) : kNoBin;
    }
};

template <class KeyT>
__host__ __device__ inline uint32_t hash_of_key(KeyT key, const HashParams &hp)
{
    uint32_t x, y;
    if (sizeof(KeyT) == 4) {
        x = (uint32_t)key >> 16;
        y = (uint32_t)key & 0xFFFFu;
    } else {
        x = (uint32_t)((uint64_t)key >> 32);
        y = (uint32_t)key;
    }
    return hash_a(hp, x) + hash_b(hp, y);
}

}  // namespace crop
