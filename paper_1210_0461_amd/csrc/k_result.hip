// Readback helpers: gather the bin-segmented exact result into arrays that
// are contiguous per partition, unpacking keys into (i, j).
#include "crop_device.hpp"
#include "crop_internal.hpp"

namespace crop {

namespace {

template <class KeyT, int SHIFT>
__global__ void __launch_bounds__(256)
k_gather(uint32_t bin0, const uint32_t *__restrict__ bin_off, const uint32_t *__restrict__ bin_size,
         const uint32_t *__restrict__ dst_off, const KeyT *__restrict__ keys,
         const uint32_t *__restrict__ cnt, const float *__restrict__ val, uint32_t *__restrict__ oi,
         uint32_t *__restrict__ oj, uint32_t *__restrict__ oc, float *__restrict__ ov)
{
    const uint32_t b = bin0 + blockIdx.x;
    const uint32_t src = bin_off[b], n = bin_size[b], dst = dst_off[blockIdx.x];
    constexpr KeyT low = (KeyT(1) << SHIFT) - 1;
    for (uint32_t k = threadIdx.x; k < n; k += 256) {
        KeyT key = keys[src + k];
        oi[dst + k] = (uint32_t)(key >> SHIFT);
        oj[dst + k] = (uint32_t)(key & low);
        if (oc) oc[dst + k] = cnt[src + k];
        if (ov) ov[dst + k] = val[src + k];
    }
}

// The partitions of grouped bin b: [first, first + 2^g), cut to the kept range.
__device__ inline uint32_t bin_first_partition(uint32_t b, const BinMap &bm)
{
    return (b + (bm.u0 >> bm.g)) << bm.g;
}

// Grouped bins (2^g partitions per bin): for every kept partition, the number
// of entries of the bin that belong to it (n) and their total weight (w:
// the counts, or 1 per entry).  One workgroup per bin, counters in LDS.
template <class KeyT>
__global__ void __launch_bounds__(256)
k_part_stats(const uint32_t *__restrict__ bin_off, const uint32_t *__restrict__ bin_n,
             const KeyT *__restrict__ keys, const uint32_t *__restrict__ wt, HashParams hp,
             BinMap bm, uint32_t *__restrict__ out_n, uint32_t *__restrict__ out_w)
{
    extern __shared__ uint32_t sm[];
    const uint32_t G = 1u << bm.g;
    uint32_t *s_n = sm, *s_w = sm + G;
    for (uint32_t i = threadIdx.x; i < G; i += 256) s_n[i] = s_w[i] = 0;
    __syncthreads();
    const uint32_t b = blockIdx.x;
    const uint32_t first = bin_first_partition(b, bm);
    const uint32_t src = bin_off[b], n = bin_n ? bin_n[b] : bin_off[b + 1] - src;
    for (uint32_t k = threadIdx.x; k < n; k += 256) {
        const uint32_t p = interval_of(hash_of_key(keys[src + k], hp), bm.M);
        atomicAdd(&s_n[p - first], 1u);
        if (out_w) atomicAdd(&s_w[p - first], wt ? wt[src + k] : 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < G; i += 256) {
        const uint32_t p = first + i;
        if (p - bm.u0 >= bm.nu) continue;
        if (out_n) out_n[p] = s_n[i];
        if (out_w) out_w[p] = s_w[i];
    }
}

// Grouped bins to partition-contiguous arrays: partition p starts at
// dst[p - dst_p0]; inside a partition the order is unspecified.  One
// workgroup per bin of [bin0, bin0 + gridDim.x), a write cursor per
// partition in LDS.
template <class KeyT, int SHIFT>
__global__ void __launch_bounds__(256)
k_gather_grouped(uint32_t bin0, const uint32_t *__restrict__ bin_off,
                 const uint32_t *__restrict__ bin_size, const KeyT *__restrict__ keys,
                 const uint32_t *__restrict__ cnt, const float *__restrict__ val, HashParams hp,
                 BinMap bm, const uint32_t *__restrict__ dst, uint32_t dst_p0,
                 uint32_t *__restrict__ oi, uint32_t *__restrict__ oj, uint32_t *__restrict__ oc,
                 float *__restrict__ ov)
{
    extern __shared__ uint32_t s_cur[];
    const uint32_t G = 1u << bm.g;
    const uint32_t b = bin0 + blockIdx.x;
    const uint32_t first = bin_first_partition(b, bm);
    for (uint32_t i = threadIdx.x; i < G; i += 256) {
        const uint32_t p = first + i;
        s_cur[i] = (p - bm.u0 < bm.nu) ? dst[p - dst_p0] : 0u;
    }
    __syncthreads();
    const uint32_t src = bin_off[b], n = bin_size[b];
    constexpr KeyT low = (KeyT(1) << SHIFT) - 1;
    for (uint32_t k = threadIdx.x; k < n; k += 256) {
        const KeyT key = keys[src + k];
        const uint32_t p = interval_of(hash_of_key(key, hp), bm.M);
        const uint32_t o = atomicAdd(&s_cur[p - first], 1u);
        oi[o] = (uint32_t)(key >> SHIFT);
        oj[o] = (uint32_t)(key & low);
        if (oc) oc[o] = cnt[src + k];
        if (ov) ov[o] = val[src + k];
    }
}

}  // namespace

hipError_t launch_part_stats(const crop_ctx *c, bool routed, uint32_t *out_n, uint32_t *out_w,
                             hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    if (pl.NB == 0) return hipSuccess;
    const size_t sm = 8u << pl.g;
    const uint32_t *bn = routed ? nullptr : c->bin_size.as<uint32_t>();
    const uint32_t *wt = routed || c->in.mode == Mode::Outer ? nullptr : c->out_cnt.as<uint32_t>();
    if (c->in.wide_keys || c->in.mode == Mode::Outer)
        hipLaunchKernelGGL(k_part_stats<uint64_t>, dim3(pl.NB), dim3(256), sm, s,
                           c->bin_off.as<uint32_t>(), bn, c->keys.as<uint64_t>(), wt, c->hp,
                           bin_map(pl), out_n, out_w);
    else
        hipLaunchKernelGGL(k_part_stats<uint32_t>, dim3(pl.NB), dim3(256), sm, s,
                           c->bin_off.as<uint32_t>(), bn, c->keys.as<uint32_t>(), wt, c->hp,
                           bin_map(pl), out_n, out_w);
    return hipGetLastError();
}

hipError_t launch_gather_grouped(const crop_ctx *c, uint32_t bin0, uint32_t n_bins,
                                 const uint32_t *dst, uint32_t dst_p0, uint32_t *out_i,
                                 uint32_t *out_j, uint32_t *out_cnt, float *out_val,
                                 hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    if (n_bins == 0) return hipSuccess;
    const bool outer = c->in.mode == Mode::Outer;
    const uint32_t *cnt = outer ? nullptr : c->out_cnt.as<uint32_t>();
    const float *val = outer ? c->vals.as<float>() : nullptr;
    const size_t sm = 4u << pl.g;
    if (!outer && !c->in.wide_keys)
        hipLaunchKernelGGL((k_gather_grouped<uint32_t, 16>), dim3(n_bins), dim3(256), sm, s, bin0,
                           c->bin_off.as<uint32_t>(), c->bin_size.as<uint32_t>(),
                           c->keys.as<uint32_t>(), cnt, val, c->hp, bin_map(pl), dst, dst_p0,
                           out_i, out_j, cnt ? out_cnt : nullptr, val ? out_val : nullptr);
    else
        hipLaunchKernelGGL((k_gather_grouped<uint64_t, 32>), dim3(n_bins), dim3(256), sm, s, bin0,
                           c->bin_off.as<uint32_t>(), c->bin_size.as<uint32_t>(),
                           c->keys.as<uint64_t>(), cnt, val, c->hp, bin_map(pl), dst, dst_p0,
                           out_i, out_j, cnt ? out_cnt : nullptr, val ? out_val : nullptr);
    return hipGetLastError();
}

// Bins [bin0, bin0 + n_bins) to partition-contiguous arrays; dst_off[k] is
// the output start of bin bin0 + k.
hipError_t launch_gather_result(const crop_ctx *c, uint32_t bin0, uint32_t n_bins,
                                const uint32_t *dst_off, uint32_t *out_i, uint32_t *out_j,
                                uint32_t *out_cnt, float *out_val, hipStream_t s)
{
    if (n_bins == 0) return hipSuccess;
    const bool outer = c->in.mode == Mode::Outer;
    const uint32_t *cnt = outer ? nullptr : c->out_cnt.as<uint32_t>();
    const float *val = outer ? c->vals.as<float>() : nullptr;
    if (!outer && !c->in.wide_keys)
        hipLaunchKernelGGL((k_gather<uint32_t, 16>), dim3(n_bins), dim3(256), 0, s, bin0,
                           c->bin_off.as<uint32_t>(), c->bin_size.as<uint32_t>(), dst_off,
                           c->keys.as<uint32_t>(), cnt, val, out_i, out_j,
                           cnt ? out_cnt : nullptr, val ? out_val : nullptr);
    else
        hipLaunchKernelGGL((k_gather<uint64_t, 32>), dim3(n_bins), dim3(256), 0, s, bin0,
                           c->bin_off.as<uint32_t>(), c->bin_size.as<uint32_t>(), dst_off,
                           c->keys.as<uint64_t>(), cnt, val, out_i, out_j,
                           cnt ? out_cnt : nullptr, val ? out_val : nullptr);
    return hipGetLastError();
}

}  // namespace crop
