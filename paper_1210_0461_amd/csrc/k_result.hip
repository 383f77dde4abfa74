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

}  // namespace

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
