// Count-Sketch per bucket (Section 4, "Frequent items mining algorithms";
// Section 6, Theorem 3).  Every bucket of every partition keeps one signed
// counter: an entry e adds s(e) w(e) to the counter of its bucket, with
// s(e) = +-1 from the sign hash, and s(e) times that counter estimates e's
// weight.  t instances with independent hash functions (instance i uses the
// parameters drawn from seed + i) give t estimates, and the reported one is
// their median.  Buckets nest in partitions as for Space-Saving: bucket =
// (h * P * B) >> 32, so partition = bucket / B.
//
// Two ways to fill the counters.  Routed (the default): each instance's
// terms are first routed with that instance's hash into bins of whole
// buckets (the exact path's count, scan and scatter), and one workgroup per
// bin sums the bin's signed weights in LDS and writes its buckets' counters
// once.  Direct (when the buckets of a partition have no divisor that gives
// enough bins): the routing kernels' enumeration (crop_enum.hpp) adds every
// term to one counter per instance with a device-scope atomic.  Transactions
// count with int32 counters (exact); outer products with fp32.
#include <algorithm>

#include "crop_device.hpp"
#include "crop_enum.hpp"
#include "crop_internal.hpp"

namespace crop {

namespace {

template <int BS>
__global__ void __launch_bounds__(BS)
k_cs_tx(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items, uint32_t T,
        uint32_t R, uint32_t max_items, CsParams cp, int32_t *__restrict__ cs)
{
    extern __shared__ uint32_t smem[];
    const TxLds L = tx_lds(smem, 0, max_items);
    const uint32_t chunk = xcd_contiguous(blockIdx.x, gridDim.x);
    const uint32_t r0 = chunk * R, r1 = min(r0 + R, T);
    const uint32_t m = stage_tx<BS>(off, items, r0, r1, cp.hp[0], L);
    enum_tx<BS>(m, L, cp.hp[0], [&](uint32_t x, uint32_t y, uint32_t h0) {
        for (uint32_t i = 0; i < cp.t; ++i) {
            const HashParams &hp = cp.hp[i];
            const uint32_t h = i == 0 ? h0 : hash_a(hp, x) + hash_b(hp, y);
            const uint64_t b = interval_of(h, cp.PB);
            atomicAdd(&cs[(uint64_t)i * cp.PB + b], sign_of(hp, x, y));
        }
    });
}

template <int BS>
__global__ void __launch_bounds__(BS)
k_cs_op(OpArgs a, uint32_t max_a, CsParams cp, float *__restrict__ cs)
{
    extern __shared__ uint32_t smem[];
    uint32_t *s_ai, *s_ha, *s_bs, *s_wp, *s_tmp;
    float *s_av;
    (void)op_smem_layout<BS>(smem, 0, max_a, &s_ai, &s_ha, &s_av, &s_bs, &s_wp, &s_tmp);
    const uint32_t chunk = xcd_contiguous(blockIdx.x, gridDim.x);
    uint32_t m;
    const uint32_t Tc = stage_op<BS>(a.chunks[chunk], a.a_off, a.a_idx, a.a_val, a.b_off,
                                     cp.hp[0], s_ai, s_ha, s_av, s_bs, s_wp, s_tmp, &m);
    walk_op<BS>(Tc, m, s_ai, s_ha, s_av, s_bs, s_wp, a.b_idx, a.b_val, cp.hp[0],
                [&](uint32_t x, uint32_t y, uint32_t h0, float v) {
                    for (uint32_t i = 0; i < cp.t; ++i) {
                        const HashParams &hp = cp.hp[i];
                        const uint32_t h = i == 0 ? h0 : hash_a(hp, x) + hash_b(hp, y);
                        const uint64_t b = interval_of(h, cp.PB);
                        atomicAdd(&cs[(uint64_t)i * cp.PB + b], sign_of(hp, x, y) > 0 ? v : -v);
                    }
                });
}

// Bin b holds buckets [b nbk, (b + 1) nbk) of the instance (bucket =
// (h * PB) >> 32 and bin = (h * NB) >> 32 with PB = NB nbk nest).  Its
// counters are summed in LDS from the bin's routed keys and written once.
template <int BS, class KeyT, bool OUTER>
__global__ void __launch_bounds__(BS)
k_cs_bins(const uint32_t *__restrict__ bin_off, const KeyT *__restrict__ keys,
          const float *__restrict__ vals, HashParams hp, uint64_t PB, uint32_t nbk, uint32_t NB,
          uint32_t *__restrict__ out)
{
    extern __shared__ uint32_t acc[];
    for (uint32_t b = blockIdx.x; b < NB; b += gridDim.x) {
        for (uint32_t q = threadIdx.x; q < nbk; q += BS) acc[q] = 0;
        __syncthreads();
        const uint64_t k1 = bin_off[b + 1];
        const uint64_t first = (uint64_t)b * nbk;
        // U keys per thread are loaded before any is summed, so their
        // latencies overlap
        constexpr int U = 4;
        for (uint64_t k = bin_off[b] + threadIdx.x; k < k1; k += (uint64_t)U * BS) {
            KeyT kv[U];
            float vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t i = k + (uint64_t)u * BS;
                kv[u] = i < k1 ? keys[i] : (KeyT)0;
                vv[u] = (OUTER && i < k1) ? vals[i] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (k + (uint64_t)u * BS >= k1) break;
                const KeyT key = kv[u];
                uint32_t x, y;
                if (sizeof(KeyT) == 4) {
                    x = (uint32_t)key >> 16;
                    y = (uint32_t)key & 0xFFFFu;
                } else {
                    x = (uint32_t)((uint64_t)key >> 32);
                    y = (uint32_t)key;
                }
                const uint32_t q =
                    (uint32_t)(interval_of(hash_a(hp, x) + hash_b(hp, y), PB) - first);
                const int sg = sign_of(hp, x, y);
                if (OUTER)
                    atomicAdd(reinterpret_cast<float *>(&acc[q]), sg > 0 ? vv[u] : -vv[u]);
                else
                    atomicAdd(reinterpret_cast<int32_t *>(&acc[q]), sg);
            }
        }
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < nbk; q += BS) out[first + q] = acc[q];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_cs_clear(uint32_t *__restrict__ p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256)
        p[i] = 0;
}

// Median of the instances' estimates s_i(e) C_i[bucket_i(e)] for every query.
template <bool FP>
__global__ void __launch_bounds__(256)
k_cs_estimate(CsParams cp, const void *__restrict__ cs, const uint32_t *__restrict__ qx,
              const uint32_t *__restrict__ qy, uint64_t n, double *__restrict__ out)
{
    for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; q < n;
         q += (uint64_t)gridDim.x * 256) {
        const uint32_t x = qx[q], y = qy[q];
        double v[kCsMaxInstances];
        for (uint32_t i = 0; i < cp.t; ++i) {
            const HashParams &hp = cp.hp[i];
            const uint64_t b = (uint64_t)i * cp.PB + interval_of(hash_a(hp, x) + hash_b(hp, y),
                                                                 cp.PB);
            const double c = FP ? (double)static_cast<const float *>(cs)[b]
                                : (double)static_cast<const int32_t *>(cs)[b];
            v[i] = sign_of(hp, x, y) > 0 ? c : -c;
        }
        // insertion sort of at most kCsMaxInstances values
        for (uint32_t i = 1; i < cp.t; ++i) {
            const double key = v[i];
            uint32_t k = i;
            while (k > 0 && v[k - 1] > key) {
                v[k] = v[k - 1];
                --k;
            }
            v[k] = key;
        }
        const uint32_t h = cp.t / 2;
        out[q] = (cp.t & 1u) ? v[h] : 0.5 * (v[h - 1] + v[h]);
    }
}

static uint32_t grid_of(uint64_t n, uint32_t cap = 4096)
{
    uint64_t g = (n + 255) / 256;
    if (g > cap) g = cap;
    return g ? (uint32_t)g : 1u;
}

}  // namespace

hipError_t launch_cs_clear(void *cs, uint64_t words, hipStream_t s)
{
    if (!words) return hipSuccess;
    hipLaunchKernelGGL(k_cs_clear, dim3(grid_of(words)), dim3(256), 0, s,
                       static_cast<uint32_t *>(cs), words);
    return hipGetLastError();
}

hipError_t launch_cs_tx(const crop_ctx *c, const CsParams &cp, int32_t *cs, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    if (!pl.n_chunks) return hipSuccess;
    const size_t sm = tx_count_smem_bytes(0, pl.max_items);
    hipLaunchKernelGGL(k_cs_tx<256>, dim3(pl.n_chunks), dim3(256), sm, s, c->in.off, c->in.items,
                       (uint32_t)c->in.T, pl.R, pl.max_items, cp, cs);
    return hipGetLastError();
}

hipError_t launch_cs_op(const crop_ctx *c, const CsParams &cp, float *cs, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    if (!pl.n_chunks) return hipSuccess;
    OpArgs a;
    a.a_off = c->in.a_off;
    a.a_idx = c->in.a_idx;
    a.a_val = c->in.a_val;
    a.b_off = c->in.b_off;
    a.b_idx = c->in.b_idx;
    a.b_val = c->in.b_val;
    a.chunks = c->in.d_op_chunks.as<OpChunk>();
    const size_t sm = sizeof(uint32_t) * (5 * (size_t)pl.max_items + 1 + 256 / kWave + 1);
    hipLaunchKernelGGL(k_cs_op<256>, dim3(pl.n_chunks), dim3(256), sm, s, a, pl.max_items, cp,
                       cs);
    return hipGetLastError();
}

// One instance's counters from the routed keys of the current plan: NB bins
// of nbk buckets each (PB = NB nbk counters at out).
hipError_t launch_cs_bins(const crop_ctx *c, const HashParams &hp, uint64_t PB, uint32_t nbk,
                          uint32_t *out, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    const uint32_t NB = pl.NB;
    const size_t sm = (size_t)nbk * 4;
    const uint32_t grid = std::min<uint32_t>(NB, 8192);
    if (c->in.mode == Mode::Outer)
        hipLaunchKernelGGL((k_cs_bins<512, uint64_t, true>), dim3(grid), dim3(512), sm, s,
                           c->bin_off.as<uint32_t>(), c->keys.as<uint64_t>(),
                           c->vals.as<float>(), hp, PB, nbk, NB, out);
    else if (c->in.wide_keys)
        hipLaunchKernelGGL((k_cs_bins<512, uint64_t, false>), dim3(grid), dim3(512), sm, s,
                           c->bin_off.as<uint32_t>(), c->keys.as<uint64_t>(), nullptr, hp, PB,
                           nbk, NB, out);
    else
        hipLaunchKernelGGL((k_cs_bins<512, uint32_t, false>), dim3(grid), dim3(512), sm, s,
                           c->bin_off.as<uint32_t>(), c->keys.as<uint32_t>(), nullptr, hp, PB,
                           nbk, NB, out);
    return hipGetLastError();
}

hipError_t launch_cs_estimate(const CsParams &cp, const void *cs, bool fp, const uint32_t *qx,
                              const uint32_t *qy, uint64_t n, double *out, hipStream_t s)
{
    if (!n) return hipSuccess;
    if (fp)
        hipLaunchKernelGGL(k_cs_estimate<true>, dim3(grid_of(n)), dim3(256), 0, s, cp, cs, qx, qy,
                           n, out);
    else
        hipLaunchKernelGGL(k_cs_estimate<false>, dim3(grid_of(n)), dim3(256), 0, s, cp, cs, qx,
                           qy, n, out);
    return hipGetLastError();
}

}  // namespace crop
