// Learned heavy-pair seeding (an addition to the method; the paper has no
// learned component).  Its Space-Saving analysis (Section 6, Theorem 2 and
// its proof) names the failure this targets: a heavy entry loses its slot
// when more than ell/2 heavy entries, or too much light weight, share its
// bucket.  Pairs predicted heavy are pinned into their bucket before the
// stream (k_topk.hip), so they are counted exactly from the start.
//
// Pieces, all on the device:
//   - per-item statistics of a stream prefix and 16 features per item;
//   - candidate pairs: all x < y among the M items most frequent in the
//     prefix (ties by smaller id);
//   - labels: exact supports of the candidates looked up in the result of
//     an exact run, y = log1p(support);
//   - an MLP [f(x), f(y)] (32) -> 64 -> 64 -> 1 with ReLU, trained with mean
//     squared error and Adam (Kingma and Ba 2015) in fp32 by one persistent
//     workgroup whose weights stay in LDS, and scored with bf16-rounded
//     weights and inputs (fp32 accumulation);
//   - seed selection: candidates ranked by score (higher first, ties by
//     candidate index).
#include <math.h>

#include "crop_device.hpp"
#include "crop_internal.hpp"

namespace crop {

namespace {

constexpr int kF = 16;       // features per item
constexpr int kIn = 2 * kF;  // network inputs
constexpr int kH = 64;       // hidden width
constexpr int oW1 = 0, oB1 = kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH, kParams = oB3 + 1;
static_assert(kParams == 6337, "parameter layout");
// The training kernels keep the weights in LDS with rows of W1 and W2 padded
// by one word (strides kIn + 1 and kH + 1), so that the lanes of a wavefront,
// which read one row each, hit different LDS banks.  lds_of maps a
// parameter index to its padded LDS position.
constexpr int kW1S = kIn + 1, kW2S = kH + 1;
constexpr int lW1 = 0, lB1 = kH * kW1S, lW2 = lB1 + kH, lB2 = lW2 + kH * kW2S, lW3 = lB2 + kH,
              lB3 = lW3 + kH, kLdsParams = lB3 + 1;
__device__ inline uint32_t lds_of(uint32_t p)
{
    if (p < (uint32_t)oB1) return lW1 + (p / kIn) * kW1S + p % kIn;
    if (p < (uint32_t)oW2) return lB1 + (p - oB1);
    if (p < (uint32_t)oB2) {
        const uint32_t q = p - oW2;
        return lW2 + (q / kH) * kW2S + q % kH;
    }
    return lB2 + (p - oB2);  // b2, w3, b3 keep their order
}

// ---------------------------------------------------------------- features

struct ItemStats {
    uint32_t *A, *S1, *LMAX, *H1, *LONG, *SHORT, *hist;  // hist: prefix_T + 2 words
    unsigned long long *S2;
};

__global__ void __launch_bounds__(256)
k_item_stats(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items, uint32_t Tp,
             ItemStats st)
{
    const uint32_t half = Tp / 2;
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < Tp; t += gridDim.x * 256) {
        const uint32_t a = off[t], e = off[t + 1], L = e - a;
        const uint32_t s1 = L ? L - 1 : 0;
        const unsigned long long s2 = L >= 2 ? (unsigned long long)(L - 1) * (L - 2) / 2 : 0;
        for (uint32_t k = a; k < e; ++k) {
            const uint32_t x = items[k];
            atomicAdd(&st.A[x], 1u);
            atomicAdd(&st.S1[x], s1);
            if (s2) atomicAdd(&st.S2[x], s2);
            atomicMax(&st.LMAX[x], L);
            if (t < half) atomicAdd(&st.H1[x], 1u);
            if (L >= 16) atomicAdd(&st.LONG[x], 1u);
            if (L <= 4) atomicAdd(&st.SHORT[x], 1u);
        }
    }
}

__global__ void __launch_bounds__(256)
k_count_hist(const uint32_t *__restrict__ A, uint32_t n, uint32_t *__restrict__ hist)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        atomicAdd(&hist[A[i]], 1u);
}

// One workgroup: hist[a] <- number of items with count >= a (suffix sums
// over a = 0..Tp), in place; hist[Tp + 1] = 0.
__global__ void __launch_bounds__(1024) k_suffix_sum(uint32_t *__restrict__ hist, uint32_t Tp)
{
    __shared__ uint32_t s_tmp[1024 / kWave + 1];
    const uint32_t m = Tp + 1;
    const uint32_t per = (m + 1023) / 1024;
    // reverse order: thread 0 owns the largest counts
    const uint32_t r0 = threadIdx.x * per, r1 = min(m, r0 + per);
    uint32_t sum = 0;
    for (uint32_t r = r0; r < r1; ++r) sum += hist[Tp - r];
    uint32_t total;
    uint32_t run = block_exclusive_scan<1024>(sum, s_tmp, &total);
    for (uint32_t r = r0; r < r1; ++r) {
        run += hist[Tp - r];
        hist[Tp - r] = run;
    }
    if (threadIdx.x == 0) hist[Tp + 1] = 0;
}

__global__ void __launch_bounds__(256)
k_features(ItemStats st, uint32_t n, uint32_t Tp, float *__restrict__ feat)
{
    const float Tpf = (float)(Tp ? Tp : 1);
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float A = (float)st.A[i];
        const float S1 = (float)st.S1[i];
        const float S2 = (float)st.S2[i];
        const float H1 = (float)st.H1[i];
        const float H2 = A - H1;
        const float rank = (float)st.hist[st.A[i] + 1];  // items with a larger count
        float *f = feat + (size_t)i * kF;
        f[0] = log1pf(A);
        f[1] = 100.0f * A / Tpf;
        f[2] = log1pf(rank);
        f[3] = log1pf(S1);
        f[4] = log1pf(S2);
        f[5] = S1 / fmaxf(A, 1.0f) / 10.0f;
        f[6] = log1pf((float)st.LMAX[i]);
        f[7] = log1pf(H1);
        f[8] = log1pf(H2);
        f[9] = (H2 - H1) / (A + 1.0f);
        f[10] = log1pf((float)st.LONG[i]);
        f[11] = log1pf((float)st.SHORT[i]);
        f[12] = sqrtf(A / Tpf);
        f[13] = log1pf(A) * log1pf(A) / 10.0f;
        f[14] = A > 0.0f ? 1.0f : 0.0f;
        f[15] = logf(Tpf) / 10.0f;
    }
}

// ---------------------------------------------------------------- candidates

// One workgroup: top[0..M) = the M items with the largest prefix counts,
// ties by smaller id, in increasing id order.  geq = suffix counts.
__global__ void __launch_bounds__(1024)
k_top_items(const uint32_t *__restrict__ A, uint32_t n, const uint32_t *__restrict__ geq,
            uint32_t Tp, uint32_t M, uint32_t *__restrict__ top)
{
    __shared__ uint32_t s_tmp[1024 / kWave + 1];
    __shared__ uint32_t s_aM, s_gt;
    if (threadIdx.x == 0) {
        // largest a with #(count >= a) >= M; a = 0 always qualifies when n >= M
        uint32_t lo = 0, hi = Tp;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            if (geq[mid] >= M) lo = mid; else hi = mid - 1;
        }
        s_aM = lo;
        s_gt = geq[lo + 1];
    }
    __syncthreads();
    const uint32_t aM = s_aM, need_ties = M - s_gt;
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t i0 = threadIdx.x * per, i1 = min(n, i0 + per);
    uint32_t ties = 0;
    for (uint32_t i = i0; i < i1; ++i) ties += A[i] == aM;
    uint32_t tot;
    uint32_t tie_before = block_exclusive_scan<1024>(ties, s_tmp, &tot);
    uint32_t sel = 0;
    {
        uint32_t tb = tie_before;
        for (uint32_t i = i0; i < i1; ++i) {
            if (A[i] > aM) ++sel;
            else if (A[i] == aM) {
                if (tb < need_ties) ++sel;
                ++tb;
            }
        }
    }
    uint32_t pos = block_exclusive_scan<1024>(sel, s_tmp, &tot);
    uint32_t tb = tie_before;
    for (uint32_t i = i0; i < i1; ++i) {
        bool take = false;
        if (A[i] > aM) take = true;
        else if (A[i] == aM) {
            take = tb < need_ties;
            ++tb;
        }
        if (take) top[pos++] = i;
    }
}

// Pairs (top[a], top[b]) for a < b in (a, b) order; one thread per a.
__global__ void __launch_bounds__(256)
k_pairs(const uint32_t *__restrict__ top, uint32_t M, uint32_t *__restrict__ cx,
        uint32_t *__restrict__ cy)
{
    const uint32_t a = blockIdx.x * 256 + threadIdx.x;
    if (a >= M) return;
    const uint64_t base = (uint64_t)a * (M - 1) - (uint64_t)a * (a - 1) / 2;  // pairs of rows < a
    for (uint32_t b = a + 1; b < M; ++b) {
        cx[base + (b - a - 1)] = top[a];
        cy[base + (b - a - 1)] = top[b];
    }
}

// ---------------------------------------------------------------- labels

// One wavefront per query: scan the query's routing bin of the exact result.
template <class KeyT>
__global__ void __launch_bounds__(256)
k_lookup(const uint32_t *__restrict__ qx, const uint32_t *__restrict__ qy, uint64_t n,
         HashParams hp, BinMap bm, uint32_t NB,
         const uint32_t *__restrict__ bin_off,
         const uint32_t *__restrict__ bin_size, const KeyT *__restrict__ keys,
         const uint32_t *__restrict__ cnt, uint32_t *__restrict__ out)
{
    const uint64_t q = ((uint64_t)blockIdx.x * 256 + threadIdx.x) / kWave;
    const uint32_t lane = lane_id();
    if (q >= n) return;
    const uint32_t x = qx[q], y = qy[q];
    // the query's bin of the run (a pair outside the owned partitions: none)
    const uint32_t b = bm.local(hash_a(hp, x) + hash_b(hp, y));
    const KeyT key = sizeof(KeyT) == 4 ? (KeyT)((x << 16) | y) : (KeyT)(((uint64_t)x << 32) | y);
    const uint32_t s0 = b < NB ? bin_off[b] : 0, ns = b < NB ? bin_size[b] : 0;
    uint32_t found = 0;
    for (uint32_t i = lane; i < ns; i += kWave) {
        if (keys[s0 + i] == key) found = cnt[s0 + i];
    }
    // at most one lane found the key
    for (int d = 32; d >= 1; d >>= 1) found |= __shfl_xor(found, d, kWave);
    if (lane == 0) out[q] = found;
}

__global__ void __launch_bounds__(256)
k_pair_inputs(const float *__restrict__ feat, const uint32_t *__restrict__ cx,
              const uint32_t *__restrict__ cy, const uint32_t *__restrict__ count, uint64_t n,
              float *__restrict__ Z, float *__restrict__ y)
{
    for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n * kIn;
         e += (uint64_t)gridDim.x * 256) {
        const uint64_t q = e / kIn;
        const uint32_t c = (uint32_t)(e % kIn);
        const uint32_t item = c < kF ? cx[q] : cy[q];
        Z[e] = feat[(size_t)item * kF + (c % kF)];
        if (y && c == 0) y[q] = log1pf((float)count[q]);
    }
}

// ---------------------------------------------------------------- MLP

constexpr int kBatch = 128;  // samples per step (LDS-resident activations)

struct MlpLds {
    float *W;   // kParams
    float *Zs;  // kBatch x kIn
    float *H1;  // kBatch x kH
    float *H2;  // kBatch x kH (reused for G1)
    float *G2;  // kBatch x kH
    float *g;   // kBatch (output gradients)
    float *red; // reduction scratch
};

// Forward and backward of one batch of nb <= kBatch samples; this thread's
// share of the gradient is accumulated into grad (kParams, global) by
// ownership: every parameter is written by exactly one thread.  Returns the
// batch's summed squared residual in *sse (thread 0).
// Gradients are written to gstage (global, kParams); with apply, Adam then
// updates the LDS weights and the moments m, v from it.
template <int BS>
__device__ void mlp_batch(const MlpLds &L, uint32_t nb, float inv_n, const float *__restrict__ y,
                          const uint32_t *idx, bool apply, float *gstage, float *m, float *v,
                          float lr, float bc1, float bc2, float *sse)
{
    const float *W1 = L.W + lW1, *b1 = L.W + lB1, *W2 = L.W + lW2, *b2 = L.W + lB2,
                *w3 = L.W + lW3;
    const float b3 = L.W[lB3];
    // layer 1
    for (uint32_t e = threadIdx.x; e < nb * kH; e += BS) {
        const uint32_t s = e / kH, i = e % kH;
        float a = b1[i];
        for (int k = 0; k < kIn; ++k) a = fmaf(W1[i * kW1S + k], L.Zs[s * kIn + k], a);
        L.H1[s * kH + i] = fmaxf(a, 0.0f);
    }
    __syncthreads();
    // layer 2
    for (uint32_t e = threadIdx.x; e < nb * kH; e += BS) {
        const uint32_t s = e / kH, i = e % kH;
        float a = b2[i];
        for (int k = 0; k < kH; ++k) a = fmaf(W2[i * kW2S + k], L.H1[s * kH + k], a);
        L.H2[s * kH + i] = fmaxf(a, 0.0f);
    }
    __syncthreads();
    // output and its gradient
    float part = 0.0f;
    for (uint32_t s = threadIdx.x; s < nb; s += BS) {
        float o = b3;
        for (int i = 0; i < kH; ++i) o = fmaf(w3[i], L.H2[s * kH + i], o);
        const float r = o - y[idx[s]];
        L.g[s] = 2.0f * r * inv_n;
        part += r * r;
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) part += __shfl_xor(part, d, kWave);
    if (lane_id() == 0) L.red[threadIdx.x / kWave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int k = 0; k < BS / kWave; ++k) t += L.red[k];
        *sse = t;
    }
    // gradients of w3, b3 (need H2), then G2 = g * w3 * [H2 > 0]
    auto stage = [&](uint32_t p, float val) { gstage[p] = val; };
    for (uint32_t i = threadIdx.x; i < kH + 1; i += BS) {
        float acc = 0.0f;
        if (i < kH) {
            for (uint32_t s = 0; s < nb; ++s) acc = fmaf(L.g[s], L.H2[s * kH + i], acc);
            stage(oW3 + i, acc);
        } else {
            for (uint32_t s = 0; s < nb; ++s) acc += L.g[s];
            stage(oB3, acc);
        }
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < nb * kH; e += BS) {
        const uint32_t s = e / kH, i = e % kH;
        L.G2[e] = L.H2[e] > 0.0f ? L.g[s] * w3[i] : 0.0f;
    }
    __syncthreads();
    // gW2, gb2
    for (uint32_t p = threadIdx.x; p < kH * kH + kH; p += BS) {
        float acc = 0.0f;
        if (p < kH * kH) {
            const uint32_t i = p / kH, k = p % kH;
            for (uint32_t s = 0; s < nb; ++s) acc = fmaf(L.G2[s * kH + i], L.H1[s * kH + k], acc);
            stage(oW2 + p, acc);
        } else {
            const uint32_t i = p - kH * kH;
            for (uint32_t s = 0; s < nb; ++s) acc += L.G2[s * kH + i];
            stage(oB2 + i, acc);
        }
    }
    // G1 = (G2 W2) * [H1 > 0], into the H2 buffer
    float *G1 = L.H2;
    for (uint32_t e = threadIdx.x; e < nb * kH; e += BS) {
        const uint32_t s = e / kH, k = e % kH;
        float acc = 0.0f;
        for (int i = 0; i < kH; ++i) acc = fmaf(L.G2[s * kH + i], W2[i * kW2S + k], acc);
        G1[e] = L.H1[e] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    // gW1, gb1
    for (uint32_t p = threadIdx.x; p < kH * kIn + kH; p += BS) {
        float acc = 0.0f;
        if (p < kH * kIn) {
            const uint32_t i = p / kIn, k = p % kIn;
            for (uint32_t s = 0; s < nb; ++s) acc = fmaf(G1[s * kH + i], L.Zs[s * kIn + k], acc);
            stage(oW1 + p, acc);
        } else {
            const uint32_t i = p - kH * kIn;
            for (uint32_t s = 0; s < nb; ++s) acc += G1[s * kH + i];
            stage(oB1 + i, acc);
        }
    }
    __syncthreads();  // weights are no longer read; gstage is complete and visible
    if (apply) {
        for (uint32_t p = threadIdx.x; p < kParams; p += BS) {
            const float gr = gstage[p];
            const float mp = 0.9f * m[p] + 0.1f * gr;
            const float vp = 0.999f * v[p] + 0.001f * gr * gr;
            m[p] = mp;
            v[p] = vp;
            L.W[lds_of(p)] -= lr * (mp / bc1) / (sqrtf(vp / bc2) + 1e-8f);
        }
        __syncthreads();
    }
}

__device__ inline MlpLds mlp_lds(float *smem)
{
    MlpLds L;
    L.W = smem;
    L.Zs = L.W + ((kLdsParams + 3) & ~3);
    L.H1 = L.Zs + kBatch * kIn;
    L.H2 = L.H1 + kBatch * kH;
    L.G2 = L.H2 + kBatch * kH;
    L.g = L.G2 + kBatch * kH;
    L.red = L.g + kBatch;
    return L;
}

constexpr int kMlpBS = 1024;  // one workgroup: as many wavefronts as a CU takes
constexpr size_t kMlpSmem =
    sizeof(float) * (((kLdsParams + 3) & ~3) + kBatch * kIn + 3 * kBatch * kH + kBatch + kMlpBS);

// Persistent single workgroup: n_steps Adam steps over consecutive slices of
// `order` (batch indices into Z/y), weights kept in LDS; Adam moments in
// global memory.  Step numbers t0+1 .. t0+n_steps give the bias corrections.
__global__ void __launch_bounds__(kMlpBS)
k_mlp_train(float *__restrict__ params, float *__restrict__ m, float *__restrict__ v,
            float *__restrict__ gstage, const float *__restrict__ Z, const float *__restrict__ y,
            const uint32_t *__restrict__ order, uint64_t n_order, uint32_t batch, float lr,
            uint64_t t0, float *__restrict__ loss_out)
{
    extern __shared__ float smem_f[];
    const MlpLds L = mlp_lds(smem_f);
    __shared__ uint32_t s_idx[kBatch];
    __shared__ float s_sse;
    for (uint32_t p = threadIdx.x; p < kParams; p += kMlpBS) L.W[lds_of(p)] = params[p];
    __syncthreads();
    const uint64_t n_steps = n_order / batch;
    float last = 0.0f;
    for (uint64_t st = 0; st < n_steps; ++st) {
        const uint64_t base = st * batch;
        for (uint32_t s = threadIdx.x; s < batch; s += kMlpBS) s_idx[s] = order[base + s];
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < batch * kIn; e += kMlpBS)
            L.Zs[e] = Z[(size_t)s_idx[e / kIn] * kIn + (e % kIn)];
        __syncthreads();
        const double t = (double)(t0 + st + 1);
        const float bc1 = (float)(1.0 - pow(0.9, t));
        const float bc2 = (float)(1.0 - pow(0.999, t));
        mlp_batch<kMlpBS>(L, batch, 1.0f / batch, y, s_idx, true, gstage, m, v, lr, bc1, bc2,
                          &s_sse);
        last = s_sse;
    }
    for (uint32_t p = threadIdx.x; p < kParams; p += kMlpBS) params[p] = L.W[lds_of(p)];
    if (threadIdx.x == 0 && loss_out) *loss_out = last / (float)batch;
}

// Gradient of the mean squared error over N <= kBatch samples (no update).
__global__ void __launch_bounds__(kMlpBS)
k_mlp_grad(const float *__restrict__ params, const float *__restrict__ Z,
           const float *__restrict__ y, uint32_t N, float *__restrict__ grad,
           float *__restrict__ loss_out)
{
    extern __shared__ float smem_f[];
    const MlpLds L = mlp_lds(smem_f);
    __shared__ uint32_t s_idx[kBatch];
    __shared__ float s_sse;
    for (uint32_t p = threadIdx.x; p < kParams; p += kMlpBS) L.W[lds_of(p)] = params[p];
    for (uint32_t s = threadIdx.x; s < N; s += kMlpBS) s_idx[s] = s;
    for (uint32_t e = threadIdx.x; e < N * kIn; e += kMlpBS) L.Zs[e] = Z[e];
    __syncthreads();
    mlp_batch<kMlpBS>(L, N, 1.0f / N, y, s_idx, false, grad, nullptr, nullptr, 0.0f, 1.0f, 1.0f,
                      &s_sse);
    if (threadIdx.x == 0) *loss_out = s_sse / (float)N;
}

__device__ inline float bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// bf16 pairs for the dot-product instruction (element 0 in the low half).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ inline uint32_t bf16_pair(float lo, float hi)
{
    return (__float_as_uint(bf16_rne(lo)) >> 16) | (__float_as_uint(bf16_rne(hi)) & 0xFFFF0000u);
}

// a.lo * b.lo + a.hi * b.hi + c with bf16 operands, in fp32
__device__ inline float dot2_bf16(uint32_t a, uint32_t b, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a),
                                           __builtin_bit_cast(bf16x2_t, b), c, false);
}

// bf16 inference: weights, inputs and each layer's activations rounded to
// bf16 (nearest even), products and sums in fp32 through the bf16
// dot-product instruction (two products per step); biases in fp32.  One
// thread per sample, the weight pairs in LDS.
__global__ void __launch_bounds__(256)
k_mlp_score(const float *__restrict__ params, const float *__restrict__ Z, uint64_t N,
            float *__restrict__ out)
{
    constexpr int P1 = kH * kIn / 2, P2 = kH * kH / 2, P3 = kH / 2;
    __shared__ uint32_t W1[P1], W2[P2], W3[P3];
    __shared__ float B1[kH], B2[kH], B3;
    for (uint32_t p = threadIdx.x; p < (uint32_t)P1; p += 256)
        W1[p] = bf16_pair(params[oW1 + 2 * p], params[oW1 + 2 * p + 1]);
    for (uint32_t p = threadIdx.x; p < (uint32_t)P2; p += 256)
        W2[p] = bf16_pair(params[oW2 + 2 * p], params[oW2 + 2 * p + 1]);
    for (uint32_t p = threadIdx.x; p < (uint32_t)P3; p += 256)
        W3[p] = bf16_pair(params[oW3 + 2 * p], params[oW3 + 2 * p + 1]);
    for (uint32_t p = threadIdx.x; p < (uint32_t)kH; p += 256) {
        B1[p] = params[oB1 + p];
        B2[p] = params[oB2 + p];
    }
    if (threadIdx.x == 0) B3 = params[oB3];
    __syncthreads();
    for (uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x; s < N;
         s += (uint64_t)gridDim.x * 256) {
        uint32_t z[kIn / 2];
#pragma unroll
        for (int k = 0; k < kIn / 2; ++k) z[k] = bf16_pair(Z[s * kIn + 2 * k], Z[s * kIn + 2 * k + 1]);
        uint32_t h1[kH / 2];
#pragma unroll
        for (int i = 0; i < kH; i += 2) {
            float a0 = B1[i], a1 = B1[i + 1];
#pragma unroll
            for (int k = 0; k < kIn / 2; ++k) {
                a0 = dot2_bf16(W1[i * (kIn / 2) + k], z[k], a0);
                a1 = dot2_bf16(W1[(i + 1) * (kIn / 2) + k], z[k], a1);
            }
            h1[i / 2] = bf16_pair(fmaxf(a0, 0.0f), fmaxf(a1, 0.0f));
        }
        float o = B3;
        for (int i = 0; i < kH; i += 2) {
            float a0 = B2[i], a1 = B2[i + 1];
#pragma unroll
            for (int k = 0; k < kH / 2; ++k) {
                a0 = dot2_bf16(W2[i * (kH / 2) + k], h1[k], a0);
                a1 = dot2_bf16(W2[(i + 1) * (kH / 2) + k], h1[k], a1);
            }
            o = dot2_bf16(W3[i / 2], bf16_pair(fmaxf(a0, 0.0f), fmaxf(a1, 0.0f)), o);
        }
        out[s] = o;
    }
}

// Seeds: the R best candidates by (score desc, index asc), in that order.
// Scores become order-preserving words (-0 taken as +0, so equal scores
// give equal words).
__device__ inline uint32_t score_word(float f)
{
    const uint32_t b = __float_as_uint(f == 0.0f ? 0.0f : f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// One workgroup: the R-th best word t by radix selection (four 8-bit digits,
// most significant first), then the selected candidates in index order:
// every word above t and the first `need` (by index) equal to t, where need
// is what R leaves after the words above t.  sel[0] = t, sel[1] = need,
// sel[2 ..] = the R selected indices.
__global__ void __launch_bounds__(1024)
k_seed_threshold(const float *__restrict__ score, uint32_t n, uint32_t R, uint32_t *__restrict__ sel)
{
    constexpr uint32_t BS = 1024;
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_tmp[BS / kWave + 1];
    __shared__ uint32_t s_prefix, s_need;
    if (threadIdx.x == 0) {
        s_prefix = 0;
        s_need = R;
    }
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (uint32_t d = threadIdx.x; d < 256; d += BS) hist[d] = 0;
        __syncthreads();
        const uint32_t prefix = s_prefix;
        for (uint32_t i = threadIdx.x; i < n; i += BS) {
            const uint32_t u = score_word(score[i]);
            // the digits above this one agree with the prefix chosen so far
            if (shift == 24 || ((u ^ prefix) >> (shift + 8)) == 0)
                atomicAdd(&hist[(u >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t need = s_need, cum = 0, d = 255;
            for (;; --d) {
                if (cum + hist[d] >= need || d == 0) break;
                cum += hist[d];
            }
            s_prefix = prefix | (d << shift);
            s_need = need - cum;
        }
        __syncthreads();
    }
    const uint32_t t = s_prefix, need = s_need;
    uint32_t eq_seen = 0, taken = 0;
    for (uint32_t base = 0; base < n; base += BS) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t u = i < n ? score_word(score[i]) : 0u;
        const bool eq = i < n && u == t;
        uint32_t n_eq;
        const uint32_t eq_before = block_exclusive_scan<BS>(eq ? 1u : 0u, s_tmp, &n_eq);
        const bool take = (i < n && u > t) || (eq && eq_seen + eq_before < need);
        uint32_t n_take;
        const uint32_t pos = block_exclusive_scan<BS>(take ? 1u : 0u, s_tmp, &n_take);
        if (take) sel[2 + taken + pos] = i;
        eq_seen += n_eq;
        taken += n_take;
    }
    if (threadIdx.x == 0) {
        sel[0] = t;
        sel[1] = need;
    }
}

// Rank of selected candidate p among the R selected (better: larger word,
// or equal word and smaller index); seeds written in rank order.
__global__ void __launch_bounds__(256)
k_seed_rank(const float *__restrict__ score, const uint32_t *__restrict__ cx,
            const uint32_t *__restrict__ cy, uint32_t R, const uint32_t *__restrict__ sel,
            uint32_t *__restrict__ sx, uint32_t *__restrict__ sy)
{
    __shared__ uint32_t tw[256], ti[256];
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    const uint32_t me = p < R ? sel[2 + p] : 0u;
    const uint32_t mw = p < R ? score_word(score[me]) : 0u;
    uint32_t rank = 0;
    for (uint32_t b = 0; b < R; b += 256) {
        __syncthreads();
        if (b + threadIdx.x < R) {
            const uint32_t j = sel[2 + b + threadIdx.x];
            ti[threadIdx.x] = j;
            tw[threadIdx.x] = score_word(score[j]);
        }
        __syncthreads();
        const uint32_t lim = min(256u, R - b);
        if (p < R)
            for (uint32_t q = 0; q < lim; ++q)
                rank += (tw[q] > mw || (tw[q] == mw && ti[q] < me)) ? 1u : 0u;
    }
    if (p < R) {
        sx[rank] = cx[me];
        sy[rank] = cy[me];
    }
}

__global__ void __launch_bounds__(256)
k_max_index(const uint32_t *__restrict__ idx, uint64_t n, uint32_t *__restrict__ out)
{
    uint32_t mx = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256)
        mx = max(mx, idx[i]);
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, d, kWave));
    if (lane_id() == 0) atomicMax(out, mx);
}

}  // namespace

// ---------------------------------------------------------------- launchers

static uint32_t grid_of(uint64_t n, uint32_t cap = 2048)
{
    uint64_t g = (n + 255) / 256;
    if (g > cap) g = cap;
    return g ? (uint32_t)g : 1u;
}

size_t item_stats_words(uint32_t n, uint32_t Tp)
{
    return 6ull * n + 2ull * n + (Tp + 2) + 64;  // six u32 arrays, S2 (u64), hist
}

// ws: zeroed workspace of item_stats_words words.
hipError_t launch_item_features(const uint32_t *off, const uint32_t *items, uint32_t n,
                                uint32_t Tp, uint32_t *ws, float *feat, hipStream_t s)
{
    ItemStats st;
    st.A = ws;
    st.S1 = ws + n;
    st.LMAX = ws + 2 * n;
    st.H1 = ws + 3 * n;
    st.LONG = ws + 4 * n;
    st.SHORT = ws + 5 * n;
    uint32_t *p8 = ws + 6 * n + ((6 * n) & 1);  // 8-byte alignment
    st.S2 = reinterpret_cast<unsigned long long *>(p8);
    st.hist = p8 + 2 * n;
    if (Tp) hipLaunchKernelGGL(k_item_stats, dim3(grid_of(Tp)), dim3(256), 0, s, off, items, Tp, st);
    hipLaunchKernelGGL(k_count_hist, dim3(grid_of(n)), dim3(256), 0, s, st.A, n, st.hist);
    hipLaunchKernelGGL(k_suffix_sum, dim3(1), dim3(1024), 0, s, st.hist, Tp);
    if (feat) hipLaunchKernelGGL(k_features, dim3(grid_of(n)), dim3(256), 0, s, st, n, Tp, feat);
    return hipGetLastError();
}

hipError_t launch_top_pairs(const uint32_t *ws, uint32_t n, uint32_t Tp, uint32_t M,
                            uint32_t *top, uint32_t *cx, uint32_t *cy, hipStream_t s)
{
    const uint32_t *A = ws;
    const uint32_t *p8 = ws + 6 * n + ((6 * n) & 1);
    const uint32_t *hist = p8 + 2 * n;
    hipLaunchKernelGGL(k_top_items, dim3(1), dim3(1024), 0, s, A, n, hist, Tp, M, top);
    hipLaunchKernelGGL(k_pairs, dim3((M + 255) / 256), dim3(256), 0, s, top, M, cx, cy);
    return hipGetLastError();
}

hipError_t launch_lookup(const crop_ctx *c, const uint32_t *qx, const uint32_t *qy, uint64_t n,
                         uint32_t *out, hipStream_t s)
{
    if (!n) return hipSuccess;
    const uint64_t blocks = (n * kWave + 255) / 256;
    if (c->in.wide_keys)
        hipLaunchKernelGGL((k_lookup<uint64_t>), dim3((uint32_t)blocks), dim3(256), 0, s, qx, qy, n,
                           c->hp, bin_map(c->plan), c->plan.NB,
                           c->bin_off.as<uint32_t>(),
                           c->bin_size.as<uint32_t>(), c->keys.as<uint64_t>(),
                           c->out_cnt.as<uint32_t>(), out);
    else
        hipLaunchKernelGGL((k_lookup<uint32_t>), dim3((uint32_t)blocks), dim3(256), 0, s, qx, qy, n,
                           c->hp, bin_map(c->plan), c->plan.NB,
                           c->bin_off.as<uint32_t>(),
                           c->bin_size.as<uint32_t>(), c->keys.as<uint32_t>(),
                           c->out_cnt.as<uint32_t>(), out);
    return hipGetLastError();
}

hipError_t launch_pair_inputs(const float *feat, const uint32_t *cx, const uint32_t *cy,
                              const uint32_t *count, uint64_t n, float *Z, float *y,
                              hipStream_t s)
{
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_pair_inputs, dim3(grid_of(n * kIn, 4096)), dim3(256), 0, s, feat, cx, cy,
                       count, n, Z, y);
    return hipGetLastError();
}

hipError_t launch_mlp_train(float *params, float *m, float *v, float *gstage, const float *Z,
                            const float *y, const uint32_t *order, uint64_t n_order,
                            uint32_t batch, float lr, uint64_t t0, float *loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(kMlpBS), kMlpSmem, s, params, m, v, gstage, Z,
                       y, order, n_order, batch, lr, t0, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *params, const float *Z, const float *y, uint32_t N,
                           float *grad, float *loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(kMlpBS), kMlpSmem, s, params, Z, y, N, grad,
                       loss);
    return hipGetLastError();
}

hipError_t launch_mlp_score(const float *params, const float *Z, uint64_t N, float *out,
                            hipStream_t s)
{
    if (!N) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_score, dim3(grid_of(N, 1024)), dim3(256), 0, s, params, Z, N, out);
    return hipGetLastError();
}

hipError_t launch_select_seeds(const float *score, const uint32_t *cx, const uint32_t *cy,
                               uint32_t n, uint32_t R, uint32_t *sx, uint32_t *sy, uint32_t *sel,
                               hipStream_t s)
{
    if (!n || !R) return hipSuccess;
    hipLaunchKernelGGL(k_seed_threshold, dim3(1), dim3(1024), 0, s, score, n, R, sel);
    hipLaunchKernelGGL(k_seed_rank, dim3((R + 255) / 256), dim3(256), 0, s, score, cx, cy, R, sel,
                       sx, sy);
    return hipGetLastError();
}

// out: one word, zeroed by the caller; receives the largest index.
hipError_t launch_max_index(const uint32_t *idx, uint64_t n, uint32_t *out, hipStream_t s)
{
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_max_index, dim3(grid_of(n, 1024)), dim3(256), 0, s, idx, n, out);
    return hipGetLastError();
}

int mlp_param_count() { return kParams; }
int mlp_batch_max() { return kBatch; }
size_t mlp_smem_bytes() { return kMlpSmem; }

}  // namespace crop
