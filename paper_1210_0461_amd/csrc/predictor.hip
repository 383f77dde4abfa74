// The learned heavy-pair predictor as one object (an addition; the paper has
// no learned component).  Its failure model is the paper's: a heavy entry is
// lost when too many heavy entries or too much light weight share its
// Space-Saving bucket (Section 6, proof of Theorem 2), so pairs predicted
// heavy are pinned into their buckets before the stream.
//
// Training, per training stream: an exact run (Section 7 supports) gives the
// labels, the stream's prefix gives 16 features per item and the candidate
// pairs (all pairs of its M most frequent prefix items); then the
// 32 -> 64 -> 64 -> 1 network is trained with Adam on log1p(support).
// Scoring a loaded stream: the same features and candidates, bf16 scores and
// the R best candidates as seeds for crop_run_topk_seeded.  Every step is one
// of the library's kernels; this file only orders them, on a private context
// so the caller's loaded input and results stay as they were.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "api_util.hpp"

using namespace crop;

struct crop_predictor {
    int device = 0;
    crop_mlp *mlp = nullptr;
    uint32_t top_items = 0;  // M of the candidates
    float last_loss = 0.0f;
};

namespace {

constexpr uint32_t kFeat = 16;

// Transactions of the prefix the features come from: ceil(T / 20).
uint32_t prefix_len(uint64_t T) { return T == 0 ? 0 : (uint32_t)std::max<uint64_t>(1, (T + 19) / 20); }

uint64_t splitmix_next(uint64_t &s)
{
    s += 0x9e3779b97f4a7c15ULL;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// Uniform in [0, n) from a SplitMix64 word (Lemire's multiply-shift range
// reduction; the bias is below n / 2^64).
uint32_t below(uint64_t &s, uint32_t n)
{
    return (uint32_t)(((unsigned __int128)splitmix_next(s) * n) >> 64);
}

// He-uniform initial weights, +-sqrt(6 / fan_in), biases zero, in the
// library's parameter order W1[64][32], b1, W2[64][64], b2, w3[64], b3.
std::vector<float> default_init(uint64_t seed)
{
    std::vector<float> w;
    w.reserve(6337);
    uint64_t s = seed;
    auto uni = [&](size_t n, double fan_in) {
        const double lim = std::sqrt(6.0 / fan_in);
        for (size_t k = 0; k < n; ++k) {
            const double u = (double)(splitmix_next(s) >> 11) * (1.0 / 9007199254740992.0);
            w.push_back((float)((2.0 * u - 1.0) * lim));
        }
    };
    auto zeros = [&](size_t n) { w.insert(w.end(), n, 0.0f); };
    uni(64 * 32, 32);
    zeros(64);
    uni(64 * 64, 64);
    zeros(64);
    uni(64, 64);
    zeros(1);
    return w;
}

// Features and candidates of the stream loaded in c, and the network inputs
// of the candidates unless Z is null.
crop_status candidate_inputs(crop_ctx *c, uint32_t M, DevBuf &feat, DevBuf &cx, DevBuf &cy,
                             DevBuf *Z, uint64_t *n_pairs)
{
    const uint32_t Tp = prefix_len(c->in.T);
    const uint64_t np = (uint64_t)M * (M - 1) / 2;
    crop_status st;
    hipError_t e = feat.ensure((size_t)c->in.n_items * kFeat * 4);
    if (e == hipSuccess) e = cx.ensure(np * 4);
    if (e == hipSuccess) e = cy.ensure(np * 4);
    if (e == hipSuccess && Z) e = Z->ensure(np * 2 * kFeat * 4);
    if (e != hipSuccess) return hip_fail(c, e, "predictor buffers");
    st = crop_item_features(c, Tp, feat.as<float>());
    if (st != CROP_OK) return st;
    st = crop_top_item_pairs(c, Tp, M, cx.as<uint32_t>(), cy.as<uint32_t>(), np, n_pairs);
    if (st != CROP_OK || !Z) return st;
    return crop_pair_inputs(c, feat.as<float>(), cx.as<uint32_t>(), cy.as<uint32_t>(), nullptr,
                            np, Z->as<float>(), nullptr);
}

// Copies the status and message of a failure on the private context to the
// caller's.
crop_status relay(crop_ctx *ctx, crop_ctx *priv, crop_status st)
{
    if (st != CROP_OK) {
        ctx->err = std::string("predictor: ") + crop_last_error_detail(priv);
        ctx->err_index = crop_last_error_index(priv);
    }
    return st;
}

}  // namespace

extern "C" {

crop_status crop_predictor_train(crop_ctx *ctx, const crop_train_set *set,
                                 const crop_train_opts *opts, crop_predictor **out)
{
    if (!ctx || !set || !opts || !out || (set->n_streams && !set->streams)) return CROP_E_ARG;
    *out = nullptr;
    if (set->n_streams == 0) return fail(ctx, CROP_E_ARG, "no training streams");
    const uint32_t M = opts->top_items ? opts->top_items : 256;
    const uint32_t epochs = opts->epochs ? opts->epochs : 4;
    const uint32_t batch = opts->batch ? opts->batch : 128;
    const float lr = opts->lr > 0.0f ? opts->lr : 1e-3f;
    if (M < 2) return fail(ctx, CROP_E_ARG, "top_items must be at least 2");
    if (batch > (uint32_t)mlp_batch_max()) return fail(ctx, CROP_E_ARG, "batch above 128");
    DeviceGuard g(ctx->device);
    CK(hipStreamSynchronize(ctx->stream));

    crop_ctx *priv = nullptr;
    crop_status st = crop_create(&priv, ctx->device);
    if (st != CROP_OK) return fail(ctx, st, "predictor: cannot create a working context");
    crop_predictor *pred = new (std::nothrow) crop_predictor();
    DevBuf feat, cx, cy, sup, order, Zall, yall;
    auto cleanup = [&]() {
        for (DevBuf *b : {&feat, &cx, &cy, &sup, &order, &Zall, &yall}) b->release();
        crop_destroy(priv);
    };
    if (!pred) {
        cleanup();
        return CROP_E_NOMEM;
    }
    pred->device = ctx->device;
    pred->top_items = M;
    st = crop_set_seed(priv, ctx->seed);
    if (st == CROP_OK) st = crop_set_partitions(priv, ctx->P);
    const uint64_t np = (uint64_t)M * (M - 1) / 2;
    const uint64_t n_samples = np * set->n_streams;
    hipError_t e = Zall.ensure(n_samples * 2 * kFeat * 4);
    if (e == hipSuccess) e = yall.ensure(n_samples * 4);
    if (e == hipSuccess) e = sup.ensure(np * 4);
    if (e != hipSuccess) st = hip_fail(ctx, e, "predictor training buffers");
    for (uint32_t k = 0; st == CROP_OK && k < set->n_streams; ++k) {
        const crop_stream_ref &r = set->streams[k];
        st = crop_load_transactions(priv, r.off, r.T, r.items, r.nnz, r.n_items, set->where,
                                    set->where == CROP_MEM_DEVICE ? CROP_OWN_BORROW
                                                                  : CROP_OWN_COPY);
        if (st == CROP_OK && M > r.n_items) st = fail(priv, CROP_E_ARG, "top_items above n_items");
        if (st == CROP_OK) st = crop_run_exact(priv);
        uint64_t got = 0;
        if (st == CROP_OK) st = candidate_inputs(priv, M, feat, cx, cy, nullptr, &got);
        if (st == CROP_OK)
            st = crop_lookup_exact(priv, cx.as<uint32_t>(), cy.as<uint32_t>(), np,
                                   sup.as<uint32_t>());
        // labels y = log1p(support), inputs written into this stream's block
        if (st == CROP_OK)
            st = crop_pair_inputs(priv, feat.as<float>(), cx.as<uint32_t>(), cy.as<uint32_t>(),
                                  sup.as<uint32_t>(), np, Zall.as<float>() + k * np * 2 * kFeat,
                                  yall.as<float>() + k * np);
        if (st == CROP_OK) {
            e = hipStreamSynchronize(priv->stream);
            if (e != hipSuccess) st = hip_fail(priv, e, "label stream");
        }
        if (st != CROP_OK) st = relay(ctx, priv, st);
    }
    if (st == CROP_OK) {
        std::vector<float> init;
        if (opts->init)
            init.assign(opts->init, opts->init + mlp_param_count());
        else
            init = default_init(opts->shuffle_seed ^ 0x5851F42D4C957F2DULL);
        st = crop_mlp_create(priv, init.data(), &pred->mlp);
        if (st != CROP_OK) st = relay(ctx, priv, st);
    }
    if (st == CROP_OK) {
        // one Fisher-Yates permutation of the samples per epoch (SplitMix64)
        std::vector<uint32_t> ord(n_samples * epochs);
        uint64_t s = opts->shuffle_seed;
        for (uint32_t ep = 0; ep < epochs; ++ep) {
            uint32_t *p = ord.data() + (size_t)ep * n_samples;
            for (uint64_t i = 0; i < n_samples; ++i) p[i] = (uint32_t)i;
            for (uint64_t i = n_samples - 1; i > 0; --i)
                std::swap(p[i], p[below(s, (uint32_t)(i + 1))]);
        }
        e = order.ensure(ord.size() * 4);
        if (e == hipSuccess)
            e = hipMemcpy(order.p, ord.data(), ord.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) st = hip_fail(ctx, e, "predictor sample order");
    }
    if (st == CROP_OK) {
        st = crop_mlp_train(priv, pred->mlp, Zall.as<float>(), yall.as<float>(), n_samples,
                            order.as<uint32_t>(), (uint64_t)n_samples * epochs, batch, lr);
        if (st == CROP_OK) st = crop_mlp_loss(priv, pred->mlp, &pred->last_loss);
        if (st != CROP_OK) st = relay(ctx, priv, st);
    }
    cleanup();
    if (st != CROP_OK) {
        crop_predictor_free(pred);
        return st;
    }
    *out = pred;
    return CROP_OK;
}

crop_status crop_predictor_score(crop_ctx *ctx, const crop_predictor *pred, uint32_t R,
                                 uint32_t *sx, uint32_t *sy, uint64_t *n_seeds)
{
    if (!ctx || !pred || !sx || !sy) return CROP_E_ARG;
    if (ctx->in.mode != Mode::Tx) return fail(ctx, CROP_E_STATE, "no transaction stream loaded");
    if (pred->device != ctx->device) return fail(ctx, CROP_E_ARG, "predictor on another GPU");
    const uint32_t M = pred->top_items;
    if (M > ctx->in.n_items) return fail(ctx, CROP_E_ARG, "stream has fewer items than top_items");
    DeviceGuard g(ctx->device);
    const uint64_t np = (uint64_t)M * (M - 1) / 2;
    const uint32_t take = (uint32_t)std::min<uint64_t>(R, np);
    if (n_seeds) *n_seeds = take;
    DevBuf feat, cx, cy, Z, score;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(ctx->stream);
        for (DevBuf *b : {&feat, &cx, &cy, &Z, &score}) b->release();
    };
    uint64_t got = 0;
    crop_status st = candidate_inputs(ctx, M, feat, cx, cy, &Z, &got);
    if (st == CROP_OK) {
        hipError_t e = score.ensure(np * 4);
        if (e != hipSuccess) st = hip_fail(ctx, e, "predictor scores");
    }
    if (st == CROP_OK) st = crop_mlp_score(ctx, pred->mlp, Z.as<float>(), np, score.as<float>());
    if (st == CROP_OK && take)
        st = crop_select_seeds(ctx, score.as<float>(), cx.as<uint32_t>(), cy.as<uint32_t>(), np,
                               take, sx, sy);
    cleanup();
    return st;
}

crop_status crop_predictor_params(crop_ctx *ctx, const crop_predictor *pred, float *out,
                                  float *last_loss)
{
    if (!ctx || !pred || !out) return CROP_E_ARG;
    if (last_loss) *last_loss = pred->last_loss;
    return crop_mlp_params(ctx, pred->mlp, out);
}

void crop_predictor_free(crop_predictor *pred)
{
    if (!pred) return;
    crop_mlp_destroy(pred->mlp);
    delete pred;
}

}  // extern "C"
