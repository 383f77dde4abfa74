// Batched exact runs: many independent transaction streams of uneven sizes
// in one pass of the hot path.  The streams are concatenated row-wise and
// planned together: every stream gets its own routing bins (consistent-hash
// partitions of its own pair space) and chunks that never cross a stream, so
// the whole batch is one count launch, one scan, one scatter and one
// persistent aggregation launch over all bins of all streams.  The launch
// sequence is captured once as a HIP graph and replayed.  An autotuner picks
// the terms aimed at per bin (how full the LDS tables get, hence the
// partition count of each stream) and the rows per chunk (how many
// wavefronts share one transaction chunk) by timing candidate plans on the
// loaded batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "api_util.hpp"
#include "crop_device.hpp"

using namespace crop;

namespace crop {

hipError_t launch_aggregate_counts(const crop_ctx *c, hipStream_t s);

namespace {

// Candidate plans of the autotuner.
constexpr uint32_t kTunerTermsPerBin[] = {15000, 30000, 60000};
constexpr uint32_t kTunerRows[] = {64, 128, 256};

// Process-wide cache of tuned plans, keyed by the batch's shape.
struct TuneKey {
    uint32_t n;
    uint64_t T, terms, nnz;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(n, T, terms, nnz) < std::tie(o.n, o.T, o.terms, o.nnz);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<uint32_t, uint32_t>> g_tuned;

void drop_graph(BatchState &b)
{
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
}

crop_status require_batch(crop_ctx *ctx)
{
    if (ctx->in.mode != Mode::Batch) return fail(ctx, CROP_E_STATE, "no batch loaded");
    return CROP_OK;
}

// The region route for the batch (packed keys, every transaction fitting a
// sub-batch): one segment per stream, with the stream's P bins (one per
// partition, the stream's own hash intervals) and its own sub-batches, which
// never cross a stream.  *done false: the chunk plan is taken instead.
crop_status plan_batch_regions(crop_ctx *ctx, uint32_t tpb, uint32_t NBmax, uint64_t NBtot,
                               bool *done)
{
    BatchState &b = ctx->batch;
    const Input &in = ctx->in;
    *done = false;
    if (in.wide_keys || in.total_terms >= (1ull << 32)) return CROP_OK;
    uint32_t S, I, R;
    if (!sb_caps(NBmax, 4, 0, &S, &I, &R)) return CROP_OK;
    const std::vector<uint64_t> cuts(b.tx_off.begin() + 1, b.tx_off.end());
    bool fits = false;
    crop_status st = plan_sb_rows(ctx, S, I, R, &fits, &cuts);
    if (st != CROP_OK || !fits) return st;
    SbPlan &sp = ctx->sb;
    const uint32_t n = b.n;
    sp.segs.assign(n, SbSeg{});
    std::vector<uint32_t> sub_seg(sp.n_sub), bin_seg(NBtot);
    uint64_t key0 = 0;
    uint32_t i = 0;  // sub-batches of the streams so far
    for (uint32_t st = 0; st < n; ++st) {
        SbSeg &g = sp.segs[st];
        g.bm = BinMap{b.P[st], 0, b.P[st], 0};
        g.NB = b.P[st];
        g.bin0 = b.bin_base[st];
        g.sub0 = i;
        while (i < sp.n_sub && sp.row[i] < b.tx_off[st + 1]) sub_seg[i++] = st;
        g.n_sub = i - g.sub0;
        g.key0 = (uint32_t)key0;
        key0 += b.terms[st];
        for (uint32_t k = 0; k < g.NB; ++k) bin_seg[g.bin0 + k] = st;
    }
    layout_sb_segments(sp);
    CK(ctx->sb_subseg.ensure(std::max<size_t>(sub_seg.size(), 1) * 4));
    CK(ctx->sb_binseg.ensure(std::max<size_t>(bin_seg.size(), 1) * 4));
    if (!sub_seg.empty())
        CK(hipMemcpy(ctx->sb_subseg.p, sub_seg.data(), sub_seg.size() * 4, hipMemcpyHostToDevice));
    if (!bin_seg.empty())
        CK(hipMemcpy(ctx->sb_binseg.p, bin_seg.data(), bin_seg.size() * 4, hipMemcpyHostToDevice));
    st = ensure_region_buffers(ctx);
    if (st != CROP_OK) return st;

    // the single-stream plan fields the shared launchers read
    RoutePlan &pl = ctx->plan;
    pl = RoutePlan{};
    pl.S = 1;
    pl.NB = (uint32_t)NBtot;
    pl.M = NBtot;
    pl.u0 = 0;
    pl.nu = (uint32_t)NBtot;
    pl.g = 0;
    pl.regions = true;
    pl.G = 1;
    pl.log2_slots = 14;
    pl.BS = 256;
    const uint64_t nt = in.total_terms;
    CK(ctx->bin_off.ensure(((size_t)NBtot + 1) * 4));
    CK(ctx->bin_size.ensure(std::max<size_t>(NBtot, 1) * 4));
    CK(ctx->bin_order.ensure(std::max<size_t>(NBtot, 1) * 4));
    CK(ctx->keys.ensure(std::max<uint64_t>(nt, 1) * 4));
    CK(ctx->out_cnt.ensure(std::max<uint64_t>(nt, 1) * 4));
    CK(ctx->spill.ensure(std::max<uint64_t>(nt, 1) * spill_entry_bytes(false, false)));
    CK(ctx->counter.ensure(64));
    b.regions = true;
    b.terms_per_bin = tpb;
    b.rows_per_chunk = 0;
    b.planned = true;
    *done = true;
    return CROP_OK;
}

// Plan the batch for (terms per bin, rows per chunk) and size the buffers:
// the region route when it applies (rows per chunk unused), else one count
// row per chunk of R transactions.
crop_status plan_batch(crop_ctx *ctx, uint32_t tpb, uint32_t R)
{
    BatchState &b = ctx->batch;
    const Input &in = ctx->in;
    drop_graph(b);
    b.planned = false;
    const uint32_t n = b.n;
    b.P.assign(n, 1);
    b.bin_base.assign(n, 0);
    b.chunk0.assign(n, 0);
    b.n_chunks.assign(n, 0);
    b.cnt_base.assign(n, 0);
    uint32_t NBmax = 1;
    uint64_t NBtot = 0;
    for (uint32_t s = 0; s < n; ++s) {
        const uint64_t want = (b.terms[s] + tpb - 1) / tpb;
        b.P[s] = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(want, 1), kMaxP);
        b.bin_base[s] = (uint32_t)NBtot;
        NBtot += b.P[s];
        NBmax = std::max(NBmax, b.P[s]);
    }
    if (NBtot >= (1ull << 31)) return fail(ctx, CROP_E_UNSUPPORTED, "too many routing bins");
    b.regions = false;
    bool done = false;
    const crop_status rst = plan_batch_regions(ctx, tpb, NBmax, NBtot, &done);
    if (rst != CROP_OK || done) return rst;
    // rows per chunk: halve until the largest chunk stages in LDS
    const size_t hist_bytes = (size_t)NBmax * 4;
    auto max_items_for = [&](uint32_t r) {
        uint32_t mx = 0;
        for (uint32_t s = 0; s < n; ++s)
            for (uint64_t t0 = b.tx_off[s]; t0 < b.tx_off[s + 1]; t0 += r) {
                const uint64_t t1 = std::min<uint64_t>(b.tx_off[s + 1], t0 + r);
                mx = std::max(mx, in.h_off[t1] - in.h_off[t0]);
            }
        return mx;
    };
    uint32_t mi = max_items_for(R);
    while (R > 1 && hist_bytes + 12ull * mi > kLdsBudget) {
        R /= 2;
        mi = max_items_for(R);
    }
    if (hist_bytes + 12ull * mi + 1024 > 150 * 1024)
        return fail(ctx, CROP_E_UNSUPPORTED, "a transaction is too long to stage in LDS");
    std::vector<uint32_t> crow, cstream;
    uint64_t cnt_words = 0;
    for (uint32_t s = 0; s < n; ++s) {
        b.chunk0[s] = (uint32_t)crow.size();
        for (uint64_t t0 = b.tx_off[s]; t0 < b.tx_off[s + 1]; t0 += R) {
            crow.push_back((uint32_t)t0);
            cstream.push_back(s);
        }
        b.n_chunks[s] = (uint32_t)crow.size() - b.chunk0[s];
        b.cnt_base[s] = cnt_words;
        cnt_words += (uint64_t)b.n_chunks[s] * b.P[s];
    }
    crow.push_back((uint32_t)in.T);
    const uint32_t n_chunks = (uint32_t)cstream.size();
    std::vector<BatchStreamDev> sd(n);
    std::vector<uint32_t> bin_stream(NBtot);
    for (uint32_t s = 0; s < n; ++s) {
        sd[s] = BatchStreamDev{b.P[s], b.bin_base[s], b.chunk0[s], b.n_chunks[s], b.cnt_base[s]};
        for (uint32_t k = 0; k < b.P[s]; ++k) bin_stream[b.bin_base[s] + k] = s;
    }
    const uint32_t stage_cap = 0;  // direct scatter writes (as for single streams)
    if (tx_scatter_smem_bytes(NBmax, mi, 0, in.wide_keys) > kStageBudget ||
        !tx_launch_layouts_ok(NBmax, mi, stage_cap, in.wide_keys))
        return fail(ctx, CROP_E_UNSUPPORTED, "routing bins and chunk do not fit in LDS");
    CK(b.d_crow.ensure(crow.size() * 4));
    CK(b.d_cstream.ensure(std::max<size_t>(cstream.size(), 1) * 4));
    CK(b.d_streams.ensure(std::max<size_t>(n, 1) * sizeof(BatchStreamDev)));
    CK(b.d_bin_stream.ensure(std::max<size_t>(NBtot, 1) * 4));
    CK(b.tot.ensure(std::max<size_t>(NBtot, 1) * 4));
    CK(b.tiles.ensure((size_t)batch_scan_tiles((uint32_t)NBtot) * 4 + 4));
    CK(hipMemcpy(b.d_crow.p, crow.data(), crow.size() * 4, hipMemcpyHostToDevice));
    if (n_chunks)
        CK(hipMemcpy(b.d_cstream.p, cstream.data(), cstream.size() * 4, hipMemcpyHostToDevice));
    if (n) CK(hipMemcpy(b.d_streams.p, sd.data(), n * sizeof(BatchStreamDev), hipMemcpyHostToDevice));
    if (NBtot)
        CK(hipMemcpy(b.d_bin_stream.p, bin_stream.data(), NBtot * 4, hipMemcpyHostToDevice));

    BatchDev &d = b.dev;
    d.crow = b.d_crow.as<uint32_t>();
    d.cstream = b.d_cstream.as<uint32_t>();
    d.streams = b.d_streams.as<BatchStreamDev>();
    d.bin_stream = b.d_bin_stream.as<uint32_t>();
    d.n_chunks = n_chunks;
    d.n_streams = n;
    d.NBtot = (uint32_t)NBtot;
    d.NBmax = NBmax;
    d.max_items = mi;
    d.stage_cap = stage_cap;
    b.cnt_words = cnt_words;
    b.terms_per_bin = tpb;
    b.rows_per_chunk = R;

    // the single-stream plan fields the shared launchers read
    RoutePlan &pl = ctx->plan;
    pl = RoutePlan{};
    pl.S = 1;
    pl.NB = (uint32_t)NBtot;
    pl.M = NBtot;
    pl.u0 = 0;
    pl.nu = (uint32_t)NBtot;
    pl.g = 0;
    pl.n_chunks = n_chunks;
    pl.R = R;
    pl.max_items = mi;
    pl.stage_cap = stage_cap;
    pl.G = 1;
    pl.log2_slots = in.wide_keys ? 13 : 14;
    pl.BS = 256;

    const uint64_t nt = in.total_terms;
    const size_t kb = in.wide_keys ? 8 : 4;
    CK(ctx->cnt_mat.ensure(std::max<uint64_t>(cnt_words, 1) * 4));
    CK(ctx->bin_off.ensure(((size_t)NBtot + 1) * 4));
    CK(ctx->bin_size.ensure(std::max<size_t>(NBtot, 1) * 4));
    CK(ctx->bin_order.ensure(std::max<size_t>(NBtot, 1) * 4));
    CK(ctx->keys.ensure(std::max<uint64_t>(nt, 1) * kb));
    CK(ctx->out_cnt.ensure(std::max<uint64_t>(nt, 1) * 4));
    CK(ctx->spill.ensure(std::max<uint64_t>(nt, 1) * spill_entry_bytes(in.wide_keys, false)));
    CK(ctx->counter.ensure(64));
    b.planned = true;
    return CROP_OK;
}

// The kernels of one batched run, in order, on stream s.
crop_status enqueue_batch(crop_ctx *ctx, hipStream_t s, bool stages)
{
    const BatchState &b = ctx->batch;
    const Input &in = ctx->in;
    uint32_t *bin_off = ctx->bin_off.as<uint32_t>();
    if (b.regions) {
        if (ctx->sb.n_sub) CK(launch_sb_route(ctx, s));
        if (stages) STAGE("route");
        CK(launch_sb_headers(ctx, s));
        // one ordered range of bins and one bin counter (cleared) per XCD
        CK(launch_bin_order(ctx->plan.NB, bin_off, ctx->bin_order.as<uint32_t>(), s, kNumXcd,
                            ctx->counter.as<uint32_t>(), kNumXcd));
        if (stages) STAGE("headers");
        CK(launch_aggregate_regions(ctx, s));
        if (stages) STAGE("aggregate");
        return CROP_OK;
    }
    uint32_t *cnt = ctx->cnt_mat.as<uint32_t>();
    CK(launch_batch_count(in.off, in.items, ctx->hp, b.dev, cnt, bin_off, s));
    if (stages) STAGE("count");
    CK(launch_batch_scan(b.dev, cnt, b.tot.as<uint32_t>(), b.tiles.as<uint32_t>(), bin_off,
                         ctx->counter.as<uint32_t>(), s));
    CK(launch_bin_order(b.dev.NBtot, bin_off, ctx->bin_order.as<uint32_t>(), s));
    if (stages) STAGE("scan");
    CK(launch_batch_scatter(in.off, in.items, ctx->hp, b.dev, cnt, bin_off, ctx->keys.p,
                            in.wide_keys, s));
    if (stages) STAGE("scatter");
    CK(launch_aggregate_counts(ctx, s));
    if (stages) STAGE("aggregate");
    return CROP_OK;
}

// One timed eager run (for the tuner); returns milliseconds.
crop_status timed_eager_run(crop_ctx *ctx, float *ms)
{
    CK(hipEventRecord(ctx->ev0, ctx->stream));
    crop_status st = enqueue_batch(ctx, ctx->stream, false);
    if (st != CROP_OK) return st;
    CK(hipEventRecord(ctx->ev1, ctx->stream));
    CK(hipEventSynchronize(ctx->ev1));
    CK(hipEventElapsedTime(ms, ctx->ev0, ctx->ev1));
    return CROP_OK;
}

}  // namespace

// The captured graph holds the kernels' arguments by value (the hash
// parameters among them): a change of any of them must capture again.
void batch_invalidate_graph(crop_ctx *ctx) { drop_graph(ctx->batch); }

void reset_batch(crop_ctx *ctx)
{
    BatchState &b = ctx->batch;
    drop_graph(b);
    b.planned = false;
    b.n = 0;
    b.tx_off.clear();
    b.n_items.clear();
    b.terms.clear();
}

}  // namespace crop

extern "C" {

crop_status crop_load_batch(crop_ctx *ctx, uint32_t n_streams, const uint64_t *tx_off,
                            const uint32_t *off, const uint32_t *items, const uint32_t *n_items,
                            crop_mem where, crop_own own)
{
    if (!ctx) return CROP_E_ARG;
    if (!tx_off || !off || !n_items) return fail(ctx, CROP_E_ARG, "null input pointer");
    if (own == CROP_OWN_BORROW && where != CROP_MEM_DEVICE)
        return fail(ctx, CROP_E_ARG, "only device buffers can be borrowed");
    const uint64_t T = tx_off[n_streams];
    if (tx_off[0] != 0) return fail(ctx, CROP_E_ARG, "tx_off[0] must be 0");
    for (uint32_t s = 0; s < n_streams; ++s)
        if (tx_off[s + 1] < tx_off[s]) {
            ctx->err_index = s;
            return fail(ctx, CROP_E_ARG, "stream boundaries decrease at stream " + std::to_string(s));
        }
    if (T >= (1ull << 32)) return fail(ctx, CROP_E_UNSUPPORTED, "more than 2^32 - 1 transactions");
    DeviceGuard g(ctx->device);
    reset_input(ctx);
    ctx->err_index = -1;
    Input &in = ctx->in;
    BatchState &b = ctx->batch;
    CK(fetch(in.h_off, off, T + 1, where));
    const uint64_t nnz = in.h_off.empty() ? 0 : in.h_off.back();
    if (nnz >= (1ull << 32)) return fail(ctx, CROP_E_UNSUPPORTED, "nnz must be below 2^32");
    if (nnz && !items) return fail(ctx, CROP_E_ARG, "null input pointer");
    crop_status st = check_offsets(ctx, in.h_off, nnz, "transactions");
    if (st != CROP_OK) return st;
    b.n = n_streams;
    b.tx_off.assign(tx_off, tx_off + n_streams + 1);
    b.n_items.assign(n_items, n_items + n_streams);
    b.terms.assign(n_streams, 0);
    uint64_t total = 0;
    bool wide = false;
    for (uint32_t s = 0; s < n_streams; ++s) {
        for (uint64_t t = tx_off[s]; t < tx_off[s + 1]; ++t) {
            const uint64_t L = in.h_off[t + 1] - in.h_off[t];
            b.terms[s] += L * (L ? L - 1 : 0) / 2;
        }
        total += b.terms[s];
        wide = wide || n_items[s] > 65536u;
    }
    if (total >= (1ull << 32))
        return fail(ctx, CROP_E_UNSUPPORTED, "more than 2^32 - 1 terms in one batch");
    in.total_terms = total;
    CK(place(off, T + 1, where, own, in.own[0], &in.off, ctx->stream));
    CK(place(items, nnz, where, own, in.own[1], &in.items, ctx->stream));
    for (uint32_t s = 0; s < n_streams; ++s) {
        int64_t bad = -1;
        const uint64_t Ts = tx_off[s + 1] - tx_off[s];
        st = validate_on_device(ctx, in.off + tx_off[s], Ts, in.items, nnz, n_items[s], &bad);
        if (st != CROP_OK) return st;
        if (bad >= 0) {
            ctx->err_index = (int64_t)tx_off[s] + bad;
            return fail(ctx, CROP_E_INPUT,
                        "stream " + std::to_string(s) + ", transaction " + std::to_string(bad) +
                            ": item id out of range or items not strictly increasing");
        }
    }
    in.T = T;
    in.nnz = nnz;
    in.n_items = 0;
    in.wide_keys = wide;
    in.mode = Mode::Batch;
    // a plan tuned earlier for a batch of this shape is reused
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(TuneKey{n_streams, T, total, nnz});
    b.terms_per_bin = it != g_tuned.end() ? it->second.first : (uint32_t)kTermsPerBin;
    b.rows_per_chunk = it != g_tuned.end() ? it->second.second : 128u;
    return CROP_OK;
}

crop_status crop_batch_set_graph(crop_ctx *ctx, int enable)
{
    if (!ctx) return CROP_E_ARG;
    ctx->batch.use_graph = enable != 0;
    drop_graph(ctx->batch);
    return CROP_OK;
}

crop_status crop_batch_autotune(crop_ctx *ctx, uint32_t reps, uint32_t *terms_per_bin,
                                uint32_t *rows_per_chunk, float *best_ms)
{
    if (!ctx) return CROP_E_ARG;
    crop_status st = require_batch(ctx);
    if (st != CROP_OK) return st;
    DeviceGuard g(ctx->device);
    ctx->result = Result::None;
    reps = std::max<uint32_t>(reps, 1);
    float best = -1.0f;
    uint32_t bt = 0, br = 0;
    for (uint32_t tpb : kTunerTermsPerBin)
        for (uint32_t R : kTunerRows) {
            st = plan_batch(ctx, tpb, R);
            if (st != CROP_OK) continue;  // a candidate that does not fit is skipped
            // the region route has no rows per chunk: one candidate per tpb
            if (ctx->batch.regions && R != kTunerRows[0]) continue;
            float ms = 0.0f;
            st = timed_eager_run(ctx, &ms);  // warm-up
            if (st != CROP_OK) return st;
            float lo = -1.0f;
            for (uint32_t k = 0; k < reps; ++k) {
                st = timed_eager_run(ctx, &ms);
                if (st != CROP_OK) return st;
                if (lo < 0 || ms < lo) lo = ms;
            }
            if (best < 0 || lo < best) {
                best = lo;
                bt = tpb;
                br = R;
            }
        }
    if (best < 0) return fail(ctx, CROP_E_UNSUPPORTED, "no candidate plan fits this batch");
    st = plan_batch(ctx, bt, br);
    if (st != CROP_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const Input &in = ctx->in;
        g_tuned[TuneKey{ctx->batch.n, in.T, in.total_terms, in.nnz}] = {bt, br};
    }
    if (terms_per_bin) *terms_per_bin = bt;
    if (rows_per_chunk) *rows_per_chunk = ctx->batch.rows_per_chunk;
    if (best_ms) *best_ms = best;
    return CROP_OK;
}

crop_status crop_batch_set_plan(crop_ctx *ctx, uint32_t terms_per_bin, uint32_t rows_per_chunk)
{
    if (!ctx) return CROP_E_ARG;
    crop_status st = require_batch(ctx);
    if (st != CROP_OK) return st;
    if (terms_per_bin == 0 || rows_per_chunk == 0)
        return fail(ctx, CROP_E_ARG, "terms_per_bin and rows_per_chunk must be positive");
    DeviceGuard g(ctx->device);
    ctx->result = Result::None;
    return plan_batch(ctx, terms_per_bin, rows_per_chunk);
}

crop_status crop_run_exact_batched(crop_ctx *ctx)
{
    if (!ctx) return CROP_E_ARG;
    crop_status st = require_batch(ctx);
    if (st != CROP_OK) return st;
    DeviceGuard g(ctx->device);
    BatchState &b = ctx->batch;
    ctx->result = Result::None;
    if (!b.planned) {
        st = plan_batch(ctx, b.terms_per_bin ? b.terms_per_bin : (uint32_t)kTermsPerBin,
                        b.rows_per_chunk ? b.rows_per_chunk : 128u);
        if (st != CROP_OK) return st;
    }
    if (b.use_graph && !b.exec) {
        // capture on the context's own stream (the null stream cannot capture)
        hipStream_t cs = ctx->own_stream;
        CK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        st = enqueue_batch(ctx, cs, false);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        if (st != CROP_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        CK(e);
        b.graph = graph;
        CK(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    }
    st = run_begin(ctx);
    if (st != CROP_OK) return st;
    if (b.use_graph) {
        CK(hipGraphLaunch(b.exec, ctx->stream));
        STAGE("graph");
    } else {
        st = enqueue_batch(ctx, ctx->stream, true);
        if (st != CROP_OK) return st;
    }
    st = run_end(ctx);
    if (st != CROP_OK) return st;
    ctx->result = Result::BatchExact;
    return CROP_OK;
}

crop_status crop_batch_info(crop_ctx *ctx, uint32_t stream, uint32_t *partitions,
                            uint64_t *terms, uint64_t *first_tx, uint64_t *n_tx)
{
    if (!ctx) return CROP_E_ARG;
    crop_status st = require_batch(ctx);
    if (st != CROP_OK) return st;
    const BatchState &b = ctx->batch;
    if (stream >= b.n) return fail(ctx, CROP_E_ARG, "stream index out of range");
    if (partitions) *partitions = b.planned ? b.P[stream] : 0;
    if (terms) *terms = b.terms[stream];
    if (first_tx) *first_tx = b.tx_off[stream];
    if (n_tx) *n_tx = b.tx_off[stream + 1] - b.tx_off[stream];
    return CROP_OK;
}

crop_status crop_batch_result_sizes(crop_ctx *ctx, uint32_t stream, uint64_t *sizes,
                                    uint64_t *terms_per_partition)
{
    if (!ctx) return CROP_E_ARG;
    if (ctx->result != Result::BatchExact)
        return fail(ctx, CROP_E_STATE, "no batched result: call crop_run_exact_batched first");
    const BatchState &b = ctx->batch;
    if (stream >= b.n) return fail(ctx, CROP_E_ARG, "stream index out of range");
    DeviceGuard g(ctx->device);
    const uint32_t P = b.P[stream], b0 = b.bin_base[stream];
    std::vector<uint32_t> bs(P), bo(P + 1);
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(bs.data(), ctx->bin_size.as<uint32_t>() + b0, P * 4, hipMemcpyDeviceToHost));
    CK(hipMemcpy(bo.data(), ctx->bin_off.as<uint32_t>() + b0, (P + 1) * 4, hipMemcpyDeviceToHost));
    for (uint32_t p = 0; p < P; ++p) {
        if (sizes) sizes[p] = bs[p];
        if (terms_per_partition) terms_per_partition[p] = bo[p + 1] - bo[p];
    }
    return CROP_OK;
}

crop_status crop_batch_read_stream(crop_ctx *ctx, uint32_t stream, crop_mem where, uint32_t *i,
                                   uint32_t *j, uint32_t *count, uint64_t cap, uint64_t *written,
                                   uint64_t *part_off)
{
    if (!ctx || !i || !j) return CROP_E_ARG;
    if (ctx->result != Result::BatchExact)
        return fail(ctx, CROP_E_STATE, "no batched result: call crop_run_exact_batched first");
    const BatchState &b = ctx->batch;
    if (stream >= b.n) return fail(ctx, CROP_E_ARG, "stream index out of range");
    DeviceGuard g(ctx->device);
    const uint32_t P = b.P[stream], b0 = b.bin_base[stream];
    std::vector<uint32_t> bs(P), dst(P);
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(bs.data(), ctx->bin_size.as<uint32_t>() + b0, P * 4, hipMemcpyDeviceToHost));
    uint64_t tot = 0;
    for (uint32_t p = 0; p < P; ++p) {
        dst[p] = (uint32_t)tot;
        if (part_off) part_off[p] = tot;
        tot += bs[p];
    }
    if (part_off) part_off[P] = tot;
    if (written) *written = tot;
    if (tot > cap) return fail(ctx, CROP_E_CAPACITY, "output capacity below the entry count");
    const size_t n = std::max<uint64_t>(tot, 1);
    const size_t head = ((size_t)P * 4 + 255) / 256 * 256;
    CK(ctx->scratch.ensure(head + (where == CROP_MEM_HOST ? 12 * n : 0)));
    uint32_t *d_dst = ctx->scratch.as<uint32_t>();
    CK(hipMemcpyAsync(d_dst, dst.data(), P * 4, hipMemcpyHostToDevice, ctx->stream));
    uint32_t *oi = i, *oj = j, *oc = count;
    if (where == CROP_MEM_HOST) {
        oi = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(d_dst) + head);
        oj = oi + n;
        oc = count ? oj + n : nullptr;
    }
    CK(launch_gather_result(ctx, b0, P, d_dst, oi, oj, oc, nullptr, ctx->stream));
    if (where == CROP_MEM_HOST) {
        CK(hipMemcpyAsync(i, oi, tot * 4, hipMemcpyDeviceToHost, ctx->stream));
        CK(hipMemcpyAsync(j, oj, tot * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (count) CK(hipMemcpyAsync(count, oc, tot * 4, hipMemcpyDeviceToHost, ctx->stream));
    }
    CK(hipStreamSynchronize(ctx->stream));
    return CROP_OK;
}

}  // extern "C"
