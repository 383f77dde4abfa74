// C ABI of the CRoP library (declared in include/crop.h): context, inputs,
// planning, run orchestration and readback.  Every step of a run is a HIP
// kernel on the context's stream; the host only plans and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "api_util.hpp"
#include "crop_device.hpp"
#include "crop_layout.hpp"

using namespace crop;

namespace crop {

crop_status fail(crop_ctx *c, crop_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

crop_status hip_fail(crop_ctx *c, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? CROP_E_NOMEM : CROP_E_HIP, m);
}

uint64_t tx_terms_of(const std::vector<uint32_t> &off)
{
    uint64_t s = 0;
    for (size_t t = 0; t + 1 < off.size(); ++t) {
        uint64_t L = off[t + 1] - off[t];
        s += L * (L ? L - 1 : 0) / 2;
    }
    return s;
}

// Validate CSR contents on the device; returns the first bad vector or -1.
crop_status validate_on_device(crop_ctx *ctx, const uint32_t *v_off, uint64_t K,
                               const uint32_t *idx, uint64_t nnz, uint32_t n, int64_t *bad_out)
{
    CK(ctx->scratch.ensure(64));
    auto *bad = ctx->scratch.as<unsigned long long>();
    unsigned long long init = ~0ull;
    CK(hipMemcpyAsync(bad, &init, sizeof(init), hipMemcpyHostToDevice, ctx->stream));
    if (K) CK(launch_validate_tx(v_off, K, idx, nnz, n, bad, ctx->stream));
    unsigned long long got = 0;
    CK(hipMemcpyAsync(&got, bad, sizeof(got), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    *bad_out = got == ~0ull ? -1 : (int64_t)got;
    return CROP_OK;
}

// First query pair breaking x < y < n_items, or -1 (synchronizes).
crop_status check_pairs_on_device(crop_ctx *ctx, const uint32_t *qx, const uint32_t *qy,
                                  uint64_t n, uint32_t n_items, int64_t *bad_out)
{
    CK(ctx->scratch.ensure(64));
    auto *bad = ctx->scratch.as<unsigned long long>();
    unsigned long long init = ~0ull;
    CK(hipMemcpyAsync(bad, &init, sizeof(init), hipMemcpyHostToDevice, ctx->stream));
    CK(launch_check_pairs(qx, qy, n, n_items, bad, ctx->stream));
    unsigned long long got = 0;
    CK(hipMemcpyAsync(&got, bad, sizeof(got), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    *bad_out = got == ~0ull ? -1 : (int64_t)got;
    return CROP_OK;
}

crop_status check_offsets(crop_ctx *ctx, const std::vector<uint32_t> &off, uint64_t nnz,
                          const char *name)
{
    if (off.empty() || off[0] != 0 || off.back() != nnz) {
        ctx->err_index = -1;
        return fail(ctx, CROP_E_INPUT, std::string(name) + ": off[0] must be 0 and off[K] = nnz");
    }
    for (size_t t = 0; t + 1 < off.size(); ++t)
        if (off[t + 1] < off[t]) {
            ctx->err_index = (int64_t)t;
            return fail(ctx, CROP_E_INPUT,
                        std::string(name) + ": offsets decrease at vector " + std::to_string(t));
        }
    return CROP_OK;
}

void reset_input(crop_ctx *ctx)
{
    Input &in = ctx->in;
    in.mode = Mode::None;
    in.off = in.items = nullptr;
    in.a_off = in.a_idx = in.b_off = in.b_idx = nullptr;
    in.a_val = in.b_val = nullptr;
    in.T = in.nnz = in.K = in.nnz_a = in.nnz_b = 0;
    in.total_terms = 0;
    in.h_off.clear();
    in.h_b_off.clear();
    ctx->sb.valid = false;
    in.op_chunks.clear();
    reset_batch(ctx);
    ctx->result = Result::None;
}

// ---- planning -------------------------------------------------------------

// Owned partitions [p0, p1) of the context (all by default).
static void owned_range(const crop_ctx *ctx, uint32_t *p0, uint32_t *p1)
{
    const bool all = ctx->own_p0 == 0 && ctx->own_p1 == 0;
    *p0 = all ? 0 : ctx->own_p0;
    *p1 = all ? ctx->P : ctx->own_p1;
}

// Bins spanned by the owned partitions [p0, p1) when a bin groups 2^g.
static uint64_t grouped_span(uint32_t p0, uint32_t p1, uint32_t g)
{
    return (uint64_t)((p1 - 1) >> g) - (p0 >> g) + 1;
}

// Bins of the run.  Up to kMaxP kept bins (the count kernels' LDS histogram):
// S bins per partition (M = P * S) while the owned partitions times S fit,
// S chosen for about terms_per_bin routed terms per bin; beyond that (P above
// 8192) one bin holds 2^g consecutive partitions (M = P), g the smallest that
// fits.  g_req >= 0 asks for that grouping with one bin per 2^g partitions.
static crop_status plan_bins(crop_ctx *ctx, uint32_t S, uint64_t terms_per_bin, int g_req = -1)
{
    Input &in = ctx->in;
    RoutePlan &pl = ctx->plan;
    const uint32_t P = ctx->P;
    uint32_t p0, p1;
    owned_range(ctx, &p0, &p1);
    const uint32_t Pown = p1 - p0;
    if (g_req < 0 && S == 0) {
        const uint64_t want = (in.total_terms + terms_per_bin - 1) / terms_per_bin;
        S = (uint32_t)std::max<uint64_t>(1, (want + P - 1) / P);
        while (S > 1 && (uint64_t)Pown * S > kMaxP) --S;
    }
    if (g_req < 0 && (uint64_t)Pown * S <= kMaxP) {
        if ((uint64_t)P * S > (1ull << 32))
            return fail(ctx, CROP_E_UNSUPPORTED, "partitions x bins_per_partition exceeds 2^32");
        pl.S = S;
        pl.g = 0;
        pl.M = (uint64_t)P * S;
        pl.u0 = p0 * S;
        pl.nu = Pown * S;
        pl.NB = Pown * S;
        return CROP_OK;
    }
    if (g_req < 0 && S > 1)
        return fail(ctx, CROP_E_UNSUPPORTED, "owned partitions x bins_per_partition exceeds 8192");
    uint32_t g = g_req < 0 ? 0u : (uint32_t)g_req;
    while (grouped_span(p0, p1, g) > kMaxP) ++g;
    if (g > kMaxGroupLog2)
        return fail(ctx, CROP_E_UNSUPPORTED, "too many partitions per routing bin");
    pl.S = 1;
    pl.g = g;
    pl.M = P;
    pl.u0 = p0;
    pl.nu = Pown;
    pl.NB = (uint32_t)grouped_span(p0, p1, g);
    return CROP_OK;
}

// An owned share of at most half the hash space enumerates through h_b
// windows (Lemma 1) instead of every term: the owned interval is [q, r) with
// q = ceil(u0 2^32 / M), r = ceil((u0 + nu) 2^32 / M), and the bucket bits
// make a bucket about a quarter of the window (at most 32 per row).
static void plan_window(crop_ctx *ctx)
{
    RoutePlan &pl = ctx->plan;
    pl.win_kb = pl.win_q = pl.win_W = 0;
    if (ctx->tune.window == CROP_WINDOW_OFF || pl.n_wg || pl.stage_cap) return;
    const uint64_t q = (((uint64_t)pl.u0 << 32) + pl.M - 1) / pl.M;
    const uint64_t r = ((((uint64_t)pl.u0 + pl.nu) << 32) + pl.M - 1) / pl.M;
    const uint64_t W = r - q;
    if (W == 0 || W > (1ull << 31)) return;
    uint32_t kb = 2;
    while (kb < 5 && (1ull << (32 - kb)) > W / 4) ++kb;
    if (!tx_win_layout_ok(pl.NB, pl.R, kb, pl.max_items)) return;
    pl.win_kb = kb;
    pl.win_q = (uint32_t)q;
    pl.win_W = (uint32_t)W;
}

crop_status plan_tx(crop_ctx *ctx, uint32_t S_force = 0, int g_req = -1)
{
    Input &in = ctx->in;
    RoutePlan &pl = ctx->plan;
    pl.regions = false;
    crop_status st = plan_bins(ctx, S_force ? S_force : ctx->tune.bins_per_partition,
                               kTermsPerBin, g_req);
    if (st != CROP_OK) return st;
    const size_t hist_bytes = (size_t)pl.NB * 4;
    // 128 transactions per chunk: about 11,000 terms at ten items per
    // transaction (measured best on the 1M-transaction stream among 64..352
    // with direct scatter writes)
    uint32_t R = ctx->tune.rows_per_chunk ? ctx->tune.rows_per_chunk : 128;
    auto max_items_for = [&](uint32_t r) {
        uint32_t mx = 0;
        for (uint64_t t0 = 0; t0 < in.T; t0 += r) {
            uint64_t t1 = std::min<uint64_t>(in.T, t0 + r);
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
    pl.R = R;
    pl.max_items = mi;
    pl.n_chunks = (uint32_t)((in.T + R - 1) / R);
    const size_t fixed = tx_scatter_smem_bytes(pl.NB, mi, 0, in.wide_keys);
    const size_t per = in.wide_keys ? 8 : 4;
    // Scatter writes go straight to their slots unless staging is requested
    // (stage_keys): measured faster, and the smaller LDS footprint lets two
    // scatter workgroups share a CU.
    pl.stage_cap = 0;
    if (ctx->tune.stage_keys) {
        const size_t room = fixed < kStageBudget ? (kStageBudget - fixed) / per : 0;
        if (room < 1024)
            return fail(ctx, CROP_E_UNSUPPORTED, "routing bins and chunk leave no LDS for staging");
        pl.stage_cap = (uint32_t)std::min<size_t>(room, ctx->tune.stage_keys);
    }
    // Range kernels (on request): one workgroup per contiguous range of
    // chunks, as many as fit on the GPU at once.  Two scatter workgroups share
    // a CU when half of the LDS still stages a typical chunk in one window.
    pl.n_wg = 0;
    if (ctx->tune.route == CROP_ROUTE_RANGES && pl.n_chunks) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const uint64_t avg_terms = pl.n_chunks ? in.total_terms / pl.n_chunks : 0;
        const size_t half = kCuLds / 2;
        const size_t room2 = fixed < half ? (half - fixed) / per : 0;
        uint32_t per_cu = 1;
        if (pl.stage_cap == 0 || (room2 >= 1024 && room2 >= avg_terms + avg_terms / 4)) {
            per_cu = 2;
            if (pl.stage_cap) pl.stage_cap = (uint32_t)std::min<size_t>(room2, pl.stage_cap);
        }
        pl.n_wg = (uint32_t)std::min<uint64_t>(pl.n_chunks, (uint64_t)cus * per_cu);
    }
    pl.G = std::max<uint32_t>(1, std::min<uint32_t>(64, pl.n_wg ? pl.n_wg / 16 : pl.n_chunks));
    if (!tx_launch_layouts_ok(pl.NB, pl.max_items, pl.stage_cap, in.wide_keys))
        return fail(ctx, CROP_E_UNSUPPORTED, "chunk image does not fit its LDS layout");
    plan_window(ctx);
    return CROP_OK;
}

// ---- region route plan

// Caps of a sub-batch for NB bins (packed keys): the terms (route threads x
// Q, Q in {24, 16}), items and rows in proportion (about ten items and 45
// terms per transaction of the 1M-transaction stream: a sub-batch is cut by
// its terms, rarely by the others); the largest that fits the LDS budget.
bool sb_caps(uint32_t NB, uint32_t key_bytes, uint32_t want, uint32_t *S, uint32_t *I,
             uint32_t *R)
{
    static const uint32_t qs[] = {24, 16};
    for (int k = 0; k < 2; ++k) {
        const uint32_t terms = sb_threads() * qs[k];
        if (want && terms != want) continue;
        const uint32_t items = terms / 8, rows = terms / 24;
        const size_t sm = sb_route_smem_bytes(NB, rows, items, terms, key_bytes);
        if (sm <= kStageBudget && sb_layout_ok(NB, rows, items, terms, key_bytes, sm)) {
            *S = terms;
            *I = items;
            *R = rows;
            return true;
        }
    }
    return false;
}

// Sub-batches of the loaded stream for these caps (greedy over the rows,
// kept until the next load); false when one transaction alone exceeds them.
// cuts (a batch's stream boundaries, ascending) start a new sub-batch, so
// that none crosses a stream; such a plan is made afresh each time.  The
// row and term boundaries go to the device once per plan.
crop_status plan_sb_rows(crop_ctx *ctx, uint32_t S, uint32_t I, uint32_t R, bool *ok,
                         const std::vector<uint64_t> *cuts)
{
    SbPlan &sp = ctx->sb;
    *ok = true;
    if (!cuts && sp.valid && sp.max_terms == S && sp.max_items == I && sp.max_rows == R)
        return CROP_OK;
    sp.valid = false;
    sp.row.assign(1, 0);
    sp.term.assign(1, 0);
    const std::vector<uint32_t> &off = ctx->in.h_off;
    const uint64_t T = ctx->in.T;
    // region bases: the term prefix with each region rounded up to four
    // keys, so that every region starts on 16 bytes
    uint64_t base = 0;
    uint32_t ct = 0, ci = 0, cr = 0;
    size_t next_cut = 0;
    for (uint64_t t = 0; t < T; ++t) {
        const uint32_t L = off[t + 1] - off[t];
        const uint64_t n = L ? (uint64_t)L * (L - 1) / 2 : 0;
        if (n > S || L > I) {
            *ok = false;
            return CROP_OK;
        }
        bool cut = false;
        while (cuts && next_cut < cuts->size() && (*cuts)[next_cut] <= t) {
            cut = cut || (*cuts)[next_cut] == t;
            ++next_cut;
        }
        if (cr && (cut || ct + n > S || ci + L > I || cr + 1 > R)) {
            base += (ct + 3) & ~3u;
            sp.row.push_back((uint32_t)t);
            sp.term.push_back((uint32_t)base);
            ct = ci = cr = 0;
        }
        ct += (uint32_t)n;
        ci += L;
        cr += 1;
    }
    if (T) {
        base += (ct + 3) & ~3u;
        sp.row.push_back((uint32_t)T);
        sp.term.push_back((uint32_t)base);
    }
    if (base >= (1ull << 32)) {
        *ok = false;
        return CROP_OK;
    }
    sp.n_sub = (uint32_t)sp.row.size() - 1;
    sp.max_terms = S;
    sp.max_items = I;
    sp.max_rows = R;
    CK(ctx->sb_row.ensure(sp.row.size() * 4));
    CK(ctx->sb_term.ensure(sp.term.size() * 4));
    CK(hipMemcpy(ctx->sb_row.p, sp.row.data(), sp.row.size() * 4, hipMemcpyHostToDevice));
    CK(hipMemcpy(ctx->sb_term.p, sp.term.data(), sp.term.size() * 4, hipMemcpyHostToDevice));
    sp.valid = true;
    return CROP_OK;
}

// The region route for an exact run of the loaded transaction stream, when
// the tuning allows it (route AUTO or REGIONS, no staged scatter), no owned
// share of at most half the hash space enumerates through windows instead,
// and every transaction fits a sub-batch.  *ok false: plan_tx decides.
static crop_status plan_regions(crop_ctx *ctx, bool *ok)
{
    *ok = false;
    const crop_tune &tu = ctx->tune;
    if (ctx->in.mode != Mode::Tx || ctx->in.wide_keys) return CROP_OK;
    if (tu.route != CROP_ROUTE_AUTO && tu.route != CROP_ROUTE_REGIONS) return CROP_OK;
    if (tu.stage_keys) return CROP_OK;
    crop_status st = plan_bins(ctx, tu.bins_per_partition, kTermsPerBin);
    if (st != CROP_OK) return st;
    RoutePlan &pl = ctx->plan;
    if (tu.window != CROP_WINDOW_OFF && tu.route == CROP_ROUTE_AUTO) {
        const uint64_t q = (((uint64_t)pl.u0 << 32) + pl.M - 1) / pl.M;
        const uint64_t r = ((((uint64_t)pl.u0 + pl.nu) << 32) + pl.M - 1) / pl.M;
        if (r - q <= (1ull << 31)) return CROP_OK;
    }
    uint32_t S, I, R;
    const uint32_t kb = ctx->in.wide_keys ? 8 : 4;
    if (!sb_caps(pl.NB, kb, tu.region_terms, &S, &I, &R)) return CROP_OK;
    bool fits = false;
    st = plan_sb_rows(ctx, S, I, R, &fits);
    if (st != CROP_OK || !fits) return st;
    SbPlan &sp = ctx->sb;
    sp.segs.assign(1, SbSeg{});
    SbSeg &sg = sp.segs[0];
    sg.bm = bin_map(pl);
    sg.NB = pl.NB;
    sg.n_sub = sp.n_sub;
    layout_sb_segments(sp);
    pl.regions = true;
    pl.n_chunks = 0;
    pl.R = 0;
    pl.max_items = 0;
    pl.stage_cap = 0;
    pl.n_wg = 0;
    pl.G = 1;
    pl.win_kb = pl.win_q = pl.win_W = 0;
    *ok = true;
    return CROP_OK;
}

crop_status plan_outer(crop_ctx *ctx, uint32_t S_force = 0, int g_req = -1)
{
    Input &in = ctx->in;
    RoutePlan &pl = ctx->plan;
    pl.regions = false;
    // outer-product entries rarely repeat and fp32 sums use 8192-slot
    // tables: aim at about 2000 routed terms per bin
    crop_status st = plan_bins(ctx, S_force ? S_force : ctx->tune.bins_per_partition,
                               kTermsPerBin / 16, g_req);
    if (st != CROP_OK) return st;
    pl.max_items = in.op_max_a;
    pl.n_chunks = (uint32_t)in.op_chunks.size();
    pl.n_wg = 0;
    pl.G = std::max<uint32_t>(1, std::min<uint32_t>(64, pl.n_chunks));
    const size_t lds = (size_t)pl.NB * 4 + 20ull * pl.max_items + 1024;
    if (lds > 150 * 1024)
        return fail(ctx, CROP_E_UNSUPPORTED, "outer-product chunk does not fit in LDS");
    return CROP_OK;
}

// Split the a-entries of the K vectors into chunks of at most kA entries and
// about kW terms; a vector with many terms is split over several chunks.
void build_outer_chunks(Input &in)
{
    constexpr uint32_t kA = 1024;
    constexpr uint64_t kW = 32768;
    in.op_chunks.clear();
    in.op_max_a = 0;
    OpChunk cur{0, 0, 0, 0};
    uint64_t work = 0;
    bool open = false;
    auto close = [&]() {
        if (open && cur.a_hi > cur.a_lo) {
            in.op_chunks.push_back(cur);
            in.op_max_a = std::max(in.op_max_a, cur.a_hi - cur.a_lo);
        }
        open = false;
        work = 0;
    };
    for (uint32_t k = 0; k < in.K; ++k) {
        uint32_t a0 = in.h_off[k], a1 = in.h_off[k + 1];
        uint64_t nb = in.h_b_off[k + 1] - in.h_b_off[k];
        if (a0 == a1 || nb == 0) continue;
        for (uint32_t a = a0; a < a1; ++a) {
            if (!open) {
                cur = OpChunk{k, k + 1, a, a};
                open = true;
            }
            if (cur.a_hi - cur.a_lo >= kA || (work + nb > kW && cur.a_hi > cur.a_lo)) {
                close();
                cur = OpChunk{k, k + 1, a, a};
                open = true;
            }
            cur.k1 = k + 1;
            cur.a_hi = a + 1;
            work += nb;
        }
    }
    close();
}

crop_status ensure_route_buffers(crop_ctx *ctx, size_t key_bytes, bool sums)
{
    const RoutePlan &pl = ctx->plan;
    const uint64_t nt = ctx->in.total_terms;
    CK(ctx->cnt_mat.ensure((size_t)std::max<uint32_t>(pl.n_chunks, 1) * pl.NB * 4));
    CK(ctx->part_buf.ensure((size_t)pl.G * pl.NB * 4));
    CK(ctx->bin_off.ensure(((size_t)pl.NB + 1) * 4));
    CK(ctx->bin_size.ensure((size_t)pl.NB * 4));
    CK(ctx->bin_order.ensure((size_t)pl.NB * 4));
    CK(ctx->keys.ensure(nt * key_bytes));
    if (sums)
        CK(ctx->vals.ensure(nt * 4));
    else
        CK(ctx->out_cnt.ensure(nt * 4));
    CK(ctx->spill.ensure(nt * spill_entry_bytes(ctx->in.wide_keys, sums)));
    CK(ctx->counter.ensure(64));
    if (pl.g) CK(ctx->part_stats.ensure((size_t)ctx->P * 8));
    return CROP_OK;
}

// Strides, tiles and offsets of the segments of a region plan (their NB,
// bin0, sub0, n_sub, bm and key0 set): header rows of NB + 1 starts rounded
// to 64, transposed rows of n_sub rounded to 64, 64 x 64 header tiles, the
// segments' blocks one after another; NBmax for the route's LDS image.
void layout_sb_segments(SbPlan &sp)
{
    sp.NBmax = 0;
    sp.n_tiles = 0;
    sp.hdr_words = sp.hdrT_words = sp.tsum_words = 0;
    for (SbSeg &g : sp.segs) {
        g.hs = (g.NB + 1 + 63) & ~63u;
        g.hts = (g.n_sub + 63) & ~63u;
        g.btiles = (g.NB + 1 + 63) / 64;
        g.tile0 = sp.n_tiles;
        g.hdr0 = sp.hdr_words;
        g.hdrT0 = sp.hdrT_words;
        g.tsum0 = sp.tsum_words;
        const uint32_t sub_tiles = (g.n_sub + 63) / 64;
        sp.n_tiles += g.btiles * sub_tiles;
        sp.hdr_words += (uint64_t)g.n_sub * g.hs;
        sp.hdrT_words += (uint64_t)(g.NB + 1) * g.hts;
        sp.tsum_words += (uint64_t)sub_tiles * (g.NB + 1);
        sp.NBmax = std::max(sp.NBmax, g.NB);
    }
}

// Region route: the routed array (the padded regions of every sub-batch;
// terms an owned share drops leave gaps), the sub-batches' bin-start rows,
// their transpose and tile sums, and the segments on the device (copied
// when they changed).
crop_status ensure_region_buffers(crop_ctx *ctx)
{
    const SbPlan &sp = ctx->sb;
    const size_t kb = ctx->in.wide_keys ? 8 : 4;
    // the padded regions, and one more 16-byte group past the last
    CK(ctx->routed.ensure((sp.term.empty() ? 0 : (size_t)sp.term.back()) * kb + 64));
    CK(ctx->sb_hdr.ensure(sp.hdr_words * 2));
    CK(ctx->sb_hdrT.ensure(sp.hdrT_words * 2));
    CK(ctx->sb_tsum.ensure(sp.tsum_words * 4));
    const size_t seg_bytes = sp.segs.size() * sizeof(SbSeg);
    std::vector<SbSeg> &up = ctx->sb_seg_host;
    auto same = [](const SbSeg &x, const SbSeg &y) {
        return x.bm.M == y.bm.M && x.bm.u0 == y.bm.u0 && x.bm.nu == y.bm.nu && x.bm.g == y.bm.g &&
               x.NB == y.NB && x.bin0 == y.bin0 && x.sub0 == y.sub0 && x.n_sub == y.n_sub &&
               x.hs == y.hs && x.hts == y.hts && x.tile0 == y.tile0 && x.btiles == y.btiles &&
               x.key0 == y.key0 && x.hdr0 == y.hdr0 && x.hdrT0 == y.hdrT0 && x.tsum0 == y.tsum0;
    };
    bool changed = up.size() != sp.segs.size() || !ctx->sb_seg.p;
    for (size_t i = 0; !changed && i < up.size(); ++i) changed = !same(up[i], sp.segs[i]);
    if (changed) {
        CK(ctx->sb_seg.ensure(std::max<size_t>(seg_bytes, 1)));
        if (seg_bytes) CK(hipMemcpy(ctx->sb_seg.p, sp.segs.data(), seg_bytes, hipMemcpyHostToDevice));
        up = sp.segs;
    }
    return CROP_OK;
}

// First local bin of partition p in the last run, or -1 when p is not owned
// (with grouped bins, the one bin p shares with its neighbours).
static int64_t partition_bin(const crop_ctx *ctx, uint32_t p)
{
    const RoutePlan &pl = ctx->plan;
    if (pl.g) {
        if (p < pl.u0 || p - pl.u0 >= pl.nu) return -1;
        return (int64_t)(p >> pl.g) - (pl.u0 >> pl.g);
    }
    const uint32_t p0 = pl.u0 / pl.S, p1 = p0 + pl.nu / pl.S;
    return (p >= p0 && p < p1) ? (int64_t)(p - p0) * pl.S : -1;
}

crop_status require_exact(crop_ctx *ctx)
{
    if (ctx->result != Result::Exact)
        return fail(ctx, CROP_E_STATE, "no exact result: call crop_run_exact first");
    return CROP_OK;
}

// Space-Saving routing: bins hold whole groups of nbk buckets (nbk divides
// the B buckets of a partition), the bucket summaries of a bin must fit in
// LDS, and there should be enough bins to occupy the GPU.  When no divisor
// keeps the bins within kMaxP (P above 8192), a bin holds the B buckets of
// 2^g consecutive partitions instead (*g_out = g; else -1); the last bin may
// then be partial, and the summary state is padded to whole bins.
crop_status plan_ss(crop_ctx *ctx, uint32_t *nbk_out, uint64_t *PB_out, int *g_out)
{
    const uint32_t P = ctx->P, ell = ctx->ss_ell;
    const uint64_t B = ctx->ss_counters / ell;
    const uint64_t PB = (uint64_t)P * B;
    if (PB > (1ull << 32))
        return fail(ctx, CROP_E_UNSUPPORTED, "P x buckets per partition exceeds 2^32");
    const bool outer = ctx->in.mode == Mode::Outer;
    const bool wide = outer || ctx->in.wide_keys;
    // Bins of nbk buckets (nbk divides B), at most kMaxP bins and within the
    // LDS budget: the largest nbk that still leaves min(kSsMinBins, P*B)
    // bins, else the smallest feasible nbk.
    std::vector<uint64_t> divs;
    for (uint64_t d = 1; d * d <= B; ++d)
        if (B % d == 0) {
            divs.push_back(d);
            if (d != B / d) divs.push_back(B / d);
        }
    std::sort(divs.begin(), divs.end());
    const uint64_t min_bins = std::min<uint64_t>(kSsMinBins, PB);
    auto pick_for = [&](uint32_t MB) {
        uint64_t pick = 0;
        for (uint64_t nbk : divs) {
            const uint64_t NB = PB / nbk;
            if (NB > kMaxP) continue;
            if (ss_bins_smem_bytes((uint32_t)nbk, ell, wide, outer, MB) > kSsLdsBudget) break;
            if (!pick || NB >= min_bins) pick = nbk;
        }
        return pick;
    };
    // Packed transaction keys merge micro-batches of kSsBatchTxLarge terms
    // when bins of several buckets fit with them (measured faster: fewer,
    // longer merged update lists per bucket).  Bins of one bucket keep
    // kSsBatchTx: the time of their run is set by the heaviest bins, and on
    // two 1M-transaction streams of the same law (P = 1, 16,384 counters)
    // the larger batch took 3.30 instead of 3.44 ms on one and 3.54 instead
    // of 3.24 ms on the other.
    uint32_t MB = outer ? kSsBatchOuter : wide ? kSsBatchWide : kSsBatchTx;
    uint64_t pick = 0;
    if (!wide) {
        pick = pick_for(kSsBatchTxLarge);
        if (pick > 1) MB = kSsBatchTxLarge;
    }
    if (MB != kSsBatchTxLarge) pick = pick_for(MB);
    *g_out = -1;
    if (!pick) {
        // grouped bins: the smallest g with ceil(P / 2^g) <= kMaxP
        uint32_t g = 0;
        while (((uint64_t)P + (1ull << g) - 1) >> g > kMaxP) ++g;
        const uint64_t nbk = B << g;
        MB = outer ? kSsBatchOuter : wide ? kSsBatchWide : kSsBatchTx;
        if (g == 0 || g > kMaxGroupLog2 || nbk > (1ull << 20) ||
            ss_bins_smem_bytes((uint32_t)nbk, ell, wide, outer, MB) > kSsLdsBudget)
            return fail(ctx, CROP_E_UNSUPPORTED, "Space-Saving summaries do not fit the LDS plan");
        pick = nbk;
        *g_out = (int)g;
    }
    ctx->plan.ss_mb = MB;
    *nbk_out = (uint32_t)pick;
    *PB_out = PB;
    return CROP_OK;
}

crop_status ensure_ss_buffers(crop_ctx *ctx, uint64_t nslots, uint32_t K, uint32_t ns)
{
    const size_t a8 = (nslots * 8 + 255) / 256 * 256, a4 = (nslots * 4 + 255) / 256 * 256;
    CK(ctx->ss_state.ensure(a8 + 3 * a4 + nslots + 256));
    char *p = static_cast<char *>(ctx->ss_state.p);
    ctx->ss.key = reinterpret_cast<uint64_t *>(p);
    ctx->ss.cnt = reinterpret_cast<uint32_t *>(p + a8);
    ctx->ss.err = reinterpret_cast<uint32_t *>(p + a8 + a4);
    ctx->ss.val = reinterpret_cast<float *>(p + a8 + 2 * a4);
    ctx->ss.flag = reinterpret_cast<uint8_t *>(p + a8 + 3 * a4);
    ctx->ss.nslots = nslots;
    // top-K: st (8) + hist (256) + pinned counter | cand | sel | outputs
    const size_t kk = std::max<uint32_t>(K, 1);
    CK(ctx->topk_buf.ensure(2048 + 2 * a4 + kk * 40 + ns + 256));
    return CROP_OK;
}

// Combined entries of an amplified run, one per slot of the t summaries:
// upper bound, lower bound, value, used flag and votes.
crop_status ensure_amp_buffers(crop_ctx *ctx, uint64_t nslots, SsState *A, uint8_t **votes)
{
    const size_t a4 = (nslots * 4 + 255) / 256 * 256, a1 = (nslots + 255) / 256 * 256;
    CK(ctx->amp_buf.ensure(4 * a4 + 2 * a1));
    char *p = static_cast<char *>(ctx->amp_buf.p);
    A->key = ctx->ss.key;
    // packed keys of the t summaries (narrow runs), for the combine's lookups
    A->key32 = reinterpret_cast<uint32_t *>(p + 3 * a4 + 2 * a1);
    A->cnt = reinterpret_cast<uint32_t *>(p);
    A->err = reinterpret_cast<uint32_t *>(p + a4);
    A->val = reinterpret_cast<float *>(p + 2 * a4);
    A->flag = reinterpret_cast<uint8_t *>(p + 3 * a4);
    A->nslots = nslots;
    *votes = reinterpret_cast<uint8_t *>(p + 3 * a4 + a1);
    return CROP_OK;
}

struct TopkViews {
    uint32_t *st, *hist, *n_pinned, *cand, *sel, *oi, *oj, *ovotes, *rank;
    double *ou, *ol, *ov;
    uint8_t *dup;
};

TopkViews topk_views(crop_ctx *ctx, uint32_t K)
{
    const uint64_t nslots = ctx->ss.nslots;
    const size_t a4 = (nslots * 4 + 255) / 256 * 256;
    const size_t kk = std::max<uint32_t>(K, 1);
    char *p = static_cast<char *>(ctx->topk_buf.p);
    TopkViews v;
    v.st = reinterpret_cast<uint32_t *>(p);
    v.hist = v.st + 8;
    v.n_pinned = v.st + 8 + 256;
    v.cand = reinterpret_cast<uint32_t *>(p + 2048);
    v.sel = reinterpret_cast<uint32_t *>(p + 2048 + a4);
    char *o = p + 2048 + 2 * a4;
    v.ou = reinterpret_cast<double *>(o);
    v.ol = v.ou + kk;
    v.ov = v.ol + kk;
    v.oi = reinterpret_cast<uint32_t *>(v.ov + kk);
    v.oj = v.oi + kk;
    v.ovotes = v.oj + kk;
    v.rank = v.ovotes + kk;
    v.dup = reinterpret_cast<uint8_t *>(v.rank + kk);
    return v;
}

// Run bracketing: ev0/ev1 around every run; with profiling on, one event
// after each stage as well, kept for the last kStageRing runs.
crop_status run_begin(crop_ctx *ctx)
{
    hipStream_t s = ctx->stream;
    CK(hipEventRecord(ctx->ev0, s));
    ctx->cur_rec = nullptr;
    if (!ctx->profiling) return CROP_OK;
    StageRec &r = ctx->ring[ctx->runs % kStageRing];
    r.n = 0;
    CK(hipEventRecord(r.ev[0], s));
    ctx->cur_rec = &r;
    return CROP_OK;
}

crop_status stage_end(crop_ctx *ctx, const char *name)
{
    StageRec *r = ctx->cur_rec;
    if (!r || r->n >= kMaxStages) return CROP_OK;
    r->names[r->n] = name;
    CK(hipEventRecord(r->ev[r->n + 1], ctx->stream));
    r->n += 1;
    return CROP_OK;
}

crop_status run_end(crop_ctx *ctx)
{
    CK(hipEventRecord(ctx->ev1, ctx->stream));
    ctx->timed = true;
    if (ctx->cur_rec) ctx->runs += 1;
    ctx->cur_rec = nullptr;
    return CROP_OK;
}

}  // namespace crop

// ============================================================== context

extern "C" {

int crop_abi_version(void) { return CROP_ABI_VERSION; }

const char *crop_status_string(crop_status s)
{
    switch (s) {
    case CROP_OK: return "ok";
    case CROP_E_ARG: return "invalid argument";
    case CROP_E_STATE: return "call out of order";
    case CROP_E_INPUT: return "invalid input";
    case CROP_E_CAPACITY: return "output buffer too small";
    case CROP_E_NOMEM: return "out of device memory";
    case CROP_E_HIP: return "HIP runtime error";
    case CROP_E_UNSUPPORTED: return "unsupported parameters";
    }
    return "unknown status";
}

crop_status crop_create(crop_ctx **out, int hip_device)
{
    if (!out) return CROP_E_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n)
        return CROP_E_ARG;
    DeviceGuard g(hip_device);
    crop_ctx *ctx = new (std::nothrow) crop_ctx();
    if (!ctx) return CROP_E_NOMEM;
    ctx->device = hip_device;
    ctx->hp = make_hash_params(ctx->seed);
    // the fixed workspace of the no-allocation entry point on this device; a
    // failure is reported by that entry point
    (void)noalloc_setup(hip_device);
    if (hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) {
        crop_destroy(ctx);
        return CROP_E_HIP;
    }
    ctx->stream = ctx->own_stream;
    *out = ctx;
    return CROP_OK;
}

void crop_destroy(crop_ctx *ctx)
{
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->own_stream) (void)hipStreamSynchronize(ctx->own_stream);
    reset_batch(ctx);
    BatchState &bt = ctx->batch;
    for (DevBuf *b : {&ctx->cnt_mat, &ctx->part_buf, &ctx->bin_off, &ctx->bin_size,
                      &ctx->bin_order, &ctx->keys,
                      &ctx->vals, &ctx->out_cnt, &ctx->spill, &ctx->counter, &ctx->ss_state,
                      &ctx->topk_buf, &ctx->scratch, &ctx->learn_ws, &ctx->seed_sel,
                      &ctx->part_stats, &ctx->routed, &ctx->sb_row, &ctx->sb_term,
                      &ctx->sb_hdr, &ctx->sb_hdrT, &ctx->sb_tsum, &ctx->sb_seg,
                      &ctx->sb_subseg, &ctx->sb_binseg, &ctx->in.d_op_chunks,
                      &bt.d_crow, &bt.d_cstream, &bt.d_streams, &bt.d_bin_stream, &bt.tot,
                      &bt.tiles, &ctx->cs_buf, &ctx->amp_buf})
        b->release();
    for (DevBuf &b : ctx->in.own) b.release();
    for (StageRec &r : ctx->ring)
        for (hipEvent_t &e : r.ev)
            if (e) (void)hipEventDestroy(e);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    delete ctx;
}

const char *crop_last_error_detail(const crop_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }
int64_t crop_last_error_index(const crop_ctx *ctx) { return ctx ? ctx->err_index : -1; }

crop_status crop_set_partitions(crop_ctx *ctx, uint32_t P)
{
    if (!ctx) return CROP_E_ARG;
    if (P < 1 || P > kMaxPartitions)
        return fail(ctx, CROP_E_UNSUPPORTED, "P must be in [1, 2^20]");
    ctx->P = P;
    ctx->own_p0 = ctx->own_p1 = 0;  // a new partition count owns all partitions again
    ctx->result = Result::None;
    return CROP_OK;
}

crop_status crop_set_seed(crop_ctx *ctx, uint64_t seed)
{
    if (!ctx) return CROP_E_ARG;
    ctx->seed = seed;
    ctx->hp = make_hash_params(seed);
    ctx->result = Result::None;
    batch_invalidate_graph(ctx);  // a captured batch graph holds the old parameters
    return CROP_OK;
}

crop_status crop_set_summary(crop_ctx *ctx, uint32_t counters_per_partition,
                             uint32_t counters_per_bucket)
{
    if (!ctx) return CROP_E_ARG;
    if (counters_per_bucket < 1 || counters_per_bucket > 64 || counters_per_partition == 0 ||
        counters_per_partition % counters_per_bucket)
        return fail(ctx, CROP_E_ARG, "need 1 <= ell <= 64 dividing counters_per_partition");
    ctx->ss_counters = counters_per_partition;
    ctx->ss_ell = counters_per_bucket;
    ctx->result = Result::None;
    return CROP_OK;
}

crop_status crop_set_owned_partitions(crop_ctx *ctx, uint32_t p_begin, uint32_t p_end)
{
    if (!ctx) return CROP_E_ARG;
    if (!(p_begin == 0 && p_end == 0) && !(p_begin < p_end && p_end <= ctx->P))
        return fail(ctx, CROP_E_ARG, "need 0 <= p_begin < p_end <= P (or 0, 0 for all)");
    ctx->own_p0 = p_begin;
    ctx->own_p1 = (p_begin == 0 && p_end == ctx->P) ? 0 : p_end;
    if (ctx->own_p1 == 0) ctx->own_p0 = 0;
    ctx->result = Result::None;
    return CROP_OK;
}

crop_status crop_set_topk_rank(crop_ctx *ctx, int rank)
{
    if (!ctx) return CROP_E_ARG;
    if (rank != CROP_RANK_UPPER && rank != CROP_RANK_LOWER)
        return fail(ctx, CROP_E_ARG, "rank must be CROP_RANK_UPPER or CROP_RANK_LOWER");
    ctx->topk_rank = rank;
    ctx->result = Result::None;
    return CROP_OK;
}

crop_status crop_set_stream(crop_ctx *ctx, void *hip_stream)
{
    if (!ctx) return CROP_E_ARG;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return CROP_OK;
}

crop_status crop_use_own_stream(crop_ctx *ctx)
{
    if (!ctx) return CROP_E_ARG;
    ctx->stream = ctx->own_stream;
    return CROP_OK;
}

crop_status crop_set_tuning(crop_ctx *ctx, const crop_tune *t)
{
    if (!ctx) return CROP_E_ARG;
    if (!t) {
        ctx->tune = crop_tune{};
        return CROP_OK;
    }
    if (t->route > CROP_ROUTE_REGIONS)
        return fail(ctx, CROP_E_ARG, "route must be CROP_ROUTE_AUTO, _CHUNKS, _RANGES or _REGIONS");
    if (t->stage_keys && t->stage_keys < 1024)
        return fail(ctx, CROP_E_ARG, "stage_keys must be 0 (automatic) or at least 1024");
    if (t->window > CROP_WINDOW_OFF)
        return fail(ctx, CROP_E_ARG, "window must be CROP_WINDOW_AUTO or CROP_WINDOW_OFF");
    if (t->region_terms && t->region_terms != 16384 && t->region_terms != 24576)
        return fail(ctx, CROP_E_ARG, "region_terms must be 0, 16384 or 24576");
    ctx->tune = *t;
    return CROP_OK;
}

crop_status crop_set_profiling(crop_ctx *ctx, int enable)
{
    if (!ctx) return CROP_E_ARG;
    DeviceGuard g(ctx->device);
    if (enable && ctx->ring.empty()) {
        ctx->ring.resize(kStageRing);
        for (StageRec &r : ctx->ring)
            for (hipEvent_t &e : r.ev) CK(hipEventCreate(&e));
    }
    ctx->profiling = enable != 0;
    ctx->runs = 0;
    return CROP_OK;
}

crop_status crop_run_stages(crop_ctx *ctx, uint32_t back, uint32_t *n_stages,
                            const char **names, float *ms, uint32_t cap)
{
    if (!ctx || !n_stages) return CROP_E_ARG;
    if (!ctx->profiling) return fail(ctx, CROP_E_STATE, "profiling is off");
    if (back >= ctx->runs || back >= (uint32_t)kStageRing)
        return fail(ctx, CROP_E_ARG, "no such recorded run");
    DeviceGuard g(ctx->device);
    const StageRec &r = ctx->ring[(ctx->runs - 1 - back) % kStageRing];
    *n_stages = (uint32_t)r.n;
    if ((uint32_t)r.n > cap) return fail(ctx, CROP_E_CAPACITY, "stage capacity too small");
    CK(hipEventSynchronize(r.ev[r.n]));
    for (int k = 0; k < r.n; ++k) {
        if (names) names[k] = r.names[k];
        if (ms) CK(hipEventElapsedTime(&ms[k], r.ev[k], r.ev[k + 1]));
    }
    return CROP_OK;
}

crop_status crop_get_tuning(const crop_ctx *ctx, crop_tune *out)
{
    if (!ctx || !out) return CROP_E_ARG;
    out->bins_per_partition = ctx->plan.S;
    out->rows_per_chunk = ctx->plan.R;
    out->stage_keys = ctx->plan.stage_cap;
    out->route = ctx->plan.regions ? CROP_ROUTE_REGIONS
                 : ctx->plan.n_wg      ? CROP_ROUTE_RANGES
                                       : CROP_ROUTE_CHUNKS;
    out->window = ctx->plan.win_kb ? CROP_WINDOW_AUTO : CROP_WINDOW_OFF;
    out->region_terms = ctx->plan.regions ? ctx->sb.max_terms : 0;
    return CROP_OK;
}

// ============================================================== input

crop_status crop_load_transactions(crop_ctx *ctx, const uint32_t *off, uint64_t T,
                                   const uint32_t *items, uint64_t nnz, uint32_t n_items,
                                   crop_mem where, crop_own own)
{
    if (!ctx) return CROP_E_ARG;
    if (!off || (nnz && !items)) return fail(ctx, CROP_E_ARG, "null input pointer");
    if (T >= (1ull << 32) || nnz >= (1ull << 32))
        return fail(ctx, CROP_E_UNSUPPORTED, "T and nnz must be below 2^32");
    if (own == CROP_OWN_BORROW && where != CROP_MEM_DEVICE)
        return fail(ctx, CROP_E_ARG, "only device buffers can be borrowed");
    DeviceGuard g(ctx->device);
    reset_input(ctx);
    ctx->err_index = -1;
    Input &in = ctx->in;
    CK(fetch(in.h_off, off, T + 1, where));
    crop_status st = check_offsets(ctx, in.h_off, nnz, "transactions");
    if (st != CROP_OK) return st;
    in.total_terms = tx_terms_of(in.h_off);
    if (in.total_terms >= (1ull << 32))
        return fail(ctx, CROP_E_UNSUPPORTED, "more than 2^32 - 1 terms in one run");
    CK(place(off, T + 1, where, own, in.own[0], &in.off, ctx->stream));
    CK(place(items, nnz, where, own, in.own[1], &in.items, ctx->stream));
    int64_t bad = -1;
    st = validate_on_device(ctx, in.off, T, in.items, nnz, n_items, &bad);
    if (st != CROP_OK) return st;
    if (bad >= 0) {
        ctx->err_index = bad;
        return fail(ctx, CROP_E_INPUT,
                    "transaction " + std::to_string(bad) +
                        ": item id out of range or items not strictly increasing");
    }
    in.T = T;
    in.nnz = nnz;
    in.n_items = n_items;
    in.wide_keys = n_items > 65536u;
    in.mode = Mode::Tx;
    return CROP_OK;
}

crop_status crop_load_outer(crop_ctx *ctx, const uint32_t *a_off, const uint32_t *a_idx,
                            const float *a_val, const uint32_t *b_off, const uint32_t *b_idx,
                            const float *b_val, uint64_t K, uint64_t nnz_a, uint64_t nnz_b,
                            uint32_t n_rows, uint32_t n_cols, crop_mem where, crop_own own)
{
    if (!ctx) return CROP_E_ARG;
    if (!a_off || !b_off || (nnz_a && (!a_idx || !a_val)) || (nnz_b && (!b_idx || !b_val)))
        return fail(ctx, CROP_E_ARG, "null input pointer");
    if (K >= (1ull << 32) || nnz_a >= (1ull << 32) || nnz_b >= (1ull << 32))
        return fail(ctx, CROP_E_UNSUPPORTED, "K and nnz must be below 2^32");
    if (own == CROP_OWN_BORROW && where != CROP_MEM_DEVICE)
        return fail(ctx, CROP_E_ARG, "only device buffers can be borrowed");
    DeviceGuard g(ctx->device);
    reset_input(ctx);
    ctx->err_index = -1;
    Input &in = ctx->in;
    CK(fetch(in.h_off, a_off, K + 1, where));
    CK(fetch(in.h_b_off, b_off, K + 1, where));
    crop_status st = check_offsets(ctx, in.h_off, nnz_a, "a vectors");
    if (st != CROP_OK) return st;
    st = check_offsets(ctx, in.h_b_off, nnz_b, "b vectors");
    if (st != CROP_OK) return st;
    uint64_t terms = 0;
    for (uint64_t k = 0; k < K; ++k)
        terms += (uint64_t)(in.h_off[k + 1] - in.h_off[k]) * (in.h_b_off[k + 1] - in.h_b_off[k]);
    if (terms >= (1ull << 32))
        return fail(ctx, CROP_E_UNSUPPORTED, "more than 2^32 - 1 terms in one run");
    in.total_terms = terms;
    CK(place(a_off, K + 1, where, own, in.own[0], &in.a_off, ctx->stream));
    CK(place(a_idx, nnz_a, where, own, in.own[1], &in.a_idx, ctx->stream));
    CK(place(a_val, nnz_a, where, own, in.own[2], &in.a_val, ctx->stream));
    CK(place(b_off, K + 1, where, own, in.own[3], &in.b_off, ctx->stream));
    CK(place(b_idx, nnz_b, where, own, in.own[4], &in.b_idx, ctx->stream));
    CK(place(b_val, nnz_b, where, own, in.own[5], &in.b_val, ctx->stream));
    int64_t bad = -1;
    st = validate_on_device(ctx, in.a_off, K, in.a_idx, nnz_a, n_rows, &bad);
    if (st != CROP_OK) return st;
    if (bad < 0) {
        st = validate_on_device(ctx, in.b_off, K, in.b_idx, nnz_b, n_cols, &bad);
        if (st != CROP_OK) return st;
    }
    if (bad >= 0) {
        ctx->err_index = bad;
        return fail(ctx, CROP_E_INPUT,
                    "vector pair " + std::to_string(bad) +
                        ": index out of range or indices not strictly increasing");
    }
    in.K = K;
    in.nnz_a = nnz_a;
    in.nnz_b = nnz_b;
    in.n_rows = n_rows;
    in.n_cols = n_cols;
    in.wide_keys = true;
    build_outer_chunks(in);
    CK(in.d_op_chunks.ensure(std::max<size_t>(1, in.op_chunks.size()) * sizeof(OpChunk)));
    if (!in.op_chunks.empty())
        CK(hipMemcpy(in.d_op_chunks.p, in.op_chunks.data(), in.op_chunks.size() * sizeof(OpChunk),
                     hipMemcpyHostToDevice));
    in.mode = Mode::Outer;
    return CROP_OK;
}

// ============================================================== runs

crop_status crop_run_exact(crop_ctx *ctx)
{
    if (!ctx) return CROP_E_ARG;
    if (ctx->in.mode == Mode::None) return fail(ctx, CROP_E_STATE, "no input loaded");
    if (ctx->in.mode == Mode::Batch)
        return fail(ctx, CROP_E_STATE, "a batch is loaded: use crop_run_exact_batched");
    DeviceGuard g(ctx->device);
    ctx->result = Result::None;
    const bool outer = ctx->in.mode == Mode::Outer;
    bool regions = false;
    crop_status st = outer ? plan_outer(ctx) : plan_regions(ctx, &regions);
    if (st != CROP_OK) return st;
    if (!outer && !regions) {
        st = plan_tx(ctx);
        if (st != CROP_OK) return st;
    }
    ctx->plan.log2_slots = (outer || ctx->in.wide_keys) ? 13 : 14;
    ctx->plan.BS = 256;
    st = ensure_route_buffers(ctx, ctx->in.wide_keys ? 8 : 4, outer);
    if (st == CROP_OK && regions) st = ensure_region_buffers(ctx);
    if (st != CROP_OK) return st;
    const RoutePlan &pl = ctx->plan;
    hipStream_t s = ctx->stream;
    uint32_t *cnt = ctx->cnt_mat.as<uint32_t>();
    st = run_begin(ctx);
    if (st != CROP_OK) return st;
    if (regions) {
        if (ctx->sb.n_sub) CK(launch_sb_route(ctx, s));
        STAGE("route");
        CK(launch_sb_headers(ctx, s));
        // one ordered range of bins and one bin counter (cleared) per XCD
        CK(launch_bin_order(pl.NB, ctx->bin_off.as<uint32_t>(), ctx->bin_order.as<uint32_t>(),
                            s, crop::kNumXcd, ctx->counter.as<uint32_t>(), crop::kNumXcd));
        STAGE("headers");
    } else {
        if (pl.n_chunks) CK(outer ? launch_op_count(ctx, cnt, s)
                                  : pl.n_wg ? launch_tx_count_ranges(ctx, cnt, s)
                                  : pl.win_kb ? launch_tx_count_win(ctx, cnt, s)
                                            : launch_tx_count(ctx, cnt, s));
        STAGE("count");
        CK(launch_scan_counts(cnt, pl.n_wg ? pl.n_wg : pl.n_chunks, pl.NB, pl.G,
                              ctx->part_buf.as<uint32_t>(),
                              ctx->bin_off.as<uint32_t>(), ctx->counter.as<uint32_t>(), s));
        CK(launch_bin_order(pl.NB, ctx->bin_off.as<uint32_t>(), ctx->bin_order.as<uint32_t>(),
                            s));
        STAGE("scan");
        if (pl.n_chunks)
            CK(outer ? launch_op_scatter(ctx, cnt, ctx->keys.p, ctx->vals.as<float>(), s)
                     : pl.n_wg ? launch_tx_scatter_ranges(ctx, cnt, ctx->keys.p, s)
                     : pl.win_kb ? launch_tx_scatter_win(ctx, cnt, ctx->keys.p, s)
                               : launch_tx_scatter(ctx, cnt, ctx->keys.p, s));
        STAGE("scatter");
    }
    // grouped bins: per-partition terms from the routed keys (outer products;
    // for transactions they are the sums of the supports, taken below)
    uint32_t *ps_n = ctx->part_stats.as<uint32_t>(), *ps_w = ps_n + (pl.g ? ctx->P : 0);
    if (pl.g) {
        CK(launch_zero32(ps_n, 2 * ctx->P, s));
        if (outer) CK(launch_part_stats(ctx, true, ps_w, nullptr, s));
    }
    CK(outer     ? launch_aggregate_sums(ctx, s)
       : regions ? launch_aggregate_regions(ctx, s)
                 : launch_aggregate_counts(ctx, s));
    STAGE("aggregate");
    if (pl.g) {
        CK(launch_part_stats(ctx, false, ps_n, outer ? nullptr : ps_w, s));
        STAGE("partitions");
    }
    st = run_end(ctx);
    if (st != CROP_OK) return st;
    ctx->result = Result::Exact;
    return CROP_OK;
}

// One top-K run: t = 1 is a single CRoP instance (optionally seeded); t > 1
// runs t instances with the hash functions of seed, seed + 1, ..., each into
// its own summaries, and reports the entries monitored by at least
// min_votes of them.
static crop_status run_topk_impl(crop_ctx *ctx, uint32_t K, const uint32_t *sx,
                                 const uint32_t *sy, uint64_t ns, uint32_t r_max,
                                 uint32_t t = 1, uint32_t min_votes = 1)
{
    if (!ctx) return CROP_E_ARG;
    if (ctx->in.mode == Mode::None) return fail(ctx, CROP_E_STATE, "no input loaded");
    if (ctx->in.mode == Mode::Batch)
        return fail(ctx, CROP_E_UNSUPPORTED, "top-K runs take one stream, not a batch");
    if (ctx->own_p0 || ctx->own_p1)
        return fail(ctx, CROP_E_UNSUPPORTED, "owned partitions apply to exact runs");
    if (K == 0) return fail(ctx, CROP_E_ARG, "K must be positive");
    if (ns && (!sx || !sy)) return fail(ctx, CROP_E_ARG, "null seed arrays");
    if (ns >= (1ull << 31)) return fail(ctx, CROP_E_UNSUPPORTED, "too many seeds");
    if (ns && ctx->in.mode != Mode::Tx)
        return fail(ctx, CROP_E_UNSUPPORTED, "seeding is defined for transaction streams");
    if (ns && r_max >= ctx->ss_ell)
        return fail(ctx, CROP_E_ARG, "r_max must be below the slots per bucket");
    DeviceGuard g(ctx->device);
    ctx->result = Result::None;
    if (ns) {
        // a seed must be a pair the stream can hold: a key outside x < y <
        // n_items would be pinned where no term ever reaches it
        int64_t bad = -1;
        crop_status cs = check_pairs_on_device(ctx, sx, sy, ns, ctx->in.n_items, &bad);
        if (cs != CROP_OK) return cs;
        if (bad >= 0) {
            ctx->err_index = bad;
            return fail(ctx, CROP_E_INPUT,
                        "seed " + std::to_string(bad) + ": need x < y < n_items");
        }
    }
    uint32_t nbk = 0;
    uint64_t PB = 0;
    int g_ss = -1;
    crop_status st = plan_ss(ctx, &nbk, &PB, &g_ss);
    if (st != CROP_OK) return st;
    const uint32_t S = g_ss < 0 ? (uint32_t)(PB / ctx->P / nbk) : 1u;
    const bool outer = ctx->in.mode == Mode::Outer;
    st = outer ? plan_outer(ctx, S, g_ss) : plan_tx(ctx, S, g_ss);
    if (st != CROP_OK) return st;
    if (g_ss >= 0 && ctx->plan.g != (uint32_t)g_ss)
        return fail(ctx, CROP_E_UNSUPPORTED, "Space-Saving bins do not match the routing bins");
    ctx->plan.log2_slots = 0;
    ctx->plan.BS = 256;
    st = ensure_route_buffers(ctx, ctx->in.wide_keys ? 8 : 4, outer);
    if (st != CROP_OK) return st;
    // grouped bins: the state covers whole bins (the last one may be partial)
    const uint64_t nslots = (g_ss < 0 ? PB : (uint64_t)ctx->plan.NB * nbk) * ctx->ss_ell;
    if (nslots * t >= (1ull << 32))
        return fail(ctx, CROP_E_UNSUPPORTED, "more than 2^32 summary slots");
    st = ensure_ss_buffers(ctx, nslots * t, K, (uint32_t)ns);
    if (st != CROP_OK) return st;
    SsState amp{};
    uint8_t *votes = nullptr;
    if (t > 1) {
        st = ensure_amp_buffers(ctx, nslots * t, &amp, &votes);
        if (st != CROP_OK) return st;
    }
    const TopkViews tv = topk_views(ctx, K);
    const RoutePlan &pl = ctx->plan;
    hipStream_t s = ctx->stream;
    uint32_t *cnt = ctx->cnt_mat.as<uint32_t>();
    CsParams ip{};
    ip.t = t;
    ip.PB = PB;
    for (uint32_t i = 0; i < t; ++i) ip.hp[i] = make_hash_params(ctx->seed + i);
    st = run_begin(ctx);
    if (st != CROP_OK) return st;
    // without seeds the summary kernel starts every bin empty and writes
    // every slot, so the state needs no clearing; pinned seeds go into
    // cleared state, which the kernel then reads
    if (ns) CK(launch_ss_clear(ctx->ss, s));
    CK(launch_zero32(tv.st, 8 + 256 + 1, s));
    if (ns)
        CK(launch_ss_pin(ctx->ss, sx, sy, (uint32_t)ns, tv.dup, r_max, ctx->hp, PB, ctx->ss_ell,
                         tv.n_pinned, s));
    STAGE("init");
    // instance i routes and summarises with its own hash functions; the
    // kernels take the parameters by value at launch
    HashGuard hg(ctx);
    for (uint32_t i = 0; i < t; ++i) {
        ctx->hp = ip.hp[i];
        SsState Si = ctx->ss;
        Si.key += i * nslots;
        Si.cnt += i * nslots;
        Si.err += i * nslots;
        Si.val += i * nslots;
        Si.flag += i * nslots;
        Si.nslots = nslots;
        const bool narrow = !outer && !ctx->in.wide_keys;
        Si.key32 = (t > 1 && narrow) ? amp.key32 + i * nslots : nullptr;
        if (pl.n_chunks) CK(outer ? launch_op_count(ctx, cnt, s)
                                  : pl.n_wg ? launch_tx_count_ranges(ctx, cnt, s)
                                            : launch_tx_count(ctx, cnt, s));
        if (i == 0) STAGE("count");
        CK(launch_scan_counts(cnt, pl.n_wg ? pl.n_wg : pl.n_chunks, pl.NB, pl.G,
                              ctx->part_buf.as<uint32_t>(),
                              ctx->bin_off.as<uint32_t>(), ctx->counter.as<uint32_t>(), s));
        CK(launch_bin_order(pl.NB, ctx->bin_off.as<uint32_t>(), ctx->bin_order.as<uint32_t>(),
                            s));
        if (i == 0) STAGE("scan");
        if (pl.n_chunks)
            CK(outer ? launch_op_scatter(ctx, cnt, ctx->keys.p, ctx->vals.as<float>(), s)
                     : pl.n_wg ? launch_tx_scatter_ranges(ctx, cnt, ctx->keys.p, s)
                               : launch_tx_scatter(ctx, cnt, ctx->keys.p, s));
        if (i == 0) STAGE("scatter");
        CK(launch_ss_bins(ctx, Si, nbk, PB, s, ns == 0));
        if (i == 0) STAGE("summaries");
    }
    ctx->hp = hg.saved;
    const bool by_lower = ctx->topk_rank == CROP_RANK_LOWER;
    if (t > 1) {
        SsState S = ctx->ss;
        S.key32 = amp.key32;
        CK(launch_amp_combine(ip, S, ctx->ss_ell, nslots, min_votes, outer,
                              !outer && !ctx->in.wide_keys, amp, votes, s));
        STAGE("majority");
        CK(launch_topk(amp, K, outer, by_lower, true, votes, tv.st, tv.hist, tv.cand, tv.sel,
                       tv.rank, tv.oi, tv.oj, tv.ou, tv.ol, tv.ov, tv.ovotes, s));
    } else {
        CK(launch_topk(ctx->ss, K, outer, by_lower, false, nullptr, tv.st, tv.hist, tv.cand,
                       tv.sel, tv.rank, tv.oi, tv.oj, tv.ou, tv.ol, tv.ov, tv.ovotes, s));
    }
    STAGE("topk");
    st = run_end(ctx);
    if (st != CROP_OK) return st;
    ctx->result = Result::TopK;
    ctx->topk_K = K;
    ctx->ss_buckets = PB;
    ctx->topk_outer = outer ? 1 : 0;
    ctx->topk_instances = t;
    return CROP_OK;
}

crop_status crop_run_topk(crop_ctx *ctx, uint32_t K)
{
    return run_topk_impl(ctx, K, nullptr, nullptr, 0, 0);
}

crop_status crop_run_topk_seeded(crop_ctx *ctx, uint32_t K, const uint32_t *sx,
                                 const uint32_t *sy, uint64_t ns, uint32_t r_max)
{
    return run_topk_impl(ctx, K, sx, sy, ns, r_max);
}

crop_status crop_run_topk_amplified(crop_ctx *ctx, uint32_t K, uint32_t instances,
                                    uint32_t min_votes)
{
    if (!ctx) return CROP_E_ARG;
    if (instances < 1 || instances > kCsMaxInstances)
        return fail(ctx, CROP_E_ARG, "instances must be 1..15");
    if (min_votes < 1 || min_votes > instances)
        return fail(ctx, CROP_E_ARG, "min_votes must be 1..instances");
    return run_topk_impl(ctx, K, nullptr, nullptr, 0, 0, instances, min_votes);
}

crop_status crop_read_topk_votes(crop_ctx *ctx, uint32_t *votes, uint64_t cap, uint64_t *written)
{
    if (!ctx || !votes) return CROP_E_ARG;
    if (ctx->result != Result::TopK) return fail(ctx, CROP_E_STATE, "no top-K result");
    DeviceGuard g(ctx->device);
    const TopkViews tv = topk_views(ctx, ctx->topk_K);
    uint32_t stv[8];
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(stv, tv.st, sizeof(stv), hipMemcpyDeviceToHost));
    const uint64_t n = stv[5];
    if (written) *written = n;
    if (n > cap) return fail(ctx, CROP_E_CAPACITY, "output capacity below K");
    if (n) CK(hipMemcpy(votes, tv.ovotes, n * 4, hipMemcpyDeviceToHost));
    return CROP_OK;
}

crop_status crop_read_topk(crop_ctx *ctx, uint32_t *i, uint32_t *j, double *upper,
                           double *lower, double *value, uint64_t cap, uint64_t *written)
{
    if (!ctx || !i || !j) return CROP_E_ARG;
    if (ctx->result != Result::TopK) return fail(ctx, CROP_E_STATE, "no top-K result");
    DeviceGuard g(ctx->device);
    const TopkViews tv = topk_views(ctx, ctx->topk_K);
    uint32_t stv[8];
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(stv, tv.st, sizeof(stv), hipMemcpyDeviceToHost));
    const uint64_t n = stv[5];
    if (written) *written = n;
    if (n > cap) return fail(ctx, CROP_E_CAPACITY, "output capacity below K");
    if (!n) return CROP_OK;
    CK(hipMemcpy(i, tv.oi, n * 4, hipMemcpyDeviceToHost));
    CK(hipMemcpy(j, tv.oj, n * 4, hipMemcpyDeviceToHost));
    if (upper) CK(hipMemcpy(upper, tv.ou, n * 8, hipMemcpyDeviceToHost));
    if (lower) CK(hipMemcpy(lower, tv.ol, n * 8, hipMemcpyDeviceToHost));
    if (value) CK(hipMemcpy(value, tv.ov, n * 8, hipMemcpyDeviceToHost));
    return CROP_OK;
}

crop_status crop_read_summary(crop_ctx *ctx, uint32_t *i, uint32_t *j, double *cnt, double *err,
                              double *value, uint8_t *flags, uint64_t cap, uint64_t *written)
{
    if (!ctx || !i || !j) return CROP_E_ARG;
    if (ctx->result != Result::TopK) return fail(ctx, CROP_E_STATE, "no top-K result");
    DeviceGuard g(ctx->device);
    const uint64_t n = ctx->ss.nslots;
    if (written) *written = n;
    if (n > cap) return fail(ctx, CROP_E_CAPACITY, "output capacity below the slot count");
    CK(hipStreamSynchronize(ctx->stream));
    std::vector<uint64_t> k(n);
    std::vector<uint32_t> c(n), e(n);
    std::vector<float> v(n);
    std::vector<uint8_t> f(n);
    CK(hipMemcpy(k.data(), ctx->ss.key, n * 8, hipMemcpyDeviceToHost));
    CK(hipMemcpy(c.data(), ctx->ss.cnt, n * 4, hipMemcpyDeviceToHost));
    CK(hipMemcpy(e.data(), ctx->ss.err, n * 4, hipMemcpyDeviceToHost));
    CK(hipMemcpy(v.data(), ctx->ss.val, n * 4, hipMemcpyDeviceToHost));
    CK(hipMemcpy(f.data(), ctx->ss.flag, n, hipMemcpyDeviceToHost));
    const bool outer = ctx->topk_outer != 0;
    for (uint64_t q = 0; q < n; ++q) {
        i[q] = (uint32_t)(k[q] >> 32);
        j[q] = (uint32_t)k[q];
        float fc, fe;
        std::memcpy(&fc, &c[q], 4);
        std::memcpy(&fe, &e[q], 4);
        if (cnt) cnt[q] = outer ? (double)fc : (double)c[q];
        if (err) err[q] = outer ? (double)fe : (double)e[q];
        if (value) value[q] = outer ? (double)v[q] : 0.0;
        if (flags) flags[q] = f[q];
    }
    return CROP_OK;
}

// ============================================================== Count-Sketch

crop_status crop_run_countsketch(crop_ctx *ctx, uint32_t buckets_per_partition,
                                 uint32_t instances)
{
    if (!ctx) return CROP_E_ARG;
    if (ctx->in.mode == Mode::None) return fail(ctx, CROP_E_STATE, "no input loaded");
    if (ctx->in.mode == Mode::Batch)
        return fail(ctx, CROP_E_UNSUPPORTED, "Count-Sketch runs take one stream, not a batch");
    if (ctx->own_p0 || ctx->own_p1)
        return fail(ctx, CROP_E_UNSUPPORTED, "owned partitions apply to exact runs");
    if (instances < 1 || instances > kCsMaxInstances)
        return fail(ctx, CROP_E_ARG, "instances must be 1..15");
    if (buckets_per_partition < 1) return fail(ctx, CROP_E_ARG, "need at least one bucket");
    const uint64_t PB = (uint64_t)ctx->P * buckets_per_partition;
    if (PB > (1ull << 32))
        return fail(ctx, CROP_E_UNSUPPORTED, "P x buckets per partition exceeds 2^32");
    if (PB * instances > (1ull << 34))
        return fail(ctx, CROP_E_UNSUPPORTED, "Count-Sketch counters exceed 64 GiB");
    DeviceGuard g(ctx->device);
    ctx->result = Result::None;
    const bool outer = ctx->in.mode == Mode::Outer;
    // Routed when the partition's buckets split into S bins (S divides B)
    // that give at least kCsMinBins bins of at most kCsMaxBinBuckets
    // buckets each; S is the divisor closest to the exact path's terms per
    // bin (the largest at or below it, else the smallest above).
    const uint32_t B = buckets_per_partition;
    const uint64_t per_bin = outer ? kTermsPerBin / 16 : kTermsPerBin;
    const uint64_t want =
        std::max<uint64_t>(1, (ctx->in.total_terms + per_bin - 1) / per_bin / ctx->P);
    uint32_t S = 0;
    for (uint64_t d = 1; d * d <= B; ++d) {
        if (B % d) continue;
        for (uint64_t c : {d, (uint64_t)B / d}) {
            if ((uint64_t)ctx->P * c > kMaxP || B / c > kCsMaxBinBuckets) continue;
            const bool better = S == 0 || (c <= want ? (S > want || c > S) : (S > want && c < S));
            if (better) S = (uint32_t)c;
        }
    }
    bool routed = S != 0 && (uint64_t)ctx->P * S >= std::min<uint64_t>(kCsMinBins, PB);
    // bins_per_partition of crop_set_tuning, when it divides B, forces the
    // routed form with that many bins per partition
    const uint32_t St = ctx->tune.bins_per_partition;
    if (St && B % St == 0 && (uint64_t)ctx->P * St <= kMaxP && B / St <= kCsMaxBinBuckets) {
        S = St;
        routed = true;
    }
    crop_status st = outer ? plan_outer(ctx, routed ? S : 0) : plan_tx(ctx, routed ? S : 0);
    if (st != CROP_OK) return st;
    if (routed) {
        ctx->plan.log2_slots = 0;
        ctx->plan.BS = 256;
        st = ensure_route_buffers(ctx, ctx->in.wide_keys || outer ? 8 : 4, outer);
        if (st != CROP_OK) return st;
    }
    CsParams &cp = ctx->cs;
    cp.t = instances;
    cp.PB = PB;
    for (uint32_t i = 0; i < instances; ++i) cp.hp[i] = make_hash_params(ctx->seed + i);
    ctx->cs_B = buckets_per_partition;
    const uint64_t words = PB * instances;
    CK(ctx->cs_buf.ensure(words * 4));
    hipStream_t s = ctx->stream;
    st = run_begin(ctx);
    if (st != CROP_OK) return st;
    if (routed) {
        const RoutePlan &pl = ctx->plan;
        uint32_t *cnt = ctx->cnt_mat.as<uint32_t>();
        HashGuard hg(ctx);
        for (uint32_t i = 0; i < instances; ++i) {
            ctx->hp = cp.hp[i];  // routing by this instance's hash
            if (pl.n_chunks) CK(outer ? launch_op_count(ctx, cnt, s)
                                      : pl.n_wg ? launch_tx_count_ranges(ctx, cnt, s)
                                                : launch_tx_count(ctx, cnt, s));
            CK(launch_scan_counts(cnt, pl.n_wg ? pl.n_wg : pl.n_chunks, pl.NB, pl.G,
                                  ctx->part_buf.as<uint32_t>(), ctx->bin_off.as<uint32_t>(),
                                  ctx->counter.as<uint32_t>(), s));
            if (pl.n_chunks)
                CK(outer ? launch_op_scatter(ctx, cnt, ctx->keys.p, ctx->vals.as<float>(), s)
                         : pl.n_wg ? launch_tx_scatter_ranges(ctx, cnt, ctx->keys.p, s)
                                   : launch_tx_scatter(ctx, cnt, ctx->keys.p, s));
            CK(launch_cs_bins(ctx, cp.hp[i], PB, B / S, ctx->cs_buf.as<uint32_t>() + i * PB, s));
        }
        STAGE("sketch");
    } else {
        CK(launch_cs_clear(ctx->cs_buf.p, words, s));
        STAGE("clear");
        if (outer)
            CK(launch_cs_op(ctx, cp, ctx->cs_buf.as<float>(), s));
        else
            CK(launch_cs_tx(ctx, cp, ctx->cs_buf.as<int32_t>(), s));
        STAGE("sketch");
    }
    ctx->cs_routed = routed ? 1u : 0u;
    st = run_end(ctx);
    if (st != CROP_OK) return st;
    ctx->result = Result::CountSketch;
    ctx->topk_outer = outer ? 1u : 0u;
    return CROP_OK;
}

crop_status crop_countsketch_estimate(crop_ctx *ctx, const uint32_t *qx, const uint32_t *qy,
                                      uint64_t n, double *est)
{
    if (!ctx || (n && (!qx || !qy || !est))) return CROP_E_ARG;
    if (ctx->result != Result::CountSketch)
        return fail(ctx, CROP_E_STATE, "no Count-Sketch: call crop_run_countsketch first");
    DeviceGuard g(ctx->device);
    CK(launch_cs_estimate(ctx->cs, ctx->cs_buf.p, ctx->topk_outer != 0, qx, qy, n, est,
                          ctx->stream));
    return CROP_OK;
}

crop_status crop_read_countsketch(crop_ctx *ctx, uint32_t instance, double *out, uint64_t cap)
{
    if (!ctx || !out) return CROP_E_ARG;
    if (ctx->result != Result::CountSketch)
        return fail(ctx, CROP_E_STATE, "no Count-Sketch: call crop_run_countsketch first");
    if (instance >= ctx->cs.t) return fail(ctx, CROP_E_ARG, "instance out of range");
    const uint64_t PB = ctx->cs.PB;
    if (cap < PB) return fail(ctx, CROP_E_CAPACITY, "capacity below P x buckets");
    DeviceGuard g(ctx->device);
    std::vector<uint32_t> raw(PB);
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(raw.data(), ctx->cs_buf.as<uint32_t>() + instance * PB, PB * 4,
                 hipMemcpyDeviceToHost));
    for (uint64_t k = 0; k < PB; ++k) {
        if (ctx->topk_outer) {
            float f;
            std::memcpy(&f, &raw[k], 4);
            out[k] = f;
        } else {
            out[k] = (double)(int32_t)raw[k];
        }
    }
    return CROP_OK;
}

// ============================================================== learned seeding

static crop_status require_tx(crop_ctx *ctx)
{
    if (ctx->in.mode != Mode::Tx) return fail(ctx, CROP_E_STATE, "no transaction stream loaded");
    return CROP_OK;
}

static crop_status stats_workspace(crop_ctx *ctx, uint32_t prefix_T)
{
    const uint32_t n = ctx->in.n_items;
    const size_t words = item_stats_words(n, prefix_T);
    CK(ctx->learn_ws.ensure(words * 4 + 4096));
    CK(launch_zero32(ctx->learn_ws.as<uint32_t>(), (uint32_t)words, ctx->stream));
    return CROP_OK;
}

crop_status crop_item_features(crop_ctx *ctx, uint32_t prefix_T, float *feat)
{
    if (!ctx || !feat) return CROP_E_ARG;
    crop_status st = require_tx(ctx);
    if (st != CROP_OK) return st;
    if (prefix_T > ctx->in.T) return fail(ctx, CROP_E_ARG, "prefix longer than the stream");
    DeviceGuard g(ctx->device);
    st = stats_workspace(ctx, prefix_T);
    if (st != CROP_OK) return st;
    CK(launch_item_features(ctx->in.off, ctx->in.items, ctx->in.n_items, prefix_T,
                            ctx->learn_ws.as<uint32_t>(), feat, ctx->stream));
    return CROP_OK;
}

crop_status crop_top_item_pairs(crop_ctx *ctx, uint32_t prefix_T, uint32_t M, uint32_t *cx,
                                uint32_t *cy, uint64_t cap, uint64_t *n_pairs)
{
    if (!ctx || !cx || !cy) return CROP_E_ARG;
    crop_status st = require_tx(ctx);
    if (st != CROP_OK) return st;
    if (prefix_T > ctx->in.T) return fail(ctx, CROP_E_ARG, "prefix longer than the stream");
    if (M < 2 || M > ctx->in.n_items) return fail(ctx, CROP_E_ARG, "need 2 <= M <= n_items");
    const uint64_t np = (uint64_t)M * (M - 1) / 2;
    if (n_pairs) *n_pairs = np;
    if (np > cap) return fail(ctx, CROP_E_CAPACITY, "pair capacity below M(M-1)/2");
    DeviceGuard g(ctx->device);
    st = stats_workspace(ctx, prefix_T);
    if (st != CROP_OK) return st;
    CK(ctx->scratch.ensure((size_t)M * 4 + 256));
    uint32_t *ws = ctx->learn_ws.as<uint32_t>();
    CK(launch_item_features(ctx->in.off, ctx->in.items, ctx->in.n_items, prefix_T, ws, nullptr,
                            ctx->stream));
    CK(launch_top_pairs(ws, ctx->in.n_items, prefix_T, M, ctx->scratch.as<uint32_t>(), cx, cy,
                        ctx->stream));
    return CROP_OK;
}

crop_status crop_lookup_exact(crop_ctx *ctx, const uint32_t *qx, const uint32_t *qy, uint64_t n,
                              uint32_t *count)
{
    if (!ctx || (n && (!qx || !qy || !count))) return CROP_E_ARG;
    if (n > (1ull << 30)) return fail(ctx, CROP_E_UNSUPPORTED, "at most 2^30 queries per call");
    crop_status st = require_exact(ctx);
    if (st != CROP_OK) return st;
    st = require_tx(ctx);
    if (st != CROP_OK) return st;
    DeviceGuard g(ctx->device);
    CK(launch_lookup(ctx, qx, qy, n, count, ctx->stream));
    return CROP_OK;
}

crop_status crop_pair_inputs(crop_ctx *ctx, const float *feat, const uint32_t *cx,
                             const uint32_t *cy, const uint32_t *count, uint64_t n, float *Z,
                             float *y)
{
    if (!ctx || (n && (!feat || !cx || !cy || !Z))) return CROP_E_ARG;
    if (y && !count) return fail(ctx, CROP_E_ARG, "labels need counts");
    DeviceGuard g(ctx->device);
    CK(launch_pair_inputs(feat, cx, cy, count, n, Z, y, ctx->stream));
    return CROP_OK;
}

crop_status crop_mlp_create(crop_ctx *ctx, const float *init, crop_mlp **out)
{
    if (!ctx || !init || !out) return CROP_E_ARG;
    *out = nullptr;
    DeviceGuard g(ctx->device);
    crop_mlp *m = new (std::nothrow) crop_mlp();
    if (!m) return CROP_E_NOMEM;
    m->device = ctx->device;
    const size_t nb = (size_t)mlp_param_count() * 4;
    hipError_t e = hipSuccess;
    for (DevBuf *b : {&m->params, &m->m, &m->v, &m->gstage})
        if (e == hipSuccess) e = b->ensure(nb);
    if (e == hipSuccess) e = m->loss.ensure(256);
    if (e == hipSuccess) e = hipMemcpy(m->params.p, init, nb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_zero32(m->m.as<uint32_t>(), mlp_param_count(), ctx->stream);
    if (e == hipSuccess) e = launch_zero32(m->v.as<uint32_t>(), mlp_param_count(), ctx->stream);
    if (e == hipSuccess) e = launch_zero32(m->loss.as<uint32_t>(), 64, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        crop_mlp_destroy(m);
        return hip_fail(ctx, e, "crop_mlp_create");
    }
    *out = m;
    return CROP_OK;
}

void crop_mlp_destroy(crop_mlp *m)
{
    if (!m) return;
    DeviceGuard g(m->device);
    for (DevBuf *b : {&m->params, &m->m, &m->v, &m->gstage, &m->loss}) b->release();
    delete m;
}

crop_status crop_mlp_params(crop_ctx *ctx, const crop_mlp *m, float *out)
{
    if (!ctx || !m || !out) return CROP_E_ARG;
    DeviceGuard g(ctx->device);
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(out, m->params.p, (size_t)mlp_param_count() * 4, hipMemcpyDeviceToHost));
    return CROP_OK;
}

crop_status crop_mlp_grad(crop_ctx *ctx, crop_mlp *m, const float *Z, const float *y, uint32_t N,
                          float *grad, float *loss)
{
    if (!ctx || !m || !Z || !y || !grad) return CROP_E_ARG;
    if (N < 1 || N > (uint32_t)mlp_batch_max())
        return fail(ctx, CROP_E_ARG, "gradient batch must hold 1..128 samples");
    DeviceGuard g(ctx->device);
    CK(launch_mlp_grad(m->params.as<float>(), Z, y, N, m->gstage.as<float>(),
                       m->loss.as<float>(), ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(grad, m->gstage.p, (size_t)mlp_param_count() * 4, hipMemcpyDeviceToHost));
    if (loss) CK(hipMemcpy(loss, m->loss.p, 4, hipMemcpyDeviceToHost));
    return CROP_OK;
}

crop_status crop_mlp_train(crop_ctx *ctx, crop_mlp *m, const float *Z, const float *y,
                           uint64_t n_samples, const uint32_t *order, uint64_t n_order,
                           uint32_t batch, float lr)
{
    if (!ctx || !m || !Z || !y || !order) return CROP_E_ARG;
    if (batch < 1 || batch > (uint32_t)mlp_batch_max())
        return fail(ctx, CROP_E_ARG, "batch must hold 1..128 samples");
    DeviceGuard g(ctx->device);
    const uint64_t steps = n_order / batch;
    if (!steps) return CROP_OK;
    // every sample index is checked before the training kernel reads Z and y
    CK(launch_zero32(m->loss.as<uint32_t>() + 1, 1, ctx->stream));
    CK(launch_max_index(order, steps * batch, m->loss.as<uint32_t>() + 1, ctx->stream));
    uint32_t mx = 0;
    CK(hipMemcpyAsync(&mx, m->loss.as<uint32_t>() + 1, 4, hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    if (mx >= n_samples) return fail(ctx, CROP_E_INPUT, "sample index beyond n_samples");
    CK(launch_mlp_train(m->params.as<float>(), m->m.as<float>(), m->v.as<float>(),
                        m->gstage.as<float>(), Z, y, order, steps * batch, batch, lr, m->t,
                        m->loss.as<float>(), ctx->stream));
    m->t += steps;
    return CROP_OK;
}

crop_status crop_mlp_loss(crop_ctx *ctx, const crop_mlp *m, float *loss)
{
    if (!ctx || !m || !loss) return CROP_E_ARG;
    DeviceGuard g(ctx->device);
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(loss, m->loss.p, 4, hipMemcpyDeviceToHost));
    return CROP_OK;
}

crop_status crop_mlp_score(crop_ctx *ctx, const crop_mlp *m, const float *Z, uint64_t N,
                           float *out)
{
    if (!ctx || !m || (N && (!Z || !out))) return CROP_E_ARG;
    DeviceGuard g(ctx->device);
    CK(launch_mlp_score(m->params.as<float>(), Z, N, out, ctx->stream));
    return CROP_OK;
}

crop_status crop_select_seeds(crop_ctx *ctx, const float *score, const uint32_t *cx,
                              const uint32_t *cy, uint64_t n, uint32_t R, uint32_t *sx,
                              uint32_t *sy)
{
    if (!ctx || (n && (!score || !cx || !cy || !sx || !sy))) return CROP_E_ARG;
    if (n >= (1ull << 32)) return fail(ctx, CROP_E_UNSUPPORTED, "too many candidates");
    if (R > n) return fail(ctx, CROP_E_ARG, "R exceeds the candidate count");
    DeviceGuard g(ctx->device);
    CK(ctx->seed_sel.ensure(((size_t)R + 2) * 4));
    CK(launch_select_seeds(score, cx, cy, (uint32_t)n, R, sx, sy, ctx->seed_sel.as<uint32_t>(),
                           ctx->stream));
    return CROP_OK;
}

crop_status crop_hash_pairs(crop_ctx *ctx, const uint32_t *qx, const uint32_t *qy, uint64_t n,
                            uint32_t *h, uint32_t *part)
{
    if (!ctx || (n && (!qx || !qy))) return CROP_E_ARG;
    DeviceGuard g(ctx->device);
    CK(launch_hash_pairs(qx, qy, n, ctx->hp, ctx->P, h, part, ctx->stream));
    return CROP_OK;
}

crop_status crop_synchronize(crop_ctx *ctx)
{
    if (!ctx) return CROP_E_ARG;
    DeviceGuard g(ctx->device);
    CK(hipStreamSynchronize(ctx->stream));
    return CROP_OK;
}

// Exact-run tuner for a loaded transaction stream: times routing bins per
// partition S in {S0 - 1, S0, S0 + 1, S0 + 2} (S0 the automatic choice) x
// rows per chunk in {64, 96, 128, 192, 256}, keeps the fastest in the
// context's tuning and leaves the result of a run with it.
crop_status crop_autotune(crop_ctx *ctx, uint32_t reps, uint32_t *bins_per_partition,
                          uint32_t *rows_per_chunk, float *best_ms)
{
    if (!ctx) return CROP_E_ARG;
    if (ctx->in.mode != Mode::Tx)
        return fail(ctx, CROP_E_STATE, "the tuner needs a loaded transaction stream");
    DeviceGuard g(ctx->device);
    reps = std::max<uint32_t>(reps, 1);
    const crop_tune saved = ctx->tune;
    ctx->tune.bins_per_partition = 0;
    ctx->tune.rows_per_chunk = 0;
    ctx->tune.region_terms = 0;
    bool regions = false;
    crop_status st = plan_regions(ctx, &regions);
    if (st == CROP_OK && !regions) st = plan_tx(ctx);
    if (st != CROP_OK) {
        ctx->tune = saved;
        return st;
    }
    const uint32_t S0 = ctx->plan.S;
    // the second axis: terms per sub-batch on the region route, else rows
    // per chunk
    std::vector<uint32_t> second;
    if (regions)
        second = {16384u, 24576u};
    else
        second = {64u, 96u, 128u, 192u, 256u};
    uint32_t p0, p1;
    owned_range(ctx, &p0, &p1);
    float best = -1.0f;
    uint32_t bS = 0, bR = 0;
    // grouped bins (P above the bin limit) have one bin per 2^g partitions:
    // only the rows per chunk are tuned
    const uint32_t S_hi = ctx->plan.g ? 1u : S0 + 2;
    for (uint32_t S = S0 > 1 ? S0 - 1 : 1; S <= S_hi; ++S) {
        if (ctx->plan.g == 0 && (uint64_t)(p1 - p0) * S > kMaxP) break;
        for (uint32_t R : second) {
            ctx->tune = saved;
            ctx->tune.bins_per_partition = S;
            if (regions)
                ctx->tune.region_terms = R;
            else
                ctx->tune.rows_per_chunk = R;
            float lo = -1.0f, ms = 0.0f;
            for (uint32_t k = 0; k <= reps; ++k) {  // the first run warms up
                st = crop_run_exact(ctx);
                if (st == CROP_OK) st = crop_last_run_ms(ctx, &ms);
                if (st != CROP_OK) break;
                if (k && (lo < 0 || ms < lo)) lo = ms;
            }
            if (st != CROP_OK) {
                if (st == CROP_E_UNSUPPORTED) continue;  // a plan that does not fit
                ctx->tune = saved;
                return st;
            }
            if (best < 0 || lo < best) {
                best = lo;
                bS = S;
                bR = R;
            }
        }
    }
    ctx->tune = saved;
    if (best < 0) return fail(ctx, CROP_E_UNSUPPORTED, "no candidate plan fits this stream");
    ctx->tune.bins_per_partition = bS;
    if (regions)
        ctx->tune.region_terms = bR;
    else
        ctx->tune.rows_per_chunk = bR;
    st = crop_run_exact(ctx);
    if (st != CROP_OK) return st;
    if (bins_per_partition) *bins_per_partition = bS;
    if (rows_per_chunk) *rows_per_chunk = ctx->plan.R;
    if (best_ms) *best_ms = best;
    return CROP_OK;
}

crop_status crop_last_run_ms(crop_ctx *ctx, float *ms)
{
    if (!ctx || !ms) return CROP_E_ARG;
    if (!ctx->timed) return fail(ctx, CROP_E_STATE, "no run recorded");
    DeviceGuard g(ctx->device);
    CK(hipEventSynchronize(ctx->ev1));
    CK(hipEventElapsedTime(ms, ctx->ev0, ctx->ev1));
    return CROP_OK;
}

// ============================================================== readback

namespace {

// Partition p of a run with grouped bins: its bin is gathered by partition
// into scratch and p's slice is copied out.
crop_status read_partition_grouped(crop_ctx *ctx, uint32_t p, uint32_t *i, uint32_t *j,
                                   uint32_t *count, float *value, uint64_t cap,
                                   uint64_t *written)
{
    const RoutePlan &pl = ctx->plan;
    CK(hipStreamSynchronize(ctx->stream));
    const int64_t b = partition_bin(ctx, p);
    if (b < 0) {
        if (written) *written = 0;
        return CROP_OK;
    }
    const uint32_t G = 1u << pl.g;
    const uint32_t first = (uint32_t)((b + (pl.u0 >> pl.g)) << pl.g);
    std::vector<uint32_t> ps(G, 0), dst(G, 0);
    const uint32_t last = std::min<uint32_t>(first + G, ctx->P);
    CK(hipMemcpy(ps.data(), ctx->part_stats.as<uint32_t>() + first, (last - first) * 4,
                 hipMemcpyDeviceToHost));
    uint32_t bs = 0;
    CK(hipMemcpy(&bs, ctx->bin_size.as<uint32_t>() + b, 4, hipMemcpyDeviceToHost));
    uint64_t run = 0;
    for (uint32_t k = 0; k < G; ++k) {
        dst[k] = (uint32_t)run;
        run += ps[k];
    }
    const uint64_t tot = ps[p - first];
    if (written) *written = tot;
    if (tot > cap) return fail(ctx, CROP_E_CAPACITY, "output capacity below the entry count");
    const size_t n = std::max<uint32_t>(bs, 1);
    const size_t head = ((size_t)G * 4 + 255) / 256 * 256;
    CK(ctx->scratch.ensure(head + 16 * n));
    uint32_t *d_dst = ctx->scratch.as<uint32_t>();
    uint32_t *oi = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(d_dst) + head);
    uint32_t *oj = oi + n, *oc = oj + n;
    float *ov = reinterpret_cast<float *>(oc + n);
    const bool outer = ctx->in.mode == Mode::Outer;
    CK(hipMemcpyAsync(d_dst, dst.data(), G * 4, hipMemcpyHostToDevice, ctx->stream));
    CK(launch_gather_grouped(ctx, (uint32_t)b, 1, d_dst, first, oi, oj, outer ? nullptr : oc,
                             outer ? ov : nullptr, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    const uint32_t at = dst[p - first];
    if (tot) {
        CK(hipMemcpy(i, oi + at, tot * 4, hipMemcpyDeviceToHost));
        CK(hipMemcpy(j, oj + at, tot * 4, hipMemcpyDeviceToHost));
        if (count && !outer) CK(hipMemcpy(count, oc + at, tot * 4, hipMemcpyDeviceToHost));
        if (value && outer) CK(hipMemcpy(value, ov + at, tot * 4, hipMemcpyDeviceToHost));
    }
    return CROP_OK;
}

}  // namespace

crop_status crop_result_sizes(crop_ctx *ctx, uint64_t *sizes, uint64_t *terms)
{
    if (!ctx) return CROP_E_ARG;
    crop_status st = require_exact(ctx);
    if (st != CROP_OK) return st;
    DeviceGuard g(ctx->device);
    const RoutePlan &pl = ctx->plan;
    CK(hipStreamSynchronize(ctx->stream));
    if (pl.g) {
        std::vector<uint32_t> v(2 * (size_t)ctx->P);
        CK(hipMemcpy(v.data(), ctx->part_stats.p, v.size() * 4, hipMemcpyDeviceToHost));
        for (uint32_t p = 0; p < ctx->P; ++p) {
            if (sizes) sizes[p] = v[p];
            if (terms) terms[p] = v[ctx->P + p];
        }
        return CROP_OK;
    }
    std::vector<uint32_t> bs(pl.NB), bo(pl.NB + 1);
    CK(hipMemcpy(bs.data(), ctx->bin_size.p, pl.NB * 4, hipMemcpyDeviceToHost));
    CK(hipMemcpy(bo.data(), ctx->bin_off.p, (pl.NB + 1) * 4, hipMemcpyDeviceToHost));
    for (uint32_t p = 0; p < ctx->P; ++p) {
        const int64_t b0 = partition_bin(ctx, p);
        uint64_t n = 0, t = 0;
        if (b0 >= 0) {
            for (uint32_t s = 0; s < pl.S; ++s) n += bs[b0 + s];
            t = (uint64_t)bo[b0 + pl.S] - bo[b0];
        }
        if (sizes) sizes[p] = n;
        if (terms) terms[p] = t;
    }
    return CROP_OK;
}

crop_status crop_read_all(crop_ctx *ctx, crop_mem where, uint32_t *i, uint32_t *j,
                          uint32_t *count, float *value, uint64_t cap, uint64_t *written,
                          uint64_t *part_off)
{
    if (!ctx || !i || !j) return CROP_E_ARG;
    crop_status st = require_exact(ctx);
    if (st != CROP_OK) return st;
    DeviceGuard g(ctx->device);
    const RoutePlan &pl = ctx->plan;
    std::vector<uint32_t> bs(pl.NB);
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(bs.data(), ctx->bin_size.p, pl.NB * 4, hipMemcpyDeviceToHost));
    std::vector<uint32_t> dst(pl.g ? ctx->P : pl.NB);
    uint64_t tot = 0;
    if (pl.g) {
        // grouped bins: partition starts from the per-partition sizes
        std::vector<uint32_t> ps(ctx->P);
        CK(hipMemcpy(ps.data(), ctx->part_stats.p, ps.size() * 4, hipMemcpyDeviceToHost));
        for (uint32_t p = 0; p < ctx->P; ++p) {
            dst[p] = (uint32_t)tot;
            if (part_off) part_off[p] = tot;
            tot += ps[p];
        }
        if (part_off) part_off[ctx->P] = tot;
    } else {
        for (uint32_t b = 0; b < pl.NB; ++b) {
            dst[b] = (uint32_t)tot;
            tot += bs[b];
        }
    }
    if (part_off && !pl.g) {
        // partitions outside the owned range are empty
        uint64_t run = 0;
        for (uint32_t p = 0; p < ctx->P; ++p) {
            const int64_t b0 = partition_bin(ctx, p);
            if (b0 >= 0) run = dst[b0];
            part_off[p] = run;
            if (b0 >= 0)
                for (uint32_t s = 0; s < pl.S; ++s) run += bs[b0 + s];
        }
        part_off[ctx->P] = tot;
    }
    if (written) *written = tot;
    if (tot > cap) return fail(ctx, CROP_E_CAPACITY, "output capacity below the entry count");
    const bool outer = ctx->in.mode == Mode::Outer;
    // device staging: dst offsets, and the four outputs when reading to host
    // scratch layout: dst offsets, then (host readback only) four arrays of n
    // words starting at the next 256-byte boundary
    const size_t n = std::max<uint64_t>(tot, 1);
    const size_t head = (dst.size() * 4 + 255) / 256 * 256;
    CK(ctx->scratch.ensure(head + (where == CROP_MEM_HOST ? 16 * n : 0)));
    uint32_t *d_dst = ctx->scratch.as<uint32_t>();
    CK(hipMemcpyAsync(d_dst, dst.data(), dst.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    uint32_t *oi = i, *oj = j, *oc = count;
    float *ov = value;
    if (where == CROP_MEM_HOST) {
        char *base = reinterpret_cast<char *>(d_dst) + head;
        oi = reinterpret_cast<uint32_t *>(base);
        oj = oi + n;
        oc = count ? oj + n : nullptr;
        ov = value ? reinterpret_cast<float *>(oj + 2 * n) : nullptr;
    }
    if (pl.g)
        CK(launch_gather_grouped(ctx, 0, pl.NB, d_dst, 0, oi, oj, outer ? nullptr : oc,
                                 outer ? ov : nullptr, ctx->stream));
    else
        CK(launch_gather_result(ctx, 0, pl.NB, d_dst, oi, oj, outer ? nullptr : oc,
                                outer ? ov : nullptr, ctx->stream));
    if (where == CROP_MEM_HOST) {
        CK(hipMemcpyAsync(i, oi, tot * 4, hipMemcpyDeviceToHost, ctx->stream));
        CK(hipMemcpyAsync(j, oj, tot * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (count && !outer) CK(hipMemcpyAsync(count, oc, tot * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (value && outer) CK(hipMemcpyAsync(value, ov, tot * 4, hipMemcpyDeviceToHost, ctx->stream));
    }
    CK(hipStreamSynchronize(ctx->stream));
    return CROP_OK;
}

crop_status crop_read_partition(crop_ctx *ctx, uint32_t p, uint32_t *i, uint32_t *j,
                                uint32_t *count, float *value, uint64_t cap, uint64_t *written)
{
    if (!ctx || !i || !j) return CROP_E_ARG;
    crop_status st = require_exact(ctx);
    if (st != CROP_OK) return st;
    if (p >= ctx->P) return fail(ctx, CROP_E_ARG, "partition index out of range");
    DeviceGuard g(ctx->device);
    const RoutePlan &pl = ctx->plan;
    if (pl.g) return read_partition_grouped(ctx, p, i, j, count, value, cap, written);
    std::vector<uint32_t> bs(pl.NB), bo(pl.NB + 1);
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(bs.data(), ctx->bin_size.p, pl.NB * 4, hipMemcpyDeviceToHost));
    CK(hipMemcpy(bo.data(), ctx->bin_off.p, (pl.NB + 1) * 4, hipMemcpyDeviceToHost));
    const int64_t b0 = partition_bin(ctx, p);
    const uint32_t nbins = b0 >= 0 ? pl.S : 0;
    uint64_t tot = 0;
    for (uint32_t s = 0; s < nbins; ++s) tot += bs[b0 + s];
    if (written) *written = tot;
    if (tot > cap) return fail(ctx, CROP_E_CAPACITY, "output capacity below the entry count");
    const bool outer = ctx->in.mode == Mode::Outer;
    const bool wide = ctx->in.wide_keys;
    uint64_t w = 0;
    for (uint32_t s = 0; s < nbins; ++s) {
        uint32_t b = (uint32_t)b0 + s, n = bs[b], src = bo[b];
        if (!n) continue;
        if (wide) {
            std::vector<uint64_t> k(n);
            CK(hipMemcpy(k.data(), ctx->keys.as<uint64_t>() + src, n * 8, hipMemcpyDeviceToHost));
            for (uint32_t e = 0; e < n; ++e) {
                i[w + e] = (uint32_t)(k[e] >> 32);
                j[w + e] = (uint32_t)k[e];
            }
        } else {
            std::vector<uint32_t> k(n);
            CK(hipMemcpy(k.data(), ctx->keys.as<uint32_t>() + src, n * 4, hipMemcpyDeviceToHost));
            for (uint32_t e = 0; e < n; ++e) {
                i[w + e] = k[e] >> 16;
                j[w + e] = k[e] & 0xFFFFu;
            }
        }
        if (count && !outer)
            CK(hipMemcpy(count + w, ctx->out_cnt.as<uint32_t>() + src, n * 4, hipMemcpyDeviceToHost));
        if (value && outer)
            CK(hipMemcpy(value + w, ctx->vals.as<float>() + src, n * 4, hipMemcpyDeviceToHost));
        w += n;
    }
    return CROP_OK;
}

}  // extern "C"
