// Host-side internals of the CRoP library: context, buffers, kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/crop.h"
#include "crop_hash.hpp"

namespace crop {

enum class Mode { None = 0, Tx = 1, Outer = 2, Batch = 3 };
enum class Result { None = 0, Exact = 1, TopK = 2, BatchExact = 3, CountSketch = 4 };

// A device allocation that grows on demand (never shrinks).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need)
    {
        if (need <= bytes && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (need == 0) need = 256;
        hipError_t e = hipMalloc(&p, need);
        if (e == hipSuccess) bytes = need;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// One enumeration workgroup's share of an outer-product stream: the
// a-entries [a_lo, a_hi) of vectors k0..k1-1.
struct OpChunk {
    uint32_t k0, k1, a_lo, a_hi;
};

// Resolved routing configuration of a run.
struct RoutePlan {
    // Bins: a hash value h maps to u = floor(h M / 2^32) with M = P * S (S
    // bins per partition) or M = P (bins that group 2^g partitions); the run
    // keeps u in [u0, u0 + nu) (the owned partitions) and routes u to bin
    // (u >> g) - (u0 >> g).
    uint32_t S = 1;          // routing bins per partition (1 when g > 0)
    uint32_t NB = 1;         // routing bins of the run
    uint64_t M = 1;          // P * S
    uint32_t u0 = 0, nu = 1; // kept range of u
    uint32_t g = 0;          // log2 of the partitions grouped in one bin
    uint32_t n_chunks = 0;   // enumeration workgroups
    uint32_t R = 256;        // vectors per chunk (transactions)
    uint32_t max_items = 0;  // largest number of staged entries in a chunk
    uint32_t stage_cap = 0;  // scatter: terms staged in LDS per window
    uint32_t G = 1;          // row groups of the count-matrix scan
    uint32_t n_wg = 0;       // transactions: workgroups of the range kernels
                             // (0: one count row per chunk)
    // windowed enumeration of an owned share (Lemma 1): the owned hash
    // interval [win_q, win_q + win_W) and the h_b bucket bits (0: off)
    uint32_t win_kb = 0, win_q = 0, win_W = 0;
    uint32_t log2_slots = 14;
    uint32_t BS = 256;
    uint32_t ss_mb = 0;      // Space-Saving micro-batch of the last top-K plan
    bool regions = false;    // transactions: the region route (k_sb_route)
};

// Region route of a transaction stream (k_sb_route): sub-batches of
// consecutive rows with at most max_terms terms, max_items items and
// max_rows rows; sub-batch s is rows [row[s], row[s+1]) and its region of
// the routed array starts at term[s] (the term prefix with every region
// rounded up to four keys; term[n_sub] = the routed array's keys).
// Computed once per loaded stream and set of caps.
// One segment of the region route: a stream with its own kept bins and
// sub-batches (an exact run is one segment, a batched run one per stream).
// Its header rows (one per sub-batch, hs >= NB + 1 bin starts), their
// transpose (one row per bin start, hts >= n_sub) and its header tile sums
// (one row of NB + 1 per 64 sub-batches) sit at their offsets in the run's
// arrays; its bins' results start after key0 kept keys.
struct SbSeg {
    BinMap bm;                     // hash -> kept bin of the segment
    uint32_t NB, bin0;             // kept bins, first bin in the run's numbering
    uint32_t sub0, n_sub;          // its sub-batches
    uint32_t hs, hts;              // header and transposed row strides (u16)
    uint32_t tile0, btiles;        // first header tile (64 x 64), bin tiles per tile row
    uint32_t key0;                 // kept keys of the segments before
    uint64_t hdr0, hdrT0, tsum0;   // offsets of its header, transpose (u16), tile sums (u32)
};

struct SbPlan {
    bool valid = false;
    uint32_t n_sub = 0, max_terms = 0, max_items = 0, max_rows = 0;
    std::vector<uint32_t> row, term;
    // segments of the last planned run, and the sizes of its header arrays
    std::vector<SbSeg> segs;
    uint32_t NBmax = 0, n_tiles = 0;
    uint64_t hdr_words = 0, hdrT_words = 0, tsum_words = 0;
};

struct Input {
    Mode mode = Mode::None;
    // transactions
    const uint32_t *off = nullptr, *items = nullptr;
    uint64_t T = 0, nnz = 0;
    uint32_t n_items = 0;
    // outer products
    const uint32_t *a_off = nullptr, *a_idx = nullptr, *b_off = nullptr, *b_idx = nullptr;
    const float *a_val = nullptr, *b_val = nullptr;
    uint64_t K = 0, nnz_a = 0, nnz_b = 0;
    uint32_t n_rows = 0, n_cols = 0;
    // derived
    uint64_t total_terms = 0;
    bool wide_keys = false;            // keys need 64 bits
    std::vector<uint32_t> h_off;       // host copy of the vector offsets
    std::vector<uint32_t> h_b_off;     // outer products: host copy of b_off
    std::vector<OpChunk> op_chunks;    // outer products: chunk plan
    uint32_t op_max_a = 0;             // largest a-range of an outer chunk
    DevBuf own[6];                     // private copies (COPY mode)
    DevBuf d_op_chunks;
};

// Batches of transaction streams (one exact run over all of them).  The
// streams are concatenated row-wise; stream s owns NB routing bins starting
// at global bin bin_base, chunks [chunk0, chunk0 + n_chunks), and its count
// matrix at cnt_base.
struct BatchStreamDev {
    uint32_t NB, bin_base, chunk0, n_chunks;
    uint64_t cnt_base;
};

struct BatchDev {
    const uint32_t *crow = nullptr;       // n_chunks + 1 row boundaries
    const uint32_t *cstream = nullptr;    // stream of each chunk
    const BatchStreamDev *streams = nullptr;
    const uint32_t *bin_stream = nullptr; // stream of each global bin
    uint32_t n_chunks = 0, n_streams = 0, NBtot = 0, NBmax = 0, max_items = 0, stage_cap = 0;
};

// Count-Sketch instances: hash parameters of instance i from seed + i.
constexpr uint32_t kCsMaxInstances = 15;
constexpr uint64_t kCsMinBins = 256;          // fewer routed bins: direct atomics
constexpr uint64_t kCsMaxBinBuckets = 16384;  // counters of one bin in LDS
struct CsParams {
    HashParams hp[kCsMaxInstances];
    uint32_t t;   // instances
    uint64_t PB;  // buckets per instance (P * B)
};

// Space-Saving state in device memory, bucket-major with ell slots per
// bucket (structure of arrays).  cnt/err hold uint32 counts (transactions)
// or fp32 bits (outer products); key holds (i << 32) | j; flag bit 0 =
// used, bit 1 = pinned.
struct SsState {
    uint64_t *key = nullptr;
    // optional copy of the used slots' keys packed as (x << 16) | y (0 for a
    // free slot), written by the summary kernel of a narrow run when set
    uint32_t *key32 = nullptr;
    uint32_t *cnt = nullptr;
    uint32_t *err = nullptr;
    float *val = nullptr;
    uint8_t *flag = nullptr;
    uint64_t nslots = 0;
};

// Per-stage HIP events of one run (profiling mode).
constexpr int kStageRing = 64;
constexpr int kMaxStages = 10;
struct StageRec {
    int n = 0;
    const char *names[kMaxStages] = {};
    hipEvent_t ev[kMaxStages + 1] = {};
};

}  // namespace crop

namespace crop {

// Host side of a loaded batch and its plan.  Stream s is rows
// [tx_off[s], tx_off[s+1]) of the concatenated CSR; its P[s] partitions are
// its routing bins [bin_base[s], bin_base[s] + P[s]) (one bin per partition).
struct BatchState {
    uint32_t n = 0;
    std::vector<uint64_t> tx_off;
    std::vector<uint32_t> n_items;
    std::vector<uint64_t> terms;
    // plan
    bool planned = false;
    bool regions = false;  // the plan takes the region route (one segment per stream)
    uint32_t terms_per_bin = 0, rows_per_chunk = 0;
    std::vector<uint32_t> P, bin_base, chunk0, n_chunks;
    std::vector<uint64_t> cnt_base;
    uint64_t cnt_words = 0;
    BatchDev dev;
    DevBuf d_crow, d_cstream, d_streams, d_bin_stream, tot, tiles;
    // captured launch sequence of one run
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace crop

struct crop_mlp {
    int device = 0;
    crop::DevBuf params, m, v, gstage, loss;
    uint64_t t = 0;  // Adam steps taken
};

struct crop_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;

    uint32_t P = 1;
    uint32_t own_p0 = 0, own_p1 = 0;  // owned partitions [own_p0, own_p1); 0, 0: all
    uint64_t seed = 0x243F6A8885A308D3ull;
    crop::HashParams hp{};
    uint32_t ss_counters = 1u << 14;  // counters per partition
    uint32_t ss_ell = 16;             // counters per bucket
    int topk_rank = CROP_RANK_LOWER;  // top-K order
    crop_tune tune{};                 // user request (0 = auto)
    crop::RoutePlan plan{};

    crop::Input in;
    crop::Result result = crop::Result::None;
    uint32_t topk_K = 0;

    // work and result buffers
    crop::DevBuf cnt_mat, part_buf, bin_off, bin_size, bin_order, keys, vals, out_cnt, spill,
        counter;
    crop::DevBuf ss_state, topk_buf, scratch, learn_ws;
    crop::DevBuf seed_sel;     // seed selection: threshold words and the selected candidates
    crop::DevBuf part_stats;   // grouped bins: entries and terms of each partition
    crop::SbPlan sb;           // region route: sub-batch plan of the loaded stream
    crop::DevBuf routed, sb_row, sb_term, sb_hdr, sb_hdrT, sb_tsum;
    crop::DevBuf sb_seg;       // the segments on the device (sb.segs)
    crop::DevBuf sb_subseg, sb_binseg;  // segment of each sub-batch / bin (several segments)
    std::vector<crop::SbSeg> sb_seg_host;  // ... as last uploaded
    crop::BatchState batch;    // batched streams
    crop::DevBuf cs_buf;       // Count-Sketch counters [t][P * B]
    crop::CsParams cs{};       // ... of the last Count-Sketch run
    uint32_t cs_B = 0;
    uint32_t cs_routed = 0;    // ... was routed into bins of buckets
    crop::SsState ss;          // views into ss_state
    uint64_t ss_buckets = 0;   // P * B of the last top-K run
    uint32_t topk_outer = 0;   // the last top-K run was on outer products
    uint32_t topk_instances = 1;  // ... and ran this many instances
    crop::DevBuf amp_buf;      // combined entries of an amplified run

    // profiling: per-stage events of the last kStageRing runs
    bool profiling = false;
    std::vector<crop::StageRec> ring;
    uint64_t runs = 0;
    crop::StageRec *cur_rec = nullptr;

    std::string err;
    int64_t err_index = -1;
};

namespace crop {

// ---- launchers (kernels live in the .hip files) ---------------------------
BinMap bin_map(const RoutePlan &pl);
hipError_t launch_validate_tx(const uint32_t *off, uint64_t T, const uint32_t *items,
                              uint64_t nnz, uint32_t n_items, unsigned long long *bad,
                              hipStream_t s);
hipError_t launch_validate_outer(const uint32_t *v_off, uint64_t K, const uint32_t *idx,
                                 uint64_t nnz, uint32_t n, unsigned long long *bad,
                                 hipStream_t s);

// *bad <- min(*bad, first q whose pair breaks x < y < n_items).
hipError_t launch_check_pairs(const uint32_t *qx, const uint32_t *qy, uint64_t n,
                              uint32_t n_items, unsigned long long *bad, hipStream_t s);
hipError_t launch_hash_pairs(const uint32_t *qx, const uint32_t *qy, uint64_t n,
                             const HashParams &hp, uint32_t P, uint32_t *h, uint32_t *part,
                             hipStream_t s);

// Region route (k_sbroute.hip): the sub-batch regions and their bin-start
// rows, then the transposed rows and bin_off (bin-contiguous offsets), then
// optionally the bin-contiguous keys themselves.
size_t sb_route_smem_bytes(uint32_t NB, uint32_t max_rows, uint32_t max_items,
                           uint32_t max_terms, uint32_t key_bytes);
uint32_t sb_threads();
void layout_sb_segments(SbPlan &sp);
bool sb_caps(uint32_t NB, uint32_t key_bytes, uint32_t want, uint32_t *S, uint32_t *I,
             uint32_t *R);
crop_status plan_sb_rows(crop_ctx *ctx, uint32_t S, uint32_t I, uint32_t R, bool *ok,
                         const std::vector<uint64_t> *cuts = nullptr);
crop_status ensure_region_buffers(crop_ctx *ctx);
hipError_t launch_sb_route(const crop_ctx *c, hipStream_t s);
hipError_t launch_sb_headers(const crop_ctx *c, hipStream_t s);

hipError_t launch_tx_count(const crop_ctx *c, uint32_t *cnt, hipStream_t s);
// Owned shares with windowed enumeration (plan.win_kb > 0).
size_t tx_win_smem_bytes(uint32_t NB, uint32_t R, uint32_t kb, uint32_t max_items);
bool tx_win_layout_ok(uint32_t NB, uint32_t R, uint32_t kb, uint32_t max_items);
hipError_t launch_tx_count_win(const crop_ctx *c, uint32_t *cnt, hipStream_t s);
hipError_t launch_tx_scatter_win(const crop_ctx *c, const uint32_t *cur, void *keys,
                                 hipStream_t s);
// Range kernels: n_wg workgroups, each over a contiguous range of chunks;
// the count matrix is [n_wg x NB].
hipError_t launch_tx_count_ranges(const crop_ctx *c, uint32_t *cnt, hipStream_t s);
hipError_t launch_tx_scatter_ranges(const crop_ctx *c, const uint32_t *cur, void *keys,
                                    hipStream_t s);
hipError_t launch_tx_scatter(const crop_ctx *c, const uint32_t *cur, void *keys, hipStream_t s);
hipError_t launch_op_count(const crop_ctx *c, uint32_t *cnt, hipStream_t s);
hipError_t launch_op_scatter(const crop_ctx *c, const uint32_t *cur, void *keys, float *vals,
                             hipStream_t s);
// Count matrix [n_chunks x NB] -> global write offsets in place; bin_off
// [NB+1] receives the bin starts; *counter is reset to 0.
hipError_t launch_scan_counts(uint32_t *cnt, uint32_t n_chunks, uint32_t NB, uint32_t G,
                              uint32_t *part, uint32_t *bin_off, uint32_t *counter,
                              hipStream_t s);

// order[] <- bins with more than twice the mean term count first.
// n_seg > 1: each of n_seg equal segments of the bins ordered on its own
// (the region aggregation's per-XCD bin ranges); zero[0 .. n_zero) <- 0
// (n_zero at most 1024)
hipError_t launch_bin_order(uint32_t NB, const uint32_t *bin_off, uint32_t *order, hipStream_t s,
                            uint32_t n_seg = 1, uint32_t *zero = nullptr, uint32_t n_zero = 0);

hipError_t launch_batch_count(const uint32_t *off, const uint32_t *items, const HashParams &hp,
                              const BatchDev &b, uint32_t *cnt, const uint32_t *bin_off,
                              hipStream_t s);
hipError_t launch_batch_scatter(const uint32_t *off, const uint32_t *items, const HashParams &hp,
                                const BatchDev &b, uint32_t *cur, const uint32_t *bin_off,
                                void *keys, bool wide, hipStream_t s);
uint32_t batch_scan_tiles(uint32_t NBtot);
hipError_t launch_batch_scan(const BatchDev &b, uint32_t *cnt, uint32_t *tot, uint32_t *tiles,
                             uint32_t *bin_off, uint32_t *counter, hipStream_t s);

hipError_t launch_aggregate_regions(const crop_ctx *c, hipStream_t s);
hipError_t launch_aggregate_counts(const crop_ctx *c, hipStream_t s);
hipError_t launch_aggregate_sums(const crop_ctx *c, hipStream_t s);

// Space-Saving and top-K (k_topk.hip).
hipError_t launch_ss_clear(const SsState &S, hipStream_t s);
hipError_t launch_ss_pin(const SsState &S, const uint32_t *sx, const uint32_t *sy, uint32_t ns,
                         uint8_t *dup, uint32_t r_max, const HashParams &hp, uint64_t PB,
                         uint32_t ell, uint32_t *n_pinned, hipStream_t s);
constexpr uint32_t kSsBatchTxLarge = 2048;  // ... of packed keys, bins of several buckets
constexpr uint32_t kSsBatchTx = 1024;    // routed terms per Space-Saving micro-batch
constexpr uint32_t kSsBatchWide = 1024;   // ... with 64-bit keys
constexpr uint32_t kSsBatchOuter = 1024;  // ... of outer-product terms
size_t ss_bins_smem_bytes(uint32_t nbk, uint32_t ell, bool wide_key, bool outer, uint32_t MB);
uint32_t ss_block_threads(uint32_t nbk, uint32_t ell);
// fresh: start every bin from empty summaries instead of reading the
// (cleared, pinned) state; every slot is written back either way
hipError_t launch_ss_bins(const crop_ctx *c, const SsState &S, uint32_t nbk, uint64_t PB,
                          hipStream_t s, bool fresh = false);
hipError_t launch_zero32(uint32_t *p, uint32_t n, hipStream_t s);
hipError_t launch_topk(const SsState &S, uint32_t K, bool outer, bool by_lower, bool err_is_lower,
                       const uint8_t *votes, uint32_t *st, uint32_t *hist, uint32_t *cand,
                       uint32_t *sel, uint32_t *rank, uint32_t *oi, uint32_t *oj, double *ou,
                       double *ol, double *ov, uint32_t *ovotes, hipStream_t s);
hipError_t launch_amp_combine(const CsParams &ip, const SsState &S, uint32_t ell, uint64_t nslots,
                              uint32_t min_votes, bool outer, bool narrow, const SsState &A,
                              uint8_t *votes, hipStream_t s);

size_t tx_count_smem_bytes(uint32_t NB, uint32_t max_items);
bool tx_launch_layouts_ok(uint32_t NB, uint32_t max_items, uint32_t cap, bool wide);

// Count-Sketch (k_cs.hip).
hipError_t launch_cs_clear(void *cs, uint64_t words, hipStream_t s);
hipError_t launch_cs_tx(const crop_ctx *c, const CsParams &cp, int32_t *cs, hipStream_t s);
hipError_t launch_cs_op(const crop_ctx *c, const CsParams &cp, float *cs, hipStream_t s);
hipError_t launch_cs_bins(const crop_ctx *c, const HashParams &hp, uint64_t PB, uint32_t nbk,
                          uint32_t *out, hipStream_t s);
hipError_t launch_cs_estimate(const CsParams &cp, const void *cs, bool fp, const uint32_t *qx,
                              const uint32_t *qy, uint64_t n, double *out, hipStream_t s);

// Learned seeding (k_learned.hip).
size_t item_stats_words(uint32_t n, uint32_t Tp);
// The fixed workspace of crop_item_features_noalloc (noalloc.hip): resolve
// this device's copy, with `device` current; once per device.
hipError_t noalloc_setup(int device);
hipError_t launch_item_features(const uint32_t *off, const uint32_t *items, uint32_t n,
                                uint32_t Tp, uint32_t *ws, float *feat, hipStream_t s);
hipError_t launch_top_pairs(const uint32_t *ws, uint32_t n, uint32_t Tp, uint32_t M,
                            uint32_t *top, uint32_t *cx, uint32_t *cy, hipStream_t s);
hipError_t launch_lookup(const crop_ctx *c, const uint32_t *qx, const uint32_t *qy, uint64_t n,
                         uint32_t *out, hipStream_t s);
hipError_t launch_pair_inputs(const float *feat, const uint32_t *cx, const uint32_t *cy,
                              const uint32_t *count, uint64_t n, float *Z, float *y,
                              hipStream_t s);
hipError_t launch_mlp_train(float *params, float *m, float *v, float *gstage, const float *Z,
                            const float *y, const uint32_t *order, uint64_t n_order,
                            uint32_t batch, float lr, uint64_t t0, float *loss, hipStream_t s);
hipError_t launch_mlp_grad(const float *params, const float *Z, const float *y, uint32_t N,
                           float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_score(const float *params, const float *Z, uint64_t N, float *out,
                            hipStream_t s);
// sel: 2 + R words of workspace.
hipError_t launch_select_seeds(const float *score, const uint32_t *cx, const uint32_t *cy,
                               uint32_t n, uint32_t R, uint32_t *sx, uint32_t *sy, uint32_t *sel,
                               hipStream_t s);
hipError_t launch_max_index(const uint32_t *idx, uint64_t n, uint32_t *out, hipStream_t s);
int mlp_param_count();
int mlp_batch_max();

// Grouped bins: entries (out_n) and weights (out_w: counts, or terms when
// `routed`, over the routed keys before aggregation) of every kept partition.
hipError_t launch_part_stats(const crop_ctx *c, bool routed, uint32_t *out_n, uint32_t *out_w,
                             hipStream_t s);
// Grouped bins [bin0, bin0 + n_bins) to partition-contiguous arrays;
// partition p starts at dst[p - dst_p0].
hipError_t launch_gather_grouped(const crop_ctx *c, uint32_t bin0, uint32_t n_bins,
                                 const uint32_t *dst, uint32_t dst_p0, uint32_t *out_i,
                                 uint32_t *out_j, uint32_t *out_cnt, float *out_val,
                                 hipStream_t s);

// Gather the bin-segmented exact result into partition-contiguous arrays.
hipError_t launch_gather_result(const crop_ctx *c, uint32_t bin0, uint32_t n_bins,
                                const uint32_t *dst_off, uint32_t *out_i, uint32_t *out_j,
                                uint32_t *out_cnt, float *out_val, hipStream_t s);

}  // namespace crop
