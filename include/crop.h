/*
 * crop.h -- C ABI of the MI355X column-row parallel (CRoP) library.
 *
 * The library computes, on one AMD MI355X (gfx950), the data-parallel hot
 * path of the column-row method of Campagna, Kutzkov and Pagh, "On
 * Parallelizing Matrix Multiplication by the Column-Row Method":
 *
 *   - enumerate the nonzero terms of C = sum_k a_k b_k^T (Section 4,
 *     notation: entry (i,j) has weight sum_k a_k(i) b_k(j)), or all item
 *     pairs of each transaction of a {0,1} stream (Section 7: the pairs of a
 *     transaction are the entries above the diagonal of v_T v_T^T);
 *   - route every entry (i,j) to one of P partitions by the consistent hash
 *     h(i,j) = (h_a(i) + h_b(j)) mod 2^32 (Section 5, Lemma 1 and its proof;
 *     Figure 1), partition = (h * P) >> 32;
 *   - accumulate each partition exactly (uint32 supports or fp32 sums), or
 *     in Space-Saving summaries of ell slots per bucket (Section 4, frequent
 *     items mining; Figure 1), bucket = (h * P * B) >> 32;
 *   - read back per-partition results or the top-K entries.
 *
 * Hash family (the paper leaves it open): seed -> (alpha_a, beta_a,
 * alpha_b, beta_b) are the first four outputs of SplitMix64 started at the
 * seed; h_a(x) = ((alpha_a * x + beta_a) mod 2^64) >> 32, likewise h_b.
 *
 * Conventions for every call:
 *   - Pointers marked "device" must be device memory of the context's GPU;
 *     pointers marked "host" must be host memory.  Where a crop_mem argument
 *     is present it says which.
 *   - Calls return a crop_status; they never throw and never abort.  On a
 *     non-OK status, crop_last_error_detail() gives a message.
 *   - Run calls are asynchronous on the context's HIP stream: they return
 *     after enqueueing.  Read calls synchronize that stream.
 *   - Results live in library-owned device memory until the next run, load
 *     or crop_destroy.  The caller owns every buffer it passes in.
 *   - One context must not be used from two threads at once; separate
 *     contexts are independent.
 */
#ifndef CROP_H
#define CROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CROP_ABI_VERSION 4

typedef enum crop_status {
    CROP_OK = 0,
    CROP_E_ARG = -1,          /* invalid argument (null pointer, bad size)   */
    CROP_E_STATE = -2,        /* call out of order, e.g. run before load     */
    CROP_E_INPUT = -3,        /* input violates the CSR contract; see
                                 crop_last_error_index()                      */
    CROP_E_CAPACITY = -4,     /* output buffer too small; *written holds the
                                 required element count                       */
    CROP_E_NOMEM = -5,        /* device allocation failed                     */
    CROP_E_HIP = -6,          /* a HIP runtime call failed; see detail        */
    CROP_E_UNSUPPORTED = -7   /* parameters outside the supported range       */
} crop_status;

typedef enum crop_mem { CROP_MEM_HOST = 0, CROP_MEM_DEVICE = 1 } crop_mem;
typedef enum crop_own { CROP_OWN_COPY = 0, CROP_OWN_BORROW = 1 } crop_own;

typedef struct crop_ctx crop_ctx;

/* Tuning knobs; a zero field means "choose automatically". */
typedef struct crop_tune {
    uint32_t bins_per_partition; /* routing bins per partition (S >= 1)       */
    uint32_t rows_per_chunk;     /* transactions per enumeration chunk        */
    uint32_t stage_keys;         /* scatter: 0 writes every key straight to
                                    its slot; >= 1024 stages up to that many
                                    keys per window in LDS, sorted by bin     */
    uint32_t route;              /* transactions: CROP_ROUTE_*                */
    uint32_t window;             /* owned shares: CROP_WINDOW_*               */
    uint32_t region_terms;       /* region route: terms per sub-batch, 16384
                                    or 24576 (largest that fits when 0)       */
} crop_tune;

/* How an exact run that owns at most half of the hash space finds its terms:
 * through h_b-bucketed windows of every transaction (Section 5, Lemma 1: the
 * owner's entries without enumerating the others; the default), or by
 * enumerating every term and keeping the owned ones. */
enum { CROP_WINDOW_AUTO = 0, CROP_WINDOW_OFF = 1 };

/* How the terms of a transaction stream reach their routing bins.  REGIONS
 * (what AUTO takes for exact runs of streams with fewer than 2^16 items,
 * whose keys pack into 32 bits, when every transaction fits a sub-batch and
 * no owned share enumerates through windows): each workgroup sorts the
 * terms of a sub-batch of consecutive transactions by bin in LDS and writes
 * them as one contiguous region with a row of bin starts, and a bin is read
 * back as one run per region; no count pass.  CHUNKS: a count pass builds a
 * [chunk x bin] matrix of offsets and a second enumeration writes every key
 * to its offset.  RANGES: as CHUNKS with one count row per workgroup that
 * walks a contiguous range of chunks. */
enum { CROP_ROUTE_AUTO = 0, CROP_ROUTE_CHUNKS = 1, CROP_ROUTE_RANGES = 2, CROP_ROUTE_REGIONS = 3 };

/* ---- context ----------------------------------------------------------- */

/* Create a context on HIP device `hip_device`.  Defaults: P = 1, seed =
 * 0x243F6A8885A308D3, 2^14 counters per partition with 16 per bucket, the
 * library's own non-blocking stream, automatic tuning. */
crop_status crop_create(crop_ctx **out, int hip_device);
void crop_destroy(crop_ctx *ctx);

/* Static strings; never freed by the caller. */
const char *crop_status_string(crop_status s);
const char *crop_last_error_detail(const crop_ctx *ctx);
/* For CROP_E_INPUT: index of the first offending vector (transaction or k),
 * or -1 when the offsets array itself is malformed. */
int64_t crop_last_error_index(const crop_ctx *ctx);
int crop_abi_version(void);

/* ---- parameters -------------------------------------------------------- */

/* Number of owners P, 1 <= P <= 2^20 (Section 6, Theorem 1: owners hold
 * disjoint equal intervals of the hash space; the paper's own runs used about
 * 2^20 buckets, Table 4).  Up to 8192 owned partitions each get one or more
 * routing bins of their own; beyond that a routing bin holds 2^g consecutive
 * partitions and each partition's entries are told apart by its hash when
 * the results are read.  Either way partition p owns exactly the hash values
 * h with floor(h P / 2^32) = p. */
crop_status crop_set_partitions(crop_ctx *ctx, uint32_t P);
/* 64-bit seed of the hash functions (Section 5: the hash description is
 * broadcast before the computation). */
crop_status crop_set_seed(crop_ctx *ctx, uint64_t seed);
/* Space-Saving sizes: counters_per_partition = B * ell, ell slots per bucket
 * (Section 4; Figure 1 keeps one summary of ell entries per bucket).
 * ell in [1, 64]; counters_per_partition a multiple of ell. */
crop_status crop_set_summary(crop_ctx *ctx, uint32_t counters_per_partition,
                             uint32_t counters_per_bucket);
/* Own only partitions [p_begin, p_end) (0, 0: all, the default): exact runs
 * then route and keep only the terms whose hash lies in the owned interval
 * [ceil(p_begin 2^32 / P), ceil(p_end 2^32 / P)) -- the share of one
 * processor in Section 5 (Lemma 1) and Section 6 (Theorem 1).  A share of at
 * most half the hash space visits only the h_b windows of each transaction
 * that can hold owned terms (window tuning CROP_WINDOW_AUTO, the default);
 * a larger share, or CROP_WINDOW_OFF, enumerates every term and drops the
 * unowned ones.
 * Partitions outside the range read back empty.  crop_set_partitions resets
 * the range; top-K and Count-Sketch runs reject an owned range. */
crop_status crop_set_owned_partitions(crop_ctx *ctx, uint32_t p_begin, uint32_t p_end);
/* Order of the top-K report: by lower bound (count - overestimation, the
 * guaranteed part of the count; Section 4), the default, or by upper bound
 * (the Space-Saving count), ties by smaller key either way.  The lower bound
 * is the default because an upper bound carries up to the bucket's minimum
 * count of overestimation, so light entries admitted late outrank heavier
 * entries whose counts are exact (pinned seeds, entries that never left the
 * summary); on the 1M-transaction stream with one partition of 16,384
 * counters the top 1,000 by lower bound recall 0.95 of the true top 1,000,
 * by upper bound 0.79. */
typedef enum { CROP_RANK_UPPER = 0, CROP_RANK_LOWER = 1 } crop_rank;
crop_status crop_set_topk_rank(crop_ctx *ctx, int rank);
/* Borrow a HIP stream (hipStream_t) for all later work; NULL is HIP's null
 * stream.  The stream must outlive its use.  A new context works on a
 * non-blocking stream of its own; crop_use_own_stream returns to it. */
crop_status crop_set_stream(crop_ctx *ctx, void *hip_stream);
crop_status crop_use_own_stream(crop_ctx *ctx);
crop_status crop_set_tuning(crop_ctx *ctx, const crop_tune *tune);
/* The configuration the next (or last) run uses, after automatic choices. */
crop_status crop_get_tuning(const crop_ctx *ctx, crop_tune *out);
/* Tune exact runs of the loaded transaction stream: time routing bins per
 * partition S in {S0-1 .. S0+2} (S0 = the automatic choice, within 8192
 * bins) x, on the region route, terms per sub-batch in {16384, 24576},
 * otherwise rows per chunk in {64, 96,
 * 128, 192, 256}; reps timed runs each after one warm-up, keep the fastest
 * as the context's tuning (other tuning fields unchanged) and leave the
 * exact result of a run with it.  Results do not depend on the plan.
 * Outputs (NULL allowed): the chosen S, the rows per chunk (after any
 * halving to fit LDS; 0 on the region route, whose choice crop_get_tuning
 * reports as region_terms) and the best time in ms.  CROP_E_STATE without a
 * loaded transaction stream. */
crop_status crop_autotune(crop_ctx *ctx, uint32_t reps, uint32_t *bins_per_partition,
                          uint32_t *rows_per_chunk, float *best_ms);

/* ---- input ------------------------------------------------------------- */

/* A {0,1} transaction stream in CSR form (Section 7; the stream order is the
 * row order, Section 7.3).  off[T+1] with off[0] = 0, non-decreasing,
 * off[T] = nnz; items[nnz] < n_items and strictly increasing inside each
 * transaction.  The input is validated on the device; a violation returns
 * CROP_E_INPUT.  BORROWed device buffers must stay valid until the next load
 * or destroy; COPY takes a private copy (host or device source). */
crop_status crop_load_transactions(crop_ctx *ctx, const uint32_t *off, uint64_t T,
                                   const uint32_t *items, uint64_t nnz, uint32_t n_items,
                                   crop_mem where, crop_own own);

/* K outer products a_k b_k^T (Section 5: A column-major, B row-major
 * triples).  a_off[K+1], a_idx[nnz_a] < n_rows, a_val[nnz_a]; likewise b.
 * Indices strictly increasing inside each vector.  Every stored pair is a
 * term, also when a value is 0.0. */
crop_status crop_load_outer(crop_ctx *ctx, const uint32_t *a_off, const uint32_t *a_idx,
                            const float *a_val, const uint32_t *b_off, const uint32_t *b_idx,
                            const float *b_val, uint64_t K, uint64_t nnz_a, uint64_t nnz_b,
                            uint32_t n_rows, uint32_t n_cols, crop_mem where, crop_own own);

/* ---- runs (asynchronous) ----------------------------------------------- */

/* Exact accumulation of every partition: uint32 supports (transactions) or
 * fp32 sums (outer products), plus the number of terms per partition. */
crop_status crop_run_exact(crop_ctx *ctx);

/* Space-Saving summaries per bucket, then the top-K monitored entries over
 * all partitions by (lower bound descending, key ascending), or by upper
 * bound (crop_set_topk_rank).  Transactions
 * use weight 1 per term; outer products use |a_k(i) b_k(j)| and keep the
 * signed sum of an entry's terms since its admission. */
crop_status crop_run_topk(crop_ctx *ctx, uint32_t K);

/* As crop_run_topk, with learned seeding: seeds (device arrays sx, sy of ns
 * transaction pairs x < y, highest priority first) are pinned into their
 * buckets before the stream, at most r_max per bucket (r_max < ell), in the
 * given order.  A pinned slot is never evicted, so its count is exact.
 * The seeds are checked on the device first (this call synchronizes once
 * for that): a pair without x < y < n_items returns CROP_E_INPUT with the
 * first offending seed in crop_last_error_index, and nothing runs. */
crop_status crop_run_topk_seeded(crop_ctx *ctx, uint32_t K, const uint32_t *sx,
                                 const uint32_t *sy, uint64_t ns, uint32_t r_max);

/* Amplification (Section 6, Theorem 2 and its proof): `instances` independent
 * CRoP runs, instance i with the hash functions of seed + i (1 <= instances
 * <= 15), each with its own Space-Saving summaries of the configured size.
 * An entry is reported when at least min_votes instances (1 <= min_votes <=
 * instances; the paper's rule is at least half, e.g. 6 of 11) monitor it
 * in the summary of its bucket.  A reported entry's bounds intersect the
 * reporting instances' bounds: upper = their least count, lower = their
 * largest count - overestimation; outer products also get the median of
 * their signed sums (mean of the two middle values for an even number).
 * The top-K over the reported entries ranks as crop_run_topk does.  Read
 * the result with crop_read_topk and crop_read_topk_votes;
 * crop_read_summary returns the instances' slots one instance after the
 * other (instances * P * B * ell slots).  Device memory: the summaries of
 * every instance plus 14 bytes per slot for the combined entries.
 * Errors: CROP_E_ARG for instances or min_votes out of range, else as
 * crop_run_topk. */
crop_status crop_run_topk_amplified(crop_ctx *ctx, uint32_t K, uint32_t instances,
                                    uint32_t min_votes);

/* ---- readback (synchronizes the context stream) ------------------------ */

/* Per-partition distinct-entry counts and term counts of the last exact run
 * (host arrays of P elements; either may be NULL). */
crop_status crop_result_sizes(crop_ctx *ctx, uint64_t *sizes, uint64_t *terms);

/* Entries of partition p of the last exact run into host arrays of
 * capacity cap: i, j (required), count (transactions, or NULL), value
 * (outer products, or NULL).  Order inside a partition is unspecified. */
crop_status crop_read_partition(crop_ctx *ctx, uint32_t p, uint32_t *i, uint32_t *j,
                                uint32_t *count, float *value, uint64_t cap,
                                uint64_t *written);

/* Every entry of the last exact run, partition by partition, into arrays in
 * `where` memory of capacity cap; part_off (host, P+1 elements, or NULL)
 * receives each partition's start. */
crop_status crop_read_all(crop_ctx *ctx, crop_mem where, uint32_t *i, uint32_t *j,
                          uint32_t *count, float *value, uint64_t cap, uint64_t *written,
                          uint64_t *part_off);

/* Top-K entries of the last top-K run into host arrays: upper and lower
 * bounds (Section 4: count and count - overestimation) and, for outer
 * products, the signed sum since admission (NULL allowed). */
crop_status crop_read_topk(crop_ctx *ctx, uint32_t *i, uint32_t *j, double *upper,
                           double *lower, double *value, uint64_t cap, uint64_t *written);

/* Number of instances that reported each entry of crop_read_topk, in the
 * same order (host array of capacity cap; 1 for single-instance runs). */
crop_status crop_read_topk_votes(crop_ctx *ctx, uint32_t *votes, uint64_t cap,
                                 uint64_t *written);

/* Every Space-Saving slot of the last top-K run (P*B*ell slots, bucket
 * major) into host arrays: entry, count, overestimation, signed sum (outer
 * products; else 0) and flags (bit 0 used, bit 1 pinned).  With P above 8192
 * the slots are padded to whole routing bins of 2^g partitions: the count
 * (*written) is then rounded up and the extra slots, at the end, are unused. */
crop_status crop_read_summary(crop_ctx *ctx, uint32_t *i, uint32_t *j, double *cnt,
                              double *err, double *value, uint8_t *flags, uint64_t cap,
                              uint64_t *written);

/* The consistent hash of query pairs under the context's seed and P
 * (Section 5: every processor can compute the owner of any entry from the
 * broadcast hash description): h[q] = (h_a(qx[q]) + h_b(qy[q])) mod 2^32 and
 * part[q] = (h[q] * P) >> 32.  qx, qy, h, part are device arrays of n
 * elements; h or part may be NULL.  Any 32-bit ids are accepted.
 * Asynchronous on the context stream. */
crop_status crop_hash_pairs(crop_ctx *ctx, const uint32_t *qx, const uint32_t *qy, uint64_t n,
                            uint32_t *h, uint32_t *part);

/* Wait for all work enqueued by this context. */
crop_status crop_synchronize(crop_ctx *ctx);

/* Device time in milliseconds of the last run, from HIP events recorded on
 * the context stream around its kernels (synchronizes). */
crop_status crop_last_run_ms(crop_ctx *ctx, float *ms);

/* ---- Count-Sketch ------------------------------------------------------- */
/* Count-Sketch per bucket (Section 4, "Frequent items mining algorithms";
 * Section 6, Theorem 3): B buckets per partition, bucket = (h * P * B) >> 32,
 * one signed counter per bucket; every term adds s(e) * w(e) (s = +-1 from the
 * sign hash; w = 1 for transactions, a_k(i) b_k(j) for outer products).
 * `instances` (1..15) independent sketches use the hash parameters of
 * seed + i.  Counters are int32 for transactions (exact), fp32 for outer
 * products.  P * B <= 2^32.  Each instance's terms are routed into bins of
 * whole buckets and summed per bin on chip when B has a suitable divisor
 * (bins_per_partition of crop_set_tuning picks it when it divides B); else
 * every term adds to its counter with a device atomic. */
crop_status crop_run_countsketch(crop_ctx *ctx, uint32_t buckets_per_partition,
                                 uint32_t instances);
/* Median over the instances of s_i(e) * C_i[bucket_i(e)] for each query pair
 * (qx[q], qy[q]); device arrays; est[n] doubles (the mean of the two middle
 * estimates for an even instance count). */
crop_status crop_countsketch_estimate(crop_ctx *ctx, const uint32_t *qx, const uint32_t *qy,
                                      uint64_t n, double *est);
/* The P * B counters of one instance into a host array (synchronizes). */
crop_status crop_read_countsketch(crop_ctx *ctx, uint32_t instance, double *out, uint64_t cap);

/* ---- batches of transaction streams ----------------------------------- */
/* Many independent streams in one exact run.  Each stream is accumulated
 * exactly as crop_run_exact would (Section 7: the pairs x < y of every
 * transaction), in partitions of its own consistent hash (Section 6,
 * Theorem 1; the same seed for every stream).  The batch is one pass: one
 * count, scan, scatter and persistent aggregation launch over every bin of
 * every stream, replayed as a captured HIP graph.
 *
 * Input: one CSR of all transactions, stream after stream; stream s is
 * transactions [tx_off[s], tx_off[s+1]).  tx_off (n_streams + 1 entries) and
 * n_items (item ids of stream s are below n_items[s]) are host arrays;
 * off (tx_off[n_streams] + 1 item offsets, off[0] = 0) and items live in
 * `where`.  Validation as crop_load_transactions, per stream; the error index
 * is the global transaction.  Totals must stay below 2^32 terms. */
crop_status crop_load_batch(crop_ctx *ctx, uint32_t n_streams, const uint64_t *tx_off,
                            const uint32_t *off, const uint32_t *items, const uint32_t *n_items,
                            crop_mem where, crop_own own);
/* Plan knobs: routed terms aimed at per bin (each stream gets
 * ceil(terms / terms_per_bin) partitions, at most 8192) and transactions per
 * chunk (rows_per_chunk; halved while a chunk does not fit in LDS).  A batch
 * whose item ids all pack into 32-bit keys takes the region route (one
 * segment per stream: its sub-batches sorted by bin in LDS and read in place
 * by the aggregation), where rows_per_chunk does not apply. */
crop_status crop_batch_set_plan(crop_ctx *ctx, uint32_t terms_per_bin, uint32_t rows_per_chunk);
/* Time every candidate plan (terms_per_bin in {15000, 30000, 60000} x
 * rows_per_chunk in {64, 128, 256}; on the region route terms_per_bin only)
 * reps times on the loaded batch, keep the fastest, and remember it for
 * later batches of the same shape in this process.  Outputs (NULL allowed):
 * the chosen knobs (rows_per_chunk 0 on the region route) and its time. */
crop_status crop_batch_autotune(crop_ctx *ctx, uint32_t reps, uint32_t *terms_per_bin,
                                uint32_t *rows_per_chunk, float *best_ms);
/* Replay the run as a captured HIP graph (default 1) or launch eagerly (0;
 * per-stage events available with crop_set_profiling). */
crop_status crop_batch_set_graph(crop_ctx *ctx, int enable);
crop_status crop_run_exact_batched(crop_ctx *ctx);
/* Stream s: its partition count (0 before a plan), terms, first transaction
 * and transaction count (NULL allowed for any output). */
crop_status crop_batch_info(crop_ctx *ctx, uint32_t stream, uint32_t *partitions,
                            uint64_t *terms, uint64_t *first_tx, uint64_t *n_tx);
/* Per partition of stream s: distinct pairs and terms (host arrays of the
 * stream's partition count). */
crop_status crop_batch_result_sizes(crop_ctx *ctx, uint32_t stream, uint64_t *sizes,
                                    uint64_t *terms_per_partition);
/* Exact result of stream s, partition by partition, as crop_read_all. */
crop_status crop_batch_read_stream(crop_ctx *ctx, uint32_t stream, crop_mem where, uint32_t *i,
                                   uint32_t *j, uint32_t *count, uint64_t cap, uint64_t *written,
                                   uint64_t *part_off);

/* ---- learned heavy-pair seeding (an addition; not in the paper) -------- */
/* All arrays below are device memory; calls are asynchronous on the context
 * stream unless they return host data.  Section 6 (Theorem 2's proof) names
 * the failure the seeding targets: a heavy entry is lost when too many heavy
 * entries or too much light weight share its bucket; pinning predicted heavy
 * pairs (crop_run_topk_seeded) counts them exactly from the start. */

/* 16 fp32 features per item (feat[n_items * 16]) from the first prefix_T
 * transactions of the loaded stream: counts, pair occurrences, lengths,
 * first/second-half counts and the rank of the item's count. */
crop_status crop_item_features(crop_ctx *ctx, uint32_t prefix_T, float *feat);
/* crop_item_features for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments and output, but the per-item statistics live
 * in a fixed per-GPU array of 2^21 32-bit words (8 MiB) inside the library
 * instead of a workspace it allocates, so 8 n_items + prefix_T + 66 must be
 * at most 2^21 (CROP_E_CAPACITY otherwise, with the size in the detail).
 * Nothing is allocated by this call.  All calls on one GPU share that
 * array: calls that overlap on one GPU (other streams or contexts) race,
 * and the caller must order them. */
crop_status crop_item_features_noalloc(crop_ctx *ctx, uint32_t prefix_T, float *feat);

/* Candidate pairs x < y among the M items with the largest prefix counts
 * (ties by smaller id), in (x, y) order: cx, cy of capacity cap >= M(M-1)/2;
 * *n_pairs receives M(M-1)/2. */
crop_status crop_top_item_pairs(crop_ctx *ctx, uint32_t prefix_T, uint32_t M, uint32_t *cx,
                                uint32_t *cy, uint64_t cap, uint64_t *n_pairs);

/* Exact supports of query pairs (qx[q] < qy[q]) in the last exact run of a
 * transaction stream; 0 for a pair that never occurs.  n <= 2^30. */
crop_status crop_lookup_exact(crop_ctx *ctx, const uint32_t *qx, const uint32_t *qy, uint64_t n,
                              uint32_t *count);

/* Network inputs Z[n * 32] = [feat[cx], feat[cy]] and, when count is given,
 * labels y[n] = log1p(count). */
crop_status crop_pair_inputs(crop_ctx *ctx, const float *feat, const uint32_t *cx,
                             const uint32_t *cy, const uint32_t *count, uint64_t n, float *Z,
                             float *y);

/* A 32 -> 64 -> 64 -> 1 ReLU network with fp32 weights kept on the device.
 * init: host array of 6337 floats in the order W1[64][32], b1[64],
 * W2[64][64], b2[64], w3[64], b3. */
typedef struct crop_mlp crop_mlp;
crop_status crop_mlp_create(crop_ctx *ctx, const float *init, crop_mlp **out);
void crop_mlp_destroy(crop_mlp *mlp);
/* Current weights into a host array of 6337 floats (synchronizes). */
crop_status crop_mlp_params(crop_ctx *ctx, const crop_mlp *mlp, float *out);
/* Gradient (host, 6337 floats) and loss of the mean squared error over the
 * N <= 128 samples Z[N * 32], y[N] at the current weights (synchronizes). */
crop_status crop_mlp_grad(crop_ctx *ctx, crop_mlp *mlp, const float *Z, const float *y,
                          uint32_t N, float *grad, float *loss);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) over the
 * minibatches order[0..batch), order[batch..2 batch), ... of sample indices
 * into Z[n_samples * 32], y[n_samples]; batch <= 128; a trailing partial
 * batch is ignored.  CROP_E_INPUT (nothing trained) if an index is
 * >= n_samples.  Synchronizes once to check the indices. */
crop_status crop_mlp_train(crop_ctx *ctx, crop_mlp *mlp, const float *Z, const float *y,
                           uint64_t n_samples, const uint32_t *order, uint64_t n_order,
                           uint32_t batch, float lr);
/* Mean loss of the last training minibatch (synchronizes). */
crop_status crop_mlp_loss(crop_ctx *ctx, const crop_mlp *mlp, float *loss);
/* Scores out[N] with weights and inputs rounded to bfloat16 (ties to even)
 * and fp32 accumulation. */
crop_status crop_mlp_score(crop_ctx *ctx, const crop_mlp *mlp, const float *Z, uint64_t N,
                           float *out);
/* The R candidates with the highest scores (ties by candidate index), in
 * rank order, as seeds sx[R], sy[R] for crop_run_topk_seeded. */
crop_status crop_select_seeds(crop_ctx *ctx, const float *score, const uint32_t *cx,
                              const uint32_t *cy, uint64_t n, uint32_t R, uint32_t *sx,
                              uint32_t *sy);

/* The predictor as one object: training and scoring composed from the calls
 * above.  A training stream is a CSR transaction stream as for
 * crop_load_transactions; the arrays of every stream of a set live in
 * `where` (device arrays are borrowed for the call, host arrays copied). */
typedef struct crop_stream_ref {
    const uint32_t *off;   /* T + 1 offsets */
    uint64_t T;
    const uint32_t *items; /* nnz item ids, strictly increasing per row */
    uint64_t nnz;
    uint32_t n_items;
} crop_stream_ref;
typedef struct crop_train_set {
    const crop_stream_ref *streams;
    uint32_t n_streams;
    crop_mem where;
} crop_train_set;
/* Zero fields take the defaults in brackets. */
typedef struct crop_train_opts {
    uint32_t top_items;    /* M: candidates are the pairs of the M items most
                              frequent in a stream's prefix [256]            */
    uint32_t epochs;       /* passes over the samples [4]                    */
    uint32_t batch;        /* Adam minibatch, <= 128 [128]                   */
    float lr;              /* Adam learning rate [1e-3]                      */
    uint64_t shuffle_seed; /* SplitMix64 seed of the minibatch order (one
                              Fisher-Yates permutation per epoch) and of the
                              default initial weights                        */
    const float *init;     /* host, 6337 initial weights in crop_mlp_create's
                              order, or NULL: He-uniform +-sqrt(6/fan_in),
                              zero biases                                    */
} crop_train_opts;
typedef struct crop_predictor crop_predictor;

/* Train a predictor: for each training stream an exact run under the
 * context's seed and P gives the labels log1p(support) of the candidate
 * pairs of its prefix (crop_item_features over the first ceil(T/20)
 * transactions, crop_top_item_pairs with M = top_items, crop_lookup_exact,
 * crop_pair_inputs); then crop_mlp_train over all samples.  The work runs on
 * a private context of the same GPU: the caller's loaded input, results and
 * stream are left as they were (this call synchronizes the caller's stream
 * first).  *out owns its device weights until crop_predictor_free.
 * Errors: CROP_E_ARG for an empty set or bad options, CROP_E_INPUT for an
 * invalid stream (crop_last_error_index: the offending transaction of that
 * stream), else as the calls it makes. */
crop_status crop_predictor_train(crop_ctx *ctx, const crop_train_set *set,
                                 const crop_train_opts *opts, crop_predictor **out);
/* Seeds for the loaded transaction stream: features and candidate pairs of
 * its prefix, bf16 scores (crop_mlp_score) and the R best candidates, in rank
 * order, into device arrays sx, sy of capacity R, for crop_run_topk_seeded.
 * *n_seeds (may be NULL) receives min(R, M(M-1)/2).  Synchronizes. */
crop_status crop_predictor_score(crop_ctx *ctx, const crop_predictor *pred, uint32_t R,
                                 uint32_t *sx, uint32_t *sy, uint64_t *n_seeds);
/* The trained weights (host array of 6337 floats, crop_mlp_create's order)
 * and the mean loss of the last training minibatch (may be NULL). */
crop_status crop_predictor_params(crop_ctx *ctx, const crop_predictor *pred, float *out,
                                  float *last_loss);
void crop_predictor_free(crop_predictor *pred);

/* Profiling: when enabled, every run also records one HIP event after each
 * of its stages (kernels or kernel groups) on the context stream, kept for
 * the last 64 runs.  Off by default. */
crop_status crop_set_profiling(crop_ctx *ctx, int enable);
/* Stage names (static strings) and device milliseconds of run number
 * `back` counted from the most recent (0) while profiling was on; names or
 * ms may be NULL.  *n_stages receives the stage count (synchronizes). */
crop_status crop_run_stages(crop_ctx *ctx, uint32_t back, uint32_t *n_stages,
                            const char **names, float *ms, uint32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* CROP_H */
