#!/usr/bin/env python3
"""Throughput of the CRoP hot path on one MI355X.

Workload: the 1,000,000-transaction stream (50,000 items, Zipf s = 1.1,
lengths Geom(mean 10) capped at 64; about 8.9e7 pair occurrences), exact
uint32 pair supports in P = 1024 partitions by the consistent hash.  One
step is one full pass of the hot path over the stream already resident in
HBM: enumerate every pair, route it to its owner by the hash, accumulate
every owner exactly (crop_run_exact: count, scan, scatter, aggregate
kernels).  The metric is term-updates per second (pair occurrences per
second).

Printed: one JSON line with the throughput, the roofline of the dominant
kernel (HIP events on the library's stream over the timed steps), the CPU
oracle timed on the same stream (single-threaded, about half a minute; its
result also gives a whole-result equality check), the paper's own method on
the host cores (multi-threaded, median of 3), and the top-1000 recall of the
Space-Saving summaries, plain and learned-seeded at equal memory, on a
held-out stream (the learned-seeding workload: 20 training streams of 1M
transactions, seeds 5000-5019, held-out seed 5100).

--batched times the 256-stream batched workload (one tuned plan replayed as
a captured HIP graph).  --learned runs the learned-seeding comparison: an MLP trained on
the GPU on 20 training streams like the one above, used to pin predicted
heavy pairs into the Space-Saving summaries of a held-out stream, against
the plain summaries at equal memory, in two regimes (P = 1024 with 2^14
counters per partition, and P = 1 with 16,384 counters).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "outer-product term-updates/sec at 1 GPU (exact) + top-1000 recall vs exact oracle"
HBM_PEAK_GBS = 8000.0
SEED = 0x243F6A8885A308D3
P = 1024


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU legs: the oracle and the host CRoP (profiling runs)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-seeding leg of the default line (profiling runs)")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="transactions of the stream the CPU oracle is timed on; the "
                         "whole stream also gives the recall and equality checks")
    ap.add_argument("--learned", action="store_true",
                    help="run the learned-seeding comparison instead of the exact bench")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the exact run's plan (crop_autotune) before timing")
    ap.add_argument("--outer", action="store_true",
                    help="the outer-product workload: exact fp32 sums and top 10,000")
    ap.add_argument("--accuracy", action="store_true",
                    help="synthetic analogs of the paper's accuracy experiments")
    ap.add_argument("--shards", type=int, default=0,
                    help="time each of G owned-partition shares of the exact run")
    ap.add_argument("--batched", action="store_true",
                    help="time the 256-stream batched exact run instead of the exact bench")
    ap.add_argument("--train-streams", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--candidates", type=int, default=256,
                    help="top prefix items M; candidates are their M(M-1)/2 pairs")
    ap.add_argument("--seeds", type=int, default=1000)
    ap.add_argument("--r-max", type=int, default=4)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB buffer 5 times (HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy():
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters of a rocprofv3 --pmc run to bytes."""
    import torch
    n = 1 << 28  # 2^28 int32 = 1 GiB each way
    a = torch.ones(n, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n}))


# The sources of the exact path's kernels: the recorded PMC traffic is used
# only while they hash to the digest it was taken with.
STEP_SOURCES = ("k_route.hip", "k_sbroute.hip", "k_exact.hip", "crop_device.hpp",
                "crop_enum.hpp", "crop_hash.hpp", "crop_layout.hpp", "crop_runs.hpp")


def source_digest(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1210_0461_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, digest):
    """HBM bytes of one launch of `kernel` from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, KiB per dispatch, scaled by the copy
    kernel calibration), or None when absent or taken on other sources.
    Lines read: `source_digest = D`, `fetch_scale = F`, `write_scale = W`
    and `traffic <kernel> fetch_kib=A write_kib=B`."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic_large1M.txt")
    if not os.path.exists(path):
        return None
    rec, per = {}, {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("traffic "):
            parts = line.split()
            per[parts[1]] = dict(kv.split("=") for kv in parts[2:])
            continue
        k, _, v = line.partition("=")
        rec[k.strip()] = v.strip()
    if rec.get("source_digest") != digest or kernel not in per:
        return None
    fetch = float(per[kernel]["fetch_kib"]) * 1024 * float(rec["fetch_scale"])
    write = float(per[kernel]["write_kib"]) * 1024 * float(rec["write_scale"])
    return round(fetch + write)


def cpu_baseline(st, n_rows):
    """The oracle timed on the first n_rows transactions; also returns its
    result (the exact supports of that sample)."""
    import oracle
    sample = st.slice(0, min(n_rows, st.T))
    t0 = time.perf_counter()
    r = oracle.tx_exact(sample.off, sample.items, P, SEED)
    dt = time.perf_counter() - t0
    return {"value": r["n_terms"] / dt, "unit": "term-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample.T} transactions of the 1M stream "
                      f"({r['n_terms']} terms), P={P}, {dt:.2f} s single-threaded",
            "seconds": round(dt, 3)}, r, sample.T


def host_cpu():
    """Model name, physical cores of the host and the threads this process
    may use (its affinity mask, at most 16: the CPU share a GPU gets)."""
    model, cores = "unknown", set()
    try:
        phys = core = None
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and model == "unknown":
                model = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                core = v
            elif not k and phys is not None:
                cores.add((phys, core))
                phys = core = None
    except OSError:
        pass
    threads = min(16, len(os.sched_getaffinity(0)))
    return model, len(cores) or None, threads


def cpu_crop_baseline(st, terms, reps=3):
    """The paper's method on the host (multi-threaded CRoP: every owner thread
    reads the whole stream, sorts each transaction by h_b and enumerates only
    the pairs of its hash interval, Lemma 1, into a private table), timed as
    the median of `reps` runs on the whole stream.  Context beside the GPU
    figure, not a target; the oracle stays the checker."""
    import numpy as np
    import oracle
    model, phys, threads = host_cpu()
    times, res = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        res = oracle.cpu_crop_tx(st.off, st.items, P, SEED, threads)
        times.append(time.perf_counter() - t0)
    med = sorted(times)[len(times) // 2]
    sizes, part_terms, distinct = res
    return {"value": terms / med, "unit": "term-updates/s", "threads": threads,
            "cpu_model": model, "physical_cores": phys, "kind": "paper's method (CRoP), "
            "owner threads with Lemma 1 windows", "seconds_median_of_3": round(med, 3),
            "seconds": [round(t, 3) for t in times],
            "sample": f"whole stream ({terms} terms), P={P}"}, sizes, part_terms


def learned_leg(streams, steps=3):
    """Learned seeding at its stated size on the default line: a predictor
    trained on the exact supports of 20 training streams (crop_predictor_*)
    seeds the Space-Saving summaries of the held-out stream with its 1,000
    best pairs (r_max 4); top-1000 recall and largest count error against
    the oracle's exact supports, plain vs seeded at equal memory, in the
    library's default report order, for one partition of 16,384 counters
    and 1,024 partitions of 2^14 counters (16 per bucket)."""
    import numpy as np
    import torch
    import oracle
    import paper_1210_0461_amd as crop
    K = 1000
    off, items, n = streams[-1]
    t0 = time.perf_counter()
    ref = oracle.tx_exact(off, items, 1, SEED)
    rk, rc = sorted_pairs(ref["x"], ref["y"], ref["cnt"])
    oracle_s = time.perf_counter() - t0
    terms = int(ref["n_terms"])
    ctx = crop.crop_create(0)
    out = {"train_streams": len(streams) - 1, "K": K, "top_items": 256, "epochs": 4,
           "r_max": 4, "oracle_seconds": round(oracle_s, 2)}
    try:
        crop.crop_set_stream(ctx, torch.cuda.current_stream())
        crop.crop_set_seed(ctx, SEED)
        crop.crop_set_partitions(ctx, P)
        t0 = time.perf_counter()
        pred = crop.crop_predictor_train(ctx, streams[:-1], top_items=256, epochs=4, batch=128,
                                         lr=1e-3, shuffle_seed=6000)
        torch.cuda.synchronize()
        out["train_seconds"] = round(time.perf_counter() - t0, 2)
        try:
            crop.crop_load_transactions(ctx, off, items, n)
            sx = torch.zeros(K, dtype=torch.int32, device="cuda")
            sy = torch.zeros(K, dtype=torch.int32, device="cuda")
            crop.crop_predictor_score(ctx, pred, K, sx, sy)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            for Pr, C in ((1, 16384), (1024, 1 << 14)):
                crop.crop_set_partitions(ctx, Pr)
                crop.crop_set_summary(ctx, C, 16)
                row = {}
                for mode in ("plain", "seeded"):
                    def once():
                        if mode == "plain":
                            crop.crop_run_topk(ctx, K)
                        else:
                            crop.crop_run_topk_seeded(ctx, K, sx, sy, 4)
                    once()
                    torch.cuda.synchronize()
                    ev0.record()
                    for _ in range(steps):
                        once()
                    ev1.record()
                    torch.cuda.synchronize()
                    ms = ev0.elapsed_time(ev1) / steps
                    i, j, up, lo, _ = crop.crop_read_topk(ctx, K)
                    rep = (i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
                    rec, exact = recall_vs(rk, rc, rep, K)
                    row[mode] = {"recall_at_1000": rec,
                                 "max_count_error": float((up - exact).max()) if up.size else 0.0,
                                 "max_lower_bound_gap": float((exact - lo).max()) if lo.size else 0.0,
                                 "ms": round(ms, 4), "term_updates_per_s": terms / (ms * 1e-3)}
                out[f"P{Pr}_C{C}"] = row
        finally:
            crop.crop_predictor_free(pred)
    finally:
        crop.crop_destroy(ctx)
    return out


def sorted_pairs(x, y, c):
    import numpy as np
    k = (np.asarray(x, np.uint64) << np.uint64(32)) | np.asarray(y, np.uint64)
    o = np.argsort(k, kind="stable")
    return k[o], np.asarray(c, np.int64)[o]


def top_keys(keys, cnt, K):
    """First K keys by (count desc, key asc) and the K-th count."""
    import numpy as np
    o = np.lexsort((keys, -cnt))[:K]
    return keys[o], int(cnt[o[-1]]) if o.shape[0] else 0


def recall_vs(ref_keys, ref_cnt, rep_keys, K):
    """Tie-tolerant recall@K of reported keys against exact supports
    (ref_keys sorted): a hit has an exact support >= the K-th largest."""
    import numpy as np
    _, cK = top_keys(ref_keys, ref_cnt, K)
    pos = np.searchsorted(ref_keys, rep_keys)
    pos = np.minimum(pos, ref_keys.shape[0] - 1)
    found = ref_keys[pos] == rep_keys
    exact = np.where(found, ref_cnt[pos], 0)
    return float((exact >= cK).sum()) / min(K, ref_keys.shape[0]), exact


def _gen_learned(i):
    import datagen
    st = datagen.config_learned_heldout() if i < 0 else datagen.config_learned_train(i)
    return st.off, st.items, st.n


def run_learned(args):
    """Plain vs learned-seeded Space-Saving top-1000 on the held-out stream."""
    import multiprocessing as mp
    import numpy as np
    t0 = time.perf_counter()
    # streams are generated in worker processes before this process touches the GPU
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        streams = pool.map(_gen_learned, list(range(args.train_streams)) + [-1])
    print(f"# generated {len(streams)} streams in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    import torch
    import datagen
    import oracle
    import paper_1210_0461_amd as crop
    from paper_1210_0461_amd import seeding

    M, K, ell = args.candidates, 1000, 16
    ctx = crop.crop_create(0)
    crop.crop_set_stream(ctx, torch.cuda.current_stream())
    out = {"experiment": "learned heavy-pair seeding vs plain Space-Saving, equal memory",
           "train_streams": args.train_streams, "candidates_per_stream": M * (M - 1) // 2,
           "top_items_M": M, "K": K, "ell": ell, "seeds": args.seeds, "r_max": args.r_max}
    try:
        crop.crop_set_seed(ctx, SEED)
        crop.crop_set_partitions(ctx, P)
        Zs, ys = [], []
        t0 = time.perf_counter()
        for off, items, n in streams[:-1]:
            crop.crop_load_transactions(ctx, off, items, n)
            Z, y, _, _, _ = seeding.training_pairs(ctx, off.shape[0] - 1, n, M)
            Zs.append(Z)
            ys.append(y)
        Z = torch.cat(Zs)
        y = torch.cat(ys)
        torch.cuda.synchronize()
        out["label_seconds"] = round(time.perf_counter() - t0, 3)
        order = torch.from_numpy(
            datagen.sample_order(6000, Z.shape[0], args.epochs).astype(np.int32)).cuda()
        mlp = crop.crop_mlp_create(ctx, seeding.flat_init(datagen.mlp_init_weights(6001)))
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        crop.crop_mlp_train(ctx, mlp, Z, y, order, 128, args.lr)
        ev1.record()
        torch.cuda.synchronize()
        steps = order.shape[0] // 128
        out["train"] = {"samples": int(Z.shape[0]), "epochs": args.epochs, "batch": 128,
                        "steps": steps, "lr": args.lr,
                        "ms": round(ev0.elapsed_time(ev1), 2),
                        "final_batch_mse": crop.crop_mlp_loss(ctx, mlp)}

        off, items, n = streams[-1]
        T = off.shape[0] - 1
        t0 = time.perf_counter()
        ref = oracle.tx_exact(off, items, 1, SEED)
        rk, rc = sorted_pairs(ref["x"], ref["y"], ref["cnt"])
        true_top, cK = top_keys(rk, rc, K)
        out["oracle_seconds"] = round(time.perf_counter() - t0, 2)
        out["kth_support"] = cK
        out["terms"] = int(ref["n_terms"])
        crop.crop_load_transactions(ctx, off, items, n)
        # predictor quality on the held-out candidates: precision of the seeds
        ev0.record()
        sx, sy, score = seeding.predict_seeds(ctx, mlp, T, n, M, args.seeds)
        ev1.record()
        torch.cuda.synchronize()
        seed_keys = ((sx.cpu().numpy().astype(np.uint32).astype(np.uint64) << np.uint64(32)) |
                     sy.cpu().numpy().astype(np.uint32).astype(np.uint64))
        out["seed_ms"] = round(ev0.elapsed_time(ev1), 3)
        out["seeds_in_true_top1000"] = int(np.isin(seed_keys, true_top).sum())

        regimes = []
        for Pr, C in ((1024, 1 << 14), (1, 16384)):
            crop.crop_set_partitions(ctx, Pr)
            crop.crop_set_summary(ctx, C, ell)
            row = {"P": Pr, "counters_per_partition": C, "total_counters": Pr * C}
            for mode, rank in (("plain", 0), ("seeded", 0), ("plain_lower", 1),
                               ("seeded_lower", 1)):
                crop.crop_set_topk_rank(ctx, rank)

                def once():
                    if mode.startswith("plain"):
                        crop.crop_run_topk(ctx, K)
                    else:
                        crop.crop_run_topk_seeded(ctx, K, sx, sy, args.r_max)
                once()
                torch.cuda.synchronize()
                ev0.record()
                for _ in range(args.steps):
                    once()
                ev1.record()
                torch.cuda.synchronize()
                ms = ev0.elapsed_time(ev1) / args.steps
                i, j, up, lo, _ = crop.crop_read_topk(ctx, K)
                rep = (i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
                rec, exact = recall_vs(rk, rc, rep, K)
                # the true top-K pairs as the summary holds them
                s = crop.crop_read_summary(ctx, Pr * C)
                sk = (s["x"].astype(np.uint64) << np.uint64(32)) | s["y"].astype(np.uint64)
                held = np.isin(true_top, sk[s["used"]])
                sel = np.isin(sk, true_top) & s["used"]
                row[mode] = {"recall_at_1000": rec,
                             "max_count_error": float((up - exact).max()) if up.size else 0.0,
                             "max_lower_bound_gap": float((exact - lo).max()) if lo.size else 0.0,
                             "true_top_monitored": int(held.sum()),
                             "true_top_with_error": int((s["err"][sel] > 0).sum()),
                             "pinned": int(s["pinned"].sum()),
                             "ms": round(ms, 4),
                             "term_updates_per_s": out["terms"] / (ms * 1e-3)}
            regimes.append(row)
            print(f"# regime P={Pr} C={C}: {json.dumps(row)}", file=sys.stderr, flush=True)
        out["regimes"] = regimes
        crop.crop_mlp_destroy(mlp)
    finally:
        crop.crop_destroy(ctx)
    print(json.dumps(out), flush=True)


def _gen_batched(s):
    import datagen
    st = datagen.config_batched_stream(s)
    return st.off, st.items, st.n


def run_batched(args):
    """The 256-stream workload as one batched exact run (tuned plan, captured
    HIP graph); throughput over all streams."""
    import multiprocessing as mp
    import numpy as np
    t0 = time.perf_counter()
    # streams are generated in worker processes before this process touches the GPU
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        streams = pool.map(_gen_batched, range(256))
    print(f"# generated 256 streams in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    import torch
    import paper_1210_0461_amd as crop
    T = np.array([o.shape[0] - 1 for o, _, _ in streams], np.int64)
    nnz = np.array([i.shape[0] for _, i, _ in streams], np.int64)
    tx = np.concatenate([[0], np.cumsum(T)]).astype(np.uint64)
    base = np.concatenate([[0], np.cumsum(nnz)])
    off = np.concatenate([o[:-1].astype(np.int64) + base[k] for k, (o, _, _) in
                          enumerate(streams)] + [[base[-1]]]).astype(np.uint32)
    items = np.concatenate([i for _, i, _ in streams])
    n_items = np.array([n for _, _, n in streams], np.uint32)
    dev = torch.device("cuda:0")
    doff = torch.from_numpy(off.view(np.int32)).to(dev)
    ditems = torch.from_numpy(items.view(np.int32)).to(dev)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize(dev)
    ctx = crop.crop_create(0)
    try:
        crop.crop_set_stream(ctx, stream)
        crop.crop_set_seed(ctx, SEED)
        crop.crop_load_batch(ctx, tx, doff, ditems, n_items, own=crop.CROP_OWN_BORROW)
        t0 = time.perf_counter()
        tpb, R, tune_ms = crop.crop_batch_autotune(ctx, 2)
        tune_s = time.perf_counter() - t0
        for _ in range(args.warmup):
            crop.crop_run_exact_batched(ctx)
        torch.cuda.synchronize(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            crop.crop_run_exact_batched(ctx)
        e1.record(stream)
        torch.cuda.synchronize(dev)
        ms = e0.elapsed_time(e1) / args.steps
        terms = 0
        distinct = 0
        parts = []
        for k in range(256):
            info = crop.crop_batch_info(ctx, k)
            sizes, pt = crop.crop_batch_result_sizes(ctx, k)
            terms += int(pt.sum())
            distinct += int(sizes.sum())
            parts.append(info["partitions"])
        # eager run with per-stage times
        crop.crop_batch_set_graph(ctx, False)
        crop.crop_set_profiling(ctx, True)
        crop.crop_run_exact_batched(ctx)
        crop.crop_synchronize(ctx)
        stages = {n: round(m, 4) for n, m in crop.crop_run_stages(ctx, 0)}
    finally:
        crop.crop_destroy(ctx)
    L = np.diff(off.astype(np.int64))
    assert terms == int((L * (L - 1) // 2).sum())
    alg = 4 * items.shape[0] + 4 * off.shape[0] + 8 * distinct
    gbs = alg / (ms * 1e-3) / 1e9
    out = {"experiment": "batched exact run, 256 streams in one captured HIP graph",
           "streams": 256, "transactions": int(T.sum()), "items": int(items.shape[0]),
           "terms": terms, "distinct_pairs": distinct, "ms_per_run": round(ms, 4),
           "term_updates_per_s": terms / (ms * 1e-3),
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes": alg},
           "autotune": {"terms_per_bin": tpb, "rows_per_chunk": R, "best_ms": round(tune_ms, 4),
                        "seconds": round(tune_s, 2)},
           "partitions": {"min": int(min(parts)), "max": int(max(parts)),
                          "total": int(sum(parts))},
           "eager_stage_ms": stages}
    print(json.dumps(out), flush=True)


def run_accuracy(args):
    """Synthetic analogs of the paper's accuracy experiments on the
    1M-transaction stream (Section 7.3):
    * bounds ratio: mean lower/upper bound of the reported top 100 against the
      number of buckets, two counters per bucket (Figure 2b);
    * counters per bucket at a fixed total of counters: reported pairs with
      lower >= 90% of upper until the 100th that is not (Figure 3, left);
    * recall of the top 10,000 with 10,000 counters per partition on P
      partitions (Table 2);
    * the Count-Sketch protocol (Figure 3, right; Theorem 2's majority
      reporting): eleven instances of 50,000 buckets x 2 pairs, pairs
      reported by at least six get the median Count-Sketch estimate;
      estimate / support for the true top 3,000."""
    import numpy as np
    import torch
    import datagen
    import oracle
    import paper_1210_0461_amd as crop
    st = datagen.config_large()
    t0 = time.perf_counter()
    ref = oracle.tx_exact(st.off, st.items, 1, SEED)
    rk, rc = sorted_pairs(ref["x"], ref["y"], ref["cnt"])
    print(f"# oracle {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    def exact_of(keys):
        pos = np.minimum(np.searchsorted(rk, keys), rk.shape[0] - 1)
        return np.where(rk[pos] == keys, rc[pos], 0)

    ctx = crop.crop_create(0)
    crop.crop_set_stream(ctx, torch.cuda.current_stream())
    crop.crop_set_seed(ctx, SEED)
    crop.crop_load_transactions(ctx, st.off, st.items, st.n)
    out = {"experiment": "accuracy analogs on the 1M-transaction stream", "terms": int(ref["n_terms"])}
    try:
        def topk(P, C, ell, K):
            crop.crop_set_partitions(ctx, P)
            crop.crop_set_summary(ctx, C, ell)
            crop.crop_run_topk(ctx, K)
            i, j, up, lo, _ = crop.crop_read_topk(ctx, K)
            keys = (i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
            return keys, up, lo

        rows = []
        for lb in range(8, 21, 2):
            B = 1 << lb
            keys, up, lo = topk(1, 2 * B, 2, 100)
            rows.append({"buckets": B, "mean_lower_over_upper": float(np.mean(lo / up))})
        out["bounds_ratio_vs_buckets"] = rows

        rows = []
        total = 1 << 17
        for ell in (2, 4, 8, 12, 16, 24):
            C = total // ell * ell
            keys, up, lo = topk(1, C, ell, 20000)
            good = lo >= 0.9 * up
            bad_pos = np.flatnonzero(~good)
            cut = bad_pos[99] if bad_pos.shape[0] >= 100 else good.shape[0]
            rows.append({"ell": ell, "counters": C, "good_before_100th_bad": int(good[:cut].sum())})
        out["good_estimates_vs_ell"] = rows

        rows = []
        _, cK = top_keys(rk, rc, 10000)
        for P in (1, 2, 4, 8, 16, 32):
            keys, up, lo = topk(P, 10000, 2, 10000)
            rec, _ = recall_vs(rk, rc, keys, 10000)
            rows.append({"P": P, "counters": 10000 * P, "recall_top10000": rec})
        out["recall_vs_P"] = rows

        # The Count-Sketch protocol of Figure 3 (right): 50,000 buckets of two
        # pairs, eleven instances; a pair reported by at least six instances'
        # summaries gets the median of its eleven Count-Sketch estimates, an
        # unreported pair the ratio 0.  Ratios to the exact count of the true
        # top 3,000; Space-Saving's intersected upper bound beside it, and a
        # single instance for comparison.
        true_top, _ = top_keys(rk, rc, 3000)
        f = exact_of(true_top).astype(np.float64)
        t_amp, votes_min, B = 11, 6, 50000
        crop.crop_set_partitions(ctx, 1)
        crop.crop_set_summary(ctx, 2 * B, 2)
        crop.crop_run_topk_amplified(ctx, 2 * B * t_amp, t_amp, votes_min)
        i, j, up, lo, _ = crop.crop_read_topk(ctx, 2 * B * t_amp)
        amp_keys = (i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
        amp_up = dict(zip(amp_keys.tolist(), up.tolist()))
        crop.crop_run_countsketch(ctx, B, t_amp)
        qx = torch.from_numpy((true_top >> np.uint64(32)).astype(np.uint32).view(np.int32)).cuda()
        qy = torch.from_numpy((true_top & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.int32)).cuda()
        est = torch.empty(3000, dtype=torch.float64, device="cuda")
        crop.crop_countsketch_estimate(ctx, qx, qy, est)
        reported = np.array([int(k) in amp_up for k in true_top])
        r_cs = np.where(reported, est.cpu().numpy() / f, 0.0)
        r_amp = np.array([amp_up.get(int(k), 0.0) for k in true_top]) / f
        keys, up1, lo1 = topk(1, 2 * B, 2, 2 * B)
        one = dict(zip(keys.tolist(), up1.tolist()))
        r_one = np.array([one.get(int(k), 0.0) for k in true_top]) / f
        q = lambda a: [round(float(x), 4) for x in np.quantile(a, [0.05, 0.5, 0.95])]
        w2 = lambda a: float(np.mean((a > 0.5) & (a < 2)))
        out["countsketch_protocol_top3000"] = {
            "buckets": B, "pairs_per_bucket": 2, "instances": t_amp, "min_votes": votes_min,
            "reported_by_majority": float(reported.mean()),
            "cs_median_ratio_q05_q50_q95": q(r_cs), "cs_within_factor_2": w2(r_cs),
            "ss_majority_upper_ratio_q05_q50_q95": q(r_amp), "ss_majority_within_factor_2": w2(r_amp),
            "ss_single_reported": float((r_one > 0).mean()),
            "ss_single_upper_ratio_q05_q50_q95": q(r_one), "ss_single_within_factor_2": w2(r_one)}
    finally:
        crop.crop_destroy(ctx)
    print(json.dumps(out), flush=True)


def run_outer(args):
    """The outer-product workload (100,000 products over 200,000 rows and
    columns, nnz per vector ~ m^-2 on [1, 2000], fp32 values; P = 8):
    exact fp32 sums with the tolerance pass rate against the oracle's fp64
    sums (|c32 - c64| <= 1e-5 sum |terms|), and the Space-Saving top 10,000
    (2^16 counters per partition, 16 per bucket, weights |a b|) with its
    recall of the exact top 10,000 by sum |a b| and by |sum a b|."""
    import numpy as np
    import torch
    import datagen
    import oracle
    import paper_1210_0461_amd as crop
    Pop = 8
    op = datagen.config_outer()
    t0 = time.perf_counter()
    ref = oracle.op_exact(op, 1, SEED)
    print(f"# oracle {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    rk = (ref["i"].astype(np.uint64) << np.uint64(32)) | ref["j"].astype(np.uint64)
    o = np.argsort(rk)
    rk, rsum, rabs = rk[o], ref["sum"][o], ref["abs"][o]
    terms = int(ref["n_terms"])
    ctx = crop.crop_create(0)
    out = {"experiment": "outer products: exact fp32 sums and Space-Saving top 10,000",
           "K": int(op.K), "terms": terms, "distinct": int(rk.shape[0]), "P": Pop}
    try:
        stream = torch.cuda.current_stream()
        crop.crop_set_stream(ctx, stream)
        crop.crop_set_partitions(ctx, Pop)
        crop.crop_set_seed(ctx, SEED)
        crop.crop_load_outer(ctx, op.a_off, op.a_idx, op.a_val, op.b_off, op.b_idx, op.b_val,
                             op.n_rows, op.n_cols)

        def timed(fn):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / args.steps

        ms = timed(lambda: crop.crop_run_exact(ctx))
        i, j, v, _ = crop.crop_read_all(ctx, Pop, outer=True)
        gk = (i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
        og = np.argsort(gk)
        same = gk.shape[0] == rk.shape[0] and bool(np.array_equal(gk[og], rk))
        err = np.abs(v[og].astype(np.float64) - rsum) if same else None
        out["exact"] = {"ms": round(ms, 4), "term_updates_per_s": terms / (ms * 1e-3),
                        "same_entries_as_oracle": same,
                        "within_tolerance": float(np.mean(err <= 1e-5 * rabs)) if same else 0.0,
                        "worst_err_over_abs": float(np.max(err / np.maximum(rabs, 1e-300)))
                        if same else None}
        crop.crop_set_summary(ctx, 1 << 16, 16)
        K = 10000
        ms = timed(lambda: crop.crop_run_topk(ctx, K))
        ti, tj, up, lo, val = crop.crop_read_topk(ctx, K)
        tk = (ti.astype(np.uint64) << np.uint64(32)) | tj.astype(np.uint64)
        kth = np.sort(rabs)[::-1][K - 1]
        kth_c = np.sort(np.abs(rsum))[::-1][K - 1]
        pos = np.minimum(np.searchsorted(rk, tk), rk.shape[0] - 1)
        found = rk[pos] == tk
        exact_abs = np.where(found, rabs[pos], 0.0)
        exact_c = np.where(found, np.abs(rsum[pos]), 0.0)
        out["topk"] = {"ms": round(ms, 4), "term_updates_per_s": terms / (ms * 1e-3), "K": K,
                       "recall_by_abs_weight": float(np.mean(exact_abs >= kth)),
                       "recall_by_abs_sum": float(np.mean(exact_c >= kth_c)),
                       "bounds_hold": bool(np.all(lo <= exact_abs * (1 + 1e-5) + 1e-6) and
                                           np.all(exact_abs <= up * (1 + 1e-5) + 1e-6))}
    finally:
        crop.crop_destroy(ctx)
    print(json.dumps(out), flush=True)


def run_shards(args):
    """One GPU's share of a G-GPU run: the exact path owning P/G partitions of
    the 1M-transaction stream (its terms found through Lemma 1's h_b windows
    of every transaction), for each of the G shares, against the whole run."""
    import numpy as np
    import torch
    import datagen
    import paper_1210_0461_amd as crop
    G = args.shards
    st = datagen.config_large()
    dev = torch.device("cuda:0")
    off = torch.from_numpy(st.off.view(np.int32)).to(dev)
    items = torch.from_numpy(st.items.view(np.int32)).to(dev)
    stream = torch.cuda.Stream(device=dev)
    ctx = crop.crop_create(0)
    out = {"experiment": f"one GPU's share of a {G}-GPU run (owned partitions)",
           "P": P, "shards": G}
    try:
        crop.crop_set_stream(ctx, stream)
        crop.crop_set_partitions(ctx, P)
        crop.crop_set_seed(ctx, SEED)
        crop.crop_load_transactions(ctx, off, items, st.n, own=crop.CROP_OWN_BORROW)
        crop.crop_set_profiling(ctx, True)

        def timed(p0, p1):
            crop.crop_set_owned_partitions(ctx, p0, p1)
            for _ in range(2):
                crop.crop_run_exact(ctx)
            torch.cuda.synchronize(dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                crop.crop_run_exact(ctx)
            e1.record(stream)
            torch.cuda.synchronize(dev)
            stages = {}
            for back in range(min(args.steps, 64)):
                for name, ms in crop.crop_run_stages(ctx, back):
                    stages.setdefault(name, []).append(ms)
            _, terms = crop.crop_result_sizes(ctx, P)
            return (e0.elapsed_time(e1) / args.steps, int(terms.sum()),
                    {k: round(sum(v) / len(v), 4) for k, v in stages.items()})

        full_ms, full_terms, full_st = timed(0, P)
        out["full"] = {"ms": round(full_ms, 4), "terms": full_terms, "stage_ms": full_st}
        # Table 3 analog: term loads (pair occurrences) per processor when
        # the P partitions are split into 2, 4 or 8 equal intervals, and per
        # partition
        _, part_terms = crop.crop_result_sizes(ctx, P)
        part_terms = part_terms.astype(np.float64)
        loads = {}
        for n in (2, 4, 8, P):
            per = part_terms.reshape(n, -1).sum(axis=1)
            loads[str(n)] = {"mean": round(float(per.mean()), 1), "max": int(per.max()),
                             "max_over_mean": round(float(per.max() / per.mean()), 4)}
        out["term_loads"] = loads
        shares = []
        for g in range(G):
            ms, terms, stg = timed(g * P // G, (g + 1) * P // G)
            shares.append({"partitions": [g * P // G, (g + 1) * P // G], "ms": round(ms, 4),
                           "terms": terms, "stage_ms": stg})
        out["shares"] = shares
        out["max_share_ms"] = max(x["ms"] for x in shares)
        out["speedup_bound_at_G"] = round(full_ms / out["max_share_ms"], 2)
    finally:
        crop.crop_destroy(ctx)
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by hash interval across GPUs with no exchange between them)",
              file=sys.stderr)
        sys.exit(2)
    if args.learned:
        run_learned(args)
        return
    if args.batched:
        run_batched(args)
        return
    if args.shards:
        run_shards(args)
        return
    if args.accuracy:
        run_accuracy(args)
        return
    if args.outer:
        run_outer(args)
        return
    import numpy as np
    import torch
    import datagen
    import paper_1210_0461_amd as crop

    learned_streams = None
    if not args.no_learned:
        import multiprocessing as mp
        t_gen = time.perf_counter()
        # generated in worker processes before this process touches the GPU
        with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
            learned_streams = pool.map(_gen_learned, list(range(20)) + [-1])
        print(f"# generated 21 learned-seeding streams in {time.perf_counter() - t_gen:.1f} s",
              file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    st = datagen.config_large()
    print(f"# generated {st.T} transactions, {st.nnz} items in "
          f"{time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    L = st.lengths()
    terms = int((L * (L - 1) // 2).sum())

    dev = torch.device("cuda:0")
    off = torch.from_numpy(st.off.view(np.int32)).to(dev)
    items = torch.from_numpy(st.items.view(np.int32)).to(dev)
    stream = torch.cuda.Stream(device=dev)  # default priority, not the null stream
    torch.cuda.synchronize(dev)
    ctx = crop.crop_create(0)
    try:
        crop.crop_set_stream(ctx, stream)
        crop.crop_set_partitions(ctx, P)
        crop.crop_set_seed(ctx, SEED)
        crop.crop_load_transactions(ctx, off, items, st.n, own=crop.CROP_OWN_BORROW)
        crop.crop_set_profiling(ctx, True)
        tuned = None
        if args.autotune:
            # before the warm-up and the timed steps, outside the timed region
            S_t, R_t, ms_t = crop.crop_autotune(ctx, 2)
            tuned = {"bins_per_partition": S_t, "rows_per_chunk": R_t, "best_ms": round(ms_t, 4)}
        for _ in range(args.warmup):
            crop.crop_run_exact(ctx)
        torch.cuda.synchronize(dev)

        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        e0.record(stream)
        for _ in range(args.steps):
            crop.crop_run_exact(ctx)
        e1.record(stream)
        torch.cuda.synchronize(dev)
        total_ms = e0.elapsed_time(e1)
        ms_per_step = total_ms / args.steps

        # per-stage device times of every timed step
        stages = {}
        for back in range(min(args.steps, 64)):
            for name, ms in crop.crop_run_stages(ctx, back):
                stages.setdefault(name, []).append(ms)
        stage_ms = {k: sum(v) / len(v) for k, v in stages.items()}
        sizes, part_terms = crop.crop_result_sizes(ctx, P)
        tune = crop.crop_get_tuning(ctx)
        gx, gy, gc, _ = crop.crop_read_all(ctx, P)   # result of the last timed step
    finally:
        crop.crop_destroy(ctx)

    distinct = int(sizes.sum())
    assert int(part_terms.sum()) == terms
    value = terms / (ms_per_step * 1e-3)

    # algorithmic bytes: every input word once + every distinct result once
    # (packed u32 key + u32 count)
    in_bytes = 4 * st.nnz + 4 * (st.T + 1)
    out_bytes = 8 * distinct
    alg_bytes = in_bytes + out_bytes
    per_term = alg_bytes / terms
    # the aggregation reads the region route's runs in place (k_aggregate_regions)
    # or the chunk route's bin-contiguous keys (k_aggregate_flat)
    regions = "route" in stage_ms
    kernel_names = {"count": "k_tx_count", "scan": "k_colsum/k_colbase/k_colapply",
                    "scatter": "k_tx_scatter_direct",
                    "aggregate": "k_aggregate_regions" if regions else "k_aggregate_flat",
                    "route": "k_sb_route", "headers": "k_sb_headers"}
    dom = max(stage_ms, key=stage_ms.get)
    dom_ms = stage_ms[dom]
    achieved = per_term * terms / (dom_ms * 1e-3) / 1e9
    digest = source_digest(*STEP_SOURCES)
    traffic = traffic_from_profiles(kernel_names[dom], digest)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": kernel_names[dom],
                "kernel_ms": round(dom_ms, 4),
                "alg_bytes_per_term": round(per_term, 4), "terms_per_launch": terms}
    path_gbs = alg_bytes / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "term-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "exact pair supports, 1M transactions over 50k items, "
                               "Zipf s=1.1, Geom(mean 10) lengths capped at 64, P=1024",
                   "transactions": st.T, "n_items": st.n, "nnz": st.nnz, "terms": terms,
                   "distinct_pairs": distinct, "P": P, "seed": SEED,
                   "bins_per_partition": tune["bins_per_partition"],
                   "rows_per_chunk": tune["rows_per_chunk"],
                   "plan": "autotuned" if tuned else "automatic"},
        "roofline": roofline,
        "path_roofline": {"bound": "hbm", "achieved": round(path_gbs, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(path_gbs / HBM_PEAK_GBS, 4),
                          "alg_bytes": alg_bytes},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "recall_top1000": {},
    }
    if traffic:
        roofline["kernel_traffic_gbs"] = round(traffic / (dom_ms * 1e-3) / 1e9, 1)
    if not args.no_cpu_baseline:
        crop_cpu, cpu_sizes, cpu_terms = cpu_crop_baseline(st, terms)
        crop_cpu["same_partition_sizes_as_gpu"] = bool(
            np.array_equal(cpu_sizes, sizes) and np.array_equal(cpu_terms, part_terms))
        out["cpu_crop"] = crop_cpu
        base, ref, rows = cpu_baseline(st, args.cpu_sample)
        out["cpu_baseline"] = base
        if rows == st.T:
            # the GPU's exact result against the oracle's: whole-result
            # equality and recall@1000 of the GPU's top 1000 pairs
            rk, rc = sorted_pairs(ref["x"], ref["y"], ref["cnt"])
            gk, gcnt = sorted_pairs(gx, gy, gc)
            top, _ = top_keys(gk, gcnt, 1000)
            out["recall_top1000"]["exact_path"], _ = recall_vs(rk, rc, top, 1000)
            out["exact_match_vs_oracle"] = bool(np.array_equal(rk, gk) and
                                                np.array_equal(rc, gcnt))
    if learned_streams is not None:
        lt = learned_leg(learned_streams)
        out["learned_top1000"] = lt
        for key in ("P1_C16384", "P1024_C16384"):
            for mode in ("plain", "seeded"):
                out["recall_top1000"][f"summary_{mode}_{key}"] = lt[key][mode]["recall_at_1000"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
