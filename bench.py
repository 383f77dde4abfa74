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
kernel (HIP events on the library's stream over the timed steps), and the
CPU oracle timed on a bounded sample of the same stream.
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
                    help="skip the CPU oracle leg (profiling runs)")
    ap.add_argument("--cpu-sample", type=int, default=500_000,
                    help="transactions of the stream the CPU oracle is timed on")
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


def source_digest(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1210_0461_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, digest, launches_bytes):
    """HBM bytes of one launch of `kernel` from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, KiB per dispatch, scaled by the copy
    kernel calibration), or None when absent or taken on other sources."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic_large1M.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, _, v = line.partition("=")
        rec[k.strip()] = v.strip()
    if rec.get("kernel") != kernel or rec.get("source_digest") != digest:
        return None
    fetch = float(rec["fetch_kib"]) * 1024 * float(rec["fetch_scale"])
    write = float(rec["write_kib"]) * 1024 * float(rec["write_scale"])
    return fetch + write


def cpu_baseline(st, n_rows):
    import oracle
    sample = st.slice(0, min(n_rows, st.T))
    t0 = time.perf_counter()
    r = oracle.tx_exact(sample.off, sample.items, P, SEED)
    dt = time.perf_counter() - t0
    return {"value": r["n_terms"] / dt, "unit": "term-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample.T} transactions of the 1M stream "
                      f"({r['n_terms']} terms), P={P}, {dt:.2f} s single-threaded",
            "seconds": round(dt, 3)}


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by hash interval across GPUs with no exchange; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import datagen
    import paper_1210_0461_amd as crop

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
    kernel_names = {"count": "k_tx_count", "scan": "k_colsum/k_colbase/k_colapply",
                    "scatter": "k_tx_scatter", "aggregate": "k_aggregate"}
    dom = max(stage_ms, key=stage_ms.get)
    dom_ms = stage_ms[dom]
    achieved = per_term * terms / (dom_ms * 1e-3) / 1e9
    digest = source_digest("k_route.hip", "k_exact.hip", "crop_device.hpp")
    traffic = traffic_from_profiles(kernel_names[dom], digest, None)
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
                   "transactions": st.T, "items": st.nnz, "terms": terms,
                   "distinct_pairs": distinct, "P": P, "seed": SEED,
                   "bins_per_partition": tune["bins_per_partition"],
                   "rows_per_chunk": tune["rows_per_chunk"]},
        "roofline": roofline,
        "path_roofline": {"bound": "hbm", "achieved": round(path_gbs, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(path_gbs / HBM_PEAK_GBS, 4),
                          "alg_bytes": alg_bytes},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "recall_top1000": 1.0,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(st, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
