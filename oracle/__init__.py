"""CPU oracle for the column-row parallel (CRoP) hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  The product library
(``paper_1210_0461_amd``) never imports, links or calls it, and this package
never imports the product library.  The two share only the seeded input
generator in ``datagen``.

The heavy lifting is plain C (``crop_oracle.c``: double loops, ``qsort``,
linear scans) reached through ctypes; the learned-seeding parts (features and
the MLP) are fp64 numpy.  Each function names the passage of the paper it
follows; where the paper is silent the reading is stated.

Parity status: every function here is pinned by tests under ``tests/``
(``test_oracle_*.py``) against closed forms, brute force or invariants, with
one exception listed in its docstring: the exact contents of a Space-Saving
summary are "parity unpinned" beyond the special cases and invariants, since
the paper prints no worked example of the summary.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32

HASH_SPACE = 1 << 32


def lib():
    global _lib
    if _lib is not None:
        return _lib
    path = os.path.join(_HERE, "liborc.so")
    src = os.path.join(_HERE, "crop_oracle.c")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        _build.build()
    L = ctypes.CDLL(path)
    L.orc_hash_params.argtypes = [_u64, _u64p]
    L.orc_splitmix64.argtypes = [_u64, _u64p, _u64]
    L.orc_hash_many.argtypes = [_u64, _u32p, _u32p, _u64, _u32,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_part_bucket_many.argtypes = [_u32p, _u64, _u32, _u32, ctypes.c_void_p,
                                       ctypes.c_void_p]
    L.orc_tx_num_terms.argtypes = [_u32p, _u64]
    L.orc_tx_num_terms.restype = _u64
    L.orc_op_num_terms.argtypes = [_u32p, _u32p, _u64]
    L.orc_op_num_terms.restype = _u64
    L.orc_tx_exact.argtypes = [_u32p, _u64, _u32p, _u32, _u64, _u64, _u64, _u64p, _u64p,
                               _u32p, _u32p, _u32p, _u64, ctypes.POINTER(_u64)]
    L.orc_tx_exact.restype = ctypes.c_int
    L.orc_tx_part_terms.argtypes = [_u32p, _u64, _u32p, _u32, _u64, _u64p]
    L.orc_op_exact.argtypes = [_u32p, _u32p, _f32p, _u32p, _u32p, _f32p, _u64, _u32, _u64,
                               _u64, _u64, _u64p, _u64p, _u32p, _u32p, _f64p, _f64p, _u32p,
                               _u64, ctypes.POINTER(_u64)]
    L.orc_op_exact.restype = ctypes.c_int
    L.orc_tx_spacesaving.argtypes = [_u32p, _u64, _u32p, _u64, _u32, _u32, _u32,
                                     ctypes.c_void_p, ctypes.c_void_p, _u64, _u32,
                                     _u32p, _u32p, _u8p, _u8p, _f64p, _f64p]
    L.orc_tx_spacesaving.restype = _u64
    L.orc_op_spacesaving.argtypes = [_u32p, _u32p, _f32p, _u32p, _u32p, _f32p, _u64, _u64,
                                     _u32, _u32, _u32, _u32p, _u32p, _u8p, _u8p, _f64p,
                                     _f64p, _f64p]
    L.orc_tx_countsketch.argtypes = [_u32p, _u64, _u32p, _u64, _u32, _u32, _f64p]
    L.orc_op_bucket_abs.argtypes = [_u32p, _u32p, _f32p, _u32p, _u32p, _f32p, _u64, _u64,
                                    _u32, _u32, _f64p]
    L.orc_sign_many.argtypes = [_u64, _u32p, _u32p, _u64, ctypes.POINTER(ctypes.c_int8)]
    L.orc_op_countsketch.argtypes = [_u32p, _u32p, _f32p, _u32p, _u32p, _f32p, _u64, _u64,
                                     _u32, _u32, _f64p]
    _lib = L
    return L


_cpu = None


def cpu_lib():
    """The paper's method on the host (oracle/crop_cpu.c): the benchmark's
    multi-core CPU baseline, not a checker."""
    global _cpu
    if _cpu is not None:
        return _cpu
    path = os.path.join(_HERE, "libcropcpu.so")
    src = os.path.join(_HERE, "crop_cpu.c")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        _build.build_cpu()
    L = ctypes.CDLL(path)
    L.cpu_crop_tx.argtypes = [_u32p, _u64, _u32p, _u32, _u64, _u32, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.POINTER(_u64)]
    L.cpu_crop_tx.restype = ctypes.c_int
    _cpu = L
    return L


def cpu_crop_tx(off, items, P: int, seed: int, n_threads: int):
    """Run the paper's multi-threaded method (each of n_threads owners reads
    every transaction, sorts it by h_b and enumerates only the pairs of its
    hash interval, Lemma 1).  Returns (part_sizes, part_terms, distinct)."""
    off = _c(off, np.uint32)
    ps = np.zeros(P, np.uint64)
    pt = np.zeros(P, np.uint64)
    d = _u64(0)
    rc = cpu_lib().cpu_crop_tx(off, off.shape[0] - 1, _c(items, np.uint32), P, seed, n_threads,
                               ps.ctypes.data, pt.ctypes.data, ctypes.byref(d))
    if rc != 0:
        raise RuntimeError("cpu_crop_tx ran out of memory")
    return ps, pt, int(d.value)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# Hash specification (Section 5, proof of Lemma 1: h = (h_a + h_b) mod kappa
# with pairwise independent h_a, h_b; the family is this project's reading,
# SplitMix64-seeded multiply-add-shift with kappa = 2^32).

def hash_params(seed: int) -> np.ndarray:
    out = np.zeros(8, dtype=np.uint64)
    lib().orc_hash_params(seed, out)
    return out


def splitmix64(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_splitmix64(seed, out, n)
    return out


def hash_many(seed: int, x, y, P: int = 1):
    """Return (h_a(x), h_b(y), h(x,y), part(h(x,y))) element-wise."""
    x = _c(x, np.uint32)
    y = _c(y, np.uint32)
    n = x.shape[0]
    ha, hb, h, part = (np.zeros(n, np.uint32) for _ in range(4))
    lib().orc_hash_many(seed, x, y, n, P, ha.ctypes.data, hb.ctypes.data,
                        h.ctypes.data, part.ctypes.data)
    return ha, hb, h, part


def part_of(h, P: int) -> np.ndarray:
    """part(h) = (h * P) >> 32 element-wise (C oracle)."""
    h = _c(h, np.uint32)
    out = np.zeros(h.shape[0], np.uint32)
    lib().orc_part_bucket_many(h, h.shape[0], P, 1, out.ctypes.data, None)
    return out


def bucket_of(h, P: int, B: int) -> np.ndarray:
    """bucket(h) = (h * P * B) >> 32 element-wise (C oracle); P*B <= 2^32."""
    h = _c(h, np.uint32)
    out = np.zeros(h.shape[0], np.uint32)
    lib().orc_part_bucket_many(h, h.shape[0], P, B, None, out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# Exact results (Section 4: entry weight sum_k a_k(i) b_k(j); Section 7: the
# pairs of a transaction are the entries above the diagonal of v_T v_T^T).

def tx_num_terms(off) -> int:
    off = _c(off, np.uint32)
    return int(lib().orc_tx_num_terms(off, off.shape[0] - 1))


def op_num_terms(a_off, b_off) -> int:
    a_off = _c(a_off, np.uint32)
    return int(lib().orc_op_num_terms(a_off, _c(b_off, np.uint32), a_off.shape[0] - 1))


def tx_exact(off, items, P: int, seed: int, q: int = 0, r: int = HASH_SPACE):
    """Exact support of every pair whose hash lies in [q, r), grouped by
    partition and sorted by (partition, x, y).

    Returns dict with part_sizes[P], part_terms[P] (uint64) and x, y, cnt
    (uint32) over the distinct pairs."""
    off = _c(off, np.uint32)
    items = _c(items, np.uint32)
    T = off.shape[0] - 1
    nt = tx_num_terms(off)
    cap = max(nt, 1)
    ps = np.zeros(P, np.uint64)
    pt = np.zeros(P, np.uint64)
    x = np.zeros(cap, np.uint32)
    y = np.zeros(cap, np.uint32)
    c = np.zeros(cap, np.uint32)
    n_out = _u64(0)
    rc = lib().orc_tx_exact(off, T, items, P, seed, q, r, ps, pt, x, y, c, cap,
                            ctypes.byref(n_out))
    if rc != 0:
        raise RuntimeError(f"orc_tx_exact failed: {rc}")
    d = n_out.value
    return dict(part_sizes=ps, part_terms=pt, x=x[:d].copy(), y=y[:d].copy(),
                cnt=c[:d].copy(), n_terms=nt)


def tx_part_terms(off, items, P: int, seed: int) -> np.ndarray:
    """Number of terms of every partition (Section 6, Theorem 1's load X)."""
    off = _c(off, np.uint32)
    out = np.zeros(P, np.uint64)
    lib().orc_tx_part_terms(off, off.shape[0] - 1, _c(items, np.uint32), P, seed, out)
    return out


def partition_interval(p: int, P: int):
    """Hash interval [q, r) owned by partition p: the h with (h*P)>>32 == p."""
    q = -(-(p << 32) // P)
    r = -(-((p + 1) << 32) // P)
    return q, min(r, HASH_SPACE)


def op_exact(op, P: int, seed: int, q: int = 0, r: int = HASH_SPACE):
    """Exact fp64 entry weights of sum_k a_k b_k^T grouped by partition.

    Returns dict with part_sizes, part_terms, i, j, sum (fp64), abs (fp64,
    sum of |terms|) and nterms (terms per entry)."""
    a_off = _c(op.a_off, np.uint32)
    b_off = _c(op.b_off, np.uint32)
    K = a_off.shape[0] - 1
    nt = op_num_terms(a_off, b_off)
    cap = max(nt, 1)
    ps = np.zeros(P, np.uint64)
    pt = np.zeros(P, np.uint64)
    oi = np.zeros(cap, np.uint32)
    oj = np.zeros(cap, np.uint32)
    s = np.zeros(cap, np.float64)
    a = np.zeros(cap, np.float64)
    m = np.zeros(cap, np.uint32)
    n_out = _u64(0)
    rc = lib().orc_op_exact(a_off, _c(op.a_idx, np.uint32), _c(op.a_val, np.float32),
                            b_off, _c(op.b_idx, np.uint32), _c(op.b_val, np.float32),
                            K, P, seed, q, r, ps, pt, oi, oj, s, a, m, cap,
                            ctypes.byref(n_out))
    if rc != 0:
        raise RuntimeError(f"orc_op_exact failed: {rc}")
    d = n_out.value
    return dict(part_sizes=ps, part_terms=pt, i=oi[:d].copy(), j=oj[:d].copy(),
                sum=s[:d].copy(), abs=a[:d].copy(), nterms=m[:d].copy(), n_terms=nt)


# ---------------------------------------------------------------------------
# Space-Saving per bucket (Section 4, frequent items mining, and Figure 1).
# The summary contents are "parity unpinned" beyond the special case of at
# most ell distinct entries per bucket and the invariants of the Section 4
# bounds, since the paper prints no worked example.

def tx_spacesaving(off, items, seed: int, P: int, B: int, ell: int,
                   seeds_x=None, seeds_y=None, r_max: int = 0):
    """Sequential Space-Saving over the canonical term order, one summary of
    ell slots per bucket, P*B buckets.  Optional seeds are pinned first."""
    off = _c(off, np.uint32)
    items = _c(items, np.uint32)
    T = off.shape[0] - 1
    ns = P * B * ell
    kx = np.zeros(ns, np.uint32)
    ky = np.zeros(ns, np.uint32)
    used = np.zeros(ns, np.uint8)
    pinned = np.zeros(ns, np.uint8)
    cnt = np.zeros(ns, np.float64)
    err = np.zeros(ns, np.float64)
    if seeds_x is not None:
        sx = _c(seeds_x, np.uint32)
        sy = _c(seeds_y, np.uint32)
        npin = lib().orc_tx_spacesaving(off, T, items, seed, P, B, ell, sx.ctypes.data,
                                        sy.ctypes.data, sx.shape[0], r_max, kx, ky, used,
                                        pinned, cnt, err)
    else:
        npin = lib().orc_tx_spacesaving(off, T, items, seed, P, B, ell, None, None, 0, 0,
                                        kx, ky, used, pinned, cnt, err)
    return dict(x=kx, y=ky, used=used.astype(bool), pinned=pinned.astype(bool),
                cnt=cnt, err=err, ell=ell, P=P, B=B, n_pinned=int(npin))


def op_spacesaving(op, seed: int, P: int, B: int, ell: int):
    """Sequential weighted Space-Saving of outer-product terms with weight
    |a_k(i) b_k(j)| and a signed sum per slot."""
    a_off = _c(op.a_off, np.uint32)
    K = a_off.shape[0] - 1
    ns = P * B * ell
    kx = np.zeros(ns, np.uint32)
    ky = np.zeros(ns, np.uint32)
    used = np.zeros(ns, np.uint8)
    pinned = np.zeros(ns, np.uint8)
    cnt = np.zeros(ns, np.float64)
    err = np.zeros(ns, np.float64)
    val = np.zeros(ns, np.float64)
    lib().orc_op_spacesaving(a_off, _c(op.a_idx, np.uint32), _c(op.a_val, np.float32),
                             _c(op.b_off, np.uint32), _c(op.b_idx, np.uint32),
                             _c(op.b_val, np.float32), K, seed, P, B, ell, kx, ky, used,
                             pinned, cnt, err, val)
    return dict(x=kx, y=ky, used=used.astype(bool), pinned=pinned.astype(bool),
                cnt=cnt, err=err, val=val, ell=ell, P=P, B=B)


def amplified_report(summaries, min_votes: int):
    """Majority reporting over t independent instances (Section 6, the proof
    of Theorem 2: run t copies with independent hash functions and report the
    entries that at least half of them report).  An instance reports an entry
    when one of its summaries monitors it.  Every instance's [count - err,
    count] holds the entry's true weight (Section 4), so a reported entry gets
    the intersection of its reporting instances' intervals; its value is the
    median of their signed sums (mean of the two middle ones for an even
    number; outer products only).

    summaries: list of t summaries as returned by tx_spacesaving /
    op_spacesaving (instance i built with its own seed).  Returns a dict of
    arrays sorted by packed key: x, y, votes, upper, lower, value.  Lower
    bounds are taken as count - err in the precision of the summary's
    counters: fp64 differences for integer counts, fp32 differences clamped
    at 0 for fp32 counters (fp32=True in the summary dict)."""
    per = {}
    for s in summaries:
        fp32 = bool(s.get("fp32", False))
        for q in np.flatnonzero(np.asarray(s["used"])):
            key = (int(s["x"][q]) << 32) | int(s["y"][q])
            c = float(s["cnt"][q])
            if fp32:
                lo = float(max(np.float32(c) - np.float32(s["err"][q]), np.float32(0.0)))
            else:
                lo = c - float(s["err"][q])
            v = float(s["val"][q]) if "val" in s else 0.0
            per.setdefault(key, []).append((c, lo, v))
    keys = sorted(k for k, r in per.items() if len(r) >= min_votes)
    out = dict(x=np.array([k >> 32 for k in keys], np.uint32),
               y=np.array([k & 0xFFFFFFFF for k in keys], np.uint32),
               votes=np.array([len(per[k]) for k in keys], np.int64),
               upper=np.array([min(r[0] for r in per[k]) for k in keys], np.float64),
               lower=np.array([max(r[1] for r in per[k]) for k in keys], np.float64))
    val = []
    for k in keys:
        vs = sorted(r[2] for r in per[k])
        n = len(vs)
        val.append(vs[n // 2] if n % 2 else 0.5 * (vs[n // 2 - 1] + vs[n // 2]))
    out["value"] = np.array(val, np.float64)
    return out


# ---------------------------------------------------------------------------
# Count-Sketch, one estimator per bucket (Section 4; Figure 1).

def tx_countsketch(off, items, seed: int, P: int, B: int):
    off = _c(off, np.uint32)
    cs = np.zeros(P * B, np.float64)
    lib().orc_tx_countsketch(off, off.shape[0] - 1, _c(items, np.uint32), seed, P, B, cs)
    return cs


def op_countsketch(op, seed: int, P: int, B: int):
    a_off = _c(op.a_off, np.uint32)
    cs = np.zeros(P * B, np.float64)
    lib().orc_op_countsketch(a_off, _c(op.a_idx, np.uint32), _c(op.a_val, np.float32),
                             _c(op.b_off, np.uint32), _c(op.b_idx, np.uint32),
                             _c(op.b_val, np.float32), a_off.shape[0] - 1, seed, P, B, cs)
    return cs


def op_bucket_abs(op, seed: int, P: int, B: int):
    """Sum of |a_k(i) b_k(j)| per bucket."""
    a_off = _c(op.a_off, np.uint32)
    s = np.zeros(P * B, np.float64)
    lib().orc_op_bucket_abs(a_off, _c(op.a_idx, np.uint32), _c(op.a_val, np.float32),
                            _c(op.b_off, np.uint32), _c(op.b_idx, np.uint32),
                            _c(op.b_val, np.float32), a_off.shape[0] - 1, seed, P, B, s)
    return s


def sign_many(seed: int, x, y) -> np.ndarray:
    """Count-Sketch sign (+1 / -1) of every pair (x[k], y[k])."""
    x = _c(x, np.uint32)
    y = _c(y, np.uint32)
    out = np.zeros(x.shape[0], np.int8)
    lib().orc_sign_many(seed, x, y, x.shape[0], out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return out.astype(np.int64)


def countsketch_estimates(sketches, seeds, P: int, B: int, x, y) -> np.ndarray:
    """Median over instances of s_i(e) C_i[bucket_i(e)] (Section 4), in fp64."""
    est = []
    for cs, seed in zip(sketches, seeds):
        _, _, h, _ = hash_many(seed, x, y, P)
        b = bucket_of(h, P, B)
        est.append(sign_many(seed, x, y) * np.asarray(cs)[b])
    return np.median(np.stack(est), axis=0)


# ---------------------------------------------------------------------------
# Top-K and recall (Section 7.3, "Scalability": recall of the top pairs).

def pack_keys(x, y) -> np.ndarray:
    return (np.asarray(x, np.uint64) << np.uint64(32)) | np.asarray(y, np.uint64)


def topk(keys, weights, K: int):
    """First K entries by (weight descending, key ascending).  Returns the
    index array into keys/weights."""
    keys = np.asarray(keys, np.uint64)
    weights = np.asarray(weights)
    order = np.lexsort((keys, -weights.astype(np.float64)))
    return order[:K]


def recall_at_k(reported_keys, exact_keys, exact_weights, K: int) -> float:
    """Tie-tolerant recall: a reported entry is a hit when its exact weight is
    at least the K-th largest exact weight c_K."""
    exact_keys = np.asarray(exact_keys, np.uint64)
    exact_weights = np.asarray(exact_weights, np.float64)
    if exact_keys.shape[0] == 0 or K == 0:
        return 1.0
    kk = min(K, exact_keys.shape[0])
    cK = np.sort(exact_weights)[::-1][kk - 1]
    lookup = dict(zip(exact_keys.tolist(), exact_weights.tolist()))
    rep = np.asarray(reported_keys, np.uint64)[:K]
    hits = sum(1 for k in rep.tolist() if lookup.get(k, 0.0) >= cK)
    return hits / kk


# ---------------------------------------------------------------------------
# Learned seeding (not in the paper).  Features, candidates and the MLP
# follow this project's reading; see learned.py.

from .learned import (  # noqa: E402,F401
    prefix_len,
    item_stats,
    item_features,
    candidates,
    mlp_forward,
    mlp_backward,
    adam_step,
    bf16_round,
)
