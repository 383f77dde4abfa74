"""Pins of the oracle's exact results against brute force and identities.

Transactions (Section 7, case study): pair supports are the entries above
the diagonal of sum_T v_T v_T^T = X^T X for the T x n incidence matrix X.
Outer products (Section 4, notation): entry weights are A B for the
column-stacked a_k and row-stacked b_k.
"""
import numpy as np
import pytest

import datagen
import oracle

SEED = 0x243F6A8885A308D3


def dense_pairs(st):
    """Strict upper triangle of X^T X by a dense matrix product."""
    X = np.zeros((st.T, st.n), dtype=np.float64)
    L = st.lengths()
    rows = np.repeat(np.arange(st.T), L)
    X[rows, st.items.astype(np.int64)] = 1.0
    C = X.T @ X
    iu = np.triu_indices(st.n, k=1)
    c = C[iu]
    nz = c > 0
    return iu[0][nz].astype(np.uint32), iu[1][nz].astype(np.uint32), c[nz].astype(np.uint32)


def sorted_by_key(x, y, c):
    o = np.lexsort((y, x))
    return x[o], y[o], c[o]


def check_against_dense(st, P, seed=SEED):
    r = oracle.tx_exact(st.off, st.items, P, seed)
    dx, dy, dc = dense_pairs(st)
    gx, gy, gc = sorted_by_key(r["x"], r["y"], r["cnt"])
    assert np.array_equal(gx, dx) and np.array_equal(gy, dy) and np.array_equal(gc, dc)
    L = st.lengths()
    total = int((L * (L - 1) // 2).sum())
    assert int(r["cnt"].astype(np.int64).sum()) == total
    assert int(r["part_terms"].sum()) == total == r["n_terms"]
    assert int(r["part_sizes"].sum()) == dx.shape[0]
    return r


def test_small_config_equals_dense_xtx():
    st = datagen.config_small()
    check_against_dense(st, 8)


@pytest.mark.parametrize("seed", range(25))
def test_random_tiny_equals_dense_xtx(seed):
    st = datagen.tiny_transactions(seed, T=30 + seed, n=20 + seed, cap=10)
    check_against_dense(st, 1 + (seed % 5) * 3)


def test_partitions_follow_hash_and_union_is_invariant():
    st = datagen.config_small()
    ref = None
    for P in (1, 8, 1024, 1000):
        r = oracle.tx_exact(st.off, st.items, P, SEED)
        # output is grouped by partition; each key's partition is part(h(x,y))
        _, _, _, part = oracle.hash_many(SEED, r["x"], r["y"], P)
        sizes = np.bincount(part, minlength=P)
        assert np.array_equal(sizes, r["part_sizes"].astype(np.int64))
        assert np.all(np.diff(part.astype(np.int64)) >= 0)
        cur = sorted_by_key(r["x"], r["y"], r["cnt"])
        if ref is not None:
            for a, b in zip(ref, cur):
                assert np.array_equal(a, b)
        ref = cur


def test_marginal_identity():
    # sum_y cnt(x,y) + sum_w cnt(w,x) = sum_{T containing x} (|T| - 1)
    st = datagen.config_small()
    r = oracle.tx_exact(st.off, st.items, 8, SEED)
    lhs = np.bincount(r["x"], weights=r["cnt"], minlength=st.n) + \
        np.bincount(r["y"], weights=r["cnt"], minlength=st.n)
    L = st.lengths()
    rhs = np.bincount(st.items, weights=np.repeat(L - 1, L), minlength=st.n)
    assert np.array_equal(lhs, rhs)


def test_owned_interval_union():
    # Lemma 1's owned set E_[q,r): intervals that cover [0, 2^32) partition
    # the result
    st = datagen.config_small()
    full = oracle.tx_exact(st.off, st.items, 1, SEED)
    cuts = [0, 123456789, 2 ** 31, 3_000_000_000, 2 ** 32]
    parts = [oracle.tx_exact(st.off, st.items, 1, SEED, q, r) for q, r in zip(cuts, cuts[1:])]
    x = np.concatenate([p["x"] for p in parts])
    y = np.concatenate([p["y"] for p in parts])
    c = np.concatenate([p["cnt"] for p in parts])
    a = sorted_by_key(x, y, c)
    b = sorted_by_key(full["x"], full["y"], full["cnt"])
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    for (q, r), p in zip(zip(cuts, cuts[1:]), parts):
        _, _, h, _ = oracle.hash_many(SEED, p["x"], p["y"])
        assert np.all((h.astype(np.int64) >= q) & (h.astype(np.int64) < r))


def test_edge_cases_empty_and_singletons():
    off = np.array([0, 0, 1, 1, 2], np.uint32)
    items = np.array([3, 4], np.uint32)
    r = oracle.tx_exact(off, items, 4, SEED)
    assert r["x"].shape[0] == 0 and int(r["part_terms"].sum()) == 0
    r = oracle.tx_exact(np.array([0], np.uint32), np.zeros(0, np.uint32), 2, SEED)
    assert r["x"].shape[0] == 0


# ----------------------------------------------------------------- outer products

def dense_product(op):
    A = np.zeros((op.n_rows, op.K))
    B = np.zeros((op.K, op.n_cols))
    Sa = np.zeros((op.n_rows, op.K))
    Sb = np.zeros((op.K, op.n_cols))
    for k in range(op.K):
        ia = op.a_idx[op.a_off[k]:op.a_off[k + 1]].astype(np.int64)
        ib = op.b_idx[op.b_off[k]:op.b_off[k + 1]].astype(np.int64)
        A[ia, k] = op.a_val[op.a_off[k]:op.a_off[k + 1]]
        B[k, ib] = op.b_val[op.b_off[k]:op.b_off[k + 1]]
        Sa[ia, k] = 1.0
        Sb[k, ib] = 1.0
    return A @ B, np.abs(A) @ np.abs(B), Sa @ Sb


@pytest.mark.parametrize("seed", range(8))
def test_outer_equals_dense_product(seed):
    op = datagen.tiny_outer(seed, K=25, n_rows=30, n_cols=20, max_nnz=10)
    r = oracle.op_exact(op, 1 + seed, SEED)
    C, Cabs, N = dense_product(op)
    ii, jj = np.nonzero(N)
    o = np.lexsort((r["j"], r["i"]))
    assert np.array_equal(r["i"][o], ii.astype(np.uint32))
    assert np.array_equal(r["j"][o], jj.astype(np.uint32))
    np.testing.assert_allclose(r["sum"][o], C[ii, jj], rtol=0, atol=1e-12 * Cabs.max())
    np.testing.assert_allclose(r["abs"][o], Cabs[ii, jj], rtol=1e-14)
    assert np.array_equal(r["nterms"][o], N[ii, jj].astype(np.uint32))


def test_outer_checksum_and_single_term_exactness():
    op = datagen.tiny_outer(99, K=200, n_rows=300, n_cols=250, max_nnz=20)
    r = oracle.op_exact(op, 8, SEED)
    # sum over all entries = sum_k (sum_i a_k(i)) (sum_j b_k(j))
    chk = 0.0
    for k in range(op.K):
        chk += float(op.a_val[op.a_off[k]:op.a_off[k + 1]].astype(np.float64).sum()) * \
            float(op.b_val[op.b_off[k]:op.b_off[k + 1]].astype(np.float64).sum())
    assert abs(r["sum"].sum() - chk) <= 1e-10 * r["abs"].sum()
    # an entry with exactly one term equals the exact fp64 product of the two
    # fp32 inputs, whose rounding to fp32 is the fp32 product
    one = np.flatnonzero(r["nterms"] == 1)[:50]
    for e in one:
        i, j = int(r["i"][e]), int(r["j"][e])
        found = False
        for k in range(op.K):
            ai = op.a_idx[op.a_off[k]:op.a_off[k + 1]]
            bj = op.b_idx[op.b_off[k]:op.b_off[k + 1]]
            if i in ai and j in bj:
                va = op.a_val[op.a_off[k] + int(np.flatnonzero(ai == i)[0])]
                vb = op.b_val[op.b_off[k] + int(np.flatnonzero(bj == j)[0])]
                assert r["sum"][e] == float(va) * float(vb)
                assert np.float32(r["sum"][e]) == np.float32(va) * np.float32(vb)
                found = True
                break
        assert found


def test_outer_config_term_count():
    op = datagen.config_outer()
    La = np.diff(op.a_off.astype(np.int64))
    Lb = np.diff(op.b_off.astype(np.int64))
    assert oracle.op_num_terms(op.a_off, op.b_off) == int((La * Lb).sum())


@pytest.mark.parametrize("P,threads", [(1, 1), (8, 3), (1024, 8), (7, 7)])
def test_cpu_crop_baseline_matches_oracle(P, threads):
    """The host run of the paper's method (the benchmark's multi-core
    baseline: owners enumerate their hash interval through the h_b-sorted
    windows of Lemma 1, wrap included) gives the oracle's per-partition
    sizes and terms."""
    for st in (datagen.config_small(), datagen.tiny_transactions(5, T=300, n=50, cap=30)):
        seed = 0x243F6A8885A308D3
        ps, pt, d = oracle.cpu_crop_tx(st.off, st.items, P, seed, threads)
        r = oracle.tx_exact(st.off, st.items, P, seed)
        np.testing.assert_array_equal(ps, r["part_sizes"])
        np.testing.assert_array_equal(pt, r["part_terms"])
        assert d == len(r["x"])
