"""Pins of the oracle's Space-Saving, Count-Sketch and top-K routines.

Space-Saving (Section 4, frequent items mining): the rules, the bound
overestimation <= m/ell, and that every item above m/ell is recorded.
Count-Sketch (Section 4): the estimate CS[h(e)] * s(e).
Top-K and recall (Section 7.3, recall of the top pairs).
The contents of a Space-Saving summary beyond these are parity unpinned.
"""
import os

import numpy as np
import pytest

import datagen
import oracle

SEED = 0x243F6A8885A308D3
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_worked_example():
    tx, final = [], []
    for line in open(os.path.join(GOLD, "spacesaving_worked_example.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("="):
            final.append(tuple(int(v) for v in line[1:].split()))
        else:
            tx.append(tuple(int(v) for v in line.split()))
    off = np.arange(0, 2 * len(tx) + 1, 2, dtype=np.uint32)
    items = np.array([v for t in tx for v in t], np.uint32)
    return off, items, final


def test_worked_example_by_hand():
    off, items, final = load_worked_example()
    s = oracle.tx_spacesaving(off, items, SEED, 1, 1, 2)
    got = [(int(s["x"][k]), int(s["y"][k]), int(s["cnt"][k]), int(s["err"][k])) for k in range(2)]
    assert got == final


def exact_lookup(st, seed=SEED):
    r = oracle.tx_exact(st.off, st.items, 1, seed)
    return dict(zip(oracle.pack_keys(r["x"], r["y"]).tolist(), r["cnt"].tolist())), r


def check_invariants(s, exact, seed=SEED):
    """I1..I5 of each bucket (Section 4 bounds), integer weights."""
    P, B, ell = s["P"], s["B"], s["ell"]
    keys = oracle.pack_keys(s["x"], s["y"]).reshape(P * B, ell)
    used = s["used"].reshape(P * B, ell)
    pinned = s["pinned"].reshape(P * B, ell)
    cnt = s["cnt"].reshape(P * B, ell)
    err = s["err"].reshape(P * B, ell)
    ek = np.array(list(exact.keys()), np.uint64)
    ef = np.array(list(exact.values()), np.float64)
    _, _, h, _ = oracle.hash_many(seed, (ek >> np.uint64(32)).astype(np.uint32),
                                  (ek & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    bk = oracle.bucket_of(h, P, B).astype(np.int64)
    m_b = np.bincount(bk, weights=ef, minlength=P * B)
    for b in range(P * B):
        u = used[b]
        assert cnt[b][u].sum() == m_b[b]                      # I1
        full = u.all()
        free = u & ~pinned[b]
        mn = cnt[b][free].min() if (full and free.any()) else 0.0
        unpinned_mass = m_b[b] - sum(exact.get(int(k), 0) for k in keys[b][u & pinned[b]])
        n_free = int((~pinned[b]).sum())
        if full and n_free:
            assert mn <= unpinned_mass / n_free + 1e-9     # I4
        for k in range(ell):
            if not u[k]:
                continue
            f = exact.get(int(keys[b][k]), 0)
            assert cnt[b][k] - err[b][k] <= f <= cnt[b][k]     # I2
            assert err[b][k] <= mn or pinned[b][k]             # I4 (err <= min)
            if pinned[b][k]:
                assert err[b][k] == 0 and cnt[b][k] == f
    mon = set(keys[used].tolist())
    for key, f, b in zip(ek.tolist(), ef.tolist(), bk.tolist()):
        if key in mon:
            continue
        full = used[b].all()
        free = used[b] & ~pinned[b]
        mn = cnt[b][free].min() if (full and free.any()) else 0.0
        assert f <= mn                                         # I3 and I5


@pytest.mark.parametrize("P,B,ell", [(1, 1, 4), (2, 4, 2), (4, 16, 3), (8, 8, 16)])
def test_invariants_small_config(P, B, ell):
    st = datagen.config_small()
    exact, _ = exact_lookup(st)
    s = oracle.tx_spacesaving(st.off, st.items, SEED, P, B, ell)
    check_invariants(s, exact)


@pytest.mark.parametrize("seed", range(10))
def test_invariants_random_tiny(seed):
    st = datagen.tiny_transactions(100 + seed, T=60, n=25, cap=9)
    exact, _ = exact_lookup(st)
    s = oracle.tx_spacesaving(st.off, st.items, SEED, 1 + seed % 3, 1 + seed % 4, 2 + seed % 3)
    check_invariants(s, exact)


def test_few_distinct_keys_per_bucket_is_exact():
    # a bucket that sees at most ell distinct entries holds exact counts
    st = datagen.tiny_transactions(7, T=50, n=12, cap=6)
    exact, _ = exact_lookup(st)
    s = oracle.tx_spacesaving(st.off, st.items, SEED, 1, 1, len(exact))
    assert s["used"].sum() == len(exact)
    for k in np.flatnonzero(s["used"]):
        key = int(oracle.pack_keys(s["x"][k], s["y"][k]))
        assert s["cnt"][k] == exact[key] and s["err"][k] == 0


def test_pinned_seeds_are_exact_and_bounded_per_bucket():
    st = datagen.config_small()
    exact, r = exact_lookup(st)
    top = oracle.topk(oracle.pack_keys(r["x"], r["y"]), r["cnt"], 40)
    sx, sy = r["x"][top], r["y"][top]
    P, B, ell, rmax = 2, 8, 6, 2
    s = oracle.tx_spacesaving(st.off, st.items, SEED, P, B, ell, sx, sy, rmax)
    per_bucket = s["pinned"].reshape(P * B, ell).sum(axis=1)
    assert per_bucket.max() <= rmax
    assert s["n_pinned"] == int(s["pinned"].sum())
    check_invariants(s, exact)


def test_outer_spacesaving_weights_and_signed_sums():
    op = datagen.tiny_outer(5, K=60, n_rows=25, n_cols=25, max_nnz=8)
    ex = oracle.op_exact(op, 1, SEED)
    P, B, ell = 2, 2, 4
    s = oracle.op_spacesaving(op, SEED, P, B, ell)
    akey = oracle.pack_keys(ex["i"], ex["j"])
    absw = dict(zip(akey.tolist(), ex["abs"].tolist()))
    sgn = dict(zip(akey.tolist(), ex["sum"].tolist()))
    keys = oracle.pack_keys(s["x"], s["y"])
    _, _, h, _ = oracle.hash_many(SEED, ex["i"], ex["j"])
    bk = oracle.bucket_of(h, P, B).astype(np.int64)
    m_b = np.bincount(bk, weights=ex["abs"], minlength=P * B)
    cnt = s["cnt"].reshape(P * B, ell)
    used = s["used"].reshape(P * B, ell)
    for b in range(P * B):
        assert abs(cnt[b][used[b]].sum() - m_b[b]) <= 1e-9 * max(m_b[b], 1)
    for k in np.flatnonzero(s["used"]):
        f = absw[int(keys[k])]
        assert s["cnt"][k] - s["err"][k] <= f * (1 + 1e-12) + 1e-12
        assert f <= s["cnt"][k] * (1 + 1e-12) + 1e-12
        if s["err"][k] == 0:
            # monitored since its first term: the signed sum is the exact weight
            assert abs(s["val"][k] - sgn[int(keys[k])]) <= 1e-9 * (1 + absw[int(keys[k])])


def test_countsketch_isolated_buckets_are_exact():
    st = datagen.tiny_transactions(3, T=30, n=15, cap=6)
    exact, r = exact_lookup(st)
    P, B = 64, 1024
    cs = oracle.tx_countsketch(st.off, st.items, SEED, P, B)
    _, _, h, _ = oracle.hash_many(SEED, r["x"], r["y"])
    bk = oracle.bucket_of(h, P, B).astype(np.int64)
    occupancy = np.bincount(bk, minlength=P * B)
    # the sign of an entry, recovered from a bucket it holds alone
    alone = occupancy[bk] == 1
    assert alone.sum() > 0.9 * bk.shape[0]
    est = np.abs(cs[bk[alone]])
    assert np.array_equal(est, r["cnt"][alone].astype(np.float64))
    assert abs(cs).sum() <= r["cnt"].sum()


def test_countsketch_linear_and_unbiased_over_seeds():
    st = datagen.config_small()
    half = st.T // 2
    a, b = st.slice(0, half), st.slice(half, st.T)
    cs = oracle.tx_countsketch(st.off, st.items, SEED, 4, 16)
    assert np.array_equal(cs, oracle.tx_countsketch(a.off, a.items, SEED, 4, 16) +
                          oracle.tx_countsketch(b.off, b.items, SEED, 4, 16))
    # unbiased estimator: mean over seeds of CS[h(e)] s(e) approaches f_e
    exact, r = exact_lookup(st)
    top = oracle.topk(oracle.pack_keys(r["x"], r["y"]), r["cnt"], 3)
    P, B = 2, 8
    ests = []
    for seed in range(60):
        cs = oracle.tx_countsketch(st.off, st.items, seed, P, B)
        _, _, h, _ = oracle.hash_many(seed, r["x"][top], r["y"][top])
        bk = oracle.bucket_of(h, P, B).astype(np.int64)
        sgn = np.array([1.0 if ((int(g) >> 31) == 0) else -1.0 for g in
                        _sign_words(seed, r["x"][top], r["y"][top])])
        ests.append(cs[bk] * sgn)
    ests = np.array(ests)
    M = float(r["cnt"].sum())
    # the estimate's noise is the sum of colliding entries with random signs
    sd = np.sqrt(float((r["cnt"].astype(np.float64) ** 2).sum()) / (P * B) / 60)
    assert np.all(np.abs(ests.mean(axis=0) - r["cnt"][top]) < 5 * sd + 1e-9 * M)


def _sign_words(seed, x, y):
    prm = oracle.hash_params(seed)
    out = []
    for a, b in zip(x.tolist(), y.tolist()):
        ga = ((int(prm[4]) * a + int(prm[5])) % (1 << 64)) >> 32
        gb = ((int(prm[6]) * b + int(prm[7])) % (1 << 64)) >> 32
        out.append((ga + gb) % (1 << 32))
    return out


def test_sign_many_matches_python_sign_words():
    x = np.array([0, 1, 5, 65535, 4000000000], np.uint32)
    y = np.array([1, 2, 9, 70000, 4000000001], np.uint32)
    want = [1 if (g >> 31) == 0 else -1 for g in _sign_words(SEED, x, y)]
    assert oracle.sign_many(SEED, x, y).tolist() == want


def test_countsketch_estimates_isolated_and_median():
    """With isolated buckets every instance's estimate is the exact weight, so
    the median is too; the median of three instances lies between their
    smallest and largest estimates."""
    st = datagen.tiny_transactions(4, T=30, n=15, cap=6)
    exact, r = exact_lookup(st)
    P, B, seeds = 16, 4096, [SEED, SEED + 1, SEED + 2]
    sk = [oracle.tx_countsketch(st.off, st.items, sd, P, B) for sd in seeds]
    est = oracle.countsketch_estimates(sk, seeds, P, B, r["x"], r["y"])
    per = []
    for cs, sd in zip(sk, seeds):
        _, _, h, _ = oracle.hash_many(sd, r["x"], r["y"])
        per.append(oracle.sign_many(sd, r["x"], r["y"]) * cs[oracle.bucket_of(h, P, B)])
    per = np.stack(per)
    assert np.all(est >= per.min(axis=0)) and np.all(est <= per.max(axis=0))
    alone = np.all(per == r["cnt"][None, :].astype(np.float64), axis=0)
    assert alone.mean() > 0.9
    assert np.array_equal(est[alone], r["cnt"][alone].astype(np.float64))


def test_op_bucket_abs_totals_and_bounds():
    op = datagen.tiny_outer(6, K=40, n_rows=30, n_cols=25, max_nnz=8)
    P, B = 2, 8
    s = oracle.op_bucket_abs(op, SEED, P, B)
    cs = oracle.op_countsketch(op, SEED, P, B)
    tot = 0.0
    for k in range(op.K):
        a = op.a_val[op.a_off[k]:op.a_off[k + 1]].astype(np.float64)
        b = op.b_val[op.b_off[k]:op.b_off[k + 1]].astype(np.float64)
        tot += np.abs(np.outer(a, b)).sum()
    assert abs(s.sum() - tot) <= 1e-9 * tot
    assert np.all(np.abs(cs) <= s + 1e-9 * tot)


def test_topk_ties_and_recall():
    keys = np.array([50, 10, 30, 20, 40, 60], np.uint64)
    w = np.array([5, 7, 5, 5, 1, 7])
    idx = oracle.topk(keys, w, 4)
    assert keys[idx].tolist() == [10, 60, 20, 30]
    # tie-tolerant recall: entries with weight >= c_K count as hits
    assert oracle.recall_at_k([10, 60, 50, 40], keys, w, 4) == 0.75
    assert oracle.recall_at_k([60, 10, 50, 30], keys, w, 4) == 1.0
    assert oracle.recall_at_k([], keys, w, 4) == 0.0


# ---------------------------------------------------------------------------
# Majority reporting over t instances (Section 6, Theorem 2 and its proof).

def _summary(entries, fp32=False):
    """A one-bucket summary from (x, y, count, err, value) tuples."""
    x, y, c, e, v = (np.array(col) for col in zip(*entries))
    return dict(x=x.astype(np.uint32), y=y.astype(np.uint32), cnt=c.astype(np.float64),
                err=e.astype(np.float64), val=v.astype(np.float64),
                used=np.ones(len(entries), bool), fp32=fp32)


def test_amplified_report_by_hand():
    s0 = _summary([(1, 2, 10, 2, -1.0), (3, 4, 5, 0, 1.0), (5, 6, 3, 3, 7.0)])
    s1 = _summary([(1, 2, 9, 0, 4.0), (5, 6, 4, 1, -2.0)])
    s2 = _summary([(1, 2, 12, 4, 2.0), (7, 8, 2, 0, 9.0), (3, 4, 6, 2, 3.0)])
    r = oracle.amplified_report([s0, s1, s2], 2)
    # (1,2): three votes, upper min(10, 9, 12) = 9, lower max(8, 9, 8) = 9,
    # value median(-1, 4, 2) = 2; (3,4): two votes, upper 5, lower max(5, 4)
    # = 5, value mean(1, 3) = 2; (5,6): upper 3, lower max(0, 3) = 3, value
    # mean(7, -2) = 2.5; (7,8) has one vote and is not reported
    assert r["x"].tolist() == [1, 3, 5] and r["y"].tolist() == [2, 4, 6]
    assert r["votes"].tolist() == [3, 2, 2]
    assert r["upper"].tolist() == [9, 5, 3]
    assert r["lower"].tolist() == [9, 5, 3]
    assert r["value"].tolist() == [2.0, 2.0, 2.5]
    r1 = oracle.amplified_report([s0, s1, s2], 1)
    assert r1["x"].tolist() == [1, 3, 5, 7] and r1["votes"].tolist() == [3, 2, 2, 1]
    assert oracle.amplified_report([s0, s1, s2], 3)["x"].tolist() == [1]
    # fp32 counters: lower = max(fp32(c - e), 0)
    f = oracle.amplified_report([_summary([(1, 2, 1.0, 1.0 + 2 ** -20, 0.0)], fp32=True)], 1)
    assert f["lower"].tolist() == [0.0]


def test_amplified_single_instance_is_the_summary():
    st = datagen.config_small()
    s = oracle.tx_spacesaving(st.off, st.items, SEED, 2, 16, 4)
    r = oracle.amplified_report([s], 1)
    u = s["used"]
    keys = oracle.pack_keys(s["x"][u], s["y"][u])
    order = np.argsort(keys)
    assert np.array_equal(oracle.pack_keys(r["x"], r["y"]), keys[order])
    assert np.array_equal(r["upper"], s["cnt"][u][order])
    assert np.array_equal(r["lower"], (s["cnt"] - s["err"])[u][order])
    assert np.all(r["votes"] == 1)


@pytest.mark.parametrize("t,min_votes", [(5, 3), (4, 2), (3, 3)])
def test_amplified_reports_every_guaranteed_entry(t, min_votes):
    """An entry heavier than m_b / ell in its bucket of instance i is
    monitored there (Section 4).  Entries with at least min_votes such
    instances are reported; every reported interval holds the exact count."""
    st = datagen.config_small()
    exact, r = exact_lookup(st)
    P, B, ell = 2, 512, 4
    seeds = [(SEED + i) & 0xFFFFFFFFFFFFFFFF for i in range(t)]
    sums = [oracle.tx_spacesaving(st.off, st.items, sd, P, B, ell) for sd in seeds]
    rep = oracle.amplified_report(sums, min_votes)
    keys = oracle.pack_keys(r["x"], r["y"])
    f = r["cnt"].astype(np.float64)
    guaranteed = np.zeros(keys.shape[0], np.int64)
    for sd in seeds:
        _, _, h, _ = oracle.hash_many(sd, r["x"], r["y"])
        b = oracle.bucket_of(h, P, B).astype(np.int64)
        m_b = np.bincount(b, weights=f, minlength=P * B)
        guaranteed += f > m_b[b] / ell
    rk = oracle.pack_keys(rep["x"], rep["y"])
    assert np.all(np.isin(keys[guaranteed >= min_votes], rk))
    assert (guaranteed >= min_votes).sum() > 10
    pos = np.searchsorted(keys, rk)
    assert np.array_equal(keys[pos], rk)
    assert np.all(rep["lower"] <= f[pos]) and np.all(f[pos] <= rep["upper"])
    assert np.all(rep["votes"] >= min_votes)
    # every vote is one monitored slot: reported * min_votes <= slots in use
    assert int(rep["votes"].sum()) <= sum(int(s["used"].sum()) for s in sums)
    assert rk.shape[0] * min_votes <= sum(int(s["used"].sum()) for s in sums)
