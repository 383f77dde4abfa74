"""GPU amplified top-K: majority reporting over t CRoP instances (Section 6,
Theorem 2 and its proof) against the oracle.

Instance i uses the hash functions of seed + i.  Space-Saving summaries are
not bit-exact (the GPU applies a bucket's updates in another order), so the
checks are:
  * every instance's summary satisfies the Section 4 invariants against the
    oracle's exact counts under that instance's hash;
  * every reported interval [lower, upper] holds the oracle's exact count;
  * every entry heavier than m_b / ell in at least min_votes instances (so
    monitored there whatever the order) is reported;
  * where every bucket sees at most ell distinct entries the summaries are
    exact, and the report equals the oracle's majority report bit for bit;
  * the report is the majority combination of the GPU's own per-instance
    summaries (a consistency check computed here with numpy).
"""
import numpy as np
import pytest

import datagen
import oracle
from _ss_checks import check_invariants  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = 0x243F6A8885A308D3


@pytest.fixture(scope="module")
def crop():
    import paper_1210_0461_amd as crop
    return crop


@pytest.fixture
def ctx(crop):
    h = crop.crop_create(0)
    yield h
    crop.crop_destroy(h)


def seeds_of(t, seed=SEED):
    return [(seed + i) & 0xFFFFFFFFFFFFFFFF for i in range(t)]


def pack(x, y):
    return (np.asarray(x, np.uint64) << np.uint64(32)) | np.asarray(y, np.uint64)


def run_amp(crop, ctx, st, P, C, ell, K, t, m, seed=SEED, outer=False):
    crop.crop_set_partitions(ctx, P)
    crop.crop_set_seed(ctx, seed)
    crop.crop_set_summary(ctx, C, ell)
    if outer:
        crop.crop_load_outer(ctx, st.a_off, st.a_idx, st.a_val, st.b_off, st.b_idx, st.b_val,
                             st.n_rows, st.n_cols)
    else:
        crop.crop_load_transactions(ctx, st.off, st.items, st.n)
    crop.crop_run_topk_amplified(ctx, K, t, m)
    ns = P * (C // ell) * ell
    whole = crop.crop_read_summary(ctx, t * ns)
    sums = []
    for i in range(t):
        s = {k: v[i * ns:(i + 1) * ns] for k, v in whole.items()}
        s.update(P=P, B=C // ell, ell=ell, fp32=outer)
        sums.append(s)
    top = crop.crop_read_topk(ctx, K)
    votes = crop.crop_read_topk_votes(ctx, K)
    return sums, top, votes


def majority_of(sums, m, outer=False):
    """Combination of the given summaries, written out with numpy: votes,
    least count, largest lower bound (fp32 difference for fp32 counters)."""
    keys = np.concatenate([pack(s["x"][s["used"]], s["y"][s["used"]]) for s in sums])
    cnt = np.concatenate([s["cnt"][s["used"]] for s in sums])
    err = np.concatenate([s["err"][s["used"]] for s in sums])
    if outer:
        lo = np.maximum(cnt.astype(np.float32) - err.astype(np.float32), 0).astype(np.float64)
    else:
        lo = cnt - err
    uk, inv, votes = np.unique(keys, return_inverse=True, return_counts=True)
    up = np.full(uk.shape[0], np.inf)
    np.minimum.at(up, inv, cnt)
    low = np.full(uk.shape[0], -np.inf)
    np.maximum.at(low, inv, lo)
    keep = votes >= m
    return uk[keep], votes[keep], up[keep], low[keep]


def first_k(keys, rank, K):
    order = np.lexsort((keys, -rank))
    return order[:K]


def exact_tx(st):
    r = oracle.tx_exact(st.off, st.items, 1, SEED)
    return pack(r["x"], r["y"]), r["cnt"].astype(np.float64), r


def guaranteed_votes(keys, f, seeds, P, B, ell):
    """Instances in which an entry outweighs m_b / ell of its bucket."""
    x = (keys >> np.uint64(32)).astype(np.uint32)
    y = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    g = np.zeros(keys.shape[0], np.int64)
    for sd in seeds:
        _, _, h, _ = oracle.hash_many(sd, x, y)
        b = oracle.bucket_of(h, P, B).astype(np.int64)
        m_b = np.bincount(b, weights=f, minlength=P * B)
        g += f > m_b[b] / ell
    return g


def check_report(top, votes, sums, m, K, by_lower=True, outer=False):
    """The top-K is the first K of the majority combination of the GPU's own
    summaries by (rank value desc, key asc)."""
    uk, v, up, lo = majority_of(sums, m, outer)
    idx = first_k(uk, lo if by_lower else up, K)
    got = pack(top[0], top[1])
    assert np.array_equal(got, uk[idx])
    assert np.array_equal(top[2], up[idx])
    assert np.array_equal(top[3], lo[idx])
    assert np.array_equal(votes, v[idx])
    return uk


@pytest.mark.parametrize("t,m", [(5, 3), (4, 2), (3, 3), (11, 6)])
def test_small_config_invariants_and_majority(crop, ctx, t, m):
    st = datagen.config_small()
    keys, f, _ = exact_tx(st)
    P, C, ell = 2, 2048, 4
    sums, top, votes = run_amp(crop, ctx, st, P, C, ell, 100000, t, m)
    exact = dict(zip(keys.tolist(), f.tolist()))
    seeds = seeds_of(t)
    for s, sd in zip(sums, seeds):
        check_invariants(s, exact, sd)
    rep = check_report(top, votes, sums, m, 100000)
    # every reported interval holds the exact count
    got = pack(top[0], top[1])
    pos = np.searchsorted(keys, got)
    assert np.array_equal(keys[pos], got)
    assert np.all(top[3] <= f[pos]) and np.all(f[pos] <= top[2])
    assert np.all((votes >= m) & (votes <= t))
    # entries guaranteed in a majority of instances are reported
    g = guaranteed_votes(keys, f, seeds, P, C // ell, ell)
    assert (g >= m).sum() > 10
    assert np.all(np.isin(keys[g >= m], rep))


@pytest.mark.parametrize("C,ell,wide", [(2048, 2, False), (1536, 6, False), (2048, 4, True)])
def test_bucket_widths_and_wide_ids(crop, ctx, C, ell, wide):
    """Bucket widths that are not a multiple of four (the combine compares
    packed keys one at a time) and more than 2^16 item ids (64-bit keys)."""
    if wide:
        st = datagen.transactions(3000, 200_000, 0.9, 8.0, 40, datagen.Raw(79), "wide")
    else:
        st = datagen.config_small()
    keys, f, _ = exact_tx(st)
    P, t, m, K = 2, 5, 3, 100000
    sums, top, votes = run_amp(crop, ctx, st, P, C, ell, K, t, m)
    exact = dict(zip(keys.tolist(), f.tolist()))
    seeds = seeds_of(t)
    for s, sd in zip(sums, seeds):
        check_invariants(s, exact, sd)
    rep = check_report(top, votes, sums, m, K)
    got = pack(top[0], top[1])
    pos = np.minimum(np.searchsorted(keys, got), keys.shape[0] - 1)
    assert np.array_equal(keys[pos], got)
    assert np.all(top[3] <= f[pos]) and np.all(f[pos] <= top[2])
    g = guaranteed_votes(keys, f, seeds, P, C // ell, ell)
    assert np.all(np.isin(keys[g >= m], rep))


def test_exact_regime_equals_oracle(crop, ctx):
    """At most ell distinct entries per bucket: every summary is exact, so
    the GPU report equals the oracle's majority report of its own
    summaries."""
    st = datagen.tiny_transactions(21, T=80, n=24, cap=8)
    P, C, ell, t, m = 1, 8 * 64, 64, 5, 3
    seeds = seeds_of(t)
    ref = [oracle.tx_spacesaving(st.off, st.items, sd, P, C // ell, ell) for sd in seeds]
    for s in ref:
        assert np.all(s["err"][s["used"]] == 0)
    want = oracle.amplified_report(ref, m)
    sums, top, votes = run_amp(crop, ctx, st, P, C, ell, 10000, t, m)
    wk = pack(want["x"], want["y"])
    idx = first_k(wk, want["upper"], 10000)
    assert np.array_equal(pack(top[0], top[1]), wk[idx])
    assert np.array_equal(top[2], want["upper"][idx])
    assert np.array_equal(top[3], want["lower"][idx])
    assert np.array_equal(votes, want["votes"][idx])
    assert np.all(votes == t)


def test_single_instance_equals_plain_topk(crop, ctx):
    st = datagen.config_small()
    P, C, ell, K = 4, 256, 8, 300
    crop.crop_set_partitions(ctx, P)
    crop.crop_set_seed(ctx, SEED)
    crop.crop_set_summary(ctx, C, ell)
    crop.crop_load_transactions(ctx, st.off, st.items, st.n)
    crop.crop_run_topk(ctx, K)
    plain = crop.crop_read_topk(ctx, K)
    sums, top, votes = run_amp(crop, ctx, st, P, C, ell, K, 1, 1)
    keys, f, _ = exact_tx(st)
    check_invariants(sums[0], dict(zip(keys.tolist(), f.tolist())), SEED)
    check_report(top, votes, sums, 1, K)
    assert np.all(votes == 1)
    # the plain run ranks the same kind of summary; both tops hold valid bounds
    for res in (plain, top):
        got = pack(res[0], res[1])
        pos = np.searchsorted(keys, got)
        assert np.all(res[3] <= f[pos]) and np.all(f[pos] <= res[2])


def test_rank_by_upper_bound(crop, ctx):
    """The report ordered by upper bound on request (the default is the
    lower bound)."""
    st = datagen.config_small()
    crop.crop_set_topk_rank(ctx, crop.CROP_RANK_UPPER)
    t, m, K = 5, 3, 500
    sums, top, votes = run_amp(crop, ctx, st, 2, 1024, 8, K, t, m)
    check_report(top, votes, sums, m, K, by_lower=False)
    assert np.all(np.diff(top[2]) <= 0)


def test_outer_products(crop, ctx):
    op = datagen.tiny_outer(5, K=300, n_rows=60, n_cols=50, max_nnz=12)
    P, C, ell, t, m, K = 2, 256, 8, 5, 3, 400
    sums, top, votes = run_amp(crop, ctx, op, P, C, ell, K, t, m, outer=True)
    check_report(top, votes, sums, m, K, outer=True)
    # bounds of |weight| sums hold the oracle's fp64 sums of |a b| within fp32
    # accumulation error: a slot's count and error are sums over its bucket,
    # so the error is bounded relative to the bucket's total |weight| (the
    # largest over the instances); the signed value is the median of the
    # instances'
    ex = oracle.op_exact(op, 1, SEED)
    ek = pack(ex["i"], ex["j"])
    order = np.argsort(ek)
    ek, eabs = ek[order], ex["abs"][order]
    got = pack(top[0], top[1])
    pos = np.searchsorted(ek, got)
    assert np.array_equal(ek[pos], got)
    mb = np.zeros(got.shape[0])
    for sd in seeds_of(t):
        _, _, h, _ = oracle.hash_many(sd, top[0], top[1])
        b = oracle.bucket_of(h, P, C // ell).astype(np.int64)
        mb = np.maximum(mb, oracle.op_bucket_abs(op, sd, P, C // ell)[b])
    tol = 1e-5 * mb + 1e-30
    assert np.all(top[3] <= eabs[pos] + tol) and np.all(eabs[pos] <= top[2] + tol)
    for n in range(got.shape[0]):
        vals = sorted(s["val"][q] for s in sums
                      for q in np.flatnonzero(s["used"] & (pack(s["x"], s["y"]) == got[n])))
        assert len(vals) == votes[n]
        h = len(vals) // 2
        med = vals[h] if len(vals) % 2 else float(np.float32(0.5) * (np.float32(vals[h - 1]) +
                                                                     np.float32(vals[h])))
        assert top[4][n] == med


def test_large_stream_sampled(crop, ctx):
    """The 1M-transaction stream, P = 1, 2^14 counters of 16 per bucket,
    eleven instances reported at six votes (the paper's protocol): every
    reported interval holds the exact count and every entry guaranteed in six
    instances is reported."""
    st = datagen.config_large()
    P, C, ell, t, m = 1, 1 << 14, 16, 11, 6
    K = 5000
    sums, top, votes = run_amp(crop, ctx, st, P, C, ell, K, t, m)
    check_report(top, votes, sums, m, K)
    keys, f, _ = exact_tx(st)
    got = pack(top[0], top[1])
    pos = np.minimum(np.searchsorted(keys, got), keys.shape[0] - 1)
    assert np.array_equal(keys[pos], got)
    assert np.all(top[3] <= f[pos]) and np.all(f[pos] <= top[2])
    # m_b counts every entry of the bucket, so the whole key set goes in
    must = keys[guaranteed_votes(keys, f, seeds_of(t), P, C // ell, ell) >= m]
    uk, _, _, _ = majority_of(sums, m)
    assert must.shape[0] > 100
    assert np.all(np.isin(must, uk))


def test_errors(crop, ctx):
    st = datagen.config_small()
    with pytest.raises(crop.CropError):
        crop.crop_run_topk_amplified(ctx, 10, 3, 2)      # nothing loaded
    crop.crop_load_transactions(ctx, st.off, st.items, st.n)
    crop.crop_set_summary(ctx, 64, 4)
    for t, m in ((0, 1), (16, 8), (3, 4)):
        with pytest.raises(crop.CropError) as e:
            crop.crop_run_topk_amplified(ctx, 10, t, m)
        assert e.value.status == -1
    with pytest.raises(crop.CropError):
        crop.crop_run_topk_amplified(ctx, 0, 3, 2)
    crop.crop_run_topk_amplified(ctx, 10, 3, 2)
    with pytest.raises(crop.CropError):
        crop.crop_read_topk_votes(ctx, 1)               # capacity below the count
