"""GPU Count-Sketch (Section 4; Section 6, Theorem 3) against the oracle.

Transactions: int32 counters, bit-exact against the oracle's sketch of every
instance (instance i uses seed + i).  Outer products: fp32 counters within
1e-5 of each bucket's sum of |terms| (the fp32 accumulation error bound read
as for the exact sums).  Estimates: the median over instances of s(e) C[b(e)],
equal to the oracle's for transactions and within the same bound otherwise.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

SEED = 0x243F6A8885A308D3


@pytest.fixture(scope="module")
def crop():
    import paper_1210_0461_amd as crop
    return crop


@pytest.fixture
def ctx(crop):
    import torch
    h = crop.crop_create(0)
    crop.crop_set_stream(h, torch.cuda.current_stream())
    yield h
    crop.crop_synchronize(h)
    crop.crop_destroy(h)


def seeds_of(t, seed=SEED):
    return [(seed + i) & 0xFFFFFFFFFFFFFFFF for i in range(t)]


def run_tx(crop, ctx, st, P, B, t, seed=SEED):
    crop.crop_set_partitions(ctx, P)
    crop.crop_set_seed(ctx, seed)
    crop.crop_load_transactions(ctx, st.off, st.items, st.n)
    crop.crop_run_countsketch(ctx, B, t)
    return [crop.crop_read_countsketch(ctx, i, P * B) for i in range(t)]


def estimate(crop, ctx, x, y):
    import torch
    qx = torch.from_numpy(np.asarray(x, np.uint32).view(np.int32)).cuda()
    qy = torch.from_numpy(np.asarray(y, np.uint32).view(np.int32)).cuda()
    est = torch.empty(qx.shape[0], dtype=torch.float64, device="cuda")
    crop.crop_countsketch_estimate(ctx, qx, qy, est)
    return est.cpu().numpy()


@pytest.mark.parametrize("P,B,t", [(8, 64, 3), (1, 1, 1), (3, 100, 2), (16, 4096, 5)])
def test_tx_counters_bit_exact(crop, ctx, P, B, t):
    st = datagen.config_small()
    got = run_tx(crop, ctx, st, P, B, t)
    for i, sd in enumerate(seeds_of(t)):
        np.testing.assert_array_equal(got[i], oracle.tx_countsketch(st.off, st.items, sd, P, B))


@pytest.mark.parametrize("P,B,t,S", [(8, 64, 3, 4), (1, 100, 2, 25), (3, 100, 2, 100),
                                     (16, 4096, 5, 8), (2, 7, 1, 7)])
def test_tx_counters_routed_bit_exact(crop, ctx, P, B, t, S):
    """The routed form (bins of B / S buckets summed on chip) forced on small
    inputs, including bins of one bucket and a prime bucket count."""
    st = datagen.config_small()
    crop.crop_set_tuning(ctx, bins_per_partition=S)
    got = run_tx(crop, ctx, st, P, B, t)
    for i, sd in enumerate(seeds_of(t)):
        np.testing.assert_array_equal(got[i], oracle.tx_countsketch(st.off, st.items, sd, P, B))


def test_tx_wide_ids_routed(crop, ctx):
    """Item ids beyond 16 bits (64-bit routed keys)."""
    st = datagen.tiny_transactions(31, T=400, n=150_000, zipf_s=0.6, mean_len=6, cap=20)
    crop.crop_set_tuning(ctx, bins_per_partition=16)
    got = run_tx(crop, ctx, st, 4, 64, 3)
    for i, sd in enumerate(seeds_of(3)):
        np.testing.assert_array_equal(got[i], oracle.tx_countsketch(st.off, st.items, sd, 4, 64))


@pytest.mark.parametrize("seed", range(4))
def test_tx_random_tiny(crop, ctx, seed):
    st = datagen.tiny_transactions(300 + seed, T=60, n=25, cap=10)
    P, B, t = 1 + seed, 5 + 7 * seed, 1 + seed
    got = run_tx(crop, ctx, st, P, B, t, seed=seed * 977 + 1)
    for i, sd in enumerate(seeds_of(t, seed * 977 + 1)):
        np.testing.assert_array_equal(got[i], oracle.tx_countsketch(st.off, st.items, sd, P, B))


@pytest.mark.parametrize("t", [1, 2, 3, 4, 7])
def test_tx_estimates_are_medians(crop, ctx, t):
    st = datagen.config_small()
    P, B = 4, 32
    sk = run_tx(crop, ctx, st, P, B, t)
    r = oracle.tx_exact(st.off, st.items, 1, SEED)
    rng = datagen.Raw(t)
    pick = rng.randint(3000, 0, r["x"].shape[0] - 1)
    x = np.concatenate([r["x"][pick], [0, 7, 499]]).astype(np.uint32)
    y = np.concatenate([r["y"][pick], [1, 400, 499]]).astype(np.uint32)
    got = estimate(crop, ctx, x, y)
    want = oracle.countsketch_estimates(sk, seeds_of(t), P, B, x, y)
    np.testing.assert_array_equal(got, want)


def test_outer_counters_and_estimates(crop, ctx):
    op = datagen.tiny_outer(5, K=300, n_rows=60, n_cols=50, max_nnz=12)
    P, B, t = 4, 16, 3
    crop.crop_set_partitions(ctx, P)
    crop.crop_set_seed(ctx, SEED)
    crop.crop_load_outer(ctx, op.a_off, op.a_idx, op.a_val, op.b_off, op.b_idx, op.b_val,
                         op.n_rows, op.n_cols)
    crop.crop_run_countsketch(ctx, B, t)
    sk = []
    for i, sd in enumerate(seeds_of(t)):
        got = crop.crop_read_countsketch(ctx, i, P * B)
        want = oracle.op_countsketch(op, sd, P, B)
        bound = 1e-5 * oracle.op_bucket_abs(op, sd, P, B) + 1e-30
        assert np.all(np.abs(got - want) <= bound), i
        sk.append(want)
    ex = oracle.op_exact(op, 1, SEED)
    x, y = ex["i"][:500].astype(np.uint32), ex["j"][:500].astype(np.uint32)
    got = estimate(crop, ctx, x, y)
    want = oracle.countsketch_estimates(sk, seeds_of(t), P, B, x, y)
    # every instance's estimate is within its bucket's bound, so the median is
    # within the largest bound
    bmax = max(oracle.op_bucket_abs(op, sd, P, B).max() for sd in seeds_of(t))
    assert np.all(np.abs(got - want) <= 1e-5 * bmax)


def test_outer_counters_routed(crop, ctx):
    op = datagen.tiny_outer(6, K=300, n_rows=60, n_cols=50, max_nnz=12)
    P, B, t = 4, 16, 3
    crop.crop_set_tuning(ctx, bins_per_partition=4)
    crop.crop_set_partitions(ctx, P)
    crop.crop_set_seed(ctx, SEED)
    crop.crop_load_outer(ctx, op.a_off, op.a_idx, op.a_val, op.b_off, op.b_idx, op.b_val,
                         op.n_rows, op.n_cols)
    crop.crop_run_countsketch(ctx, B, t)
    for i, sd in enumerate(seeds_of(t)):
        got = crop.crop_read_countsketch(ctx, i, P * B)
        want = oracle.op_countsketch(op, sd, P, B)
        bound = 1e-5 * oracle.op_bucket_abs(op, sd, P, B) + 1e-30
        assert np.all(np.abs(got - want) <= bound), i


def test_outer_config(crop, ctx):
    """The 100,000-product workload, P = 8, 2^13 buckets per partition,
    three instances."""
    op = datagen.config_outer()
    P, B, t = 8, 1 << 13, 3
    crop.crop_set_partitions(ctx, P)
    crop.crop_set_seed(ctx, SEED)
    crop.crop_load_outer(ctx, op.a_off, op.a_idx, op.a_val, op.b_off, op.b_idx, op.b_val,
                         op.n_rows, op.n_cols)
    crop.crop_run_countsketch(ctx, B, t)
    for i, sd in enumerate(seeds_of(t)):
        got = crop.crop_read_countsketch(ctx, i, P * B)
        want = oracle.op_countsketch(op, sd, P, B)
        bound = 1e-5 * oracle.op_bucket_abs(op, sd, P, B) + 1e-30
        assert np.all(np.abs(got - want) <= bound), i


def test_large_stream_full_sketch(crop, ctx):
    """The 1M-transaction stream, P = 1024, 1024 buckets per partition, three
    instances (routed into 2,048 bins): every counter equal to the
    oracle's."""
    st = datagen.config_large()
    P, B, t = 1024, 1024, 3
    got = run_tx(crop, ctx, st, P, B, t)
    for i, sd in enumerate(seeds_of(t)):
        np.testing.assert_array_equal(got[i], oracle.tx_countsketch(st.off, st.items, sd, P, B))


def test_errors(crop, ctx):
    st = datagen.config_small()
    with pytest.raises(crop.CropError):
        crop.crop_run_countsketch(ctx, 16, 1)          # nothing loaded
    crop.crop_load_transactions(ctx, st.off, st.items, st.n)
    with pytest.raises(crop.CropError):
        crop.crop_run_countsketch(ctx, 16, 0)
    with pytest.raises(crop.CropError):
        crop.crop_run_countsketch(ctx, 16, 16)
    with pytest.raises(crop.CropError):
        crop.crop_run_countsketch(ctx, 0, 3)
    with pytest.raises(crop.CropError):
        crop.crop_read_countsketch(ctx, 0, 16)         # no sketch yet
    crop.crop_run_countsketch(ctx, 16, 2)
    with pytest.raises(crop.CropError):
        crop.crop_read_countsketch(ctx, 2, 16)
    with pytest.raises(crop.CropError):
        crop.crop_read_countsketch(ctx, 0, 15)
