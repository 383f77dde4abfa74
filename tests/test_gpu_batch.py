"""GPU batched exact runs against the oracle, stream by stream.

Each stream of a batch must get exactly what a single exact run gives: the
oracle's supports of every pair x < y, in the stream's own partitions of the
consistent hash (Section 6, Theorem 1), bit-exact.  Graph replays must equal
the eager run; the tuner's choice must not change any result.
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
    h = crop.crop_create(0)
    crop.crop_set_seed(h, SEED)
    yield h
    crop.crop_destroy(h)


def make_batch(streams):
    off, items, rows = datagen.concat_transactions(streams)
    return rows.astype(np.uint64), off, items, np.array([s.n for s in streams], np.uint32)


def check_stream(crop, ctx, k, st, seed=SEED):
    info = crop.crop_batch_info(ctx, k)
    P = info["partitions"]
    assert info["n_tx"] == st.T
    i, j, c, part_off = crop.crop_batch_read_stream(ctx, k)
    r = oracle.tx_exact(st.off, st.items, P, seed)
    assert info["terms"] == int(r["part_terms"].sum())
    sizes, terms = crop.crop_batch_result_sizes(ctx, k)
    np.testing.assert_array_equal(sizes, r["part_sizes"])
    np.testing.assert_array_equal(terms, r["part_terms"])
    # partition by partition: the same (x, y, count) sets
    ro = np.concatenate([[0], np.cumsum(r["part_sizes"].astype(np.int64))])
    for p in range(P):
        a, b = int(part_off[p]), int(part_off[p + 1])
        got = np.lexsort((j[a:b], i[a:b]))
        np.testing.assert_array_equal(i[a:b][got], r["x"][ro[p]:ro[p + 1]])
        np.testing.assert_array_equal(j[a:b][got], r["y"][ro[p]:ro[p + 1]])
        np.testing.assert_array_equal(c[a:b][got], r["cnt"][ro[p]:ro[p + 1]])


def canonical(res):
    """A stream's result with each partition sorted by (i, j): the order
    inside a partition is unspecified."""
    i, j, c, part_off = res
    order = np.concatenate([int(part_off[p]) + np.lexsort((j[part_off[p]:part_off[p + 1]],
                                                             i[part_off[p]:part_off[p + 1]]))
                            for p in range(part_off.shape[0] - 1)] + [np.zeros(0, np.int64)])
    order = order.astype(np.int64)
    return i[order], j[order], c[order], part_off


def small_batch():
    """Uneven streams: empty, one transaction, tiny, mid-sized, and two that
    differ only in seed."""
    s = [datagen.tiny_transactions(1, T=0, n=10),
         datagen.tiny_transactions(2, T=1, n=10),
         datagen.tiny_transactions(3, T=40, n=30)]
    s += datagen.config_batched(n_streams=12, base_seed=4100, t_lo=50, t_hi=3000)
    s.append(datagen.config_small())
    return s


@pytest.mark.parametrize("graph", [False, True])
def test_small_batch_matches_oracle(crop, ctx, graph):
    streams = small_batch()
    tx, off, items, n = make_batch(streams)
    crop.crop_load_batch(ctx, tx, off, items, n)
    crop.crop_batch_set_graph(ctx, graph)
    crop.crop_batch_set_plan(ctx, 2000, 64)   # several partitions even for small streams
    crop.crop_run_exact_batched(ctx)
    for k, st in enumerate(streams):
        check_stream(crop, ctx, k, st)
    assert any(crop.crop_batch_info(ctx, k)["partitions"] > 1 for k in range(len(streams)))


def test_graph_replays_equal_eager(crop, ctx):
    """Replays of the captured graph, with eager work and synchronisation in
    between, all equal the eager run."""
    import torch
    streams = datagen.config_batched(n_streams=16, base_seed=4200, t_lo=100, t_hi=5000)
    tx, off, items, n = make_batch(streams)
    crop.crop_load_batch(ctx, tx, off, items, n)
    crop.crop_batch_set_graph(ctx, False)
    crop.crop_run_exact_batched(ctx)
    ref = [canonical(crop.crop_batch_read_stream(ctx, k)) for k in range(len(streams))]
    crop.crop_batch_set_graph(ctx, True)
    x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
    for rep in range(3):
        crop.crop_run_exact_batched(ctx)
        crop.crop_synchronize(ctx)
        y = (x * 2 + rep).sum()          # unrelated eager work between replays
        torch.cuda.synchronize()
        assert float(y) > 0
        for k in range(len(streams)):
            got = canonical(crop.crop_batch_read_stream(ctx, k))
            for a, b in zip(got, ref[k]):
                np.testing.assert_array_equal(a, b)


def test_autotune_choice_and_invariance(crop, ctx):
    streams = datagen.config_batched(n_streams=24, base_seed=4300, t_lo=200, t_hi=8000)
    tx, off, items, n = make_batch(streams)
    crop.crop_load_batch(ctx, tx, off, items, n)
    tpb, R, ms = crop.crop_batch_autotune(ctx, 1)
    # R is 0 on the region route (no chunks), else the chunk's rows
    assert tpb in (15000, 30000, 60000) and R in (0, 64, 128, 256, 32, 16, 8, 4, 2, 1)
    assert ms > 0
    crop.crop_run_exact_batched(ctx)
    for k in (0, 5, 11, 23):
        check_stream(crop, ctx, k, streams[k])
    # a second context reuses the cached choice for a batch of the same shape
    h2 = crop.crop_create(0)
    try:
        crop.crop_set_seed(h2, SEED)
        crop.crop_load_batch(h2, tx, off, items, n)
        crop.crop_run_exact_batched(h2)
        t = crop.crop_batch_info(h2, 7)
        assert t["partitions"] == crop.crop_batch_info(ctx, 7)["partitions"]
        for a, b in zip(canonical(crop.crop_batch_read_stream(h2, 7)),
                        canonical(crop.crop_batch_read_stream(ctx, 7))):
            np.testing.assert_array_equal(a, b)
    finally:
        crop.crop_destroy(h2)


def test_wide_item_ids(crop, ctx):
    """A stream with item ids beyond 16 bits switches the batch to 64-bit keys."""
    streams = [datagen.tiny_transactions(11, T=300, n=200_000, zipf_s=0.6, mean_len=6, cap=20),
               datagen.tiny_transactions(12, T=200, n=40, mean_len=6, cap=20)]
    tx, off, items, n = make_batch(streams)
    crop.crop_load_batch(ctx, tx, off, items, n)
    crop.crop_batch_set_plan(ctx, 500, 32)
    crop.crop_run_exact_batched(ctx)
    for k, st in enumerate(streams):
        check_stream(crop, ctx, k, st)


def test_device_input_borrowed(crop, ctx):
    import torch
    streams = small_batch()[3:9]
    tx, off, items, n = make_batch(streams)
    doff = torch.from_numpy(off.view(np.int32)).cuda()
    ditems = torch.from_numpy(items.view(np.int32)).cuda()
    crop.crop_load_batch(ctx, tx, doff, ditems, n, own=crop.CROP_OWN_BORROW)
    crop.crop_run_exact_batched(ctx)
    for k, st in enumerate(streams):
        check_stream(crop, ctx, k, st)


def test_errors(crop, ctx):
    streams = small_batch()[2:6]
    tx, off, items, n = make_batch(streams)
    with pytest.raises(crop.CropError) as e:
        crop.crop_run_exact_batched(ctx)              # nothing loaded
    assert e.value.status == -2
    bad = items.copy()
    row = int(tx[2]) + 3                              # a non-empty transaction of stream 2
    while off[row + 1] == off[row]:
        row += 1
    assert row < int(tx[3])
    bad[off[row]] = n[2] + 5                          # id beyond that stream's items
    with pytest.raises(crop.CropError) as e:
        crop.crop_load_batch(ctx, tx, off, bad, n)
    assert e.value.status == -3 and e.value.index == row
    with pytest.raises(crop.CropError):
        crop.crop_load_batch(ctx, tx[::-1].copy(), off, items, n)
    crop.crop_load_batch(ctx, tx, off, items, n)
    with pytest.raises(crop.CropError):
        crop.crop_run_exact(ctx)                      # single-stream run on a batch
    with pytest.raises(crop.CropError):
        crop.crop_batch_read_stream(ctx, 0)           # no result yet
    crop.crop_run_exact_batched(ctx)
    with pytest.raises(crop.CropError):
        crop.crop_batch_info(ctx, len(streams))


def test_full_batched_config_sampled(crop, ctx):
    """The 256-stream workload (sizes log-uniform in [1e3, 2e5] transactions)
    in the configuration the bench times: the tuned plan and the captured
    graph.  Eight streams are checked whole against the oracle (the smallest,
    the largest and six between); every stream's terms and supports add up."""
    streams = datagen.config_batched()
    tx, off, items, n = make_batch(streams)
    crop.crop_load_batch(ctx, tx, off, items, n)
    crop.crop_batch_autotune(ctx, 1)
    crop.crop_run_exact_batched(ctx)
    crop.crop_run_exact_batched(ctx)                  # a graph replay
    sizes_T = np.array([s.T for s in streams])
    order = np.argsort(sizes_T)
    pick = sorted(set([int(order[0]), int(order[-1])] +
                      [int(order[q]) for q in np.linspace(10, 245, 6).astype(int)]))
    for k in pick:
        check_stream(crop, ctx, k, streams[k])
    for k, st in enumerate(streams):
        L = st.lengths()
        want = int((L * (L - 1) // 2).sum())
        sizes, terms = crop.crop_batch_result_sizes(ctx, k)
        assert int(terms.sum()) == want
        assert crop.crop_batch_info(ctx, k)["terms"] == want


def test_seed_change_recaptures_graph(crop, ctx):
    """The captured graph holds the hash parameters by value: after
    crop_set_seed a replay must partition by the new seed's hash, the same
    as the oracle under that seed."""
    streams = small_batch()[3:9]
    tx, off, items, n = make_batch(streams)
    crop.crop_load_batch(ctx, tx, off, items, n)
    crop.crop_batch_set_graph(ctx, True)
    crop.crop_batch_set_plan(ctx, 2000, 64)
    crop.crop_run_exact_batched(ctx)          # captures with SEED
    for k, st in enumerate(streams):
        check_stream(crop, ctx, k, st, SEED)
    new_seed = 0x9E3779B97F4A7C15
    crop.crop_set_seed(ctx, new_seed)
    crop.crop_run_exact_batched(ctx)          # must not replay the old capture
    for k, st in enumerate(streams):
        check_stream(crop, ctx, k, st, new_seed)
