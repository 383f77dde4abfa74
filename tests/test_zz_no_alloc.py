"""The no-allocation entry point (crop_item_features_noalloc) against the
allocating one (crop_item_features): the same per-item features, bit for
bit, on two calls in a row -- the second on a smaller stream and prefix, so
the fixed per-GPU workspace holds the first call's statistics when the
second starts -- and a clear capacity error beyond its fixed size."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crop():
    import paper_1210_0461_amd as crop
    return crop


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.fixture
def ctx(crop, torch):
    h = crop.crop_create(0)
    crop.crop_set_stream(h, torch.cuda.current_stream())
    yield h
    crop.crop_synchronize(h)
    crop.crop_destroy(h)


def features_both_ways(crop, ctx, torch, st, Tp):
    crop.crop_load_transactions(ctx, st.off, st.items, st.n)
    want = torch.full((st.n, 16), float("nan"), device="cuda")
    got = torch.full((st.n, 16), float("nan"), device="cuda")
    crop.crop_item_features(ctx, Tp, want)
    crop.crop_item_features_noalloc(ctx, Tp, got)
    torch.cuda.synchronize()
    return want.cpu().numpy(), got.cpu().numpy()


def test_noalloc_features_match_allocating_entry_point(crop, ctx, torch):
    big = datagen.config_small()                       # 2,000 transactions, 500 items
    small = datagen.tiny_transactions(77, T=300, n=120, cap=12, mean_len=5.0)
    for st, Tp in ((big, big.T // 20), (small, 30)):
        want, got = features_both_ways(crop, ctx, torch, st, Tp)
        assert np.isfinite(want).all()
        assert np.array_equal(want.view(np.uint32), got.view(np.uint32))
    # the whole stream as the prefix, then an empty prefix
    for Tp in (small.T, 0):
        want = torch.empty((small.n, 16), device="cuda")
        got = torch.empty((small.n, 16), device="cuda")
        crop.crop_item_features(ctx, Tp, want)
        crop.crop_item_features_noalloc(ctx, Tp, got)
        torch.cuda.synchronize()
        assert torch.equal(want.view(torch.int32), got.view(torch.int32))


def test_noalloc_refuses_more_than_its_workspace(crop, ctx, torch):
    """8 n_items + prefix_T + 66 words must fit 2^21: 262,135 items with a
    prefix of 2 transactions do (2,097,148 words), 262,144 do not."""
    st = datagen.tiny_transactions(5, T=50, n=40, cap=8, mean_len=4.0)
    feat = torch.empty((262144, 16), device="cuda")
    crop.crop_load_transactions(ctx, st.off, st.items, 262135)
    crop.crop_item_features_noalloc(ctx, 2, feat[:262135])
    crop.crop_load_transactions(ctx, st.off, st.items, 262144)
    with pytest.raises(crop.CropError) as e:
        crop.crop_item_features_noalloc(ctx, 2, feat)
    assert e.value.status == -4                        # CROP_E_CAPACITY
    crop.crop_item_features(ctx, 2, feat)              # the allocating one still serves it
