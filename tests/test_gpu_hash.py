"""The consistent hash computed by the library's kernels against the oracle
on every id below 2^20, for three seeds (Section 5, proof of Lemma 1:
h = h_a + h_b mod 2^32; Section 6, Theorem 1: part = floor(h P / 2^32)).
Together with the Python-integer restatement pinned on the CPU this makes
three independent implementations that agree."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crop():
    import paper_1210_0461_amd as crop
    return crop


@pytest.mark.parametrize("seed", [0, 1, 0x243F6A8885A308D3])
@pytest.mark.parametrize("P", [1000, 65537])
def test_hash_pairs_equal_oracle_on_all_ids_below_2_20(crop, seed, P):
    import torch
    x = np.arange(1 << 20, dtype=np.uint32)
    y = x[::-1].copy()
    ctx = crop.crop_create(0)
    try:
        crop.crop_set_partitions(ctx, P)
        crop.crop_set_seed(ctx, seed)
        dx = torch.from_numpy(x.view(np.int32)).cuda()
        dy = torch.from_numpy(y.view(np.int32)).cuda()
        h = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
        part = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
        crop.crop_hash_pairs(ctx, dx, dy, h, part)
        crop.crop_synchronize(ctx)
        gh = h.cpu().numpy().view(np.uint32)
        gp = part.cpu().numpy().view(np.uint32)
    finally:
        crop.crop_destroy(ctx)
    _, _, oh, op = oracle.hash_many(seed, x, y, P)
    np.testing.assert_array_equal(gh, oh)
    np.testing.assert_array_equal(gp, op)
