"""Learned heavy-pair seeding as a sequence of C-ABI calls.

Every step runs in the library's kernels; this module only allocates the
device tensors that carry data between the calls and orders the calls.

Training data for one stream: features of the first prefix_len(T)
transactions, candidate pairs among the M most frequent prefix items, and
labels log1p(exact support) from an exact run over the whole stream.
Seeding a new stream: features and candidates of its prefix, bf16 scores,
and the R best candidates as pinned Space-Saving seeds.

The tensors are allocated on torch's current stream; give the context that
stream (crop_set_stream(ctx, torch.cuda.current_stream())) so the library's
kernels and torch's use of the tensors are ordered.
"""
from __future__ import annotations

from . import (MLP_PARAMS, crop_item_features, crop_lookup_exact, crop_pair_inputs,
               crop_mlp_score, crop_run_exact, crop_select_seeds, crop_top_item_pairs)

N_FEAT = 16


def prefix_len(T: int) -> int:
    """Transactions in the prefix the features are taken from: ceil(T / 20)."""
    return 0 if T <= 0 else max(1, (T + 19) // 20)


def _torch():
    import torch
    return torch


def candidate_inputs(ctx, T: int, n_items: int, M: int, device="cuda"):
    """Features, candidate pairs and network inputs of the loaded stream.
    Returns (feat [n,16], cx [np], cy [np], Z [np,32]) as device tensors."""
    torch = _torch()
    Tp = prefix_len(T)
    feat = torch.empty((n_items, N_FEAT), dtype=torch.float32, device=device)
    crop_item_features(ctx, Tp, feat)
    n_pairs = M * (M - 1) // 2
    cx = torch.empty(n_pairs, dtype=torch.int32, device=device)
    cy = torch.empty(n_pairs, dtype=torch.int32, device=device)
    crop_top_item_pairs(ctx, Tp, M, cx, cy)
    Z = torch.empty((n_pairs, 2 * N_FEAT), dtype=torch.float32, device=device)
    crop_pair_inputs(ctx, feat, cx, cy, None, Z, None)
    return feat, cx, cy, Z


def training_pairs(ctx, T: int, n_items: int, M: int, device="cuda"):
    """(Z, y, cx, cy, support) of the loaded stream; runs the exact pass
    for the labels."""
    torch = _torch()
    crop_run_exact(ctx)
    feat, cx, cy, _ = candidate_inputs(ctx, T, n_items, M, device)
    support = torch.empty(cx.shape[0], dtype=torch.int32, device=device)
    crop_lookup_exact(ctx, cx, cy, support)
    Z = torch.empty((cx.shape[0], 2 * N_FEAT), dtype=torch.float32, device=device)
    y = torch.empty(cx.shape[0], dtype=torch.float32, device=device)
    crop_pair_inputs(ctx, feat, cx, cy, support, Z, y)
    return Z, y, cx, cy, support


def predict_seeds(ctx, mlp, T: int, n_items: int, M: int, R: int, device="cuda"):
    """The R candidate pairs of the loaded stream with the highest scores,
    as device tensors (sx, sy), and the scores of all candidates."""
    torch = _torch()
    _, cx, cy, Z = candidate_inputs(ctx, T, n_items, M, device)
    score = torch.empty(cx.shape[0], dtype=torch.float32, device=device)
    crop_mlp_score(ctx, mlp, Z, score)
    R = min(R, cx.shape[0])
    sx = torch.empty(R, dtype=torch.int32, device=device)
    sy = torch.empty(R, dtype=torch.int32, device=device)
    crop_select_seeds(ctx, score, cx, cy, R, sx, sy)
    return sx, sy, score


def flat_init(w) -> "list":
    """Concatenate W1, b1, W2, b2, w3, b3 in the library's parameter order."""
    import numpy as np
    flat = np.concatenate([np.asarray(w[k], np.float32).reshape(-1)
                           for k in ("W1", "b1", "W2", "b2", "w3", "b3")])
    assert flat.shape[0] == MLP_PARAMS
    return flat
