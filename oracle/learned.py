"""fp64 oracle for the learned heavy-pair seeding (test infrastructure only).

The paper has no learned component.  Its Space-Saving analysis (Section 6,
Theorem 2 and its proof) names the failure mode seeding targets: a heavy
entry is lost when more than ell/2 heavy entries, or too much light mass,
share its bucket.  The reading used here (features, candidates, network,
loss and optimiser) is this project's own:

* prefix: the first ceil(5% of T) transactions of the stream;
* per-item statistics over the prefix (t in the prefix, L_t its length):
    A     transactions containing the item
    S1    sum of (L_t - 1)               pair occurrences involving the item
    S2    sum of (L_t - 1)(L_t - 2)/2
    LMAX  max L_t
    H1    transactions containing it among the first floor(T_p/2)
    LONG  transactions containing it with L_t >= 16
    SHORT transactions containing it with L_t <= 4
    RANK  number of items with a strictly larger A
* 16 features per item (item_features below);
* candidates: all pairs x < y among the top-M items by (A desc, id asc);
* network: [f(x), f(y)] (32) -> 64 -> 64 -> 1 with ReLU, fp32 weights,
  trained on y = log1p(exact support) with mean squared error and Adam
  (Kingma and Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8).
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 16
HIDDEN = 64


def prefix_len(T: int) -> int:
    return 0 if T <= 0 else max(1, (T + 19) // 20)


def item_stats(off, items, n: int, Tp: int):
    """Per-item prefix statistics as int64 arrays, by plain loops over the
    prefix transactions (numpy only to hold the arrays)."""
    off = np.asarray(off, np.int64)
    items = np.asarray(items, np.int64)
    A = np.zeros(n, np.int64)
    S1 = np.zeros(n, np.int64)
    S2 = np.zeros(n, np.int64)
    LMAX = np.zeros(n, np.int64)
    H1 = np.zeros(n, np.int64)
    LONG = np.zeros(n, np.int64)
    SHORT = np.zeros(n, np.int64)
    half = Tp // 2
    for t in range(Tp):
        seg = items[off[t]:off[t + 1]]
        L = seg.shape[0]
        A[seg] += 1
        S1[seg] += L - 1
        S2[seg] += (L - 1) * (L - 2) // 2
        LMAX[seg] = np.maximum(LMAX[seg], L)
        if t < half:
            H1[seg] += 1
        if L >= 16:
            LONG[seg] += 1
        if L <= 4:
            SHORT[seg] += 1
    # RANK[i] = #{j : A[j] > A[i]}
    order = np.sort(A)
    RANK = n - np.searchsorted(order, A, side="right")
    return dict(A=A, S1=S1, S2=S2, LMAX=LMAX, H1=H1, LONG=LONG, SHORT=SHORT,
                RANK=RANK.astype(np.int64))


def item_features(st, Tp: int) -> np.ndarray:
    """16 fp64 features per item from the prefix statistics.

    Parity unpinned: the features are this project's own definition (the
    paper has no learned component), so nothing outside it fixes their
    values; the statistics they are computed from are pinned against dense
    forms, the features themselves only by shape and finiteness."""
    A = st["A"].astype(np.float64)
    S1 = st["S1"].astype(np.float64)
    S2 = st["S2"].astype(np.float64)
    H1 = st["H1"].astype(np.float64)
    H2 = A - H1
    Tpf = float(max(Tp, 1))
    F = np.zeros((A.shape[0], N_FEAT), np.float64)
    F[:, 0] = np.log1p(A)
    F[:, 1] = 100.0 * A / Tpf
    F[:, 2] = np.log1p(st["RANK"].astype(np.float64))
    F[:, 3] = np.log1p(S1)
    F[:, 4] = np.log1p(S2)
    F[:, 5] = S1 / np.maximum(A, 1.0) / 10.0
    F[:, 6] = np.log1p(st["LMAX"].astype(np.float64))
    F[:, 7] = np.log1p(H1)
    F[:, 8] = np.log1p(H2)
    F[:, 9] = (H2 - H1) / (A + 1.0)
    F[:, 10] = np.log1p(st["LONG"].astype(np.float64))
    F[:, 11] = np.log1p(st["SHORT"].astype(np.float64))
    F[:, 12] = np.sqrt(A / Tpf)
    F[:, 13] = np.log1p(A) ** 2 / 10.0
    F[:, 14] = (A > 0).astype(np.float64)
    F[:, 15] = math.log(Tpf) / 10.0
    return F


def candidates(A, M: int):
    """Top-M items by (A desc, id asc); all pairs x < y among them in
    (x, y) lexicographic order.  Returns (top_items, cx, cy)."""
    A = np.asarray(A, np.int64)
    ids = np.arange(A.shape[0], dtype=np.int64)
    order = np.lexsort((ids, -A))
    top = np.sort(order[:M])
    cx, cy = [], []
    for a in range(top.shape[0]):
        for b in range(a + 1, top.shape[0]):
            cx.append(top[a])
            cy.append(top[b])
    return top, np.array(cx, np.uint32), np.array(cy, np.uint32)


def mlp_forward(params, Z):
    """Z: [N, 32].  Returns (out[N], cache) in fp64."""
    W1 = np.asarray(params["W1"], np.float64)
    b1 = np.asarray(params["b1"], np.float64)
    W2 = np.asarray(params["W2"], np.float64)
    b2 = np.asarray(params["b2"], np.float64)
    w3 = np.asarray(params["w3"], np.float64)
    b3 = float(np.asarray(params["b3"], np.float64).reshape(-1)[0])
    Z = np.asarray(Z, np.float64)
    a1 = Z @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    out = h2 @ w3 + b3
    return out, dict(Z=Z, a1=a1, h1=h1, a2=a2, h2=h2, W2=W2, w3=w3)


def mlp_score_bf16(params, Z):
    """bf16 scoring (this project's reading of a bf16 inference pass; the
    paper has none): the weights W1, W2, w3, the inputs and both hidden
    layers' activations are rounded to bfloat16 (nearest even); biases stay
    as given; products and sums in fp64.  Returns out[N]."""
    rb = lambda a: np.asarray(bf16_round(np.asarray(a, np.float32)), np.float64)
    W1, W2, w3 = rb(params["W1"]), rb(params["W2"]), rb(params["w3"])
    b1 = np.asarray(params["b1"], np.float64)
    b2 = np.asarray(params["b2"], np.float64)
    b3 = float(np.asarray(params["b3"], np.float64).reshape(-1)[0])
    h1 = rb(np.maximum(rb(Z) @ W1.T + b1, 0.0))
    h2 = rb(np.maximum(h1 @ W2.T + b2, 0.0))
    return h2 @ w3 + b3


def mlp_backward(params, Z, y):
    """Loss = mean((out - y)^2).  Returns (loss, grads dict) in fp64, by the
    chain rule written out layer by layer."""
    out, c = mlp_forward(params, Z)
    N = out.shape[0]
    y = np.asarray(y, np.float64)
    r = out - y
    loss = float(np.mean(r * r))
    g_out = 2.0 * r / N
    g_w3 = c["h2"].T @ g_out
    g_b3 = np.array([g_out.sum()])
    g_h2 = np.outer(g_out, c["w3"])
    g_a2 = g_h2 * (c["a2"] > 0)
    g_W2 = g_a2.T @ c["h1"]
    g_b2 = g_a2.sum(axis=0)
    g_h1 = g_a2 @ c["W2"]
    g_a1 = g_h1 * (c["a1"] > 0)
    g_W1 = g_a1.T @ c["Z"]
    g_b1 = g_a1.sum(axis=0)
    return loss, dict(W1=g_W1, b1=g_b1, W2=g_W2, b2=g_b2, w3=g_w3, b3=g_b3)


def adam_step(params, grads, m, v, t: int, lr: float = 1e-3, b1: float = 0.9,
              b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (fp64) of every tensor; returns new (params, m, v)."""
    newp, newm, newv = {}, {}, {}
    for k in params:
        g = np.asarray(grads[k], np.float64)
        mk = b1 * np.asarray(m[k], np.float64) + (1.0 - b1) * g
        vk = b2 * np.asarray(v[k], np.float64) + (1.0 - b2) * g * g
        mh = mk / (1.0 - b1 ** t)
        vh = vk / (1.0 - b2 ** t)
        newp[k] = np.asarray(params[k], np.float64) - lr * mh / (np.sqrt(vh) + eps)
        newm[k] = mk
        newv[k] = vk
    return newp, newm, newv


def bf16_round(a) -> np.ndarray:
    """Round fp32 values to the nearest bfloat16 (ties to even); returns fp32.
    NaN is not expected here."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32)
