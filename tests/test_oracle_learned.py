"""Pins of the fp64 learned-seeding oracle (features, candidates, MLP, Adam).

The paper has no learned component; these pin the oracle to finite
differences, to torch's CPU autograd and optimiser (independent library
routines), to bfloat16 rounding in torch, and to dense-matrix forms of the
prefix statistics.
"""
import math

import numpy as np
import pytest
import torch

import datagen
import oracle
from oracle import learned


def small_params(seed=1):
    return {k: v.astype(np.float64) for k, v in datagen.mlp_init_weights(seed).items()}


def test_parameter_count():
    p = datagen.mlp_init_weights(0)
    assert sum(v.size for v in p.values()) == 6337


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    p = small_params(3)
    p["b1"] = rng.normal(0, 0.1, 64)
    p["b2"] = rng.normal(0, 0.1, 64)
    p["b3"] = np.array([0.3])
    Z = rng.normal(0, 1, (9, 32))
    y = rng.normal(2, 1, 9)
    loss, g = learned.mlp_backward(p, Z, y)
    eps = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            q = {k: v.copy() for k, v in p.items()}
            q[name].reshape(-1)[idx] += eps
            lp, _ = learned.mlp_backward(q, Z, y)
            q[name].reshape(-1)[idx] -= 2 * eps
            lm, _ = learned.mlp_backward(q, Z, y)
            fd = (lp - lm) / (2 * eps)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_backward_matches_torch_autograd():
    rng = np.random.default_rng(1)
    p = small_params(4)
    p["b1"] = rng.normal(0, 0.1, 64)
    Z = rng.normal(0, 1, (33, 32))
    y = rng.normal(1, 1, 33)
    loss, g = learned.mlp_backward(p, Z, y)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    tz = torch.tensor(Z, dtype=torch.float64)
    h1 = torch.relu(tz @ tp["W1"].T + tp["b1"])
    h2 = torch.relu(h1 @ tp["W2"].T + tp["b2"])
    out = h2 @ tp["w3"] + tp["b3"]
    tl = ((out - torch.tensor(y, dtype=torch.float64)) ** 2).mean()
    tl.backward()
    assert abs(float(tl.detach()) - loss) < 1e-12
    for k in p:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-10, atol=1e-12)


def test_zero_weights_special_case():
    p = {k: np.zeros_like(v) for k, v in small_params(0).items()}
    p["b3"] = np.array([0.7])
    Z = np.random.default_rng(2).normal(0, 1, (5, 32))
    y = np.arange(5.0)
    out, _ = learned.mlp_forward(p, Z)
    assert np.all(out == 0.7)
    _, g = learned.mlp_backward(p, Z, y)
    for k in p:
        if k == "b3":
            assert abs(g[k][0] - np.mean(2 * (0.7 - y))) < 1e-12
        else:
            assert np.all(g[k] == 0)


def test_adam_matches_torch():
    rng = np.random.default_rng(3)
    p = small_params(5)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    tp = [torch.tensor(p[k], dtype=torch.float64, requires_grad=True) for k in p]
    opt = torch.optim.Adam(tp, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 4):
        grads = {k: rng.normal(0, 1, p[k].shape) for k in p}
        p, m, v = learned.adam_step(p, grads, m, v, t)
        for tt, k in zip(tp, grads):
            tt.grad = torch.tensor(grads[k], dtype=torch.float64)
        opt.step()
    for tt, k in zip(tp, p):
        np.testing.assert_allclose(p[k], tt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(4)
    a = np.concatenate([rng.normal(0, 1, 10000), rng.normal(0, 1e4, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]]).astype(np.float32)
    ref = torch.tensor(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(learned.bf16_round(a), ref)


def test_bf16_score_matches_torch_bf16_layers():
    """bf16 scoring against torch's own bfloat16 Linear layers (fp32
    accumulation, every layer's output rounded to bfloat16): with biases
    that bfloat16 represents, the two readings coincide up to the rare
    activation that rounds the other way from an fp32 sum."""
    rng = np.random.default_rng(5)
    p = {k: v.astype(np.float32) for k, v in datagen.mlp_init_weights(8).items()}
    for k in ("b1", "b2", "b3"):
        p[k] = learned.bf16_round(rng.normal(0, 0.3, p[k].shape).astype(np.float32))
    Z = rng.normal(0, 2, (2000, 32)).astype(np.float32)
    got = learned.mlp_score_bf16(p, Z)
    bf = torch.bfloat16
    z = torch.tensor(Z).to(bf)
    h1 = torch.relu(torch.nn.functional.linear(z, torch.tensor(p["W1"]).to(bf), torch.tensor(p["b1"]).to(bf)))
    h2 = torch.relu(torch.nn.functional.linear(h1, torch.tensor(p["W2"]).to(bf), torch.tensor(p["b2"]).to(bf)))
    w3 = torch.tensor(learned.bf16_round(p["w3"])).to(torch.float64)
    want = (h2.to(torch.float64) @ w3 + float(p["b3"][0])).numpy()
    err = np.abs(got - want)
    scale = np.abs(want).max() + 1
    assert np.quantile(err, 0.99) <= 1e-6 * scale
    assert err.max() <= 1e-2 * scale


def test_bf16_score_equals_fp64_network_without_rounding():
    """Weights, inputs and every activation exactly representable in
    bfloat16 (small dyadic values, one hidden unit path): no rounding
    happens and the bf16 score is the fp64 network's."""
    p = {"W1": np.zeros((64, 32), np.float32), "b1": np.zeros(64, np.float32),
         "W2": np.zeros((64, 64), np.float32), "b2": np.zeros(64, np.float32),
         "w3": np.zeros(64, np.float32), "b3": np.array([0.25], np.float32)}
    p["W1"][0, :4] = [0.5, -0.25, 1.0, 0.125]
    p["W2"][3, 0] = 2.0
    p["w3"][3] = -0.75
    Z = np.array([[1.0, 2.0, 0.5, 4.0] + [0.0] * 28, [-1.0, 0.0, 0.0, 0.0] + [0.0] * 28],
                 np.float32)
    want, _ = learned.mlp_forward(p, Z)
    assert np.array_equal(learned.mlp_score_bf16(p, Z), want)
    assert want[0] == 0.25 + (-0.75) * 2.0 * 1.0  # relu(0.5 - 0.5 + 0.5 + 0.5) = 1.0


def test_item_stats_match_dense_forms():
    st = datagen.tiny_transactions(11, T=80, n=30, cap=20, mean_len=7.0)
    Tp = learned.prefix_len(st.T)
    assert Tp == math.ceil(0.05 * st.T)
    s = learned.item_stats(st.off, st.items, st.n, Tp)
    X = np.zeros((Tp, st.n))
    L = st.lengths()[:Tp]
    for t in range(Tp):
        X[t, st.items[st.off[t]:st.off[t + 1]].astype(np.int64)] = 1
    assert np.array_equal(s["A"], X.sum(0))
    assert np.array_equal(s["S1"], X.T @ (L - 1))
    assert np.array_equal(s["S2"], X.T @ ((L - 1) * (L - 2) // 2))
    assert np.array_equal(s["LMAX"], (X * L[:, None]).max(0))
    assert np.array_equal(s["H1"], X[:Tp // 2].sum(0))
    assert np.array_equal(s["LONG"], X.T @ (L >= 16))
    assert np.array_equal(s["SHORT"], X.T @ (L <= 4))
    for i in range(st.n):
        assert s["RANK"][i] == sum(1 for j in range(st.n) if s["A"][j] > s["A"][i])
    F = learned.item_features(s, Tp)
    assert F.shape == (st.n, 16)
    assert np.all(np.isfinite(F))


def test_candidates_are_pairs_of_top_items():
    A = np.array([5, 9, 9, 1, 0, 7, 9])
    top, cx, cy = learned.candidates(A, 4)
    # by (A desc, id asc): 1, 2, 6, 5
    assert top.tolist() == [1, 2, 5, 6]
    assert list(zip(cx.tolist(), cy.tolist())) == [(1, 2), (1, 5), (1, 6), (2, 5), (2, 6), (5, 6)]
