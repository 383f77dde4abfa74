"""Pins of the oracle's hash specification.

The paper fixes the structure h(i,j) = (h_a(i) + h_b(j)) mod kappa with
pairwise independent h_a, h_b (Section 5, proof of Lemma 1) and the load
balance that follows (Section 6, Theorem 1); the family itself is this
project's reading (SplitMix64-seeded multiply-add-shift, kappa = 2^32).
"""
import math
import os

import numpy as np
import pytest

import datagen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_words(name):
    vals = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#") and not line.startswith("="):
            vals.append(int(line, 16))
    return vals


def test_splitmix64_published_vector():
    ref = _golden_words("splitmix64_seed0.txt")
    got = oracle.splitmix64(0, len(ref))
    assert [int(v) for v in got] == ref


def test_hash_params_are_splitmix_stream():
    for seed in (0, 1, 0x243F6A8885A308D3):
        assert np.array_equal(oracle.hash_params(seed), oracle.splitmix64(seed, 8))


def test_zero_key_gives_top_of_beta():
    # h_a(0) = ((alpha*0 + beta) mod 2^64) >> 32 = beta >> 32
    for seed in (3, 77):
        prm = oracle.hash_params(seed)
        ha, hb, h, _ = oracle.hash_many(seed, [0], [0])
        assert int(ha[0]) == int(prm[1]) >> 32
        assert int(hb[0]) == int(prm[3]) >> 32
        assert int(h[0]) == ((int(prm[1]) >> 32) + (int(prm[3]) >> 32)) % (1 << 32)


def test_h_is_sum_mod_2_32():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 2 ** 32, 5000, dtype=np.uint64).astype(np.uint32)
    y = rng.integers(0, 2 ** 32, 5000, dtype=np.uint64).astype(np.uint32)
    ha, hb, h, _ = oracle.hash_many(11, x, y)
    assert np.array_equal(h, (ha.astype(np.uint64) + hb.astype(np.uint64)).astype(np.uint32))


@pytest.mark.parametrize("P", [1, 2, 8, 1024, 1000, 7])
def test_part_is_equal_interval_and_nested_bucket(P):
    h = np.array([0, 1, 2 ** 31, 2 ** 32 - 1] + list(range(0, 2 ** 32, 2 ** 32 // 997)),
                 dtype=np.uint64)
    part = oracle.part_of(h, P).astype(np.int64)
    # each owner holds the interval [p*2^32/P, (p+1)*2^32/P) of hash values
    for v, p in zip(h.tolist(), part.tolist()):
        assert 0 <= p < P
        assert p * (1 << 32) <= v * P < (p + 1) * (1 << 32)
    assert part[0] == 0 and part[3] == P - 1
    for B in (1, 3, 16, 1024):
        b = oracle.bucket_of(h, P, B).astype(np.int64)
        assert np.all(b < P * B)
        assert np.array_equal(b // B, part)


def test_power_of_two_part_is_top_bits():
    rng = np.random.default_rng(9)
    x = rng.integers(0, 50000, 20000).astype(np.uint32)
    y = rng.integers(0, 50000, 20000).astype(np.uint32)
    for k in (0, 3, 10):
        _, _, h, part = oracle.hash_many(123, x, y, 1 << k)
        assert np.array_equal(part, (h.astype(np.uint64) >> np.uint64(32 - k)).astype(np.uint32)
                              if k else np.zeros_like(part))


def test_part_uniform_chi_square():
    st = datagen.config_small()
    r = oracle.tx_exact(st.off, st.items, 1, 0x243F6A8885A308D3)
    for P in (8, 64):
        _, _, _, part = oracle.hash_many(0x243F6A8885A308D3, r["x"], r["y"], P)
        obs = np.bincount(part, minlength=P).astype(np.float64)
        exp = r["x"].shape[0] / P
        chi2 = float(((obs - exp) ** 2 / exp).sum())
        # 99.9% quantile of chi-square with P-1 dof (Wilson-Hilferty)
        k = P - 1
        q = k * (1 - 2 / (9 * k) + 3.09 * math.sqrt(2 / (9 * k))) ** 3
        assert chi2 < q, (P, chi2, q)


def test_pair_collision_rate_is_one_over_P():
    # pairwise independence: Pr[part(e) = part(e')] = 1/P for distinct e, e'
    rng = np.random.default_rng(21)
    P = 16
    n = 4000
    x1 = rng.integers(0, 50000, n).astype(np.uint32)
    y1 = rng.integers(0, 50000, n).astype(np.uint32)
    x2 = rng.integers(0, 50000, n).astype(np.uint32)
    y2 = rng.integers(0, 50000, n).astype(np.uint32)
    same = ~((x1 == x2) & (y1 == y2))
    hits = 0
    total = 0
    for seed in range(40):
        _, _, _, p1 = oracle.hash_many(seed, x1, y1, P)
        _, _, _, p2 = oracle.hash_many(seed, x2, y2, P)
        hits += int(((p1 == p2) & same).sum())
        total += int(same.sum())
    rate = hits / total
    sd = math.sqrt((1 / P) * (1 - 1 / P) / total)
    assert abs(rate - 1 / P) < 5 * sd, (rate, 1 / P, sd)


def test_theorem1_load_mean_and_variance_over_seeds():
    # Section 6, Theorem 1 (its proof): X_p = sum_e f_e [part(e)=p] has mean
    # M/P and, for a pairwise independent hash, variance
    # (1/P)(1-1/P) sum_e f_e^2.
    st = datagen.config_small()
    r = oracle.tx_exact(st.off, st.items, 1, 1)
    f = r["cnt"].astype(np.float64)
    M = f.sum()
    P = 8
    dev2 = []
    means = []
    for seed in range(64):
        _, _, _, part = oracle.hash_many(1000 + seed, r["x"], r["y"], P)
        X = np.bincount(part, weights=f, minlength=P)
        means.append(X.mean())
        dev2.extend(((X - M / P) ** 2).tolist())
    var_theory = (1 / P) * (1 - 1 / P) * float((f * f).sum())
    assert abs(np.mean(means) - M / P) < 1e-9 * M
    ratio = float(np.mean(dev2)) / var_theory
    assert 0.75 < ratio < 1.3, ratio
