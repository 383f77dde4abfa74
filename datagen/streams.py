"""Seeded synthetic transaction streams and sparse outer-product sums.

Every random number comes from the raw 64-bit outputs of numpy's PCG64 bit
generator (``random_raw``), which is fixed by the PCG64 algorithm and does not
depend on numpy's distribution methods.  The transforms below are this
project's own:

* uniform      u = (raw >> 11) * 2^-53                     in [0, 1)
* geometric    L = 1 + floor(ln(1-u) / ln(1-p)),  p = 1/mean, then min(L, cap)
* Zipf rank    binary search of u * W in the fp64 prefix sums of r^-s, r = 1..n
* item id      pi(rank - 1) for a seeded permutation pi (argsort of raw words)
* distinctness duplicates inside a vector are redrawn until none remain,
               then each vector is sorted ascending
* normal       Box-Muller on two uniforms

The workloads stand in for the paper's datasets (FIMI, UCI bag-of-words and
Wikipedia in Section 7.3, Table 1), which are not reproduced: power-law item
popularity gives the skew that the paper's analysis assumes (Section 6,
Zipfian entry weights).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


class Raw:
    """A stream of raw 64-bit words from PCG64(seed) plus derived uniforms."""

    def __init__(self, seed: int):
        self.seed = int(seed)
        self._bg = np.random.PCG64(self.seed)

    def raw(self, n: int) -> np.ndarray:
        if n <= 0:
            return np.zeros(0, dtype=np.uint64)
        return self._bg.random_raw(int(n)).astype(np.uint64, copy=False)

    def uniform(self, n: int) -> np.ndarray:
        r = self.raw(n)
        return (r >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def randint(self, n: int, lo: int, hi_incl: int) -> np.ndarray:
        """Integers in [lo, hi_incl] by scaling a uniform (bias < 2^-40)."""
        u = self.uniform(n)
        span = hi_incl - lo + 1
        v = np.floor(u * span).astype(np.int64)
        return lo + np.minimum(v, span - 1)


@dataclasses.dataclass
class Transactions:
    """A {0,1} transaction stream in CSR form.

    off:   uint32[T+1], off[0] = 0, non-decreasing, off[T] = nnz
    items: uint32[nnz], strictly increasing inside each transaction
    n:     number of item ids (every id < n)
    """

    off: np.ndarray
    items: np.ndarray
    n: int
    seed: int = 0
    label: str = ""

    @property
    def T(self) -> int:
        return int(self.off.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.items.shape[0])

    def lengths(self) -> np.ndarray:
        return np.diff(self.off.astype(np.int64))

    def slice(self, t0: int, t1: int) -> "Transactions":
        a, b = int(self.off[t0]), int(self.off[t1])
        off = (self.off[t0:t1 + 1].astype(np.int64) - a).astype(np.uint32)
        return Transactions(off, self.items[a:b].copy(), self.n, self.seed,
                            f"{self.label}[{t0}:{t1}]")


@dataclasses.dataclass
class OuterProducts:
    """K pairs of sparse vectors (a_k, b_k) in CSR form.

    a_off/b_off: uint32[K+1]; a_idx < n_rows, b_idx < n_cols, strictly
    increasing inside each vector; a_val/b_val float32.
    """

    a_off: np.ndarray
    a_idx: np.ndarray
    a_val: np.ndarray
    b_off: np.ndarray
    b_idx: np.ndarray
    b_val: np.ndarray
    n_rows: int
    n_cols: int
    seed: int = 0
    label: str = ""

    @property
    def K(self) -> int:
        return int(self.a_off.shape[0] - 1)


# --------------------------------------------------------------------------
# helpers

def _geometric(rng: Raw, count: int, mean: float, cap: int) -> np.ndarray:
    u = rng.uniform(count)
    p = 1.0 / float(mean)
    if p >= 1.0:
        L = np.ones(count, dtype=np.int64)
    else:
        L = 1 + np.floor(np.log1p(-u) / math.log1p(-p)).astype(np.int64)
    return np.minimum(L, cap)


def _power_law_sampler(n: int, s: float):
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
    cum = np.cumsum(w)
    return cum


def _draw_ranks(rng: Raw, cum: np.ndarray, count: int) -> np.ndarray:
    u = rng.uniform(count)
    r = np.searchsorted(cum, u * cum[-1], side="right")
    return np.minimum(r, cum.shape[0] - 1).astype(np.int64)


def _make_distinct(rows_len: np.ndarray, vals: np.ndarray, redraw) -> np.ndarray:
    """Sort each vector's values and redraw duplicates until none remain.

    rows_len: lengths of the vectors (their concatenation is ``vals``)
    redraw(k): returns k fresh values (int64), drawn in position order.
    """
    T = rows_len.shape[0]
    row_of = np.repeat(np.arange(T, dtype=np.int64), rows_len)
    shift = int(max(1, int(vals.max(initial=0)) + 1).bit_length())
    # first pass: sort whole array by (row, value)
    comb = (row_of << shift) | vals
    comb.sort()
    vals = comb & ((1 << shift) - 1)
    while True:
        dup = np.zeros(vals.shape[0], dtype=bool)
        if vals.shape[0] > 1:
            dup[1:] = (vals[1:] == vals[:-1]) & (row_of[1:] == row_of[:-1])
        pos = np.flatnonzero(dup)
        if pos.shape[0] == 0:
            return vals
        fresh = redraw(pos.shape[0])
        vals = vals.copy()
        vals[pos] = fresh
        # re-sort only the vectors that changed
        rows = np.unique(row_of[pos])
        starts = np.zeros(T + 1, dtype=np.int64)
        np.cumsum(rows_len, out=starts[1:])
        seg_len = rows_len[rows]
        seg_pos = np.repeat(starts[rows], seg_len) + (
            np.arange(int(seg_len.sum()), dtype=np.int64)
            - np.repeat(np.cumsum(seg_len) - seg_len, seg_len))
        sub = (row_of[seg_pos] << shift) | vals[seg_pos]
        sub.sort()
        vals[seg_pos] = sub & ((1 << shift) - 1)


def _offsets(lengths: np.ndarray) -> np.ndarray:
    off = np.zeros(lengths.shape[0] + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    if off[-1] >= 2 ** 32:
        raise ValueError("stream too large for uint32 offsets")
    return off.astype(np.uint32)


# --------------------------------------------------------------------------
# generators

def transactions(T: int, n: int, zipf_s: float, mean_len: float, cap: int,
                 rng: Raw, label: str = "") -> Transactions:
    """T transactions over n items, Zipf(s) popularity, geometric lengths."""
    cap = min(int(cap), int(n))
    perm = np.argsort(rng.raw(n), kind="stable").astype(np.int64)
    L = _geometric(rng, T, mean_len, cap)
    cum = _power_law_sampler(n, zipf_s)
    nnz = int(L.sum())
    ranks = _draw_ranks(rng, cum, nnz)

    def redraw(k):
        return perm[_draw_ranks(rng, cum, k)]

    items = _make_distinct(L, perm[ranks], redraw)
    return Transactions(_offsets(L), items.astype(np.uint32), int(n), rng.seed, label)


def outer_products(K: int, n_rows: int, n_cols: int, alpha: float, max_nnz: int,
                   rng: Raw, label: str = "") -> OuterProducts:
    """K pairs (a_k, b_k): lengths ~ m^-alpha on [1, max_nnz], uniform
    distinct indices, values fl32(+-exp(N(0,1))) with a random sign."""
    cum = _power_law_sampler(max_nnz, alpha)
    La = np.minimum(_draw_ranks(rng, cum, K) + 1, n_rows)
    Lb = np.minimum(_draw_ranks(rng, cum, K) + 1, n_cols)

    def idx(L, n):
        first = rng.randint(int(L.sum()), 0, n - 1)
        return _make_distinct(L, first, lambda k: rng.randint(k, 0, n - 1))

    a_idx = idx(La, n_rows)
    b_idx = idx(Lb, n_cols)

    def vals(count):
        u1 = rng.uniform(count)
        u2 = rng.uniform(count)
        sgn = rng.raw(count) & np.uint64(1)
        z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)
        v = np.exp(z) * np.where(sgn == 1, -1.0, 1.0)
        return v.astype(np.float32)

    return OuterProducts(_offsets(La), a_idx.astype(np.uint32), vals(a_idx.shape[0]),
                         _offsets(Lb), b_idx.astype(np.uint32), vals(b_idx.shape[0]),
                         int(n_rows), int(n_cols), rng.seed, label)


# --------------------------------------------------------------------------
# named workloads (sizes and distributions of the paper-scale benchmarks)

def config_small(seed: int = 1) -> Transactions:
    """2,000 transactions over 500 items, Zipf s=1.0, length Geom(mean 8) <= 32."""
    return transactions(2000, 500, 1.0, 8.0, 32, Raw(seed), "small")


def config_large(seed: int = 2, T: int = 1_000_000) -> Transactions:
    """1,000,000 transactions over 50,000 items, Zipf s=1.1, Geom(mean 10) <= 64."""
    return transactions(T, 50_000, 1.1, 10.0, 64, Raw(seed), "large")


def config_outer(seed: int = 3, K: int = 100_000, n: int = 200_000) -> OuterProducts:
    """K = 100,000 outer products over 200,000 rows/cols, nnz ~ m^-2 on [1,2000]."""
    return outer_products(K, n, n, 2.0, 2000, Raw(seed), "outer")


def config_batched_stream(s: int, base_seed: int = 4000, t_lo: float = 1e3,
                          t_hi: float = 2e5) -> Transactions:
    """Stream s of the batched configuration: T log-uniform in [t_lo, t_hi],
    n ~ U[5e3, 5e4], Zipf s ~ U[0.8, 1.3], lengths Geom(mean 10) <= 64, seed
    base_seed + s."""
    rng = Raw(base_seed + s)
    u = rng.uniform(2)
    T = int(math.floor(math.exp(math.log(t_lo) + u[0] * (math.log(t_hi) - math.log(t_lo)))))
    n = int(rng.randint(1, 5000, 50000)[0])
    zs = 0.8 + 0.5 * float(u[1])
    return transactions(T, n, zs, 10.0, 64, rng, f"batched{s}")


def config_batched(n_streams: int = 256, base_seed: int = 4000,
                   t_lo: float = 1e3, t_hi: float = 2e5):
    """Independent streams (config_batched_stream), one seed per stream."""
    return [config_batched_stream(s, base_seed, t_lo, t_hi) for s in range(n_streams)]


def config_learned_train(i: int, T: int = 1_000_000) -> Transactions:
    """Training stream i (0..19): like the large configuration, seed 5000+i."""
    return transactions(T, 50_000, 1.1, 10.0, 64, Raw(5000 + i), f"train{i}")


def config_learned_heldout(T: int = 1_000_000) -> Transactions:
    """Held-out stream for learned seeding, seed 5100."""
    return transactions(T, 50_000, 1.1, 10.0, 64, Raw(5100), "heldout")


def tiny_transactions(seed: int, T: int = 40, n: int = 30, zipf_s: float = 1.0,
                      mean_len: float = 5.0, cap: int = 12) -> Transactions:
    return transactions(T, n, zipf_s, mean_len, cap, Raw(seed), f"tiny{seed}")


def tiny_outer(seed: int, K: int = 20, n_rows: int = 40, n_cols: int = 30,
               max_nnz: int = 12) -> OuterProducts:
    return outer_products(K, n_rows, n_cols, 1.5, max_nnz, Raw(seed), f"tinyop{seed}")


def concat_transactions(streams):
    """Concatenate streams into one CSR plus per-stream row offsets."""
    offs, items, row_base = [], [], [0]
    base = 0
    for st in streams:
        offs.append(st.off[:-1].astype(np.int64) + base)
        items.append(st.items)
        base += st.nnz
        row_base.append(row_base[-1] + st.T)
    offs.append(np.array([base], dtype=np.int64))
    off = np.concatenate(offs)
    if base >= 2 ** 32:
        raise ValueError("batch too large for uint32 offsets")
    return off.astype(np.uint32), np.concatenate(items), np.array(row_base, dtype=np.int64)


# --------------------------------------------------------------------------
# random inputs of the learned seeding: initial weights and sample order

def mlp_init_weights(seed: int, n_in: int = 32, hidden: int = 64):
    """Initial weights uniform(+-sqrt(6/fan_in)) from PCG64(seed), biases 0.
    Shapes: W1 [hidden, n_in], b1 [hidden], W2 [hidden, hidden], b2 [hidden],
    w3 [hidden], b3 [1]; fp32."""
    rng = Raw(seed)

    def uni(shape, fan_in):
        u = rng.uniform(int(np.prod(shape))).reshape(shape)
        lim = math.sqrt(6.0 / fan_in)
        return ((2.0 * u - 1.0) * lim).astype(np.float32)

    return dict(W1=uni((hidden, n_in), n_in), b1=np.zeros(hidden, np.float32),
                W2=uni((hidden, hidden), hidden), b2=np.zeros(hidden, np.float32),
                w3=uni((hidden,), hidden), b3=np.zeros(1, np.float32))


def sample_order(seed: int, n_samples: int, epochs: int) -> np.ndarray:
    """One seeded permutation of range(n_samples) per epoch, concatenated."""
    rng = Raw(seed)
    return np.concatenate([np.argsort(rng.raw(n_samples), kind="stable")
                           for _ in range(epochs)]).astype(np.uint32)
