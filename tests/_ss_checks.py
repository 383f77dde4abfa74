"""Shared checks of Space-Saving summaries against exact counts.

Section 4 (frequent items mining): a summary of ell slots over a stream of
total weight m has overestimation at most m/ell, and every entry heavier
than m/ell is monitored.  Per bucket b with exact weights f_e:
  I1  sum of the counts = m_b (the bucket's routed weight)
  I2  count - err <= f_e <= count for every monitored e
  I3  every e with f_e > min_b (full bucket) is monitored
  I4  min_b <= m_b / ell (over unpinned slots) and err <= min_b
  I5  an unmonitored e has f_e <= min_b
Pinned slots (learned seeding) have err = 0 and count = f_e.
"""
import numpy as np

import oracle


def check_invariants(s, exact, seed, rtol=0.0):
    """s: dict with x, y, used, pinned, cnt, err, P, B, ell (bucket-major
    slots); exact: {packed key: weight}.  rtol > 0 for fp32 weights."""
    P, B, ell = s["P"], s["B"], s["ell"]
    keys = oracle.pack_keys(s["x"], s["y"]).reshape(P * B, ell)
    used = np.asarray(s["used"]).reshape(P * B, ell)
    pinned = np.asarray(s["pinned"]).reshape(P * B, ell)
    cnt = np.asarray(s["cnt"], np.float64).reshape(P * B, ell)
    err = np.asarray(s["err"], np.float64).reshape(P * B, ell)
    ek = np.array(list(exact.keys()), np.uint64)
    ef = np.array(list(exact.values()), np.float64)
    _, _, h, _ = oracle.hash_many(seed, (ek >> np.uint64(32)).astype(np.uint32),
                                  (ek & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    bk = oracle.bucket_of(h, P, B).astype(np.int64)
    m_b = np.bincount(bk, weights=ef, minlength=P * B)
    tol = lambda v: rtol * max(abs(v), 1.0) + (1e-9 if rtol else 0.0)
    mins = np.zeros(P * B)
    for b in np.flatnonzero(used.any(axis=1) | (m_b > 0)):
        u = used[b]
        assert abs(cnt[b][u].sum() - m_b[b]) <= tol(m_b[b]), f"I1 bucket {b}"
        free = u & ~pinned[b]
        full = u.all()
        mn = cnt[b][free].min() if (full and free.any()) else 0.0
        mins[b] = mn
        pinned_mass = sum(exact.get(int(k), 0.0) for k in keys[b][u & pinned[b]])
        n_unpinned = int((~pinned[b]).sum())
        if full and n_unpinned:
            assert mn <= (m_b[b] - pinned_mass) / n_unpinned + tol(m_b[b]), f"I4 bucket {b}"
        for k in np.flatnonzero(u):
            f = exact.get(int(keys[b][k]), 0.0)
            assert cnt[b][k] - err[b][k] <= f + tol(f), f"I2 low bucket {b}"
            assert f <= cnt[b][k] + tol(f), f"I2 high bucket {b}"
            if pinned[b][k]:
                assert err[b][k] == 0 and abs(cnt[b][k] - f) <= tol(f), f"pinned bucket {b}"
            else:
                assert err[b][k] <= mn + tol(mn), f"I4 err bucket {b}"
    mon = set(keys[used].tolist())
    for key, f, b in zip(ek.tolist(), ef.tolist(), bk.tolist()):
        if key not in mon:
            assert f <= mins[b] + tol(f), f"I3/I5 bucket {b}"
