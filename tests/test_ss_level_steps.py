"""The level-step rule of the one-bucket Space-Saving chain, checked by brute
force against single Space-Saving steps (Section 4, Algorithm 1's update:
a monitored key takes the weight, else a free counter, else the counter of
minimum count is overwritten and its count becomes the overestimation).

The summary kernel applies a bucket's missed updates in level steps: the
slots at the minimum level (free slots below every count, count c at level
c + 1; ties broken by the lowest slot) all take the next updates at once, in
slot order.  This host model of that rule must reach exactly the state of
the single steps, including free, pinned and unequal-weight cases.
"""
import random

import pytest


def single_steps(state, updates):
    """One Space-Saving step per update (every update is a miss)."""
    c, k, e, used, pinned = (list(x) for x in state)
    for key, w in updates:
        best = None
        for j in range(len(c)):
            if pinned[j]:
                continue
            offer = (0, j) if not used[j] else (1, c[j], j)
            if best is None or offer < best[0]:
                best = (offer, j)
        if best is None:
            continue  # every slot pinned: the update drops
        j = best[1]
        if used[j]:
            e[j] = c[j]
            c[j] += w
        else:
            e[j], c[j], used[j] = 0, w, True
        k[j] = key
    return c, k, e, used


def level_steps(state, updates):
    """All slots at the minimum level take the next updates in slot order."""
    c, k, e, used, pinned = (list(x) for x in state)
    pos = 0
    while pos < len(updates):
        lvl = [None if pinned[j] else (c[j] + 1 if used[j] else 0) for j in range(len(c))]
        live = [v for v in lvl if v is not None]
        if not live:
            break
        mn = min(live)
        at = [j for j in range(len(c)) if lvl[j] == mn]
        take = min(len(at), len(updates) - pos)
        for r in range(take):
            j = at[r]
            key, w = updates[pos + r]
            if mn:
                e[j] = c[j]
                c[j] += w
            else:
                e[j], c[j], used[j] = 0, w, True
            k[j] = key
        pos += take
    return c, k, e, used


@pytest.mark.parametrize("seed", range(4))
def test_level_steps_equal_single_steps(seed):
    rng = random.Random(seed)
    for _ in range(2500):
        n = rng.choice([1, 4, 16, 32])
        used = [rng.random() < 0.8 for _ in range(n)]
        pinned = [u and rng.random() < rng.choice([0.0, 0.2, 1.0]) for u in used]
        c = [rng.randrange(1, 6) if u else 0 for u in used]
        state = (c, list(range(n)), [0] * n, used, pinned)
        ups = [(100 + t, rng.choice([1, 1, 1, 2, 3, 7])) for t in range(rng.randrange(0, 70))]
        assert level_steps(state, ups) == single_steps(state, ups)


def test_unit_updates_on_equal_counts_take_every_slot_per_step():
    # 16 slots at count 5, 32 unit misses: two steps of 16, every slot twice
    state = ([5] * 16, list(range(16)), [0] * 16, [True] * 16, [False] * 16)
    ups = [(100 + t, 1) for t in range(32)]
    c, k, e, _ = level_steps(state, ups)
    assert c == [7] * 16 and e == [6] * 16 and k == [116 + j for j in range(16)]
    assert (c, k, e) == single_steps(state, ups)[:3]
