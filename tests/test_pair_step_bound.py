"""The bound on the steps of the one-wave pair walk that sizes the pair-mask
workspace: ((m^2 + n_el m) + 63) // 64 + n_el (n_el + 1) / 2 for a centre
with m neighbours of n_el elements.  The walk (k_triplet) takes, per class
of element pair (e1 <= e2) and per chunk of up to 64 j of block e1, one step
per group of R = 64 // mJ (mJ <= 32) or 1 lane groups of deltas.  Counted
here by brute force for every split of m over the elements (small m) and
for random splits (large m)."""
import itertools

import numpy as np


def bound(m, n_el):
    return (m * m + n_el * m + 63) // 64 + n_el * (n_el + 1) // 2


def walk_steps(cnt):
    steps = 0
    n_el = len(cnt)
    for e1 in range(n_el):
        for e2 in range(e1, n_el):
            same = e1 == e2
            mA, mB = cnt[e1], cnt[e2]
            if (mA < 2) if same else (mA == 0 or mB == 0):
                continue
            d_lo, d_hi = (1, mA >> 1) if same else (0, mB - 1)
            for jc in range(0, mA, 64):
                mJ = min(64, mA - jc)
                R = 64 // mJ if mJ <= 32 else 1
                if d_hi >= d_lo:
                    steps += (d_hi - d_lo) // R + 1
    return steps


def test_bound_every_split_small():
    for n_el in (1, 2, 3):
        for m in range(0, 90 if n_el < 3 else 40):
            for split in itertools.product(range(m + 1), repeat=n_el - 1):
                if sum(split) > m:
                    continue
                cnt = list(split) + [m - sum(split)]
                assert walk_steps(cnt) <= bound(m, n_el), (cnt, walk_steps(cnt), bound(m, n_el))


def test_bound_random_splits_large():
    rng = np.random.default_rng(5)
    for _ in range(3000):
        n_el = int(rng.integers(1, 5))
        m = int(rng.integers(0, 1200))
        cuts = np.sort(rng.integers(0, m + 1, n_el - 1))
        cnt = np.diff(np.concatenate([[0], cuts, [m]])).tolist()
        assert walk_steps(cnt) <= bound(m, n_el)


def test_bound_is_near_tight_for_water_rows():
    """About 86 neighbours of two elements (a water row): the bound is within
    a factor of two of the walk, so the workspace is not oversized."""
    s = walk_steps([57, 29])
    assert s <= bound(86, 2) <= 2.5 * s
