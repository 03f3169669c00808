"""Host check of the candidate-list rule the RandGreedi pick launch uses.

A partition keeps a list of the positions whose count exceeded a threshold
tau when the list was built; counts only fall, so a list entry whose count
is above tau has a larger count than any position outside the list and the
list's best (count, lowest position) key is the partition's argmax.  When
the list's best is not above tau the partition is scanned again: its argmax
is the pick, and the list is rebuilt from a histogram of the counts (the
highest bins that together hold at most `cap` positions).  This module runs
that rule in plain Python, with the same integer bin arithmetic as the
kernel but small lists and few bins so that rebuilds, ties and exhausted
partitions are frequent, and checks every pick against a full argmax while
counts fall between picks.  No GPU.
"""
import numpy as np
import pytest


def _key(c, pos):
    return (int(c) << 32) | (0xFFFFFFFF - int(pos))


def _rebuild(cnt, lo, hi, cap, bins):
    """The kernel's rebuild: (argmax key, list, tau), or (0, [], None) when
    every count of the partition is 0."""
    best = max((_key(cnt[q], q) for q in range(lo, hi)), default=0)
    mx = best >> 32
    if mx == 0:
        return 0, [], None
    hist = [0] * bins
    for q in range(lo, hi):
        if cnt[q] > 0:
            hist[(int(cnt[q]) * bins) // (mx + 1)] += 1
    suffix = np.cumsum(hist[::-1])[::-1]
    cut = int(sum(1 for x in suffix if x > cap))
    cmin = (cut * (mx + 1) + bins - 1) // bins
    tau = cmin - 1 if cmin > 0 else 0
    lst = [q for q in range(lo, hi) if cnt[q] > tau]
    assert len(lst) <= cap
    return best, lst, tau


def _run(seed, n, m, k, cap, bins):
    rng = np.random.default_rng(seed)
    bounds = np.concatenate([[0], np.sort(rng.choice(np.arange(1, n), m - 1, replace=False)), [n]])
    cnt = np.minimum(rng.zipf(1.6, n).astype(np.int64), 10 ** 6)
    cnt[rng.random(n) < 0.2] = 0
    lists = [[] for _ in range(m)]
    taus = [0] * m  # None: the partition has nothing left to gain
    rebuilds = 0
    for _ in range(k):
        for p in range(m):
            lo, hi = int(bounds[p]), int(bounds[p + 1])
            want = max((_key(cnt[q], q) for q in range(lo, hi)), default=0)
            if taus[p] is None:
                got = 0
            else:
                got = max((_key(cnt[q], q) for q in lists[p]), default=0)
                if (got >> 32) <= taus[p]:
                    rebuilds += 1
                    got, lists[p], taus[p] = _rebuild(cnt, lo, hi, cap, bins)
            if (want >> 32) == 0:
                assert (got >> 32) == 0
                continue
            assert got == want
            pick = 0xFFFFFFFF - (got & 0xFFFFFFFF)
            cnt[pick] = 0
            # other counts of the partition fall by 0..3
            idx = rng.integers(lo, hi, size=max(1, (hi - lo) // 3))
            cnt[idx] = np.maximum(0, cnt[idx] - rng.integers(0, 4, size=idx.size))
    return rebuilds


@pytest.mark.parametrize("seed", range(12))
def test_list_rule_equals_full_argmax(seed):
    cap = [4, 8, 16, 64][seed % 4]
    bins = [4, 8, 16, 64][(seed // 4) % 4]
    assert _run(seed, 600, 5, 40, cap, bins) > 0


def test_list_rule_partition_runs_out():
    """Few positive counts: every partition's counts reach 0 before k picks."""
    assert _run(99, 60, 3, 40, 4, 4) > 0
