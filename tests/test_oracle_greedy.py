"""Pins of the oracle's greedy max coverage (Find_Most_Influential_Set,
Algorithm 2, with ties to the lowest vertex id over unselected vertices).

* A recompute-from-scratch greedy (every marginal gain recounted from the
  pool at every step) gives the same seeds and gains as the oracle's
  counter-decrement greedy.
* Exhaustive optimum on tiny pools: greedy >= (1 - 1/e) OPT (the guarantee
  from submodularity, Section II-A), with equality for k = 1.
"""

import itertools
import math

import numpy as np
import pytest

import oracle


def _random_pool(rng, n, n_sets, max_size):
    sets = []
    for _ in range(n_sets):
        sz = int(rng.integers(1, max_size + 1))
        sets.append(np.sort(rng.choice(n, size=min(sz, n), replace=False)))
    so = np.zeros(n_sets + 1, dtype=np.uint64)
    so[1:] = np.cumsum([s.size for s in sets])
    sv = np.concatenate(sets).astype(np.uint32) if sets else np.zeros(0, np.uint32)
    return sets, so, sv


def _naive_greedy(n, sets, k):
    covered = [False] * len(sets)
    chosen = []
    gains = []
    for _ in range(k):
        best, best_gain = None, -1
        for v in range(n):
            if v in chosen:
                continue
            gain = sum(1 for j, s in enumerate(sets) if not covered[j] and v in s)
            if gain > best_gain:
                best, best_gain = v, gain
        chosen.append(best)
        gains.append(best_gain)
        for j, s in enumerate(sets):
            if best in s:
                covered[j] = True
    return chosen, gains


@pytest.mark.parametrize("seed", range(12))
def test_matches_recompute_greedy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    sets, so, sv = _random_pool(rng, n, int(rng.integers(1, 150)), int(rng.integers(1, 8)))
    k = int(rng.integers(1, n + 1))
    seeds, gains, cov = oracle.greedy(n, so, sv, k)
    want_s, want_g = _naive_greedy(n, [set(s.tolist()) for s in sets], k)
    assert seeds.tolist() == want_s
    assert gains.tolist() == want_g
    assert cov == sum(want_g)


@pytest.mark.parametrize("seed", range(10))
def test_approximation_bound_exhaustive(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(4, 11))
    sets, so, sv = _random_pool(rng, n, int(rng.integers(3, 40)), 4)
    ss = [set(s.tolist()) for s in sets]
    for k in (1, 2, 3):
        if k > n:
            continue
        _, _, cov = oracle.greedy(n, so, sv, k)
        opt = max(sum(1 for s in ss if s & set(c)) for c in itertools.combinations(range(n), k))
        assert cov <= opt
        assert cov >= (1 - 1 / math.e) * opt
        if k == 1:
            assert cov == opt


def test_ties_and_exhaustion():
    # vertex 0 is in every set; afterwards every count is 0, so the remaining
    # picks are the lowest unselected ids with gain 0
    sets = [[0, 3], [0, 5], [0], [0, 2, 4]]
    so = np.array([0, 2, 4, 5, 8], dtype=np.uint64)
    sv = np.array(sum(sets, []), dtype=np.uint32)
    seeds, gains, cov = oracle.greedy(6, so, sv, 4)
    assert seeds.tolist() == [0, 1, 2, 3]
    assert gains.tolist() == [4, 0, 0, 0]
    assert cov == 4
    # equal counts: the lower id wins
    so2 = np.array([0, 1, 2], dtype=np.uint64)
    sv2 = np.array([7, 2], dtype=np.uint32)
    seeds, gains, _ = oracle.greedy(8, so2, sv2, 2)
    assert seeds.tolist() == [2, 7] and gains.tolist() == [1, 1]


def test_empty_pool():
    seeds, gains, cov = oracle.greedy(5, np.zeros(1, np.uint64), np.zeros(0, np.uint32), 3)
    assert seeds.tolist() == [0, 1, 2] and gains.tolist() == [0, 0, 0] and cov == 0
