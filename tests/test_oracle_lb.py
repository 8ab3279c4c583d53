"""Closed-form pins of the oracle's lower-bound step (IMM's OPT_Lower_Bound
with early break, Algorithm 1 with Tang et al.'s schedule): graphs whose
coverage follows from the graph alone, so the break round, LB, theta, the
targets and the seeds are derived here without the oracle's sampling or
greedy.

* Every edge certain (threshold 2^32 - 1) on a strongly connected graph:
  every RRR set is the whole vertex set, so F_R(S) = 1 for any non-empty S.
  The test n F >= (1 + sqrt(2) eps) n / 2^i first passes at the smallest i
  with 2^i >= 1 + sqrt(2) eps, and LB = n / (1 + sqrt(2) eps).
* Every edge dead (threshold 0): every RRR set is its root alone, so the
  greedy's coverage is the sum of the k largest root multiplicities (ties to
  the lowest id), computed from the roots alone; a case with no break keeps
  LB = 1.
The roots come from the root draw (pinned to Philox's published vectors and
to uniformity elsewhere); the theta constants from the theta plan (pinned to
their closed forms elsewhere)."""

import math

import numpy as np
import pytest

import oracle
import synth

T32 = 1 << 32


def _strongly_connected(n, rng, thr):
    edges = [(v, (v + 1) % n) for v in range(n)]
    while len(edges) < 3 * n:
        u, v = (int(x) for x in rng.integers(0, n, 2))
        if u != v and (u, v) not in edges:
            edges.append((u, v))
    return synth.tiny_graph(n, edges, "ic", [thr] * len(edges))


@pytest.mark.parametrize("eps,brk", [(0.5, 1), (0.7, 1), (0.75, 2), (2.0, 2), (3.0, 3)])
def test_certain_edges_break_in_closed_form(eps, brk):
    n, k = 100, 3
    g = _strongly_connected(n, np.random.default_rng(5), T32 - 1)
    r = oracle.imm(g, k, eps, 1.0, 77, keep_pool=True)
    sizes = np.diff(r["set_off"])
    assert np.all(sizes == n), "every set is the whole graph"
    lp, ls, i_max = oracle.theta_plan(n, k, eps, 1.0)
    epsp = math.sqrt(2.0) * eps
    # the smallest i with 2^i >= 1 + sqrt(2) eps
    i = 1
    while 2.0 ** i < 1.0 + epsp:
        i += 1
    assert i == brk and i <= i_max
    targets = [math.ceil(lp / math.ldexp(n, -j)) for j in range(1, i + 1)]
    lb = n / (1.0 + epsp)
    theta = math.ceil(ls / lb)
    assert r["rounds"] == i
    assert r["targets"] == targets + [theta]
    assert r["round_cov"] == targets[:]  # one seed covers every set
    assert r["lb"] == lb
    assert r["theta"] == max(targets[-1], theta)
    # all counts equal: lowest id first, then every set is covered
    assert r["seeds"].tolist() == list(range(k))
    assert r["gains"].tolist() == [r["theta"]] + [0] * (k - 1)
    assert r["covered"] == r["theta"]


def _dead_edges(n, rng):
    edges = set()
    while len(edges) < 2 * n:
        u, v = (int(x) for x in rng.integers(0, n, 2))
        if u != v:
            edges.add((u, v))
    edges = sorted(edges)
    return synth.tiny_graph(n, edges, "ic", [0] * len(edges))


def _topk_cover(roots, n, k):
    c = np.bincount(roots, minlength=n)
    order = np.lexsort((np.arange(n), -c))  # count descending, then id ascending
    return order[:k], c[order[:k]]


@pytest.mark.parametrize("n,k,eps,seed", [(300, 5, 0.5, 11), (64, 1, 0.5, 3), (256, 1, 0.9, 5),
                                          (500, 20, 0.3, 8), (40, 8, 0.2, 2)])
def test_dead_edges_follow_root_multiplicities(n, k, eps, seed):
    g = _dead_edges(n, np.random.default_rng(seed))
    r = oracle.imm(g, k, eps, 1.0, seed, keep_pool=True)
    lp, ls, i_max = oracle.theta_plan(n, k, eps, 1.0)
    epsp = math.sqrt(2.0) * eps
    T_last = math.ceil(lp / math.ldexp(n, -i_max))
    theta_max = math.ceil(ls)  # LB >= 1
    ids = max(T_last, theta_max)
    roots = np.array([oracle.root(seed, s, n) for s in range(ids)], dtype=np.int64)
    # the pool is the roots themselves
    np.testing.assert_array_equal(np.diff(r["set_off"]), 1)
    lb, targets, covs, rounds = 1.0, [], [], i_max
    for i in range(1, i_max + 1):
        x = math.ldexp(n, -i)
        T = math.ceil(lp / x)
        targets.append(T)
        _, top = _topk_cover(roots[:T], n, k)
        cov = int(top.sum())
        covs.append(cov)
        if n * (cov / T) >= (1.0 + epsp) * x:
            lb = n * (cov / T) / (1.0 + epsp)
            rounds = i
            break
    theta = math.ceil(ls / lb)
    final = max(targets[-1], theta)
    assert r["rounds"] == rounds
    assert r["targets"] == targets + [theta]
    assert r["round_cov"] == covs
    assert r["lb"] == lb
    assert r["theta"] == final
    seeds, top = _topk_cover(roots[:final], n, k)
    assert r["seeds"].tolist() == seeds.tolist()
    assert r["gains"].tolist() == top.tolist()
    assert r["covered"] == int(top.sum())


def test_dead_edges_cases_cover_break_and_no_break():
    """The parameter sets above include a run that breaks early, one that
    breaks in its last round or never, and LB = 1 (no break) at least once."""
    seen = set()
    for n, k, eps, seed in [(300, 5, 0.5, 11), (64, 1, 0.5, 3), (256, 1, 0.9, 5),
                            (500, 20, 0.3, 8), (40, 8, 0.2, 2)]:
        g = _dead_edges(n, np.random.default_rng(seed))
        r = oracle.imm(g, k, eps, 1.0, seed)
        _, _, i_max = oracle.theta_plan(n, k, eps, 1.0)
        seen.add("lb1" if r["lb"] == 1.0 else ("early" if r["rounds"] < i_max else "last"))
    assert "lb1" in seen and "early" in seen
