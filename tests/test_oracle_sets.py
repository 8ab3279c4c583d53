"""Pins of the oracle's RRR sets (Generate_RRRsets, Algorithm 3; IC and LT
models of Section II-A).

* Exact invariants: every IC set equals the reverse reachability of its root
  in the sample's materialised live-edge graph (scipy BFS); every LT set is
  the backward chain of live in-edges chosen by a library search
  (numpy.searchsorted) over the cumulative table.
* Special cases with known answers.
* Brute force: on graphs of at most 12 edges the exact distribution of the
  RR set (enumerating every live-edge world with exact Fractions) and the
  reverse-influence identity E[n 1{S meets R}] = sigma(S), where sigma is
  computed from the forward diffusion definitions (IC by exact world
  enumeration, LT by forward threshold simulation), agree with oracle samples
  within 5 standard errors.
"""

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order

import oracle
import synth

T32 = 1 << 32


def _dst(g):
    return np.repeat(np.arange(g.n), np.diff(g.col_off).astype(np.int64))


@pytest.mark.parametrize("name,count", [("rmat12_wc", 300), ("rmat12_p10", 120),
                                        ("youtube_ic_s", 200)])
def test_ic_set_is_reverse_reachability(name, count):
    g = synth.make_graph(name)
    dst = _dst(g)
    src = g.row_src.astype(np.int64)
    sizes = []
    for s in range(count):
        live = oracle.ic_live(g, 42, s).astype(bool)
        # reverse edges dst -> src of the live in-edges
        a = sp.csr_matrix((np.ones(int(live.sum())), (dst[live], src[live])), shape=(g.n, g.n))
        root = oracle.root(42, s, g.n)
        reach = breadth_first_order(a, root, directed=True, return_predecessors=False)
        got = oracle.rrr_set(g, 42, s)
        assert got[0] == root
        assert len(set(got.tolist())) == got.size
        assert set(got.tolist()) == set(reach.tolist())
        sizes.append(got.size)
    assert max(sizes) > 1


@pytest.mark.parametrize("name", ["rmat12_lt", "cl_lt_xs"])
def test_lt_set_is_live_edge_chain(name):
    g = synth.make_graph(name)
    co = g.col_off.astype(np.int64)
    lens = []
    for s in range(400):
        cur = oracle.root(42, s, g.n)
        chain = [cur]
        seen = {cur}
        while True:
            b, e = co[cur], co[cur + 1]
            if b == e:
                break
            r = oracle.lt_draw(42, s, cur)
            j = int(np.searchsorted(g.weight[b:e], r, side="right"))  # first cum > r
            if j == e - b:
                break
            w = int(g.row_src[b + j])
            if w in seen:
                break
            chain.append(w)
            seen.add(w)
            cur = w
        got = oracle.rrr_set(g, 42, s)
        assert got.tolist() == chain
        lens.append(len(chain))
    assert max(lens) > 3


def test_zero_thresholds_give_roots_only():
    n = 50
    edges = [(u, v) for u in range(n) for v in range(n) if u != v and (u * v) % 7 == 1]
    g = synth.tiny_graph(n, edges, "ic", [0] * len(edges))
    so, sv = oracle.sample(g, 3, 0, 2000)
    assert np.all(np.diff(so) == 1)
    roots = np.array([oracle.root(3, s, n) for s in range(2000)])
    np.testing.assert_array_equal(sv, roots)
    np.testing.assert_array_equal(oracle.counts(n, so, sv), np.bincount(roots, minlength=n))


def test_certain_path_gives_whole_upstream():
    n = 40
    g = synth.tiny_graph(n, [(v, v + 1) for v in range(n - 1)], "ic", [T32 - 1] * (n - 1))
    for s in range(300):
        got = oracle.rrr_set(g, 8, s)
        root = oracle.root(8, s, n)
        assert sorted(got.tolist()) == list(range(root + 1))


def test_lt_single_in_edge_cycle():
    n = 30
    # v's only in-edge comes from v-1 with weight 1 (cum = 2^32 - 1)
    g = synth.tiny_graph(n, [((v - 1) % n, v) for v in range(n)], "lt", [T32 - 1] * n)
    for s in range(100):
        got = oracle.rrr_set(g, 1, s)
        root = oracle.root(1, s, n)
        assert got.tolist() == [(root - i) % n for i in range(n)]


def test_lt_no_in_edges_stops():
    g = synth.tiny_graph(4, [(0, 1), (1, 2)], "lt", [T32 - 1, T32 - 1])
    for s in range(50):
        got = oracle.rrr_set(g, 2, s).tolist()
        root = got[0]
        # 2 <- 1 <- 0 is a certain chain; 0 and 3 have no in-edges
        assert got == ([3] if root == 3 else list(range(root, -1, -1)))


# ---------------------------------------------------------------- brute force


def _tiny_ic():
    # 6 vertices, 10 edges, probabilities 1/4, 1/2, 3/4
    edges = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 5), (5, 3), (1, 4), (0, 5), (4, 1)]
    q = [1, 2, 3, 2, 1, 3, 2, 1, 3, 2]
    g = synth.tiny_graph(6, edges, "ic", [k << 30 for k in q])
    return g


def _ic_worlds(g):
    dst = _dst(g)
    p = [Fraction(int(t), T32) for t in g.weight]
    for bits in itertools.product((0, 1), repeat=g.m):
        pr = Fraction(1)
        for b, pe in zip(bits, p):
            pr *= pe if b else 1 - pe
        if pr:
            yield pr, [(int(g.row_src[e]), int(dst[e])) for e in range(g.m) if bits[e]]


def _reach(n, live_edges, starts):
    adj = {v: [] for v in range(n)}
    for u, v in live_edges:
        adj[u].append(v)
    seen = set(starts)
    todo = list(starts)
    while todo:
        u = todo.pop()
        for v in adj[u]:
            if v not in seen:
                seen.add(v)
                todo.append(v)
    return seen


def _rev_reach(n, live_edges, root):
    return _reach(n, [(v, u) for u, v in live_edges], [root])


def _check_distribution(exact, so, sv):
    N = so.size - 1
    counts = {}
    for j in range(N):
        t = frozenset(sv[so[j]:so[j + 1]].tolist())
        counts[t] = counts.get(t, 0) + 1
    assert set(counts) <= set(exact), set(counts) - set(exact)
    for t, pr in exact.items():
        p = float(pr)
        se = math.sqrt(N * p * (1 - p)) + 1e-12
        assert abs(counts.get(t, 0) - N * p) <= 5 * se + 2, (sorted(t), counts.get(t, 0), N * p)


def test_ic_rr_distribution_brute_force():
    g = _tiny_ic()
    exact = {}
    for pr, live in _ic_worlds(g):
        for r in range(g.n):
            t = frozenset(_rev_reach(g.n, live, r))
            exact[t] = exact.get(t, 0) + pr / g.n
    assert sum(exact.values()) == 1
    so, sv = oracle.sample(g, 77, 0, 200_000, threads=4)
    _check_distribution(exact, so, sv)


def test_ic_ris_identity_brute_force():
    g = _tiny_ic()
    worlds = list(_ic_worlds(g))
    so, sv = oracle.sample(g, 78, 0, 200_000, threads=4)
    N = so.size - 1
    for S in ([0], [3], [1, 4], [2, 5]):
        sigma = sum(pr * len(_reach(g.n, live, S)) for pr, live in worlds)  # forward IC
        hit = np.zeros(N, dtype=bool)
        for v in S:
            hit |= np.add.reduceat((sv == v).astype(np.int64), so[:-1].astype(np.int64)) > 0
        est = g.n * hit.mean()
        se = g.n * math.sqrt(hit.mean() * (1 - hit.mean()) / N)
        assert abs(est - float(sigma)) <= 5 * se + 1e-9, (S, est, float(sigma))


def _tiny_lt():
    # in-weights in sixteenths (one quantum less where a column would reach
    # 2^32); vertex 1 has no live in-edge with probability 1/16, vertex 5
    # with 3/16, vertex 0 has no in-edges
    edges = [(0, 1), (2, 1), (1, 2), (3, 2), (4, 2), (2, 3), (5, 4), (3, 4), (4, 5), (0, 5)]
    quanta = [6 << 28, 9 << 28, 4 << 28, 4 << 28, (8 << 28) - 1, (16 << 28) - 1, 9 << 28,
              (7 << 28) - 1, 5 << 28, 8 << 28]
    return synth.tiny_graph(6, edges, "lt", quanta)


def _lt_worlds(g):
    co = g.col_off.astype(np.int64)
    per_v = []
    for v in range(g.n):
        opts = []
        prev = 0
        for e in range(co[v], co[v + 1]):
            opts.append((Fraction(int(g.weight[e]) - prev, T32), int(g.row_src[e])))
            prev = int(g.weight[e])
        opts.append((Fraction(T32 - prev, T32), None))
        per_v.append(opts)
    for combo in itertools.product(*per_v):
        pr = Fraction(1)
        for p, _ in combo:
            pr *= p
        if pr:
            yield pr, [(u, v) for v, (_, u) in enumerate(combo) if u is not None]


def test_lt_rr_distribution_brute_force():
    g = _tiny_lt()
    exact = {}
    for pr, live in _lt_worlds(g):
        for r in range(g.n):
            t = frozenset(_rev_reach(g.n, live, r))
            exact[t] = exact.get(t, 0) + pr / g.n
    assert sum(exact.values()) == 1
    so, sv = oracle.sample(g, 91, 0, 200_000, threads=4)
    _check_distribution(exact, so, sv)


def test_lt_ris_identity_vs_forward_threshold_model():
    """Forward LT (random thresholds, activation when the active in-weight
    reaches the threshold) against the oracle's reverse live-edge sets."""
    g = _tiny_lt()
    co = g.col_off.astype(np.int64)
    W = np.zeros((g.n, g.n))
    for v in range(g.n):
        prev = 0
        for e in range(co[v], co[v + 1]):
            W[int(g.row_src[e]), v] = (int(g.weight[e]) - prev) / T32
            prev = int(g.weight[e])
    rng = np.random.default_rng(5)
    so, sv = oracle.sample(g, 92, 0, 200_000, threads=4)
    N = so.size - 1
    trials = 100_000
    for S in ([0], [2], [4, 5]):
        th = rng.random((trials, g.n))
        act = np.zeros((trials, g.n), dtype=bool)
        act[:, S] = True
        while True:
            new = act | ((act.astype(float) @ W) >= th)
            if np.array_equal(new, act):
                break
            act = new
        spread = act.sum(axis=1)
        fwd, fse = spread.mean(), spread.std() / math.sqrt(trials)
        hit = np.zeros(N, dtype=bool)
        for v in S:
            hit |= np.add.reduceat((sv == v).astype(np.int64), so[:-1].astype(np.int64)) > 0
        est = g.n * hit.mean()
        se = g.n * math.sqrt(hit.mean() * (1 - hit.mean()) / N)
        assert abs(est - fwd) <= 5 * math.hypot(se, fse), (S, est, fwd)


def test_thread_count_does_not_change_pool():
    g = synth.make_graph("rmat12_p10")
    a = oracle.sample(g, 5, 0, 1500, threads=1)
    b = oracle.sample(g, 5, 0, 1500, threads=7)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_counts_are_bincount():
    g = synth.make_graph("rmat12_wc")
    so, sv = oracle.sample(g, 42, 0, 3000)
    c = oracle.counts(g.n, so, sv)
    np.testing.assert_array_equal(c, np.bincount(sv, minlength=g.n))
    assert int(c.sum()) == int(so[-1])
