"""End-to-end pins of the oracle's IMM driver (Algorithm 1).

On graphs of at most 12 edges the expected spread sigma(S) of any seed set is
computed exactly from the forward diffusion models by enumerating every
live-edge world; the seeds IMM returns must reach (1 - 1/e - eps) of the best
k-set's spread (IMM's guarantee, which holds with probability >= 1 - n^-l;
the fixed seeds below make the check deterministic)."""

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

T32 = 1 << 32


def _ic_sigma_table(g):
    dst = np.repeat(np.arange(g.n), np.diff(g.col_off).astype(np.int64))
    probs = [Fraction(int(t), T32) for t in g.weight]
    worlds = []
    for bits in itertools.product((0, 1), repeat=g.m):
        pr = Fraction(1)
        for b, p in zip(bits, probs):
            pr *= p if b else 1 - p
        if pr:
            adj = {v: [] for v in range(g.n)}
            for e in range(g.m):
                if bits[e]:
                    adj[int(g.row_src[e])].append(int(dst[e]))
            worlds.append((pr, adj))

    def sigma(S):
        tot = Fraction(0)
        for pr, adj in worlds:
            seen = set(S)
            todo = list(S)
            while todo:
                u = todo.pop()
                for v in adj[u]:
                    if v not in seen:
                        seen.add(v)
                        todo.append(v)
            tot += pr * len(seen)
        return tot

    return sigma


def _random_tiny_ic(rng, n, m):
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    idx = rng.choice(len(pairs), size=m, replace=False)
    edges = [pairs[i] for i in idx]
    thr = [int(rng.integers(1, 4)) << 30 for _ in edges]
    return synth.tiny_graph(n, edges, "ic", thr)


@pytest.mark.parametrize("case", range(8))
def test_imm_spread_guarantee_ic(case):
    rng = np.random.default_rng(700 + case)
    n = int(rng.integers(5, 9))
    g = _random_tiny_ic(rng, n, int(rng.integers(6, 13)))
    sigma = _ic_sigma_table(g)
    for k, eps in ((1, 0.3), (2, 0.5)):
        r = oracle.imm(g, k, eps, 1.0, 1000 + case)
        got = sigma(r["seeds"].tolist())
        opt = max(sigma(list(c)) for c in itertools.combinations(range(n), k))
        assert float(got) >= (1 - 1 / math.e - eps) * float(opt)
        assert len(set(r["seeds"].tolist())) == k


def test_threads_do_not_change_run():
    g = synth.make_graph("rmat12_wc")
    a = oracle.imm(g, 10, 0.5, 1.0, 42, threads=1, keep_pool=True)
    b = oracle.imm(g, 10, 0.5, 1.0, 42, threads=6, keep_pool=True)
    for key in ("theta", "rounds", "lb", "covered", "targets", "round_cov"):
        assert a[key] == b[key]
    np.testing.assert_array_equal(a["seeds"], b["seeds"])
    np.testing.assert_array_equal(a["set_vtx"], b["set_vtx"])


def test_run_is_consistent_with_its_pool():
    """theta = |R|; the final seeds are the greedy over the returned pool; the
    LB test passed in the last sampling round or LB = 1."""
    g = synth.make_graph("rmat12_wc")
    r = oracle.imm(g, 10, 0.5, 1.0, 42, keep_pool=True)
    assert r["theta"] == r["set_off"].size - 1 == max(r["targets"])
    s, ga, cov = oracle.greedy(g.n, r["set_off"], r["set_vtx"], 10)
    np.testing.assert_array_equal(s, r["seeds"])
    assert cov == r["covered"]
    lp, ls, _ = oracle.theta_plan(g.n, 10, 0.5, 1.0)
    epsp = math.sqrt(2) * 0.5
    i = r["rounds"]
    x = g.n / 2 ** i
    T = r["targets"][i - 1]
    frac = r["round_cov"][-1] / T
    if g.n * frac >= (1 + epsp) * x:
        assert r["lb"] == g.n * frac / (1 + epsp)
    else:
        assert r["lb"] == 1.0
    assert r["targets"][-1] == math.ceil(ls / r["lb"])


def test_errors():
    g = synth.make_graph("rmat12_wc")
    with pytest.raises(RuntimeError, match="EINVAL"):
        oracle.imm(g, 0, 0.5, 1.0, 1)
    with pytest.raises(RuntimeError, match="EINVAL"):
        oracle.imm(g, 10, -0.5, 1.0, 1)
    # LB = 1 on a 4096-vertex graph at tiny eps needs more than 2^32 sets
    with pytest.raises(RuntimeError, match="EOVERFLOW"):
        oracle.imm(g, 10, 1e-4, 1.0, 1)
