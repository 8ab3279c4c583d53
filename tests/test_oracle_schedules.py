"""Pins of the oracle's two variant sampling schedules.

* Fresh final pool (IMM with the correction of Chen, 2018): the rounds are
  IMM's own; the final selection runs over theta sets drawn afresh, sample
  ids right after the rounds' ids. Pinned by the IMM run it shares its rounds
  with, by the sets recomputed one at a time at those ids, by the greedy over
  them, and by the spread guarantee on graphs small enough for exact spread.
* Early stopping in the manner of OPIM: two independent pools, the greedy
  seeds of the first, a lower bound on their spread from the second and an
  upper bound on OPT from the first. Pinned by the Chernoff conditions each
  bound is the root of (solved numerically here, not by re-evaluating the
  closed forms), by the relation of its theta_0 to IMM's lambda* (Tang et
  al. 2015, Eq. 6) at the failure probability it uses, by the pools' sets
  recomputed one by one, by the validity of both bounds against exact spread
  on tiny graphs, and by the spread guarantee.
"""

import itertools
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
import synth
from test_oracle_imm import _ic_sigma_table, _random_tiny_ic

TWO32 = 1 << 32


def test_coverage_is_sets_hit():
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = int(rng.integers(2, 40))
        sizes = rng.integers(0, 6, size=int(rng.integers(1, 60)))
        sets = [rng.choice(n, size=min(int(s), n), replace=False) for s in sizes]
        so = np.concatenate([[0], np.cumsum([len(x) for x in sets])]).astype(np.uint64)
        sv = (np.concatenate(sets) if so[-1] else np.zeros(0)).astype(np.uint32)
        seeds = rng.choice(n, size=int(rng.integers(1, n + 1)), replace=False)
        want = sum(1 for x in sets if set(x.tolist()) & set(seeds.tolist()))
        assert oracle.coverage(n, so, sv, seeds) == want
    # the greedy's seeds cover exactly the sum of their gains
    g = synth.make_graph("rmat12_p10")
    so, sv = oracle.sample(g, 42, 0, 3000, threads=4)
    s, gains, cov = oracle.greedy(g.n, so, sv, 10)
    assert oracle.coverage(g.n, so, sv, s) == cov == int(gains.sum())


@pytest.mark.parametrize("name", ["rmat12_wc", "rmat12_lt", "rmat12_p10"])
def test_fresh_final_pool(name):
    g = synth.make_graph(name)
    sp = synth.WORKLOADS[name]
    base = oracle.imm(g, sp["k"], sp["eps"], sp["ell"], sp["seed"], threads=4)
    r = oracle.imm(g, sp["k"], sp["eps"], sp["ell"], sp["seed"], threads=4, keep_pool=True,
                   schedule=oracle.SCHED_FRESH)
    # the same rounds, LB and theta as IMM's
    for key in ("rounds", "lb", "targets", "round_cov"):
        assert r[key] == base[key]
    theta = r["targets"][-1]
    assert r["theta"] == theta == r["set_off"].size - 1
    # the final pool: sample ids after the rounds' ids, set by set
    first = r["targets"][r["rounds"] - 1]
    so, sv = oracle.sample(g, sp["seed"], first, theta)
    np.testing.assert_array_equal(r["set_off"], so)
    np.testing.assert_array_equal(r["set_vtx"], sv)
    s, gains, cov = oracle.greedy(g.n, so, sv, sp["k"])
    np.testing.assert_array_equal(r["seeds"], s)
    np.testing.assert_array_equal(r["gains"], gains)
    assert r["covered"] == cov


@pytest.mark.parametrize("case", range(6))
@pytest.mark.parametrize("schedule", [oracle.SCHED_FRESH, oracle.SCHED_EARLY])
def test_spread_guarantee(case, schedule):
    rng = np.random.default_rng(900 + case)
    n = int(rng.integers(5, 9))
    g = _random_tiny_ic(rng, n, int(rng.integers(6, 12)))
    sigma = _ic_sigma_table(g)
    for k, eps in ((1, 0.3), (2, 0.5)):
        r = oracle.imm(g, k, eps, 1.0, 3000 + case, schedule=schedule)
        got = sigma(r["seeds"].tolist())
        opt = max(sigma(list(c)) for c in itertools.combinations(range(n), k))
        assert float(got) >= (1 - 1 / math.e - eps) * float(opt)
        assert len(set(r["seeds"].tolist())) == k


@pytest.mark.parametrize("n,k,eps,ell", [(4096, 10, 0.5, 1.0), (1134890, 50, 0.13, 1.0),
                                         (8, 2, 0.5, 1.0), (1000, 1, 0.1, 2.0)])
def test_early_plan_constants(n, k, eps, ell):
    """theta_max = theta_0 n / (eps^2 k) is IMM's lambda* / k at the failure
    probability delta / 3, delta = n^-ell: Tang et al.'s lambda* with l' ln n
    + ln 2 = ln 6 + ell ln n, obtained here from the oracle's own IMM theta
    plan with the ell that gives that l'."""
    t0, i_max, a = oracle.early_plan(n, k, eps, ell)
    ln_n = math.log(n)
    ell2 = (math.log(3) + ell * ln_n) / (ln_n + math.log(2))
    _, ls, _ = oracle.theta_plan(n, k, eps, ell2)
    assert t0 * n / (eps * eps * k) == pytest.approx(ls / k, rel=1e-12)
    assert 2 ** (i_max - 1) < max(2, n / (eps * eps * k)) <= 2 ** i_max
    assert math.exp(-a) == pytest.approx(n ** -ell / (3 * i_max), rel=1e-12)


def _chernoff_roots(cov1, cov2, theta, a, k, n):
    """The upper bound on OPT and the lower bound on the seeds' spread as the
    roots of the Chernoff conditions they come from (per-sample means mu):
      lower tail: (mu - c)^2 / (2 mu) = a at mu >= c, with c = cov1 / g_k,
      upper tail: (c - mu)^2 / (2 mu + 2 (c - mu) / 3) = a at mu <= c, c = cov2."""
    gk = 1 - (1 - 1 / k) ** k
    c1 = cov1 / gk
    up = brentq(lambda mu: (mu - c1) ** 2 / (2 * mu) - a, c1, c1 + 10 * a + 10 * math.sqrt(a * c1) + 1,
                xtol=1e-13, rtol=1e-14)
    # 3 (c - mu)^2 / (4 mu + 2 c) falls from 1.5 c at mu = 0 to 0 at mu = c
    f = lambda mu: 3 * (cov2 - mu) ** 2 / (4 * mu + 2 * cov2) - a  # noqa: E731
    lo = brentq(f, 0.0, cov2, xtol=1e-13, rtol=1e-14) if cov2 > 0 and f(0.0) > 0 else 0.0
    return up * n / theta, lo * n / theta


@pytest.mark.parametrize("name", ["rmat12_wc", "rmat12_lt", "rmat12_p10", "cl_lt_xs"])
def test_early_stop_bounds(name):
    g = synth.make_graph(name)
    sp = synth.WORKLOADS[name]
    r = oracle.imm(g, sp["k"], sp["eps"], sp["ell"], sp["seed"], threads=4, keep_pool=True,
                   schedule=oracle.SCHED_EARLY)
    t0, i_max, a = oracle.early_plan(g.n, sp["k"], sp["eps"], sp["ell"])
    i = r["rounds"]
    assert r["targets"] == [math.ceil(math.ldexp(t0, j)) for j in range(i)]
    theta = r["targets"][-1]
    assert r["theta"] == theta == r["set_off"].size - 1
    # pool 1 is sample ids [0, theta), pool 2 ids 2^32 + [0, theta)
    so1, sv1 = oracle.sample(g, sp["seed"], 0, theta, threads=4)
    np.testing.assert_array_equal(r["set_off"], so1)
    np.testing.assert_array_equal(r["set_vtx"], sv1)
    s, gains, cov1 = oracle.greedy(g.n, so1, sv1, sp["k"])
    np.testing.assert_array_equal(r["seeds"], s)
    assert r["round_cov"][-1] == cov1 == r["covered"]
    so2, sv2 = oracle.sample(g, sp["seed"], TWO32, theta)
    cov2 = sum(1 for j in range(theta)
               if set(sv2[so2[j]:so2[j + 1]].tolist()) & set(s.tolist()))
    assert r["round_cov2"][-1] == cov2
    up, lo = _chernoff_roots(cov1, cov2, theta, a, sp["k"], g.n)
    assert r["sigma_up"] == pytest.approx(up, rel=1e-9)
    assert r["lb"] == pytest.approx(lo, rel=1e-9, abs=1e-9)
    assert r["alpha"] == pytest.approx(r["lb"] / r["sigma_up"], rel=1e-12)
    # stopped as soon as the ratio allowed it, or at the last iteration
    assert r["alpha"] >= 1 - 1 / math.e - sp["eps"] or i == i_max


@pytest.mark.parametrize("case", range(8))
def test_early_stop_bounds_hold(case):
    """On tiny graphs with exact spread: the upper bound is above OPT and the
    lower bound below the spread of the returned seeds (each may fail with
    probability at most n^-ell / (3 i_max); ell = 3 here, so never in these
    fixed cases)."""
    rng = np.random.default_rng(1200 + case)
    n = int(rng.integers(5, 9))
    g = _random_tiny_ic(rng, n, int(rng.integers(6, 12)))
    sigma = _ic_sigma_table(g)
    for k, eps in ((1, 0.2), (2, 0.4)):
        r = oracle.imm(g, k, eps, 3.0, 5000 + case, schedule=oracle.SCHED_EARLY)
        opt = max(sigma(list(c)) for c in itertools.combinations(range(n), k))
        assert r["sigma_up"] >= float(opt)
        assert r["lb"] <= float(sigma(r["seeds"].tolist()))
        assert r["lb"] > 0.0
