"""Pins of the oracle's theta constants (Theta_Estimation / Set_Theta of
Algorithm 1, whose formulas the paper takes from Tang, Shi and Xiao 2015).

lambda' and lambda* are checked against the probability bounds they are
derived from, evaluated with exact binomial coefficients (math.comb), not by
re-evaluating the closed forms:
  * lambda' makes the Chernoff bound of the sampling phase (their Corollary 1
    with deviation eps' theta p, p = x/n) equal n^-l' / (C(n,k) log2 n);
  * lambda* = 2n ((1-1/e) alpha + beta)^2 / eps^2 is the threshold at which
    the two error budgets eps1 = alpha sqrt(2n/lambda*) and
    eps2 = beta sqrt(2n/lambda*) of their Theorem 1 add up to eps, with
    exp(-alpha^2) = n^-l'/2 and exp(-beta^2/(1-1/e)) = n^-l'/(2 C(n,k)),
where l' = l (1 + ln 2 / ln n)."""

import math

import numpy as np
import pytest

import oracle

CASES = [(4096, 10, 0.5, 1.0), (1134890, 50, 0.13, 1.0), (4800000, 50, 0.13, 1.0),
         (8, 2, 0.5, 1.0), (12, 2, 0.3, 1.0), (1000, 1, 0.1, 2.0), (3, 3, 0.9, 0.5)]


def _log_comb(n, k):
    return math.log(math.comb(n, k))


@pytest.mark.parametrize("n,k,eps,ell", CASES)
def test_lambda_prime_meets_sampling_bound(n, k, eps, ell):
    lp, _, _ = oracle.theta_plan(n, k, eps, ell)
    ellp = ell * (1 + math.log(2) / math.log(n))
    epsp = math.sqrt(2) * eps
    # exponent of exp(-d^2 / (2 theta p + 2/3 d)) with d = eps' theta p,
    # theta p = lambda' / n
    tp = lp / n
    expo = (epsp * tp) ** 2 / (2 * tp + 2.0 / 3.0 * epsp * tp)
    target = _log_comb(n, k) + ellp * math.log(n) + math.log(math.log2(n))
    assert expo == pytest.approx(target, rel=1e-9)


@pytest.mark.parametrize("n,k,eps,ell", CASES)
def test_lambda_star_splits_eps(n, k, eps, ell):
    _, ls, _ = oracle.theta_plan(n, k, eps, ell)
    ellp = ell * (1 + math.log(2) / math.log(n))
    one_m = 1 - 1 / math.e
    alpha2 = math.log(2) + ellp * math.log(n)                       # exp(-a^2) = n^-l'/2
    beta2 = one_m * (math.log(2) + _log_comb(n, k) + ellp * math.log(n))
    eps1 = math.sqrt(alpha2 * 2 * n / ls)
    eps2 = math.sqrt(beta2 * 2 * n / ls)
    assert one_m * eps1 + eps2 == pytest.approx(eps, rel=1e-9)
    # and both error budgets are positive and meet the stated failure bounds
    assert math.exp(-alpha2) == pytest.approx(n ** -ellp / 2, rel=1e-9)
    assert math.exp(-beta2 / one_m) * math.comb(n, k) == pytest.approx(n ** -ellp / 2,
                                                                        rel=1e-6)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7, 8, 9, 1023, 1024, 1025, 4096, 1134890, 2**31])
def test_round_count(n):
    """Sampling rounds run i = 1 .. ceil(log2 n) - 1 (x = n / 2^i stays >= 1)."""
    _, _, im = oracle.theta_plan(n, 1, 0.5, 1.0)
    assert im == math.ceil(math.log2(n)) - 1
    assert 2 ** im < n <= 2 ** (im + 1)


@pytest.mark.parametrize("n,k,eps,ell", [(8, 2, 0.5, 1.0), (4096, 10, 0.5, 1.0)])
def test_imm_targets_follow_schedule(n, k, eps, ell):
    """On a graph whose sets never reach the LB threshold early, every
    sampling round's target is ceil(lambda' 2^i / n)."""
    import synth
    # all thresholds zero: every set is just its root, coverage stays tiny
    g = synth.tiny_graph(n, [(u, (u + 1) % n) for u in range(n)], "ic", [0] * n)
    r = oracle.imm(g, k, eps, ell, 1)
    lp, ls, im = oracle.theta_plan(n, k, eps, ell)
    for i, t in enumerate(r["targets"][:-1], start=1):
        assert t == math.ceil(lp / (n / 2 ** i))
    assert r["targets"][-1] == math.ceil(ls / r["lb"])
    assert r["theta"] == max(r["targets"])


def test_invalid_arguments():
    for args in [(1, 1, 0.5, 1.0), (10, 0, 0.5, 1.0), (10, 11, 0.5, 1.0), (10, 2, 0.0, 1.0),
                 (10, 2, 0.5, 0.0), (10, 2, -1.0, 1.0)]:
        with pytest.raises(RuntimeError, match="EINVAL"):
            oracle.theta_plan(*args)
