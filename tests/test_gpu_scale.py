"""GPU vs oracle at the workload sizes the benchmark uses.

* LiveJournal-shaped LT (n = 4.8M, m = 69M, k = 50, eps = 0.13): the whole
  IMM run, bit-exact (theta trajectory, LB, seeds, gains, canonical pool).
* Youtube-shaped IC (n = 1,134,890, m = 2,987,624, p = 0.01, k = 50,
  eps = 0.13): the whole 21.6 M-set run, bit-exact, and the fused counts of
  a sampling call over the same ids.
* One-tenth-size versions of both, bit-exact on the whole run.
* The LiveJournal-shaped steady-state sampling call (2^22 ids) in the
  benchmark's launch configuration: sampled sets one by one, and the fused
  counts against the whole returned pool.
"""

import numpy as np
import pytest

import synth
from conftest import oracle_threads
from gpu_util import canonical, say

pytestmark = pytest.mark.gpu


def _run(imm, name, stream, flags=0):
    spec = synth.WORKLOADS[name]
    g = synth.make_graph(name)
    dg = imm.graph_from(g, stream=stream)
    r = imm.imm_run(dg, spec["k"], spec["eps"], spec["ell"], spec["seed"], flags=flags,
                    stream=stream)
    return g, spec, r


def _full_parity(imm, orc, name, stream, pool):
    say(f"full-run parity {name}")
    g, spec, r = _run(imm, name, stream, imm.IMM_KEEP_POOL if pool else 0)
    o = orc.imm(g, spec["k"], spec["eps"], spec["ell"], spec["seed"],
                threads=oracle_threads(), keep_pool=pool)
    assert r.targets == o["targets"]
    assert r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered, r.lb) == (o["theta"], o["rounds"], o["covered"], o["lb"])
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])
    if pool:
        so, sv = r.pool()
        cso, csv = canonical(o["set_off"], o["set_vtx"], g.n)
        np.testing.assert_array_equal(so, cso)
        np.testing.assert_array_equal(sv, csv)


@pytest.mark.timeout(300)
def test_lj_lt_full_size_bit_exact(imm, orc, stream):
    _full_parity(imm, orc, "lj_lt", stream, pool=True)


def test_lj_lt_small_bit_exact(imm, orc, stream):
    _full_parity(imm, orc, "lj_lt_s", stream, pool=True)


@pytest.mark.timeout(300)
def test_youtube_small_bit_exact(imm, orc, stream):
    _full_parity(imm, orc, "youtube_ic_s", stream, pool=False)


@pytest.mark.timeout(900)
def test_youtube_full_size_bit_exact(imm, orc, stream):
    """The benchmark's Youtube-shaped IC configuration at full size (theta
    about 21.6 M sets, 9 rounds): the whole run against the oracle's, bit for
    bit (targets, per-round coverage, LB, theta, seeds, gains, the canonical
    pool), and the fused counts of a sampling call over the same theta ids
    against the occurrences in the oracle's pool."""
    name = "youtube_ic"
    spec = synth.WORKLOADS[name]
    g = synth.make_graph(name)
    say("full-size Youtube-shaped IC run (benchmark configuration)")
    dg = imm.graph_from(g, stream=stream)
    r = imm.imm_run(dg, spec["k"], spec["eps"], spec["ell"], spec["seed"],
                    flags=imm.IMM_KEEP_POOL, stream=stream)
    say(f"oracle IMM run, {oracle_threads()} threads")
    o = orc.imm(g, spec["k"], spec["eps"], spec["ell"], spec["seed"],
                threads=oracle_threads(), keep_pool=True)
    lp, ls, im = orc.theta_plan(g.n, spec["k"], spec["eps"], spec["ell"])
    assert (o["lambda_prime"], o["lambda_star"], o["i_max"]) == (lp, ls, im)
    assert r.targets == o["targets"]
    assert r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered, r.lb) == (o["theta"], o["rounds"], o["covered"], o["lb"])
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])
    say(f"canonical pools, {o['set_vtx'].size} entries")
    so, sv = r.pool()
    r.close()
    cso, csv = canonical(o["set_off"], o["set_vtx"], g.n)
    np.testing.assert_array_equal(so, cso)
    np.testing.assert_array_equal(sv, csv)
    del so, sv, cso, csv
    say(f"fused counts of imm_sample over ids [0, {o['theta']})")
    pool = imm.imm_sample(dg, spec["seed"], 0, o["theta"], stream=stream)
    _, _, cn = pool.export()
    pool.close()
    np.testing.assert_array_equal(cn, orc.counts(g.n, o["set_off"], o["set_vtx"]))


@pytest.mark.timeout(300)
def test_lj_lt_steady_state_sampled(imm, orc, stream):
    """The steady-state sampling call the benchmark times on the
    LiveJournal-shaped graph (2^22 ids, seed 42, the autotuned walk shape):
    sampled sets recomputed one by one by the oracle, and the fused counts
    equal to the occurrences in the whole returned pool."""
    spec = synth.WORKLOADS["lj_lt"]
    g = synth.make_graph("lj_lt")
    dg = imm.graph_from(g, stream=stream)
    count = 1 << 22
    say(f"steady-state LT sampling, {count} ids")
    pool = imm.imm_sample(dg, spec["seed"], 0, count, stream=stream)
    assert pool.stats["walk_lanes"] in (2, 4)
    so, sv, cn = pool.export()
    pool.close()
    assert so.size - 1 == count
    rng = np.random.default_rng(2025)
    ids = np.concatenate([[0, 1, count - 1], rng.integers(0, count, 2000)])
    for s in ids:
        want = np.sort(orc.rrr_set(g, spec["seed"], int(s)))
        np.testing.assert_array_equal(sv[so[s]:so[s + 1]], want, err_msg=f"set {s}")
    np.testing.assert_array_equal(cn, np.bincount(sv, minlength=g.n).astype(cn.dtype))
