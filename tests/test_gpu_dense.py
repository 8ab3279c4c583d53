"""Adaptive set representation (dense IC sets kept as vertex bitmaps) against
the oracle, bit for bit, on the Youtube-shaped graph at one tenth of its size
with edge probabilities p ~ U[0,1) per edge: about a third of its sets hold
more than n/32 vertices. Whole IMM runs with and without the bitmap form
(IMM_LIST_SETS), with their pools; a sampling call's pool and fused counts;
the path that adds bitmap slots and redoes the sets that found none; the
fresh-final-pool schedule (which empties the pool between phases); and a
batch that mixes dense and list-only instances."""

import numpy as np
import pytest

import oracle as _orc_mod
import synth
from conftest import oracle_threads
from gpu_util import canonical, say

pytestmark = pytest.mark.gpu

NAME = "youtube_icu_s"


@pytest.fixture(scope="module")
def dense_graph(imm, stream):
    g = synth.make_graph(NAME)
    return g, imm.graph_from(g, stream=stream)


def _check_run(r, o, g):
    assert r.targets == o["targets"]
    assert r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered, r.lb) == (o["theta"], o["rounds"], o["covered"], o["lb"])
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])
    so, sv = r.pool()
    cso, csv = canonical(o["set_off"], o["set_vtx"], g.n)
    np.testing.assert_array_equal(so, cso)
    np.testing.assert_array_equal(sv, csv)


@pytest.fixture(scope="module")
def oracle_run(orc, dense_graph):
    g, _ = dense_graph
    sp = synth.WORKLOADS[NAME]
    say(f"oracle IMM on {NAME}")
    return orc.imm(g, sp["k"], sp["eps"], sp["ell"], sp["seed"], threads=oracle_threads(),
                   keep_pool=True)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("list_only", [False, True])
def test_dense_imm_run(imm, stream, dense_graph, oracle_run, list_only):
    g, dg = dense_graph
    sp = synth.WORKLOADS[NAME]
    fl = imm.IMM_KEEP_POOL | (imm.IMM_LIST_SETS if list_only else 0)
    say(f"IMM on {NAME}, list_only={list_only}")
    r = imm.imm_run(dg, sp["k"], sp["eps"], sp["ell"], sp["seed"], flags=fl, stream=stream)
    if list_only:
        assert r.stats["dense_sets"] == 0
    else:
        # about a third of the sets are at least n/32 large
        assert r.stats["dense_sets"] > r.theta // 5
    _check_run(r, oracle_run, g)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("scale", ["1", "0"])
def test_dense_sample_pool_and_counts(imm, orc, stream, dense_graph, monkeypatch, scale):
    """Sampling call: pool and fused counts; with IMM_DENSE_SCALE=0 the first
    bitmap reservation is minimal, so most dense sets find no slot and are
    redone after more slots are added."""
    monkeypatch.setenv("IMM_DENSE_SCALE", scale)
    g, dg = dense_graph
    count = 1 << 13
    say(f"sampling {count} ids on {NAME}, dense scale {scale}")
    pool = imm.imm_sample(dg, 7, 0, count, stream=stream)
    assert pool.stats["dense_sets"] > count // 5
    so, sv, cn = pool.export()
    pool.close()
    oso, osv = orc.sample(g, 7, 0, count, threads=oracle_threads())
    cso, csv = canonical(oso, osv, g.n)
    np.testing.assert_array_equal(so, cso)
    np.testing.assert_array_equal(sv, csv)
    np.testing.assert_array_equal(cn, orc.counts(g.n, oso, osv))


@pytest.mark.timeout(600)
def test_dense_fresh_schedule(imm, orc, stream, dense_graph):
    g, dg = dense_graph
    sp = synth.WORKLOADS[NAME]
    say(f"fresh-final-pool schedule on {NAME}")
    r = imm.imm_run(dg, sp["k"], sp["eps"], sp["ell"], sp["seed"],
                    flags=imm.IMM_FRESH_FINAL | imm.IMM_KEEP_POOL, stream=stream)
    o = orc.imm(g, sp["k"], sp["eps"], sp["ell"], sp["seed"], threads=oracle_threads(),
                keep_pool=True, schedule=_orc_mod.SCHED_FRESH)
    assert r.stats["dense_sets"] > 0
    _check_run(r, o, g)


@pytest.mark.timeout(600)
def test_dense_in_batch(imm, orc, stream, dense_graph):
    g, dg = dense_graph
    small = synth.make_graph("rmat12_p10")
    ds = imm.graph_from(small, stream=stream)
    qs = [(dg, g, dict(k=10, epsilon=0.5, seed=3)),
          (ds, small, dict(k=10, epsilon=0.5, seed=4)),
          (dg, g, dict(k=5, epsilon=0.6, seed=5, flags=imm.IMM_LIST_SETS))]
    say("batch mixing dense and list-only instances")
    res = imm.imm_run_batch([(d, q) for d, _, q in qs], stream=stream)
    for (_, hg, q), r in zip(qs, res):
        o = orc.imm(hg, q["k"], q["epsilon"], 1.0, q["seed"], threads=oracle_threads())
        assert (r.theta, r.rounds, r.covered, r.lb) == (o["theta"], o["rounds"], o["covered"],
                                                        o["lb"])
        np.testing.assert_array_equal(r.seeds, o["seeds"])
        np.testing.assert_array_equal(r.gains, o["gains"])
    assert res[0].stats["dense_sets"] > 0 and res[2].stats["dense_sets"] == 0
