"""Speculative rounds (LT): when a round's launch draws the next round's ids
ahead, that next round's compaction, index segment and selection run on a
second stream beside the round's own selection, and are kept only if the
round fails its test. Every run must equal the oracle's, whether the
speculation is kept (runs of several rounds), dropped (runs whose first round
passes), turned off (IMM_SPEC=0), or halts inside its candidate steps."""

import numpy as np
import pytest

import synth
from conftest import oracle_threads
from gpu_util import canonical, say

pytestmark = pytest.mark.gpu


def _check(r, o, g):
    assert r.targets == o["targets"]
    assert r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered, r.lb) == (o["theta"], o["rounds"], o["covered"], o["lb"])
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])
    so, sv = r.pool()
    cso, csv = canonical(o["set_off"], o["set_vtx"], g.n)
    np.testing.assert_array_equal(so, cso)
    np.testing.assert_array_equal(sv, csv)


# (graph, k, eps): several rounds (speculation kept), or a first round that
# passes its test (speculation dropped)
CASES = [("lj_lt_s", 10, 0.5), ("rmat12_lt", 10, 0.5), ("cl_lt_xs", 2, 0.3),
         ("rmat12_lt", 2, 0.3), ("lj_lt_s", 50, 0.13), ("cl_lt_xs", 50, 0.13)]


@pytest.mark.parametrize("name,k,eps", CASES)
def test_spec_rounds_match_oracle(imm, orc, stream, monkeypatch, name, k, eps):
    g = synth.make_graph(name)
    dg = imm.graph_from(g, stream=stream)
    o = orc.imm(g, k, eps, 1.0, 42, threads=oracle_threads(), keep_pool=True)
    say(f"speculative rounds {name} k={k} eps={eps}: oracle rounds {o['rounds']}, "
        f"theta {o['theta']}")
    monkeypatch.delenv("IMM_SPEC", raising=False)
    r = imm.imm_run(dg, k, eps, 1.0, 42, flags=imm.IMM_KEEP_POOL, stream=stream)
    _check(r, o, g)
    monkeypatch.setenv("IMM_SPEC", "0")
    r0 = imm.imm_run(dg, k, eps, 1.0, 42, flags=imm.IMM_KEEP_POOL, stream=stream)
    _check(r0, o, g)
    say(f"  speculative rounds kept: {r.stats['spec_rounds']} (off: {r0.stats['spec_rounds']})")
    assert r0.stats["spec_rounds"] == 0
    if o["rounds"] >= 2:
        assert r.stats["spec_rounds"] >= 1
    else:
        assert r.stats["spec_rounds"] == 0
    dg.close()


@pytest.mark.parametrize("cand_max", ["1", "3"])
def test_spec_round_with_halting_selection(imm, orc, stream, monkeypatch, cand_max):
    """Candidate lists of one or three vertices: the kept speculative round's
    selection halts and is finished in full by the host, as the round's own."""
    monkeypatch.delenv("IMM_SPEC", raising=False)
    monkeypatch.setenv("IMM_CAND_MAX", cand_max)
    name, k, eps = "lj_lt_s", 10, 0.5
    g = synth.make_graph(name)
    dg = imm.graph_from(g, stream=stream)
    say(f"speculative round with halting selections, list bound {cand_max}")
    r = imm.imm_run(dg, k, eps, 1.0, 42, flags=imm.IMM_KEEP_POOL, stream=stream)
    o = orc.imm(g, k, eps, 1.0, 42, threads=oracle_threads(), keep_pool=True)
    _check(r, o, g)
    assert r.stats["spec_rounds"] >= 1
    assert r.stats["cand_halts"] >= 1
    dg.close()


def test_spec_repeated_runs_reuse_workspace(imm, orc, stream, monkeypatch):
    """Runs of several rounds and runs whose first round passes, alternating
    on one graph (its cached workspace and both selection buffer sets
    reused): each equals the oracle."""
    monkeypatch.delenv("IMM_SPEC", raising=False)
    g = synth.make_graph("cl_lt_xs")
    dg = imm.graph_from(g, stream=stream)
    for k, eps in ((2, 0.3), (50, 0.13), (10, 0.5), (2, 0.3)):
        say(f"  cl_lt_xs k={k} eps={eps}")
        r = imm.imm_run(dg, k, eps, 1.0, 42, flags=imm.IMM_KEEP_POOL, stream=stream)
        o = orc.imm(g, k, eps, 1.0, 42, threads=oracle_threads(), keep_pool=True)
        _check(r, o, g)
    dg.close()
