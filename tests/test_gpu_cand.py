"""Candidate steps of the greedy (the argmax over a short list of the vertices
whose count reaches tau at the start of a selection, with decrements only for
them; a step whose best listed count falls below tau halts the selection and
the host finishes it in full). Every result must equal the oracle's, whether
the steps use the list, halt early (a list bound of a few vertices, set with
IMM_CAND_MAX), or are turned off."""

import numpy as np
import pytest

import synth
from conftest import oracle_threads
from gpu_util import say

pytestmark = pytest.mark.gpu


def _check(r, o):
    assert r.targets == o["targets"]
    assert r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered, r.lb) == (o["theta"], o["rounds"], o["covered"], o["lb"])
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])


@pytest.mark.parametrize("cand_max", [None, "0", "1", "3", "64"])
@pytest.mark.parametrize("name", ["rmat12_wc", "rmat12_lt", "cl_lt_xs", "lj_lt_s", "youtube_ic_s"])
def test_cand_steps_match_oracle(imm, orc, stream, monkeypatch, name, cand_max):
    if cand_max is None:
        monkeypatch.delenv("IMM_CAND_MAX", raising=False)
    else:
        monkeypatch.setenv("IMM_CAND_MAX", cand_max)
    sp = synth.WORKLOADS[name]
    g = synth.make_graph(name)
    dg = imm.graph_from(g, stream=stream)
    say(f"candidate steps {name} list bound {cand_max or 'default'}")
    r = imm.imm_run(dg, sp["k"], sp["eps"], sp["ell"], sp["seed"], stream=stream)
    o = orc.imm(g, sp["k"], sp["eps"], sp["ell"], sp["seed"], threads=oracle_threads())
    say(f"  candidate steps {r.stats['cand_steps']}, halts {r.stats['cand_halts']}")
    _check(r, o)
    if cand_max == "0":
        assert r.stats["cand_steps"] == 0 and r.stats["cand_halts"] == 0
    if cand_max == "1":
        # one listed vertex: step 1 finds it selected (or below tau) and halts
        assert r.stats["cand_steps"] == 0
    if name == "lj_lt_s" and cand_max is None:
        # the LiveJournal-shaped run's selections keep to the list
        assert r.stats["cand_halts"] == 0
        assert r.stats["cand_steps"] >= sp["k"] - 1
    dg.close()


def test_cand_halts_in_batch_and_server(imm, orc, stream, monkeypatch):
    """A list bound of two vertices makes most selections halt after a step
    or two: batched and served queries (each halted query finished on its
    own) still equal the oracle, and the run alone."""
    monkeypatch.setenv("IMM_CAND_MAX", "2")
    names = ["rmat12_wc", "rmat12_lt", "cl_lt_xs"]
    graphs = {nm: synth.make_graph(nm) for nm in names}
    dev = {nm: imm.graph_from(g, stream=stream) for nm, g in graphs.items()}
    qs = []
    for nm in names:
        sp = synth.WORKLOADS[nm]
        qs.append((nm, dict(k=sp["k"], epsilon=sp["eps"], ell=sp["ell"], seed=sp["seed"])))
    qs.append(("rmat12_wc", dict(k=25, epsilon=0.3, ell=1.0, seed=7)))
    say("halting selections in a batch")
    res = imm.imm_run_batch([(dev[nm], q) for nm, q in qs], stream=stream)
    halts = 0
    for (nm, q), r in zip(qs, res):
        o = orc.imm(graphs[nm], q["k"], q["epsilon"], q["ell"], q["seed"],
                    threads=oracle_threads())
        _check(r, o)
        halts += r.stats["cand_halts"]
    assert halts > 0
    say("halting selections through the server")
    srv = imm.Server(budget_bytes=64 << 30, max_slots=4)
    tickets = [srv.submit(dev[nm], **q) for nm, q in qs]
    sres = [srv.poll(t) for t in tickets]
    srv.close()
    for a, b in zip(res, sres):
        assert a.theta == b.theta and a.covered == b.covered
        np.testing.assert_array_equal(a.seeds, b.seeds)
        np.testing.assert_array_equal(a.gains, b.gains)


def test_cand_greedy_on_oracle_pool(imm, orc, stream, monkeypatch):
    """imm_greedy over a pool the oracle drew (LiveJournal-shaped, one tenth
    size), with the default list, a list of three and none: the oracle's
    seeds and gains each time."""
    name = "lj_lt_s"
    sp = synth.WORKLOADS[name]
    g = synth.make_graph(name)
    so, sv = orc.sample(g, sp["seed"], 0, 1 << 15, threads=oracle_threads())
    seeds_o, gains_o, cov_o = orc.greedy(g.n, so, sv, sp["k"])
    for cm in (None, "3", "0"):
        if cm is None:
            monkeypatch.delenv("IMM_CAND_MAX", raising=False)
        else:
            monkeypatch.setenv("IMM_CAND_MAX", cm)
        say(f"greedy on the oracle pool, list bound {cm or 'default'}")
        seeds, gains, cov = imm.imm_greedy(g.n, so, sv, sp["k"], stream=stream)
        assert cov == cov_o
        np.testing.assert_array_equal(seeds, seeds_o)
        np.testing.assert_array_equal(np.asarray(gains, dtype=np.uint64),
                                      np.asarray(gains_o, dtype=np.uint64))


def test_cand_list_longer_than_the_argmax_grid(imm, orc, stream, monkeypatch):
    """Every vertex of a zero-threshold R-MAT-12 graph (all sets single roots)
    with a count of one or more is listed: thousands of listed vertices,
    against an argmax launch of one workgroup on this graph."""
    monkeypatch.delenv("IMM_CAND_MAX", raising=False)
    base = synth.make_graph("rmat12_wc")
    g = synth.Graph("rmat12_zero", base.n, base.m, base.col_off, base.row_src,
                    np.zeros(base.m, np.uint32), "ic")
    dg = imm.graph_from(g, stream=stream)
    say("zero thresholds: long candidate list")
    r = imm.imm_run(dg, 10, 0.5, 1.0, 42, stream=stream)
    o = orc.imm(g, 10, 0.5, 1.0, 42, threads=oracle_threads())
    say(f"  candidate steps {r.stats['cand_steps']}, halts {r.stats['cand_halts']}")
    _check(r, o)
    assert r.stats["cand_steps"] > 0
    dg.close()
