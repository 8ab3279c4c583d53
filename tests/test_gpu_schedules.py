"""The two variant sampling schedules on the GPU against the oracle, bit for
bit: IMM with a fresh final pool (IMM_FRESH_FINAL) and early stopping with
two pools (IMM_EARLY_STOP), alone, in a batch with plain IMM queries, and
through the query server."""

import numpy as np
import pytest

import oracle as _orc_mod
import synth
from conftest import oracle_threads
from gpu_util import canonical, say

pytestmark = pytest.mark.gpu

SCHED = {"fresh": _orc_mod.SCHED_FRESH, "early": _orc_mod.SCHED_EARLY}


def _flag(imm, name):
    return {"fresh": imm.IMM_FRESH_FINAL, "early": imm.IMM_EARLY_STOP}[name]


def _check(r, o, sched, g=None):
    assert r.targets == o["targets"]
    assert r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered, r.lb) == (o["theta"], o["rounds"], o["covered"], o["lb"])
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])
    if sched == "early":
        assert (r.sigma_up, r.alpha) == (o["sigma_up"], o["alpha"])
        assert r.round_cov2 == o["round_cov2"]
    if g is not None:
        so, sv = r.pool()
        cso, csv = canonical(o["set_off"], o["set_vtx"], g.n)
        np.testing.assert_array_equal(so, cso)
        np.testing.assert_array_equal(sv, csv)


@pytest.mark.parametrize("sched", ["fresh", "early"])
@pytest.mark.parametrize("name", ["rmat12_wc", "rmat12_lt", "rmat12_p10", "cl_lt_xs",
                                  "youtube_ic_s", "lj_lt_s"])
def test_schedule_matches_oracle(imm, orc, stream, sched, name):
    g = synth.make_graph(name)
    sp = synth.WORKLOADS[name]
    dg = imm.graph_from(g, stream=stream)
    keep = g.n <= 20000
    say(f"{sched} schedule on {name}")
    r = imm.imm_run(dg, sp["k"], sp["eps"], sp["ell"], sp["seed"],
                    flags=_flag(imm, sched) | (imm.IMM_KEEP_POOL if keep else 0), stream=stream)
    o = orc.imm(g, sp["k"], sp["eps"], sp["ell"], sp["seed"], threads=oracle_threads(),
                keep_pool=keep, schedule=SCHED[sched])
    _check(r, o, sched, g if keep else None)


def test_schedules_in_batch_and_server(imm, orc, stream):
    names = ["rmat12_wc", "rmat12_lt", "rmat12_p10"]
    graphs = {nm: synth.make_graph(nm) for nm in names}
    dev = {nm: imm.graph_from(g, stream=stream) for nm, g in graphs.items()}
    qs = []
    for i, nm in enumerate(names):
        for j, sched in enumerate([None, "fresh", "early"]):
            qs.append((nm, sched, dict(k=10, epsilon=0.4, ell=1.0, seed=100 + 3 * i + j)))
    say(f"batch of {len(qs)} queries with mixed schedules")
    res = imm.imm_run_batch([(dev[nm], dict(q, flags=_flag(imm, sc) if sc else 0))
                             for nm, sc, q in qs], stream=stream)
    srv = imm.Server(budget_bytes=64 << 30, max_slots=4)
    tickets = [srv.submit(dev[nm], flags=_flag(imm, sc) if sc else 0, **q) for nm, sc, q in qs]
    served = [srv.poll(t) for t in tickets]
    srv.close()
    for (nm, sc, q), rb, rs in zip(qs, res, served):
        o = orc.imm(graphs[nm], q["k"], q["epsilon"], q["ell"], q["seed"],
                    threads=oracle_threads(), schedule=SCHED.get(sc, 0))
        _check(rb, o, sc)
        _check(rs, o, sc)


def test_schedule_flags_exclusive(imm, stream):
    g = synth.make_graph("rmat12_wc")
    dg = imm.graph_from(g, stream=stream)
    with pytest.raises(imm.ImmError) as e:
        imm.imm_run(dg, 5, 0.5, 1.0, 1, flags=imm.IMM_FRESH_FINAL | imm.IMM_EARLY_STOP,
                    stream=stream)
    assert e.value.status == imm.IMM_EINVAL
