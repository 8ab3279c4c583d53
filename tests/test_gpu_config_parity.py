"""GPU vs oracle on the graphs of the multi-instance and served workloads, at
their real sizes.

* Multi-instance batch (64 weighted-cascade R-MAT instances, scale 12..20,
  average degree 4..32): every instance of scale 14 and above is checked on
  the prefix of its sampling, the first 2^16 sample ids through imm_sample
  (canonical pool and fused counts, bit-exact); every instance of scale 16 or
  less is run whole, all of them in one imm_run_batch call, and compared with
  the oracle's IMM run (targets, per-round coverage, LB, theta, seeds, gains).
* Served stream graphs (R-MAT scale 18 IC and the Orkut-shaped LT graph,
  n = 3 M, m = 117 M): the same 2^16-id prefix check, and one query on each
  of the three served graphs through the query server against the oracle's
  IMM run.
"""

import numpy as np
import pytest

import synth
from conftest import oracle_threads
from gpu_util import canonical, say

pytestmark = pytest.mark.gpu

PREFIX = 1 << 16


def _inst_kw(i, s):
    return dict(name=f"batch{i}", gen=s["gen"], model=s["model"], enc=s["enc"], gseed=s["gseed"])


def _prefix_parity(imm, orc, g, dg, seed, stream, label):
    say(f"prefix parity {label}: n={g.n} m={g.m}, ids [0, {PREFIX})")
    pool = imm.imm_sample(dg, seed, 0, PREFIX, stream=stream)
    so, sv, cn = pool.export()
    pool.close()
    oso, osv = orc.sample(g, seed, 0, PREFIX, threads=oracle_threads())
    cso, csv = canonical(oso, osv, g.n)
    np.testing.assert_array_equal(so, cso, err_msg=label)
    np.testing.assert_array_equal(sv, csv, err_msg=label)
    np.testing.assert_array_equal(cn, orc.counts(g.n, oso, osv), err_msg=label)


def _check_run(r, o, label):
    assert r.targets == o["targets"], label
    assert r.round_cov == o["round_cov"], label
    assert (r.theta, r.rounds, r.covered) == (o["theta"], o["rounds"], o["covered"]), label
    assert r.lb == o["lb"], label
    np.testing.assert_array_equal(r.seeds, o["seeds"], err_msg=label)
    np.testing.assert_array_equal(r.gains, o["gains"], err_msg=label)


@pytest.mark.timeout(1200)
def test_batch_instances_prefix_parity(imm, orc, stream):
    insts = synth.batch_instances(64)
    sel = [(i, s) for i, s in enumerate(insts) if s["gen"][1] >= 14]
    say(f"generating {len(sel)} batch graphs of scale 14..20")
    synth.make_graphs([_inst_kw(i, s) for i, s in sel])
    for i, s in sel:
        g = synth.make_graph(**_inst_kw(i, s))
        dg = imm.graph_from(g, stream=stream)
        _prefix_parity(imm, orc, g, dg, s["seed"], stream,
                       f"instance {i} (scale {s['gen'][1]}, degree {g.m >> s['gen'][1]})")
        dg.close()


@pytest.mark.timeout(900)
def test_batch_instances_to_scale16_bit_exact(imm, orc, stream):
    insts = synth.batch_instances(64)
    sel = [(i, s) for i, s in enumerate(insts) if s["gen"][1] <= 16]
    say(f"generating {len(sel)} batch graphs of scale 12..16")
    synth.make_graphs([_inst_kw(i, s) for i, s in sel])
    graphs = [synth.make_graph(**_inst_kw(i, s)) for i, s in sel]
    dev = [imm.graph_from(g, stream=stream) for g in graphs]
    say(f"imm_run_batch of {len(sel)} instances")
    res = imm.imm_run_batch([(d, dict(k=s["k"], epsilon=s["eps"], ell=s["ell"], seed=s["seed"]))
                             for d, (_, s) in zip(dev, sel)], stream=stream)
    for (i, s), g, r in zip(sel, graphs, res):
        label = f"instance {i}: n={g.n} m={g.m} k={s['k']} eps={s['eps']} theta={r.theta}"
        say(f"  check {label}")
        o = orc.imm(g, s["k"], s["eps"], s["ell"], s["seed"], threads=oracle_threads())
        _check_run(r, o, label)


@pytest.fixture(scope="module")
def served(imm, stream):
    names = ["rmat18_wc", "youtube_ic", "orkut_lt"]
    say("generating the served graphs")
    synth.make_graphs([dict(name=nm) for nm in names], workers=3)
    hg = {nm: synth.make_graph(nm) for nm in names}
    dg = {nm: imm.graph_from(g, stream=stream) for nm, g in hg.items()}
    yield hg, dg
    for d in dg.values():
        d.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["rmat18_wc", "orkut_lt"])
def test_served_graph_prefix_parity(imm, orc, stream, served, name):
    hg, dg = served
    _prefix_parity(imm, orc, hg[name], dg[name], synth.WORKLOADS[name]["seed"], stream, name)


@pytest.mark.timeout(900)
def test_served_query_per_graph(imm, orc, stream, served):
    """The first query of the served stream on each graph, all three in the
    server at once, each against the oracle's IMM run."""
    hg, dg = served
    first = {}
    for q in synth.served_queries(1000):
        first.setdefault(q["graph"], q)
    srv = imm.Server(budget_bytes=192 << 30, max_slots=4)
    tickets = {nm: srv.submit(dg[nm], k=q["k"], epsilon=q["eps"], ell=q["ell"], seed=q["seed"])
               for nm, q in first.items()}
    res = {nm: srv.poll(t) for nm, t in tickets.items()}
    srv.close()
    for nm, q in first.items():
        label = f"{nm} k={q['k']} eps={q['eps']} seed={q['seed']}"
        say(f"  oracle IMM {label}")
        o = orc.imm(hg[nm], q["k"], q["eps"], q["ell"], q["seed"], threads=oracle_threads())
        _check_run(res[nm], o, label)
