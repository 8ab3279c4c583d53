"""Batched IMM (imm_run_batch): many independent queries advanced together
on one GPU. Every query's result must equal the CPU oracle's IMM run with
the same arguments, bit for bit, and equal imm_run of that query alone."""

import numpy as np
import pytest

import synth
from conftest import oracle_threads
from gpu_util import canonical, say

pytestmark = pytest.mark.gpu


def _check(r, o, g=None):
    assert r.targets == o["targets"]
    assert r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered) == (o["theta"], o["rounds"], o["covered"])
    assert r.lb == o["lb"]
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])
    if g is not None:
        so, sv = r.pool()
        cso, csv = canonical(o["set_off"], o["set_vtx"], g.n)
        np.testing.assert_array_equal(so, cso)
        np.testing.assert_array_equal(sv, csv)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_mixed_models(imm, orc, stream, graph):
    """IC and LT queries, giant sets, a graph shared by several queries, and
    kept pools, in one batch; with graph, the seed steps run as captured
    graphs, recaptured or updated as the batch's shape changes."""
    if graph:
        import torch
        stream = torch.cuda.Stream()  # a capturable stream (default priority)
    names = ["rmat12_wc", "rmat12_lt", "cl_lt_xs", "rmat12_p10"]
    graphs = {nm: synth.make_graph(nm) for nm in names}
    dev = {nm: imm.graph_from(g, stream=stream) for nm, g in graphs.items()}
    qs = []
    for nm in names:
        sp = synth.WORKLOADS[nm]
        qs.append((nm, dict(k=sp["k"], epsilon=sp["eps"], ell=sp["ell"], seed=sp["seed"],
                            flags=imm.IMM_KEEP_POOL)))
    qs.append(("rmat12_wc", dict(k=25, epsilon=0.3, seed=7)))
    qs.append(("rmat12_wc", dict(k=1, epsilon=0.5, seed=8, ell=2.0)))
    qs.append(("rmat12_lt", dict(k=40, epsilon=0.25, seed=9)))
    if graph:
        for _, q in qs:
            q["flags"] = q.get("flags", 0) | imm.IMM_GRAPH_SELECT
    say(f"batch of {len(qs)}: " + ", ".join(f"{nm} k={q['k']}" for nm, q in qs))
    res = imm.imm_run_batch([(dev[nm], q) for nm, q in qs], stream=stream)
    for (nm, q), r in zip(qs, res):
        say(f"  check {nm} k={q['k']} seed={q['seed']}")
        keep = bool(q.get("flags", 0) & imm.IMM_KEEP_POOL)
        o = orc.imm(graphs[nm], q["k"], q["epsilon"], q.get("ell", 1.0), q["seed"],
                    threads=oracle_threads(), keep_pool=keep)
        _check(r, o, graphs[nm] if keep else None)
        one = imm.imm_run(dev[nm], q["k"], q["epsilon"], q.get("ell", 1.0), q["seed"],
                          stream=stream)
        np.testing.assert_array_equal(one.seeds, r.seeds)
        assert one.theta == r.theta
        if graph:
            assert r.stats["select_graphs"] == r.rounds + 1
        else:
            assert r.stats["select_graphs"] == 0


def test_batch_graph_select_replays(imm, orc):
    """IMM_GRAPH_SELECT on a one-run batch: the batch's shape is the same every
    round, so the seed steps are captured once and the graph is replayed in
    every later round, with that round's sampling, compaction and index (run
    eagerly) between replays. Every round's coverage and the final seeds
    equal the oracle's, and the eager batch's."""
    import torch
    s = torch.cuda.Stream()  # a capturable stream (default priority)
    for nm in ("rmat12_wc", "rmat12_lt"):
        g = synth.make_graph(nm)
        sp = synth.WORKLOADS[nm]
        dg = imm.graph_from(g, stream=s)
        q = dict(k=sp["k"], epsilon=sp["eps"], ell=sp["ell"], seed=sp["seed"])
        say(f"graph replays {nm}")
        rg = imm.imm_run_batch([(dg, dict(q, flags=imm.IMM_GRAPH_SELECT))], stream=s)[0]
        re_ = imm.imm_run_batch([(dg, q)], stream=s)[0]
        o = orc.imm(g, q["k"], q["epsilon"], q["ell"], q["seed"], threads=oracle_threads())
        _check(rg, o)
        _check(re_, o)
        assert rg.rounds >= 2
        assert rg.stats["select_graphs"] == rg.rounds + 1
        assert rg.stats["select_captures"] == 1
        assert re_.stats["select_graphs"] == 0


@pytest.mark.parametrize("select_graph", [False, True])
def test_batch_graph_sample_replays(imm, orc, select_graph):
    """IMM_GRAPH_SAMPLE: the IC queries of a batch sample each round through
    one captured multi-instance launch, relaunched while the set of sampling
    queries repeats and updated or captured anew when it changes (queries of
    different k and eps stop sampling at different rounds), with each round's
    compaction, index and selection run eagerly (or, with select_graph, as
    their own captured graph) between the replays. Every round's coverage and
    the seeds equal the oracle's and the eager batch's."""
    import torch
    s = torch.cuda.Stream()  # a capturable stream (default priority)
    names = ["rmat12_wc", "rmat12_p10", "youtube_ic_s"]
    graphs = {nm: synth.make_graph(nm) for nm in names}
    dev = {nm: imm.graph_from(g, stream=s) for nm, g in graphs.items()}
    qs = []
    for nm in names:
        sp = synth.WORKLOADS[nm]
        qs.append((nm, dict(k=sp["k"], epsilon=sp["eps"], ell=sp["ell"], seed=sp["seed"])))
    qs.append(("rmat12_wc", dict(k=25, epsilon=0.3, ell=1.0, seed=7)))
    qs.append(("rmat12_p10", dict(k=5, epsilon=0.5, ell=1.0, seed=11)))
    fl = imm.IMM_GRAPH_SAMPLE | (imm.IMM_GRAPH_SELECT if select_graph else 0)
    say(f"graph-captured sampling rounds, {len(qs)} IC queries, select graph {select_graph}")
    rg = imm.imm_run_batch([(dev[nm], dict(q, flags=fl)) for nm, q in qs], stream=s)
    re_ = imm.imm_run_batch([(dev[nm], q) for nm, q in qs], stream=s)
    replays = 0
    for (nm, q), a, b in zip(qs, rg, re_):
        say(f"  check {nm} k={q['k']} eps={q['epsilon']} seed={q['seed']}: rounds {a.rounds}, "
            f"sample graphs {a.stats['sample_graphs']} ({a.stats['sample_captures']} captured)")
        o = orc.imm(graphs[nm], q["k"], q["epsilon"], q["ell"], q["seed"],
                    threads=oracle_threads())
        _check(a, o)
        _check(b, o)
        assert a.stats["sample_graphs"] >= 1
        assert b.stats["sample_graphs"] == 0 and b.stats["sample_captures"] == 0
        replays += a.stats["sample_graphs"] - a.stats["sample_captures"]
        if select_graph:
            assert a.stats["select_graphs"] == a.rounds + 1
        else:
            assert a.stats["select_graphs"] == 0
    # the set of sampling queries repeated at least once: a graph was relaunched
    assert replays > 0


def test_batch_of_64_instances(imm, orc, stream):
    """The multi-instance workload's draws (k, eps, degree, seeds) at graph
    scale <= 13: 64 queries on 64 graphs in one call."""
    insts = synth.batch_instances(64, max_scale=13)
    graphs = [synth.make_graph(f"batch{i}", gen=s["gen"], model=s["model"], enc=s["enc"],
                               gseed=s["gseed"]) for i, s in enumerate(insts)]
    dev = [imm.graph_from(g, stream=stream) for g in graphs]
    say("batch of 64 (scale <= 13)")
    res = imm.imm_run_batch([(d, dict(k=s["k"], epsilon=s["eps"], ell=s["ell"], seed=s["seed"]))
                             for d, s in zip(dev, insts)], stream=stream)
    for i, (g, s, r) in enumerate(zip(graphs, insts, res)):
        say(f"  check {i}: n={g.n} m={g.m} k={s['k']} eps={s['eps']} theta={r.theta}")
        o = orc.imm(g, s["k"], s["eps"], s["ell"], s["seed"], threads=oracle_threads())
        _check(r, o)


def test_batch_repeat_and_single_after(imm, orc, stream):
    """Workspaces cached by a batch are reused by later batches and by a
    lone imm_run with identical results."""
    g = synth.make_graph("rmat12_wc")
    dg = imm.graph_from(g, stream=stream)
    q = [(dg, dict(k=10, epsilon=0.5, seed=s)) for s in (1, 2, 3, 4, 5, 6, 7, 8, 9)]
    a = imm.imm_run_batch(q, stream=stream)
    b = imm.imm_run_batch(q[::-1], stream=stream)[::-1]
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.seeds, y.seeds)
        assert (x.theta, x.covered) == (y.theta, y.covered)
    for s, x in zip((1, 2, 3, 4, 5, 6, 7, 8, 9), a):
        one = imm.imm_run(dg, 10, 0.5, 1.0, s, stream=stream)
        o = orc.imm(g, 10, 0.5, 1.0, s, threads=oracle_threads())
        _check(one, o)
        _check(x, o)


def test_batch_errors(imm, stream):
    g = synth.make_graph("rmat12_wc")
    dg = imm.graph_from(g, stream=stream)
    with pytest.raises(imm.ImmError) as e:
        imm.imm_run_batch([(dg, dict(k=5, epsilon=0.5, seed=1)),
                           (dg, dict(k=g.n + 1, epsilon=0.5, seed=2))], stream=stream)
    assert e.value.status == imm.IMM_EINVAL
    with pytest.raises(imm.ImmError) as e:
        imm.imm_run_batch([(dg, dict(k=5, epsilon=0.5, seed=1)),
                           (dg, dict(k=5, epsilon=0.5, seed=2, max_device_bytes=1 << 16))],
                          stream=stream)
    assert e.value.status == imm.IMM_ENOMEM
    # the library is still usable
    r = imm.imm_run_batch([(dg, dict(k=5, epsilon=0.5, seed=1))], stream=stream)
    one = imm.imm_run(dg, 5, 0.5, 1.0, 1, stream=stream)
    np.testing.assert_array_equal(r[0].seeds, one.seeds)


@pytest.mark.parametrize("stage_scale", ["1", "0.01"])
def test_batch_multi_instance_launch(imm, orc, stream, monkeypatch, stage_scale):
    """More IC queries than one multi-instance launch takes (64), so each
    sampling round is two launches; with a tiny first staging estimate, most
    sets find the staging full and are redone by each query's own retry
    passes. Every query equals imm_run alone; a sample of them equals the
    oracle."""
    monkeypatch.setenv("IMM_STAGE_SCALE", stage_scale)
    names = ["rmat12_wc", "rmat12_p10", "youtube_ic_s"]
    graphs = {nm: synth.make_graph(nm) for nm in names}
    dev = {nm: imm.graph_from(g, stream=stream) for nm, g in graphs.items()}
    qs = []
    for i in range(70):
        nm = names[i % len(names)]
        qs.append((nm, dict(k=[5, 10, 25][i % 3], epsilon=[0.5, 0.3][i % 2], ell=1.0,
                            seed=500 + i)))
    say(f"batch of {len(qs)} IC queries, stage scale {stage_scale}")
    res = imm.imm_run_batch([(dev[nm], q) for nm, q in qs], stream=stream)
    monkeypatch.delenv("IMM_STAGE_SCALE")
    for i, ((nm, q), r) in enumerate(zip(qs, res)):
        one = imm.imm_run(dev[nm], q["k"], q["epsilon"], q["ell"], q["seed"], stream=stream)
        np.testing.assert_array_equal(one.seeds, r.seeds)
        np.testing.assert_array_equal(one.gains, r.gains)
        assert (one.theta, one.rounds, one.lb) == (r.theta, r.rounds, r.lb)
        if i % 7 == 0:
            o = orc.imm(graphs[nm], q["k"], q["epsilon"], q["ell"], q["seed"],
                        threads=oracle_threads())
            _check(r, o)
