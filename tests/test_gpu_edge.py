"""Edge cases of the GPU path, each checked against the oracle: graphs without
edges, every vertex selected, certain and impossible edges, sample ids that
cross 2^32, the staging-growth path, device-memory budgets, device-pointer
inputs, and repeated runs on a resident graph."""

import os

import numpy as np
import pytest

import synth
from gpu_util import canonical, say

pytestmark = pytest.mark.gpu

T32 = 1 << 32


def _parity(imm, orc, g, k, eps, seed, stream, pool=True):
    dg = imm.graph_from(g, stream=stream)
    r = imm.imm_run(dg, k, eps, 1.0, seed, flags=imm.IMM_KEEP_POOL if pool else 0,
                    stream=stream)
    o = orc.imm(g, k, eps, 1.0, seed, keep_pool=pool)
    assert r.targets == o["targets"] and r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered, r.lb) == (o["theta"], o["rounds"], o["covered"], o["lb"])
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])
    if pool:
        so, sv = r.pool()
        cso, csv = canonical(o["set_off"], o["set_vtx"], g.n)
        np.testing.assert_array_equal(so, cso)
        np.testing.assert_array_equal(sv, csv)
    return r


@pytest.mark.parametrize("model", ["ic", "lt"])
def test_no_edges(imm, orc, stream, model):
    g = synth.tiny_graph(2, [], model, [])
    say(f"no edges {model}")
    for k in (1, 2):
        _parity(imm, orc, g, k, 0.5, 3, stream)


def test_select_every_vertex(imm, orc, stream):
    g = synth.tiny_graph(6, [(0, 1), (1, 2), (2, 0), (3, 4)], "ic", [1 << 31] * 4)
    _parity(imm, orc, g, 6, 0.5, 11, stream)


@pytest.mark.parametrize("team", [1, 2, 4])
def test_certain_and_impossible_edges(imm, orc, stream, monkeypatch, team):
    # a certain chain 0 -> 1 -> ... -> n-1 (the set of root v is {0..v}) plus
    # impossible back edges; sets longer than every team's on-chip limit
    monkeypatch.setenv("IMM_IC_TEAM", str(team))
    n = 1300
    edges = [(v, v + 1) for v in range(n - 1)] + [(v + 2, v) for v in range(0, n - 2, 7)]
    thr = [T32 - 1] * (n - 1) + [0] * len(range(0, n - 2, 7))
    g = synth.tiny_graph(n, edges, "ic", thr)
    say(f"certain chain n={n} team={team}")
    r = _parity(imm, orc, g, 3, 0.3, 5, stream)
    assert r.stats["team"] == team
    assert r.stats["deferred"] > 0  # chains longer than the on-chip set limit


@pytest.mark.parametrize("big", [256, 1024])
def test_sets_beyond_bounded_giant_queue(imm, orc, stream, monkeypatch, big):
    """A certain chain longer than the giant-set queue bound (65536 members):
    the sets of roots beyond it go through the full-size second pass. (The
    launch shapes are fixed: every BFS level of a chain holds one vertex.)"""
    monkeypatch.setenv("IMM_IC_TEAM", "4")
    monkeypatch.setenv("IMM_IC_BIG", str(big))
    n = 70000
    g = synth.tiny_graph(n, [(v, v + 1) for v in range(n - 1)], "ic", [T32 - 1] * (n - 1))
    say(f"certain chain n={n}, 300 samples")
    dg = imm.graph_from(g, stream=stream)
    pool = imm.imm_sample(dg, 4, 0, 300, stream=stream)
    so, sv, cn = pool.export()
    oso, osv = orc.sample(g, 4, 0, 300)
    cso, csv = canonical(oso, osv, g.n)
    np.testing.assert_array_equal(so, cso)
    np.testing.assert_array_equal(sv, csv)
    np.testing.assert_array_equal(cn, orc.counts(g.n, oso, osv))
    assert int(np.diff(so).max()) > 65536


def test_lt_with_no_live_edge_mass(imm, orc, stream):
    # every column keeps 1/4 probability of no live in-edge
    rng = np.random.default_rng(3)
    n = 400
    edges = sorted({(int(u), int(v)) for u, v in rng.integers(0, n, size=(3000, 2)) if u != v})
    deg = np.bincount([v for _, v in edges], minlength=n)
    q = [(3 << 30) // int(deg[v]) for _, v in edges]
    g = synth.tiny_graph(n, edges, "lt", q)
    _parity(imm, orc, g, 5, 0.3, 9, stream)


def _lt_long_graph(kind):
    # chain: v's one in-edge comes from v - 1 with weight just below 1, so the
    # walk from root r is r, r-1, ..., 0 (r + 1 vertices; most are longer
    # than a walk kernel's staging chunk). ring: the chain closed by the edge
    # n-1 -> 0, so every walk goes once round and stops at its own root.
    n = 3000 if kind == "chain" else 700
    edges = [(v, v + 1) for v in range(n - 1)]
    if kind == "ring":
        edges.append((n - 1, 0))
    return synth.tiny_graph(n, sorted(edges, key=lambda e: (e[1], e[0])), "lt",
                            [T32 - 1] * len(edges))


@pytest.mark.parametrize("lanes", [1, 2, 4])
@pytest.mark.parametrize("kind", ["chain", "ring"])
def test_lt_long_walks(imm, orc, stream, monkeypatch, kind, lanes):
    """Walks that outgrow the staging chunk (moved to a fresh chunk, or handed
    to the long-walk kernel) and walks that close a cycle, in every walk
    shape, give the oracle's sets and counts."""
    monkeypatch.setenv("IMM_LT_LANES", str(lanes))
    g = _lt_long_graph(kind)
    say(f"LT long walks {kind} n={g.n} lanes={lanes}")
    dg = imm.graph_from(g, stream=stream)
    pool = imm.imm_sample(dg, 31, 0, 2500, stream=stream)
    so, sv, cn = pool.export()
    assert pool.stats["walk_lanes"] == lanes
    if kind == "chain":
        assert pool.stats["deferred"] > 0
    else:
        assert pool.stats["deferred"] == 0
    oso, osv = orc.sample(g, 31, 0, 2500)
    cso, csv = canonical(oso, osv, g.n)
    np.testing.assert_array_equal(so, cso)
    np.testing.assert_array_equal(sv, csv)
    np.testing.assert_array_equal(cn, orc.counts(g.n, oso, osv))


@pytest.mark.parametrize("lanes", [1, 4])
def test_lt_long_walks_with_staging_growth(imm, orc, stream, monkeypatch, lanes):
    """Chain walks of up to 3000 vertices with a first staging guess far too
    small. A walk handed to the long-walk kernel leaves its first 1024
    members in its chunk, and that kernel continues from there; when it
    then finds the staging buffer full, the walk is retried after growth,
    from its root, and handed over again."""
    monkeypatch.setenv("IMM_LT_LANES", str(lanes))
    monkeypatch.setenv("IMM_STAGE_SCALE", "0.001")
    g = _lt_long_graph("chain")
    say(f"LT long walks with staging growth lanes={lanes}")
    dg = imm.graph_from(g, stream=stream)
    pool = imm.imm_sample(dg, 31, 0, 2500, stream=stream)
    so, sv, cn = pool.export()
    assert pool.stats["deferred"] > 0
    oso, osv = orc.sample(g, 31, 0, 2500)
    cso, csv = canonical(oso, osv, g.n)
    np.testing.assert_array_equal(so, cso)
    np.testing.assert_array_equal(sv, csv)
    np.testing.assert_array_equal(cn, orc.counts(g.n, oso, osv))


def test_zero_thresholds(imm, orc, stream):
    base = synth.make_graph("rmat12_wc")
    g = synth.Graph("rmat12_zero", base.n, base.m, base.col_off, base.row_src,
                    np.zeros(base.m, np.uint32), "ic")
    _parity(imm, orc, g, 10, 0.5, 42, stream)


def test_sample_ids_across_2_32(imm, orc, stream):
    for name in ("rmat12_p10", "rmat12_lt"):
        g = synth.make_graph(name)
        dg = imm.graph_from(g, stream=stream)
        first = (1 << 32) - 300
        pool = imm.imm_sample(dg, 77, first, 600, stream=stream)
        so, sv, cn = pool.export()
        oso, osv = orc.sample(g, 77, first, 600)
        cso, csv = canonical(oso, osv, g.n)
        np.testing.assert_array_equal(so, cso)
        np.testing.assert_array_equal(sv, csv)
        np.testing.assert_array_equal(cn, orc.counts(g.n, oso, osv))


@pytest.mark.parametrize("name,lanes", [("rmat12_p10", None), ("cl_lt_xs", None),
                                        ("cl_lt_xs", 1), ("cl_lt_xs", 2), ("cl_lt_xs", 4)])
def test_staging_growth_path(imm, orc, stream, monkeypatch, name, lanes):
    """A first staging guess far too small: sets are retried after growth
    and the result is unchanged. In the LT walk kernel, every walk of a wave
    can then fail to start at once while the wave still holds claimed sample
    positions; each of those must still be walked or listed for a retry."""
    spec = synth.WORKLOADS[name]
    if lanes:
        monkeypatch.setenv("IMM_LT_LANES", str(lanes))
    monkeypatch.setenv("IMM_STAGE_SCALE", "0.001")
    say(f"staging growth {name} lanes={lanes}")
    r = _parity(imm, orc, synth.make_graph(name), spec["k"], spec["eps"], 42, stream)
    if lanes:
        assert r.stats["walk_lanes"] == lanes


def test_budget_enomem_then_retry(imm, orc, stream):
    g = synth.make_graph("rmat12_wc")
    dg = imm.graph_from(g, stream=stream)
    with pytest.raises(imm.ImmError) as e:
        imm.imm_run(dg, 10, 0.5, 1.0, 42, max_device_bytes=1 << 16, stream=stream)
    assert e.value.status == imm.IMM_ENOMEM
    r = imm.imm_run(dg, 10, 0.5, 1.0, 42, max_device_bytes=1 << 30, stream=stream)
    o = orc.imm(g, 10, 0.5, 1.0, 42)
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    assert r.theta == o["theta"]


def test_overflow_is_reported(imm, stream):
    g = synth.make_graph("rmat12_wc")
    dg = imm.graph_from(g, stream=stream)
    with pytest.raises(imm.ImmError) as e:
        imm.imm_run(dg, 10, 1e-4, 1.0, 42, stream=stream)
    assert e.value.status == imm.IMM_EOVERFLOW


def test_device_pointer_inputs(imm, orc, stream):
    import torch
    g = synth.make_graph("rmat12_wc")
    t = lambda a, dt: torch.from_numpy(a.astype(dt).view(np.int64 if dt == np.uint64 else np.int32)).cuda()
    dg = imm.imm_graph_create(g.n, g.m, t(g.col_off, np.uint64), t(g.row_src, np.uint32),
                              t(g.weight, np.uint32), "ic", stream=stream)
    torch.cuda.synchronize()
    r = imm.imm_run(dg, 10, 0.5, 1.0, 42, stream=stream)
    o = orc.imm(g, 10, 0.5, 1.0, 42)
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    so, sv = orc.sample(g, 42, 0, 3000)
    s, ga, cov = imm.imm_greedy(g.n, t(so, np.uint64), t(sv, np.uint32), 10, stream=stream)
    os_, og, ocov = orc.greedy(g.n, so, sv, 10)
    np.testing.assert_array_equal(s, os_)
    assert cov == ocov


def test_repeated_runs_reuse_workspace(imm, orc, stream):
    """The resident graph's cached workspace gives identical results run
    after run, across models and different k on the same graph."""
    g = synth.make_graph("rmat12_wc")
    dg = imm.graph_from(g, stream=stream)
    o10 = orc.imm(g, 10, 0.5, 1.0, 42)
    o3 = orc.imm(g, 3, 0.3, 1.0, 7)
    for _ in range(3):
        r = imm.imm_run(dg, 10, 0.5, 1.0, 42, stream=stream)
        np.testing.assert_array_equal(r.seeds, o10["seeds"])
        r = imm.imm_run(dg, 3, 0.3, 1.0, 7, stream=stream)
        np.testing.assert_array_equal(r.seeds, o3["seeds"])
        assert r.theta == o3["theta"]
    # a larger k first, then smaller ones: per-step selection state sized for
    # the larger k must start clean for every later run
    for k, eps, seed in [(25, 0.3, 100), (5, 0.3, 100), (1, 0.5, 3), (5, 0.5, 101), (25, 0.3, 5)]:
        say(f"reuse k={k} eps={eps} seed={seed}")
        o = orc.imm(g, k, eps, 1.0, seed)
        r = imm.imm_run(dg, k, eps, 1.0, seed, stream=stream)
        np.testing.assert_array_equal(r.seeds, o["seeds"])
        np.testing.assert_array_equal(r.gains, o["gains"])


def _sample_parity(imm, orc, g, seed, count, stream):
    dg = imm.graph_from(g, stream=stream)
    pool = imm.imm_sample(dg, seed, 0, count, stream=stream)
    so, sv, cn = pool.export()
    oso, osv = orc.sample(g, seed, 0, count)
    cso, csv = canonical(oso, osv, g.n)
    np.testing.assert_array_equal(so, cso)
    np.testing.assert_array_equal(sv, csv)
    np.testing.assert_array_equal(cn, orc.counts(g.n, oso, osv))
    return so


def _hub_graph(n, p_in):
    # vertex 0 has an in-edge from every other vertex (probability p_in) and
    # an out-edge to every other vertex (certain): every set reaches the hub
    # and sweeps its whole column
    edges = [(v, 0) for v in range(1, n)] + [(0, v) for v in range(1, n)]
    thr = [int(p_in * T32)] * (n - 1) + [T32 - 1] * (n - 1)
    return synth.tiny_graph(n, edges, "ic", thr)


@pytest.mark.parametrize("team", [1, 2, 4])
def test_hub_column_spans_several_pages(imm, orc, stream, monkeypatch, team):
    """A hub of 70,000 in-edges (17,500 groups of four) in every small set: the
    BFS team sweeps it over several pages of its owner bitmap (4096 * team
    groups per page)."""
    monkeypatch.setenv("IMM_IC_TEAM", str(team))
    g = _hub_graph(70001, 1e-4)
    say(f"hub column n={g.n} team={team}")
    so = _sample_parity(imm, orc, g, 9, 400, stream)
    assert int(np.diff(so).max()) < 256 * team  # stayed in the team pass


@pytest.mark.parametrize("big", [256, 1024])
def test_giant_set_hub_column_spans_two_pages(imm, orc, stream, monkeypatch, big):
    """Giant sets (thousands of members) that sweep a hub of 270,000 in-edges:
    67,500 groups, more than one page (65,536) of the giant-set kernel's
    owner bitmap."""
    monkeypatch.setenv("IMM_IC_TEAM", "4")
    monkeypatch.setenv("IMM_IC_BIG", str(big))
    g = _hub_graph(270001, 1e-2)
    say(f"giant hub column n={g.n} big={big}")
    so = _sample_parity(imm, orc, g, 5, 60, stream)
    assert int(np.diff(so).max()) > 1024  # went through the giant-set pass


@pytest.mark.parametrize("eps,min_first_gain", [(0.1, 2 * 4096), (0.07, 4 * 4096)])
def test_recount_with_long_index_lists(imm, orc, stream, eps, min_first_gain):
    """Two hubs, each in most sets of its own parity class and in some of the
    other's: the first seed covers more than a quarter of the pool, so the
    next counts are rebuilt by a recount in which the other hub (10,000 or
    more index entries, partly covered) is a work item of its own. The
    first seed's lists hold about 10,000 positions at eps = 0.1 and about
    20,000 at eps = 0.07."""
    rng = np.random.default_rng(21)
    n = 20002
    edges, thr = [], []
    for v in range(2, n):
        edges.append((v % 2, v))
        thr.append(T32 - 1)
    for hub in (0, 1):
        same = np.arange(2 + hub, n, 2)
        other = np.arange(3 - hub, n, 2)
        src = np.concatenate([rng.choice(same, size=4500, replace=False),
                              rng.choice(other, size=500, replace=False)])
        for u in src:
            edges.append((int(u), hub))
            thr.append(int(1e-3 * T32))
    g = synth.tiny_graph(n, edges, "ic", thr)
    say(f"two-hub recount eps={eps}")
    r = _parity(imm, orc, g, 5, eps, 17, stream, pool=False)
    # the run equals the oracle's (checked in _parity); the first seed's
    # index list is longer than two (four) long-list thresholds of 4096
    assert r.theta > 2 * 4096 and r.gains[1] > 0 and r.gains[0] > min_first_gain


def test_lt_ids_drawn_ahead_and_dropped(imm, orc, stream):
    """An LT graph whose first round already passes IMM's lower-bound test:
    every vertex but the hub has an in-edge from the hub (weight 0.7) and from
    two random vertices (0.1 each), so a seed at the hub covers most sets.
    The first round also draws ids ahead (the second round's, and more); the
    final theta lies between the first two targets, so some of those sets
    join the pool and the rest are dropped. The run, its pool and its counts
    must equal the oracle's."""
    rng = np.random.default_rng(33)
    n = 2048
    edges, w = [], []
    for v in range(1, n):
        srcs = [0] + [int(x) for x in rng.choice(np.arange(1, n), size=2, replace=False) if x != v]
        for j, u in enumerate(srcs):
            edges.append((u, v))
            w.append(int(0.7 * T32) if j == 0 else int(0.1 * T32))
    g = synth.tiny_graph(n, edges, "lt", w)
    k, eps = 5, 0.5
    say("LT run that breaks in its first round")
    r = _parity(imm, orc, g, k, eps, 11, stream, pool=True)
    assert r.rounds == 1
    assert r.targets[0] < r.theta < 2 * r.targets[0]


@pytest.mark.parametrize("name,k,eps", [("rmat12_lt", 10, 0.5), ("rmat12_lt", 5, 0.2),
                                        ("cl_lt_xs", 10, 0.3), ("cl_lt_xs", 5, 0.2)])
def test_lt_ids_drawn_ahead_taken_over_rounds(imm, orc, stream, name, k, eps):
    """LT runs of two or three rounds: the first round draws ids up to the
    final theta that a pass of the next round would allow, and the later
    rounds and the final selection take them a part at a time, without a
    launch of their own. Targets, coverage, LB, seeds, gains and the pool
    must equal the oracle's."""
    g = synth.make_graph(name)
    say(f"LT run on {name}, k={k}, eps={eps}")
    r = _parity(imm, orc, g, k, eps, 3, stream, pool=True)
    assert r.rounds >= 2
