"""The vertex->sets index (Algorithm 2's "if v in R" test done by list
lookups) built either way, the radix partition or the per-entry atomic
scatter, forced for every segment: whole IMM runs of one to several rounds
(one index segment each), graphs whose vertex count is not a multiple of the
bucket width or is below the bucket count, graphs without edges, and the
greedy alone on a pool the oracle drew. Seeds, gains, coverage and LB must
equal the oracle's either way."""

import numpy as np
import pytest

import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

T32 = 1 << 32
BUILDS = ["partition", "atomic"]


@pytest.fixture
def build(monkeypatch, request):
    monkeypatch.delenv("IMM_INDEX_ATOMIC", raising=False)
    monkeypatch.delenv("IMM_INDEX_PARTITION", raising=False)
    monkeypatch.setenv("IMM_INDEX_PARTITION" if request.param == "partition"
                       else "IMM_INDEX_ATOMIC", "1")
    return request.param


def _run(imm, orc, g, k, eps, seed, stream):
    dg = imm.graph_from(g, stream=stream)
    r = imm.imm_run(dg, k, eps, 1.0, seed, stream=stream)
    o = orc.imm(g, k, eps, 1.0, seed)
    assert r.targets == o["targets"] and r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered, r.lb) == (o["theta"], o["rounds"], o["covered"], o["lb"])
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])
    return r


@pytest.mark.parametrize("build", BUILDS, indirect=True)
@pytest.mark.parametrize("name,k,eps", [("rmat12_wc", 10, 0.5), ("rmat12_p10", 25, 0.3),
                                        ("rmat12_lt", 5, 0.2), ("cl_lt_xs", 5, 0.2)])
def test_index_imm_runs(imm, orc, stream, build, name, k, eps):
    g = synth.make_graph(name)
    say(f"{build} index, {name} k={k} eps={eps}")
    _run(imm, orc, g, k, eps, 5, stream)


@pytest.mark.parametrize("build", BUILDS, indirect=True)
@pytest.mark.parametrize("n", [2, 7, 2047, 2049, 5000])
def test_index_vertex_counts(imm, orc, stream, build, n):
    """A ring plus chords (edge probabilities 1/2 and 1/4): n below, at and
    above the 2048 buckets (one vertex per bucket, then two), and n = 2."""
    rng = np.random.default_rng(n)
    edges, thr = [], []
    for v in range(n):
        if n > 1:
            edges.append(((v + 1) % n, v))
            thr.append(T32 // 2)
        for u in rng.choice(n, size=min(n, 3), replace=False):
            if int(u) != v:
                edges.append((int(u), v))
                thr.append(T32 // 4)
    g = synth.tiny_graph(n, edges, "ic", thr)
    say(f"{build} index, ring of {n}")
    _run(imm, orc, g, min(3, n), 0.5, 9, stream)


@pytest.mark.parametrize("build", BUILDS, indirect=True)
@pytest.mark.parametrize("n", [2, 7, 2047, 2049, 5000])
def test_index_vertex_counts_lt(imm, orc, stream, build, n):
    """The same rings as LT graphs (in-weights 1/3 for the ring edge, 1/5
    per chord): their later rounds and final selections take ids drawn
    ahead, whose segments the partition builds from the sets alone."""
    rng = np.random.default_rng(n + 1)
    edges, wq = [], []
    for v in range(n):
        if n > 1:
            edges.append(((v + 1) % n, v))
            wq.append(T32 // 3)
        for u in rng.choice(n, size=min(n, 3), replace=False):
            if int(u) != v and int(u) != (v + 1) % n:
                edges.append((int(u), v))
                wq.append(T32 // 5)
    g = synth.tiny_graph(n, edges, "lt", wq)
    say(f"{build} index, LT ring of {n}")
    _run(imm, orc, g, min(3, n), 0.3, 9, stream)


@pytest.mark.parametrize("build", BUILDS, indirect=True)
def test_index_lt_hub(imm, orc, stream, build):
    """An LT graph whose walks nearly all pass through vertex 0 (in-weight
    0.9 from it at every other vertex): vertex 0's bucket holds most of a
    segment's entries, far more than one placement slice, and the counting
    build gives that bucket to one workgroup."""
    n = 20000
    rng = np.random.default_rng(77)
    edges, wq = [], []
    for v in range(1, n):
        edges.append((0, v))
        wq.append(int(0.9 * T32))
        edges.append(((v + 1) % n if (v + 1) % n != 0 else 1, v))
        wq.append(T32 // 20)
    for u in rng.choice(np.arange(1, n), 3, replace=False):
        edges.append((int(u), 0))
        wq.append(T32 // 4)
    g = synth.tiny_graph(n, edges, "lt", wq)
    say(f"{build} index, LT hub")
    _run(imm, orc, g, 5, 0.05, 3, stream)


@pytest.mark.parametrize("build", BUILDS, indirect=True)
def test_index_no_edges(imm, orc, stream, build):
    g = synth.tiny_graph(3000, [], "ic", [])
    say(f"{build} index, no edges")
    _run(imm, orc, g, 4, 0.5, 2, stream)


@pytest.mark.parametrize("build", BUILDS, indirect=True)
def test_index_greedy_on_oracle_pool(imm, orc, stream, build):
    g = synth.make_graph("rmat12_wc")
    so, sv = orc.sample(g, 17, 0, 30000)
    say(f"{build} index, greedy on an oracle pool")
    for k in (1, 20):
        s, ga, cov = imm.imm_greedy(g.n, so, sv, k, stream=stream)
        os_, og, ocov = orc.greedy(g.n, so, sv, k)
        np.testing.assert_array_equal(s, os_)
        np.testing.assert_array_equal(ga, og)
        assert cov == ocov
