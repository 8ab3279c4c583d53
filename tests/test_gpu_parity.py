"""GPU path vs CPU oracle: bit-exact parity of Philox streams, RRR pools,
counts, greedy seeds and full IMM runs (every call goes through the C ABI)."""

import numpy as np
import pytest

import synth
from conftest import oracle_threads
from gpu_util import canonical, say

pytestmark = pytest.mark.gpu


def test_philox_matches_oracle(imm, orc, stream):
    """All 2^24 outputs of a counter set per key: random counters, the edge
    cases, and the sampler's own counter shapes (root, IC group, LT vertex
    counters of consecutive sample ids)."""
    rng = np.random.default_rng(5)
    count = 1 << 24
    ctr = rng.integers(0, 2**32, size=(count, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 2, 3, 4], [0, 7, 0, 1]]
    j = np.arange(1 << 20, dtype=np.uint64)
    shapes = np.stack([(j >> 8).astype(np.uint32), (j & 0xFF).astype(np.uint32),
                       np.zeros(j.size, np.uint32), (j % 3).astype(np.uint32)], axis=1)
    ctr[4:4 + shapes.shape[0]] = shapes
    for key in (0, 42, 0xFFFFFFFFFFFFFFFF, 0x123456789ABCDEF0):
        say(f"philox key={key:#x} count={count}")
        dev = imm.imm_philox4x32_10(ctr, key, stream=stream)
        np.testing.assert_array_equal(dev, orc.philox_many(ctr, key))


def test_philox_known_answers(imm, stream):
    """The library's Philox against the generator's published known-answer
    vectors (tests/golden/philox4x32_10_kat.txt)."""
    from pathlib import Path
    rows = []
    for line in (Path(__file__).parent / "golden" / "philox4x32_10_kat.txt").read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            rows.append([int(x, 16) for x in line.split()])
    for w in rows:
        ctr = np.array([w[0:4]], dtype=np.uint32)
        out = imm.imm_philox4x32_10(ctr, w[4] | (w[5] << 32), stream=stream)
        assert [int(x) for x in out[0]] == w[6:10]


def _pool_parity(imm, orc, g, seed, first, count, stream):
    say(f"pool parity {g.name} model={g.model} ids=[{first},{first + count})")
    dg = imm.graph_from(g, stream=stream)
    pool = imm.imm_sample(dg, seed, first, count, stream=stream)
    so, sv, cn = pool.export()
    if first == 0:
        oso, osv = orc.sample(g, seed, 0, count, threads=oracle_threads())
    else:
        oso, osv = orc.sample(g, seed, first, count)
    cso, csv = canonical(oso, osv, g.n)
    np.testing.assert_array_equal(so, cso)
    np.testing.assert_array_equal(sv, csv)
    np.testing.assert_array_equal(cn, orc.counts(g.n, oso, osv))
    assert pool.stats["sets"] == count
    assert pool.stats["entries"] == int(oso[-1])
    return pool


def test_ic_pool_rmat12(imm, orc, stream):
    g = synth.make_graph("rmat12_wc")
    p = _pool_parity(imm, orc, g, 42, 0, 4387, stream)
    # coins evaluated: sum of in-degrees over all members
    so, sv, _ = p.export()
    assert p.stats["edges"] == int(np.diff(g.col_off)[sv.astype(np.int64)].sum())


def test_ic_pool_offset_ids(imm, orc, stream):
    g = synth.make_graph("rmat12_wc")
    _pool_parity(imm, orc, g, 7, 123456789, 700, stream)


def test_ic_pool_youtube_small(imm, orc, stream):
    g = synth.make_graph("youtube_ic_s")
    _pool_parity(imm, orc, g, 42, 0, 60000, stream)


def test_ic_pool_giant_sets(imm, orc, stream):
    g = synth.make_graph("rmat12_p10")
    p = _pool_parity(imm, orc, g, 42, 0, 3000, stream)
    assert p.stats["deferred"] > 0  # giant sets went through the large-set kernel


@pytest.mark.parametrize("big", [256, 1024])
@pytest.mark.parametrize("team", [1, 2, 4])
@pytest.mark.parametrize("name", ["rmat12_wc", "rmat12_p10"])
def test_ic_pool_each_shape(imm, orc, stream, monkeypatch, team, big, name):
    """Every IC launch shape the autotuner can pick (1, 2 or 4 waves per BFS
    sample; 256 or 1024 threads per giant set) gives the same pool."""
    monkeypatch.setenv("IMM_IC_TEAM", str(team))
    monkeypatch.setenv("IMM_IC_BIG", str(big))
    g = synth.make_graph(name)
    p = _pool_parity(imm, orc, g, 9, 0, 3000, stream)
    assert (p.stats["team"], p.stats["big_block"]) == (team, big)


@pytest.mark.parametrize("lanes", [1, 2, 4])
@pytest.mark.parametrize("bloom", [10, 11, 12])
@pytest.mark.parametrize("name", ["cl_lt_xs", "rmat12_lt"])
def test_lt_pool_each_filter_size(imm, orc, stream, monkeypatch, lanes, bloom, name):
    """Every LT walk shape (lanes per walk, path-filter size) gives the same
    pool."""
    monkeypatch.setenv("IMM_LT_BLOOM", str(bloom))
    monkeypatch.setenv("IMM_LT_LANES", str(lanes))
    g = synth.make_graph(name)
    p = _pool_parity(imm, orc, g, 13, 0, 6000, stream)
    assert (p.stats["bloom_bits"], p.stats["walk_lanes"]) == (bloom, lanes)


def test_lt_pool_small(imm, orc, stream):
    g = synth.make_graph("cl_lt_xs")
    _pool_parity(imm, orc, g, 42, 0, 20000, stream)


def test_lt_pool_rmat12(imm, orc, stream):
    g = synth.make_graph("rmat12_lt")
    _pool_parity(imm, orc, g, 3, 0, 5000, stream)


def test_greedy_on_oracle_pool(imm, orc, stream):
    g = synth.make_graph("rmat12_wc")
    so, sv = orc.sample(g, 42, 0, 4000)
    for k in (1, 10, 50):
        say(f"greedy parity k={k}")
        s, ga, cov = imm.imm_greedy(g.n, so, sv, k, stream=stream)
        os_, og, ocov = orc.greedy(g.n, so, sv, k)
        np.testing.assert_array_equal(s, os_)
        np.testing.assert_array_equal(ga, og)
        assert cov == ocov


def _imm_parity(imm, orc, name, stream, threads=None, keep_pool=False):
    spec = synth.WORKLOADS[name]
    g = synth.make_graph(name)
    say(f"imm parity {name} k={spec['k']} eps={spec['eps']}")
    dg = imm.graph_from(g, stream=stream)
    flags = imm.IMM_KEEP_POOL if keep_pool else 0
    r = imm.imm_run(dg, spec["k"], spec["eps"], spec["ell"], spec["seed"], flags=flags,
                    stream=stream)
    o = orc.imm(g, spec["k"], spec["eps"], spec["ell"], spec["seed"],
                threads=threads or oracle_threads(), keep_pool=keep_pool)
    assert r.targets == o["targets"]
    assert r.round_cov == o["round_cov"]
    assert (r.theta, r.rounds, r.covered) == (o["theta"], o["rounds"], o["covered"])
    assert r.lb == o["lb"]
    np.testing.assert_array_equal(r.seeds, o["seeds"])
    np.testing.assert_array_equal(r.gains, o["gains"])
    if keep_pool:
        so, sv = r.pool()
        cso, csv = canonical(o["set_off"], o["set_vtx"], g.n)
        np.testing.assert_array_equal(so, cso)
        np.testing.assert_array_equal(sv, csv)
    return r, o


def test_imm_rmat12(imm, orc, stream):
    _imm_parity(imm, orc, "rmat12_wc", stream, keep_pool=True)


def test_imm_giant_sets(imm, orc, stream):
    _imm_parity(imm, orc, "rmat12_p10", stream, keep_pool=True)


def test_imm_rmat12_lt(imm, orc, stream):
    _imm_parity(imm, orc, "rmat12_lt", stream, keep_pool=True)


def test_imm_lt_small(imm, orc, stream):
    _imm_parity(imm, orc, "cl_lt_xs", stream)
