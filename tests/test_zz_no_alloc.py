"""imm_greedy_static, the greedy entry point that allocates nothing (its
scratch is the library's fixed per-device array): the same seeds, gains and
coverage as imm_greedy, bit for bit, on two calls in a row (the second on a
smaller pool, so the array holds the first call's leftovers), with the pool
in device memory and in host memory; and a clear refusal of a size beyond the
array."""

import numpy as np
import pytest

import synth
from conftest import oracle_threads
from gpu_util import say

pytestmark = pytest.mark.gpu


def _pool(orc, name, count):
    g = synth.make_graph(name)
    so, sv = orc.sample(g, synth.WORKLOADS[name]["seed"], 0, count, threads=oracle_threads())
    return g, so, sv


def _same(a, b):
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert a[2] == b[2]


@pytest.mark.parametrize("device", [True, False])
def test_static_greedy_equals_greedy(imm, orc, stream, device):
    import torch
    big = _pool(orc, "rmat12_p10", 40000)
    small = _pool(orc, "rmat12_wc", 3000)
    for (g, so, sv), k in ((big, 25), (small, 10)):
        say(f"greedy_static {g.name}: {so.size - 1} sets, {sv.size} entries, k={k}, "
            f"device={device}")
        want = imm.imm_greedy(g.n, so, sv, k, stream=stream)
        if device:
            a0 = torch.from_numpy(so.view(np.int64)).cuda()
            a1 = torch.from_numpy(sv.view(np.int32)).cuda()
            torch.cuda.synchronize()
            got = imm.imm_greedy_static(g.n, a0, a1, k, stream=stream)
        else:
            got = imm.imm_greedy_static(g.n, so, sv, k, stream=stream)
        _same(got, want)
        _same(got, orc.greedy(g.n, so, sv, k))


def test_static_greedy_limits(imm, stream):
    so = np.array([0, 2, 3], dtype=np.uint64)
    sv = np.array([0, 1, 1], dtype=np.uint32)
    # counts and index offsets alone of 40 M vertices exceed the array
    with pytest.raises(imm.ImmError) as e:
        imm.imm_greedy_static(40_000_000, so, sv, 1, stream=stream)
    assert e.value.status == imm.IMM_ENOMEM and "scratch" in str(e.value)
    with pytest.raises(imm.ImmError) as e:
        imm.imm_greedy_static(1, so, sv, 1, stream=stream)  # vertex 1 out of range
    assert e.value.status == imm.IMM_EINVAL
    # still usable, and equal to imm_greedy
    _same(imm.imm_greedy_static(4, so, sv, 2, stream=stream),
          imm.imm_greedy(4, so, sv, 2, stream=stream))
