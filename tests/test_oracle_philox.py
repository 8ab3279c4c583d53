"""Pins of the oracle's Philox4x32-10 and of the random decisions built on it
(reading R1/R2 of the oracle header).

Philox is pinned against rocRAND's own implementation of the same published
generator (Salmon et al., SC'11), compiled here as a small host program from
rocRAND's header; the sample roots and IC coins are pinned statistically
against their intended distributions."""

import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

import oracle

KAT_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
    Probe p;
    unsigned a, b, c, d, k0, k1;
    while (scanf("%x %x %x %x %x %x", &a, &b, &c, &d, &k0, &k1) == 6) {
        uint4 o = p.run(make_uint4(a, b, c, d), make_uint2(k0, k1));
        printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    hdr = Path("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h")
    if not Path(hipcc).exists() or not hdr.exists():
        pytest.skip("rocRAND header / hipcc not available")
    d = tmp_path_factory.mktemp("kat")
    (d / "kat.cpp").write_text(KAT_SRC)
    subprocess.run([hipcc, "-O1", "-o", str(d / "kat"), str(d / "kat.cpp")], check=True,
                   capture_output=True)

    def run(rows):
        inp = "\n".join(" ".join(f"{x:x}" for x in r) for r in rows) + "\n"
        out = subprocess.run([str(d / "kat")], input=inp, capture_output=True, text=True,
                             check=True).stdout.split("\n")
        return np.array([[int(x, 16) for x in line.split()] for line in out if line.strip()],
                        dtype=np.uint64)

    return run


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(11)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 2, 3, 4, 5, 6]]
    rows += rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64).tolist()
    # the counter shapes the sampler uses: (group, s_lo, s_hi, stream tag)
    rows += [[e, s, 0, tag, 42, 0] for e in (0, 1, 7, 1 << 30) for s in (0, 5, 2**32 - 1)
             for tag in (0, 1, 2)]
    ref = rocrand_philox(rows)
    for r, want in zip(rows, ref):
        got = oracle.philox4x32_10(r[:4], int(r[4]) | (int(r[5]) << 32))
        np.testing.assert_array_equal(got.astype(np.uint64), want)


def _kat_rows():
    path = Path(__file__).parent / "golden" / "philox4x32_10_kat.txt"
    rows = []
    for line in path.read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4] | (w[5] << 32), w[6:10]))
    return rows


def test_philox_known_answers():
    """The published known-answer vectors of the generator (golden fixture)."""
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle.philox4x32_10(np.array(ctr, dtype=np.uint32), key)
        assert [int(x) for x in got] == want


def test_draw_word_selection():
    """Edge e uses word e&3 of counter (e>>2, s_lo, s_hi, 1); vertex v uses
    word v&3 of (v>>2, s_lo, s_hi, 2); the root uses words 0,1 of
    (0, s_lo, s_hi, 0)."""
    seed, s = 0x1234_5678_9ABC_DEF0, (7 << 32) | 99
    for e in range(16):
        w = oracle.philox4x32_10([e >> 2, s & 0xFFFFFFFF, s >> 32, 1], seed)
        assert oracle.ic_draw(seed, s, e) == int(w[e & 3])
        w = oracle.philox4x32_10([e >> 2, s & 0xFFFFFFFF, s >> 32, 2], seed)
        assert oracle.lt_draw(seed, s, e) == int(w[e & 3])
    w = oracle.philox4x32_10([0, s & 0xFFFFFFFF, s >> 32, 0], seed)
    full = int(w[0]) | (int(w[1]) << 32)
    for n in (2, 3, 1000, 4_800_000, 2**32 - 2):
        assert oracle.root(seed, s, n) == (full * n) >> 64


def test_root_uniform():
    n, N = 16, 160_000
    hist = np.zeros(n)
    for s in range(N):
        hist[oracle.root(42, s, n)] += 1
    chi2 = ((hist - N / n) ** 2 / (N / n)).sum()
    assert chi2 < 45.0  # 15 dof, p ~ 1e-4


@pytest.mark.parametrize("thr", [1 << 30, 3 << 30, 42949672, (1 << 32) - 1])
def test_ic_coin_rate(thr):
    N = 100_000
    live = sum(oracle.ic_draw(9, s, 5 + (s % 13)) < thr for s in range(N))
    p = thr / 2**32
    se = np.sqrt(N * p * (1 - p)) + 1e-9
    assert abs(live - N * p) < 5 * se + 1
