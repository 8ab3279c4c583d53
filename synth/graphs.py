"""Graph generators and parameter encodings (inputs only; no IMM arithmetic).

Layout produced for every graph (the C-ABI's input format):

* ``col_off``  uint64[n+1]  CSC offsets of the in-edges of each vertex,
* ``row_src``  uint32[m]    source vertex of each in-edge; within a column the
                            sources are ascending, and the edge id is the CSC
                            position,
* ``weight``   uint32[m]    IC: live-edge threshold ``thr`` (edge live iff a
                            uniform 32-bit draw ``r < thr``, i.e. probability
                            ``thr / 2**32``); LT: cumulative in-weight table
                            ``cum`` (non-decreasing within a column, last entry
                            of every non-empty column is ``2**32 - 1``).

The diffusion models these encode are the IC and LT models of the paper's
Section II-A; the weighted-cascade rule ``p(u,v) = 1/indeg(v)`` and the uniform
LT in-weights normalised to sum to one are the workload definitions used for
the synthetic stand-ins of the paper's SNAP graphs (Section V-A, Table I).
"""

from __future__ import annotations

import dataclasses
import hashlib
import os
from pathlib import Path

import numpy as np

TWO32 = 1 << 32
U32_MAX = TWO32 - 1
_CACHE_VERSION = "v3"


@dataclasses.dataclass
class Graph:
    name: str
    n: int
    m: int
    col_off: np.ndarray  # uint64[n+1]
    row_src: np.ndarray  # uint32[m]
    weight: np.ndarray  # uint32[m]
    model: str  # "ic" | "lt"

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.uint64(self.n).tobytes())
        h.update(np.uint64(self.m).tobytes())
        h.update(self.model.encode())
        for a in (self.col_off, self.row_src, self.weight):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def indeg(self) -> np.ndarray:
        return np.diff(self.col_off).astype(np.int64)

    def nbytes(self) -> int:
        return self.col_off.nbytes + self.row_src.nbytes + self.weight.nbytes


# ---------------------------------------------------------------------------
# Edge-list generators: directed, self-loops and duplicate edges removed.
# Candidate edges are drawn independently; among the distinct non-loop
# candidates exactly m are kept (a seeded uniform choice), and vertex ids are
# relabelled by a seeded random permutation (the Graph500 practice).
# ---------------------------------------------------------------------------


def _keep_m_distinct(n: int, draw, m: int, rng: np.random.Generator):
    """Draw candidate (src, dst) batches until at least m distinct non-loop
    pairs exist, keep a uniform random m of them, permute vertex ids."""
    keys = np.empty(0, dtype=np.int64)
    batch = int(m * 1.06) + 1024
    while True:
        s, d = draw(batch)
        ok = s != d
        keys = np.unique(np.concatenate([keys, s[ok].astype(np.int64) * n + d[ok]]))
        if keys.size >= m:
            break
        batch = max(1024, int((m - keys.size) * 1.5) + 1024)
    if keys.size > m:
        keep = rng.choice(keys.size, size=m, replace=False)
        keep.sort()
        keys = keys[keep]
    src = keys // n
    dst = keys % n
    perm = rng.permutation(n).astype(np.int64)
    return perm[src], perm[dst]


def _rmat_code_table(levels: int, quanta) -> np.ndarray:
    """Joint quadrant codes of `levels` R-MAT levels for every integer in
    [0, 100**levels): base-100 digit i picks level i's quadrant (a, b, c, d
    cover quanta[0..3] of the 100 values); the code holds the source bits
    in bits [levels, 2*levels) and the destination bits in [0, levels)."""
    per = np.repeat(np.arange(4, dtype=np.uint8), quanta)  # 100 entries
    x = np.arange(100 ** levels, dtype=np.int64)
    sbits = np.zeros(x.size, dtype=np.uint8)
    dbits = np.zeros(x.size, dtype=np.uint8)
    for _ in range(levels):
        qd = per[x % 100]
        x //= 100
        sbits = (sbits << 1) | (qd >> 1)
        dbits = (dbits << 1) | (qd & 1)
    return (sbits << levels) | dbits


def rmat_edges(scale: int, m: int, a=0.57, b=0.19, c=0.19, seed: int = 1):
    """R-MAT edges (Chakrabarti et al.) on 2**scale vertices; quadrant
    probabilities a (src bit 0, dst bit 0), b (0,1), c (1,0), d = 1-a-b-c.
    The probabilities are whole percentages, so up to three levels are drawn
    at once, exactly, from one uniform integer in [0, 10**6)."""
    n = 1 << scale
    rng = np.random.Generator(np.random.PCG64(seed))
    quanta = [int(round(100 * x)) for x in (a, b, c)]
    quanta.append(100 - sum(quanta))
    assert all(abs(q / 100 - x) < 1e-12 for q, x in zip(quanta, (a, b, c, 1 - a - b - c)))
    tables = {}

    def draw(bsz):
        s = np.zeros(bsz, dtype=np.uint32)
        d = np.zeros(bsz, dtype=np.uint32)
        left = scale
        while left:
            lv = min(3, left)
            left -= lv
            if lv not in tables:
                tables[lv] = _rmat_code_table(lv, quanta)
            code = tables[lv][rng.integers(0, 100 ** lv, size=bsz, dtype=np.uint32)]
            np.left_shift(s, lv, out=s)
            np.bitwise_or(s, code >> lv, out=s)
            np.left_shift(d, lv, out=d)
            np.bitwise_or(d, code & ((1 << lv) - 1), out=d)
        return s.astype(np.int64), d.astype(np.int64)

    src, dst = _keep_m_distinct(n, draw, m, rng)
    return n, src, dst, rng


def _chung_lu_weights(n: int, m: int, gamma: float) -> np.ndarray:
    """Expected degrees d_i = c (i + i0)^(-1/(gamma-1)) with sum m and d_0 = sqrt(m)."""
    alpha = 1.0 / (gamma - 1.0)
    idx = np.arange(n, dtype=np.float64)
    target = np.sqrt(float(m))

    def f(i0):
        return np.sum((i0 / (idx + i0)) ** alpha) - target

    lo, hi = 1e-9, float(n) * 1e6
    for _ in range(80):
        mid = np.sqrt(lo * hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    i0 = np.sqrt(lo * hi)
    w = (i0 / (idx + i0)) ** alpha
    return w * (float(m) / w.sum())


def chung_lu_edges(n: int, m: int, gamma: float, seed: int = 1):
    """Directed Chung-Lu edges: both endpoints of a candidate edge are drawn
    with probability proportional to the same expected-degree sequence
    (correlated in/out degrees). A batch of B candidates is drawn as
    multinomial endpoint counts, with the sources randomly paired to the
    targets, which is the same distribution as B independent draws."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = _chung_lu_weights(n, m, gamma)
    p = w / w.sum()
    ids = np.arange(n, dtype=np.int64)

    def draw(bsz):
        s = np.repeat(ids, rng.multinomial(bsz, p))
        d = np.repeat(ids, rng.multinomial(bsz, p))
        rng.shuffle(s)
        return s, d

    src, dst = _keep_m_distinct(n, draw, m, rng)
    return n, src, dst, rng


def to_csc(n: int, src: np.ndarray, dst: np.ndarray):
    """CSC of in-edges: columns by destination, sources ascending in a column."""
    key = np.sort(dst.astype(np.int64) * n + src.astype(np.int64))
    row_src = (key % n).astype(np.uint32)
    cnt = np.bincount(key // n, minlength=n).astype(np.uint64)
    col_off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(cnt, out=col_off[1:])
    return col_off, row_src


# ---------------------------------------------------------------------------
# Parameter encodings
# ---------------------------------------------------------------------------


def ic_wc_thresholds(col_off: np.ndarray) -> np.ndarray:
    """Weighted cascade p(u,v) = 1/indeg(v) as thr = min(2^32-1, floor(2^32/indeg))."""
    deg = np.diff(col_off).astype(np.int64)
    per_col = np.minimum(U32_MAX, np.where(deg > 0, TWO32 // np.maximum(deg, 1), 0))
    return np.repeat(per_col, deg).astype(np.uint32)


def ic_uniform_thresholds(m: int, p: float) -> np.ndarray:
    """Uniform edge probability p as thr = min(2^32-1, floor(p * 2^32))."""
    t = min(U32_MAX, int(np.floor(p * float(TWO32))))
    return np.full(m, t, dtype=np.uint32)


def ic_random_thresholds(m: int, rng: np.random.Generator) -> np.ndarray:
    """Edge probabilities p ~ U[0,1) drawn per edge (the paper's IC setting),
    as thr = floor(p * 2^32)."""
    return rng.integers(0, TWO32, size=m, dtype=np.uint64).astype(np.uint32)


def lt_cumulative(col_off: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """LT in-weights w ~ U[0,1) per in-edge (CSC order), normalised per column
    to sum to 1, encoded as a cumulative table cum = min(2^32-1,
    floor(2^32 * prefix)), with the last entry of each column set to 2^32-1."""
    m = int(col_off[-1])
    n = col_off.size - 1
    w = rng.random(m)
    deg = np.diff(col_off).astype(np.int64)
    beg = col_off[:-1].astype(np.int64)
    csum = np.cumsum(w)
    base = np.zeros(n, dtype=np.float64)
    nz = deg > 0
    base[nz & (beg > 0)] = csum[beg[nz & (beg > 0)] - 1]
    tot = np.zeros(n, dtype=np.float64)
    tot[nz] = csum[beg[nz] + deg[nz] - 1] - base[nz]
    col = np.repeat(np.arange(n), deg)
    prefix = csum - base[col]
    t = tot[col]
    # a column whose weights are all exactly zero gets equal weights
    zero_col = t <= 0.0
    if np.any(zero_col):
        pos = np.arange(m) - beg[col] + 1
        prefix = np.where(zero_col, pos, prefix)
        t = np.where(zero_col, deg[col].astype(np.float64), t)
    frac = prefix / t
    cum = np.minimum(float(U32_MAX), np.floor(frac * float(TWO32))).astype(np.uint64)
    last = (beg + deg - 1)[nz]
    cum[last] = U32_MAX
    return cum.astype(np.uint32)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

#: name -> (generator spec, model, encoding, IMM parameters)
WORKLOADS = {
    # R-MAT scale 12, 32768 edges, weighted cascade; k=10, eps=0.5, ell=1, seed 42
    "rmat12_wc": dict(gen=("rmat", 12, 32768), model="ic", enc=("wc",),
                      k=10, eps=0.5, ell=1.0, seed=42),
    # Youtube-shaped directed Chung-Lu (gamma 2.1), IC p = 0.01; k=50, eps=0.13
    "youtube_ic": dict(gen=("chunglu", 1134890, 2987624, 2.1), model="ic",
                       enc=("uniform", 0.01), k=50, eps=0.13, ell=1.0, seed=42),
    # LiveJournal-shaped directed Chung-Lu (gamma 2.0), LT; k=50, eps=0.13
    "lj_lt": dict(gen=("chunglu", 4800000, 69000000, 2.0), model="lt",
                  enc=("lt",), k=50, eps=0.13, ell=1.0, seed=42),
    # one-tenth-size versions of the two above (same shape rules)
    "youtube_ic_s": dict(gen=("chunglu", 113489, 298762, 2.1), model="ic",
                         enc=("uniform", 0.01), k=50, eps=0.13, ell=1.0, seed=42),
    "lj_lt_s": dict(gen=("chunglu", 480000, 6900000, 2.0), model="lt",
                    enc=("lt",), k=50, eps=0.13, ell=1.0, seed=42),
    # smaller LT graph for fast parity runs
    "cl_lt_xs": dict(gen=("chunglu", 20000, 160000, 2.0), model="lt",
                     enc=("lt",), k=10, eps=0.3, ell=1.0, seed=42),
    # R-MAT scale 12 with uniform p = 0.1: a quarter of the sets are giant
    # (hundreds to ~1000 vertices), the rest tiny
    "rmat12_p10": dict(gen=("rmat", 12, 32768), model="ic", enc=("uniform", 0.1),
                       k=10, eps=0.5, ell=1.0, seed=42),
    # R-MAT scale 12 under LT (same topology rule as rmat12_wc)
    "rmat12_lt": dict(gen=("rmat", 12, 32768), model="lt", enc=("lt",),
                      k=10, eps=0.5, ell=1.0, seed=42),
    # the largest instance shape of the multi-instance batch (scale 20,
    # average degree 32, weighted cascade)
    "rmat20_wc": dict(gen=("rmat", 20, 32 << 20), model="ic", enc=("wc",),
                      k=50, eps=0.13, ell=1.0, seed=42),
    # dense IC sets: the Youtube-shaped graph with p ~ U[0,1) per edge (the
    # paper's IC edge weights), and its one-tenth-size version
    "youtube_icu": dict(gen=("chunglu", 1134890, 2987624, 2.1), model="ic",
                        enc=("urand",), k=50, eps=0.13, ell=1.0, seed=42),
    "youtube_icu_s": dict(gen=("chunglu", 113489, 298762, 2.1), model="ic",
                          enc=("urand",), k=50, eps=0.5, ell=1.0, seed=42),
    # served-stream graphs
    "rmat18_wc": dict(gen=("rmat", 18, 2097152), model="ic", enc=("wc",),
                      k=50, eps=0.13, ell=1.0, seed=42),
    "orkut_lt": dict(gen=("chunglu", 3000000, 117000000, 2.0), model="lt",
                     enc=("lt",), k=50, eps=0.13, ell=1.0, seed=42),
}


def _cache_dir() -> Path:
    d = os.environ.get("IMM_GRAPH_CACHE")
    if d:
        return Path(d)
    return Path(__file__).resolve().parent.parent / ".graph_cache"


def _build(name: str, gen, model: str, enc, gseed: int) -> Graph:
    if gen[0] == "rmat":
        _, scale, m = gen
        n, src, dst, rng = rmat_edges(scale, m, seed=gseed)
    elif gen[0] == "chunglu":
        _, n, m, gamma = gen
        n, src, dst, rng = chung_lu_edges(n, m, gamma, seed=gseed)
    else:
        raise ValueError(gen)
    col_off, row_src = to_csc(n, src, dst)
    if enc[0] == "wc":
        w = ic_wc_thresholds(col_off)
    elif enc[0] == "uniform":
        w = ic_uniform_thresholds(row_src.size, enc[1])
    elif enc[0] == "lt":
        w = lt_cumulative(col_off, rng)
    elif enc[0] == "urand":
        w = ic_random_thresholds(row_src.size, rng)
    else:
        raise ValueError(enc)
    return Graph(name, int(n), int(row_src.size), col_off, row_src, w, model)


def make_graph(name: str, gen=None, model=None, enc=None, gseed: int = 1,
               cache: bool = True) -> Graph:
    """Build (or load from the on-disk cache) a named synthetic graph."""
    if gen is None:
        spec = WORKLOADS[name]
        gen, model, enc = spec["gen"], spec["model"], spec["enc"]
    key = f"{name}-{_CACHE_VERSION}-" + hashlib.sha1(
        repr((gen, model, enc, gseed)).encode()).hexdigest()[:12]
    path = _cache_dir() / f"{key}.npz"
    if cache and path.exists():
        z = np.load(path, allow_pickle=False)
        return Graph(name, int(z["n"]), int(z["m"]), z["col_off"], z["row_src"],
                     z["weight"], str(z["model"]))
    g = _build(name, gen, model, enc, gseed)
    if cache:
        path.parent.mkdir(parents=True, exist_ok=True)
        tmp = path.with_suffix(f".{os.getpid()}.tmp.npz")
        np.savez(tmp, n=g.n, m=g.m, col_off=g.col_off, row_src=g.row_src,
                 weight=g.weight, model=np.array(g.model))
        os.replace(tmp, path)
    return g


def _make_cached(kw: dict) -> str:
    make_graph(**kw)
    return kw["name"]


def make_graphs(specs, workers: int = 8) -> None:
    """Build the graphs of ``specs`` (keyword dicts of make_graph) into the
    on-disk cache, in fresh worker processes (spawned, so a caller that has
    already initialised a GPU runtime forks nothing); make_graph then loads
    each one from the cache."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    todo = [dict(kw, cache=True) for kw in specs]
    if not todo:
        return
    with ProcessPoolExecutor(max_workers=max(1, min(workers, len(todo))),
                             mp_context=mp.get_context("spawn")) as ex:
        for _ in ex.map(_make_cached, todo):
            pass


def tiny_graph(n: int, edges, model: str, params) -> Graph:
    """Explicit small graph. ``edges`` is a list of (u, v); ``params`` gives,
    per edge in the same order, the IC probability numerator thr (int) or, for
    LT, the raw (non-cumulative) 32-bit weight quanta; LT columns are turned
    into cumulative tables here (the caller keeps sum <= 2^32 - 1)."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    prm = np.asarray(params, dtype=np.int64)
    order = np.lexsort((e[:, 0], e[:, 1]))
    e, prm = e[order], prm[order]
    col_off, row_src = to_csc(n, e[:, 0], e[:, 1])
    if model == "ic":
        w = prm.astype(np.uint32)
    else:
        w = np.zeros(len(prm), dtype=np.uint64)
        for v in range(n):
            b, t = int(col_off[v]), int(col_off[v + 1])
            acc = 0
            for i in range(b, t):
                acc += int(prm[i])
                w[i] = acc
        assert np.all(w <= U32_MAX)
        w = w.astype(np.uint32)
    return Graph("tiny", n, int(row_src.size), col_off, row_src, w, model)


def batch_instances(count: int = 64, master_seed: int = 2024, max_scale: int = 20):
    """The multi-instance workload: per instance a weighted-cascade R-MAT graph
    with scale ~ U{12..20} and average degree ~ U{4..32}, k ~ {5,10,25,50},
    eps ~ {0.5,0.3,0.13}, ell = 1 and Philox seed 42 + i. ``max_scale`` caps
    the scale (the other draws are unchanged) for test-sized batches."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    out = []
    for i in range(count):
        scale = min(int(rng.integers(12, 21)), max_scale)
        deg = int(rng.integers(4, 33))
        k = int(rng.choice([5, 10, 25, 50]))
        eps = float(rng.choice([0.5, 0.3, 0.13]))
        gseed = int(rng.integers(1, 1 << 31))
        out.append(dict(name=f"rmat{scale}x{deg}_s{gseed}",
                        gen=("rmat", scale, (1 << scale) * deg), model="ic",
                        enc=("wc",), gseed=gseed, k=k, eps=eps, ell=1.0,
                        seed=42 + i))
    return out


def served_queries(count: int = 1000, rate: float = 50.0, arrival_seed: int = 7,
                   graphs=("rmat18_wc", "youtube_ic", "orkut_lt")):
    """Poisson query stream: arrival times (s), graph name, k ~ {10,50,100},
    eps ~ {0.5,0.13}, ell = 1 and seed 1000 + query index."""
    rng = np.random.Generator(np.random.PCG64(arrival_seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for i in range(count):
        out.append(dict(t=float(t[i]), graph=str(rng.choice(list(graphs))),
                        k=int(rng.choice([10, 50, 100])),
                        eps=float(rng.choice([0.5, 0.13])), ell=1.0,
                        seed=1000 + i))
    return out
