"""CPU oracle of the IMM hot path (ctypes binding of ``imm_oracle.c``).

TEST INFRASTRUCTURE: only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module. It shares no code with
the GPU library. See ``imm_oracle.c`` for what each function computes and the
passage of the paper it follows.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "imm_oracle.c"
_LIB = _HERE / "liboracle.so"

IC, LT = 0, 1
_ERR = {1: "EINVAL", 2: "ENOMEM", 3: "EOVERFLOW"}


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (plain C11, no FP contraction, OpenMP)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(f".so.tmp{os.getpid()}")
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp",
                        "-shared", "-fPIC", "-o", str(tmp), str(_SRC), "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


class ImmInfo(C.Structure):
    _fields_ = [("theta", C.c_uint64), ("rounds", C.c_uint32), ("n_targets", C.c_uint32),
                ("lb", C.c_double), ("covered", C.c_uint64),
                ("lambda_prime", C.c_double), ("lambda_star", C.c_double),
                ("i_max", C.c_uint32), ("pad", C.c_uint32),
                ("targets", C.c_uint64 * 64), ("round_cov", C.c_uint64 * 64),
                ("sigma_up", C.c_double), ("alpha", C.c_double),
                ("round_cov2", C.c_uint64 * 64)]


#: sampling schedules of imm(): IMM as in Algorithm 1 (the rounds' sets are
#: reused by the final selection), IMM with a fresh final pool, early stopping
SCHED_IMM, SCHED_FRESH, SCHED_EARLY = 0, 1, 2


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(str(_LIB))
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        L.oracle_philox4x32_10.argtypes = [u32p, C.c_uint64, u32p]
        L.oracle_philox_many.argtypes = [u32p, C.c_uint64, C.c_uint64, u32p]
        L.oracle_philox_many.restype = None
        L.oracle_root.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32]
        L.oracle_root.restype = C.c_uint32
        L.oracle_ic_draw.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.oracle_ic_draw.restype = C.c_uint32
        L.oracle_lt_draw.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32]
        L.oracle_lt_draw.restype = C.c_uint32
        L.oracle_ic_live.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, u32p,
                                     np.ctypeslib.ndpointer(np.uint8, flags="C")]
        L.oracle_ic_live.restype = None
        L.oracle_rrr_set.argtypes = [C.c_uint32, u64p, u32p, u32p, C.c_int, C.c_uint64,
                                     C.c_uint64, u32p]
        L.oracle_rrr_set.restype = C.c_uint32
        L.oracle_pool_create.restype = C.c_void_p
        L.oracle_pool_destroy.argtypes = [C.c_void_p]
        L.oracle_pool_nsets.argtypes = [C.c_void_p]
        L.oracle_pool_nsets.restype = C.c_uint64
        L.oracle_pool_nentries.argtypes = [C.c_void_p]
        L.oracle_pool_nentries.restype = C.c_uint64
        L.oracle_pool_work.argtypes = [C.c_void_p]
        L.oracle_pool_work.restype = C.c_uint64
        L.oracle_pool_copy.argtypes = [C.c_void_p, u64p, u32p]
        L.oracle_pool_extend.argtypes = [C.c_void_p, C.c_uint32, u64p, u32p, u32p, C.c_int,
                                         C.c_uint64, C.c_uint64, C.c_int]
        L.oracle_pool_extend.restype = C.c_int
        L.oracle_counts.argtypes = [C.c_uint32, u64p, u32p, C.c_uint64, u32p]
        L.oracle_greedy.argtypes = [C.c_uint32, u64p, u32p, C.c_uint64, C.c_uint32, u32p, u64p]
        L.oracle_greedy.restype = C.c_uint64
        L.oracle_theta_plan.argtypes = [C.c_uint32, C.c_uint32, C.c_double, C.c_double,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_uint32)]
        L.oracle_theta_plan.restype = C.c_int
        L.oracle_imm.argtypes = [C.c_uint32, u64p, u32p, u32p, C.c_int, C.c_uint32,
                                 C.c_double, C.c_double, C.c_uint64, C.c_int, C.c_void_p,
                                 u32p, u64p, C.POINTER(ImmInfo)]
        L.oracle_imm.restype = C.c_int
        L.oracle_imm_ex.argtypes = [C.c_uint32, u64p, u32p, u32p, C.c_int, C.c_uint32,
                                    C.c_double, C.c_double, C.c_uint64, C.c_int, C.c_int,
                                    C.c_void_p, u32p, u64p, C.POINTER(ImmInfo)]
        L.oracle_imm_ex.restype = C.c_int
        L.oracle_coverage.argtypes = [C.c_uint32, u64p, u32p, C.c_uint64, u32p, C.c_uint32]
        L.oracle_coverage.restype = C.c_uint64
        L.oracle_early_plan.argtypes = [C.c_uint32, C.c_uint32, C.c_double, C.c_double,
                                        C.POINTER(C.c_double), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_double)]
        L.oracle_early_plan.restype = C.c_int
        L.oracle_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc:
        raise RuntimeError(f"oracle error {_ERR.get(rc, rc)}")


def _model(g):
    return IC if g.model == "ic" else LT


def _arrays(g):
    return (np.ascontiguousarray(g.col_off, dtype=np.uint64),
            np.ascontiguousarray(g.row_src, dtype=np.uint32),
            np.ascontiguousarray(g.weight, dtype=np.uint32))


def philox4x32_10(ctr, key: int) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(4)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(c, int(key), out)
    return out


def philox_many(ctr, key: int) -> np.ndarray:
    """Philox4x32-10 of every row of ctr (uint32[count, 4]) under one key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    lib().oracle_philox_many(c, c.shape[0], int(key), out)
    return out


def root(seed: int, s: int, n: int) -> int:
    return int(lib().oracle_root(seed, s, n))


def ic_draw(seed: int, s: int, e: int) -> int:
    return int(lib().oracle_ic_draw(seed, s, e))


def lt_draw(seed: int, s: int, v: int) -> int:
    return int(lib().oracle_lt_draw(seed, s, v))


def ic_live(g, seed: int, s: int) -> np.ndarray:
    """Live-edge mask (uint8[m]) of sample s under IC."""
    w = np.ascontiguousarray(g.weight, dtype=np.uint32)
    out = np.zeros(max(g.m, 1), dtype=np.uint8)
    lib().oracle_ic_live(seed, s, g.m, w if g.m else np.zeros(1, np.uint32), out)
    return out[: g.m]


def rrr_set(g, seed: int, s: int) -> np.ndarray:
    """One RRR set of sample s, in discovery order."""
    co, rs, w = _arrays(g)
    buf = np.zeros(g.n, dtype=np.uint32)
    size = lib().oracle_rrr_set(g.n, co, rs, w, _model(g), seed, s, buf)
    return buf[:size].copy()


class Pool:
    """Sets in sample-id order, appended by ``extend``."""

    def __init__(self):
        self._p = lib().oracle_pool_create()
        if not self._p:
            raise MemoryError

    def __del__(self):
        if getattr(self, "_p", None):
            lib().oracle_pool_destroy(self._p)
            self._p = None

    def extend(self, g, seed: int, target: int, threads: int = 1):
        co, rs, w = _arrays(g)
        _check(lib().oracle_pool_extend(self._p, g.n, co, rs, w, _model(g), seed, target,
                                        threads))

    @property
    def n_sets(self) -> int:
        return int(lib().oracle_pool_nsets(self._p))

    @property
    def n_entries(self) -> int:
        return int(lib().oracle_pool_nentries(self._p))

    @property
    def work(self) -> int:
        return int(lib().oracle_pool_work(self._p))

    def arrays(self):
        so = np.zeros(self.n_sets + 1, dtype=np.uint64)
        sv = np.zeros(max(self.n_entries, 1), dtype=np.uint32)
        lib().oracle_pool_copy(self._p, so, sv)
        return so, sv[: self.n_entries]


def sample(g, seed: int, first: int, count: int, threads: int = 1):
    """Sets of sample ids [first, first+count): (set_off, set_vtx), discovery order."""
    if first:
        # a pool appends from its own size, so other ranges go set by set
        offs = [0]
        vt = []
        for s in range(first, first + count):
            m = rrr_set(g, seed, s)
            vt.append(m)
            offs.append(offs[-1] + m.size)
        return (np.asarray(offs, dtype=np.uint64),
                np.concatenate(vt).astype(np.uint32) if vt else np.zeros(0, np.uint32))
    p = Pool()
    p.extend(g, seed, count, threads)
    return p.arrays()


def counts(n: int, set_off, set_vtx) -> np.ndarray:
    so = np.ascontiguousarray(set_off, dtype=np.uint64)
    sv = np.ascontiguousarray(set_vtx, dtype=np.uint32)
    if sv.size == 0:
        sv = np.zeros(1, dtype=np.uint32)
    out = np.zeros(n, dtype=np.uint32)
    lib().oracle_counts(n, so, sv, so.size - 1, out)
    return out


def greedy(n: int, set_off, set_vtx, k: int):
    """Algorithm 2 greedy: (seeds uint32[k], gains uint64[k], covered)."""
    so = np.ascontiguousarray(set_off, dtype=np.uint64)
    sv = np.ascontiguousarray(set_vtx, dtype=np.uint32)
    if sv.size == 0:
        sv = np.zeros(1, dtype=np.uint32)
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    cov = lib().oracle_greedy(n, so, sv, so.size - 1, k, seeds, gains)
    if cov == (1 << 64) - 1:
        raise MemoryError
    return seeds, gains, int(cov)


def theta_plan(n: int, k: int, eps: float, ell: float):
    lp, ls, im = C.c_double(), C.c_double(), C.c_uint32()
    _check(lib().oracle_theta_plan(n, k, eps, ell, C.byref(lp), C.byref(ls), C.byref(im)))
    return lp.value, ls.value, im.value


def imm(g, k: int, eps: float, ell: float, seed: int, threads: int = 1,
        keep_pool: bool = False, schedule: int = SCHED_IMM):
    """Full IMM run. Returns a dict with seeds, gains, theta, rounds, lb,
    covered, targets, round_cov and (optionally) the pool arrays of the final
    selection; with SCHED_EARLY also sigma_up, alpha and round_cov2."""
    co, rs, w = _arrays(g)
    pool = Pool() if keep_pool else None
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    info = ImmInfo()
    _check(lib().oracle_imm_ex(g.n, co, rs, w, _model(g), k, eps, ell, seed, threads, schedule,
                               pool._p if pool else None, seeds, gains, C.byref(info)))
    out = dict(seeds=seeds, gains=gains, theta=int(info.theta), rounds=int(info.rounds),
               lb=float(info.lb), covered=int(info.covered),
               lambda_prime=info.lambda_prime, lambda_star=info.lambda_star,
               i_max=int(info.i_max),
               targets=[int(info.targets[i]) for i in range(info.n_targets)],
               round_cov=[int(info.round_cov[i]) for i in range(info.rounds)])
    if schedule == SCHED_EARLY:
        out["sigma_up"] = info.sigma_up
        out["alpha"] = info.alpha
        out["round_cov2"] = [int(info.round_cov2[i]) for i in range(info.rounds)]
    if pool is not None:
        out["set_off"], out["set_vtx"] = pool.arrays()
        out["work"] = pool.work
    return out


def coverage(n: int, set_off, set_vtx, seeds) -> int:
    """Number of sets with at least one member among seeds."""
    so = np.ascontiguousarray(set_off, dtype=np.uint64)
    sv = np.ascontiguousarray(set_vtx, dtype=np.uint32)
    if sv.size == 0:
        sv = np.zeros(1, dtype=np.uint32)
    sd = np.ascontiguousarray(seeds, dtype=np.uint32)
    c = lib().oracle_coverage(n, so, sv, so.size - 1, sd, sd.size)
    if c == (1 << 64) - 1:
        raise MemoryError
    return int(c)


def early_plan(n: int, k: int, eps: float, ell: float):
    """The early-stopping schedule's (theta_0, i_max, a)."""
    t0, im, a = C.c_double(), C.c_uint32(), C.c_double()
    _check(lib().oracle_early_plan(n, k, eps, ell, C.byref(t0), C.byref(im), C.byref(a)))
    return t0.value, im.value, a.value


def max_threads() -> int:
    return int(lib().oracle_max_threads())
