"""Python binding of libimm (include/imm.h): argument marshalling only.

Every entry point has the name of the C function it calls. Arrays may be
numpy arrays (host memory) or torch CUDA tensors (device memory; the call then
passes IMM_DEVICE_PTRS). ``stream`` may be None (the null stream), an int
holding a hipStream_t, or a ``torch.cuda.Stream``.

The compiled library must be present: importing this package fails loudly
when ``libimm.so`` has not been built (``python -m paper_2411_09473_amd.build``).
"""

from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "libimm.so"
# One HIP runtime per process: PyTorch ships its own libamdhip64 (soname
# libamdhip64.so.7). Loading it first lets libimm's dependency on that soname
# resolve to the same runtime instead of a second copy from /opt/rocm.
try:
    import torch  # noqa: F401
except ImportError:
    pass
if not _LIB_PATH.exists():
    raise ImportError(
        f"libimm.so not found at {_LIB_PATH}; build it with "
        "`python -m paper_2411_09473_amd.build` (hipcc, gfx950)")
_lib = C.CDLL(str(_LIB_PATH))

IMM_OK, IMM_EINVAL, IMM_ENOMEM, IMM_EOVERFLOW, IMM_EDEVICE, IMM_EBUSY, IMM_ECANCELLED = range(7)
IMM_IC, IMM_LT = 0, 1
IMM_DEVICE_PTRS, IMM_KEEP_POOL, IMM_TIMING, IMM_GRAPH_SELECT = 0x1, 0x2, 0x4, 0x8
IMM_FRESH_FINAL, IMM_EARLY_STOP = 0x10, 0x20
IMM_UPDATE_DECREMENT, IMM_UPDATE_RECOUNT = 0x40, 0x80
IMM_LIST_SETS = 0x100
IMM_GRAPH_SAMPLE = 0x200
_NAMES = {1: "IMM_EINVAL", 2: "IMM_ENOMEM", 3: "IMM_EOVERFLOW", 4: "IMM_EDEVICE",
          5: "IMM_EBUSY", 6: "IMM_ECANCELLED"}


class ImmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class imm_params(C.Structure):
    _fields_ = [("k", C.c_uint32), ("flags", C.c_uint32), ("epsilon", C.c_double),
                ("ell", C.c_double), ("seed", C.c_uint64), ("max_device_bytes", C.c_uint64)]


class imm_stats(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_sample", C.c_double), ("ms_compact", C.c_double),
                ("ms_index", C.c_double), ("ms_select", C.c_double),
                ("ms_sample_main", C.c_double), ("main_launches", C.c_uint64),
                ("sets", C.c_uint64), ("entries", C.c_uint64), ("edges", C.c_uint64),
                ("live", C.c_uint64), ("deferred", C.c_uint64), ("main_sets", C.c_uint64),
                ("main_entries", C.c_uint64), ("main_edges", C.c_uint64),
                ("main_live", C.c_uint64), ("ms_sample_big", C.c_double),
                ("big_launches", C.c_uint64), ("rounds", C.c_uint32), ("team", C.c_uint32),
                ("ms_sample_lane", C.c_double), ("lane_launches", C.c_uint64),
                ("lane_sets", C.c_uint64), ("lane_edges", C.c_uint64),
                ("big_block", C.c_uint32), ("bloom_bits", C.c_uint32),
                ("device_bytes", C.c_uint64), ("ms_queue", C.c_double),
                ("walk_lanes", C.c_uint32), ("select_graphs", C.c_uint32),
                ("select_captures", C.c_uint32), ("dense_sets", C.c_uint32),
                ("sample_graphs", C.c_uint32), ("sample_captures", C.c_uint32),
                ("cand_steps", C.c_uint32), ("cand_halts", C.c_uint32),
                ("spec_rounds", C.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


_vp = C.c_void_p
_u32, _u64, _dbl, _int = C.c_uint32, C.c_uint64, C.c_double, C.c_int
_P = C.POINTER

_lib.imm_last_error.restype = C.c_char_p
_sig = {
    "imm_graph_create": [_u32, _u64, _vp, _vp, _vp, _int, _u32, _vp, _P(_vp)],
    "imm_graph_destroy": [_vp],
    "imm_graph_info": [_vp, _P(_u32), _P(_u64), _P(_int), _P(_u64)],
    "imm_theta_plan": [_u32, _u32, _dbl, _dbl, _P(_dbl), _P(_dbl), _P(_u32)],
    "imm_run": [_vp, _P(imm_params), _vp, _P(_vp)],
    "imm_run_batch": [_vp, _vp, _u32, _vp, _vp],
    "imm_result_info": [_vp, _P(_u64), _P(_u32), _P(_dbl), _P(_u64)],
    "imm_result_seeds": [_vp, _vp, _vp],
    "imm_result_targets": [_vp, _P(_u32), _vp, _vp],
    "imm_result_pool": [_vp, _P(_u64), _P(_u64), _vp, _vp],
    "imm_result_early": [_vp, _P(_dbl), _P(_dbl), _vp],
    "imm_result_stats": [_vp, _P(imm_stats)],
    "imm_sample": [_vp, _u64, _u64, _u64, _u32, _vp, _P(_vp)],
    "imm_pool_info": [_vp, _P(_u64), _P(_u64), _P(imm_stats)],
    "imm_pool_export": [_vp, _vp, _vp, _vp],
    "imm_greedy": [_u32, _vp, _vp, _u64, _u32, _u32, _vp, _vp, _vp, _P(_u64)],
    "imm_greedy_static": [_u32, _vp, _vp, _u64, _u32, _u32, _vp, _vp, _vp, _P(_u64)],
    "imm_philox4x32_10": [_vp, _u64, _u64, _u32, _vp, _vp],
    "imm_server_create": [_u64, _u32, _P(_vp)],
    "imm_server_submit": [_vp, _vp, _P(imm_params), _P(_u64)],
    "imm_server_poll": [_vp, _u64, _int, _P(_vp)],
    "imm_server_cancel": [_vp, _u64],
    "imm_server_info": [_vp, _P(_u64), _P(_u32), _P(_u64)],
    "imm_server_destroy": [_vp],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _int
_lib.imm_result_destroy.argtypes = [_vp]
_lib.imm_result_destroy.restype = None
_lib.imm_pool_destroy.argtypes = [_vp]
_lib.imm_pool_destroy.restype = None

#: exported C symbols, as declared in include/imm.h
SYMBOLS = tuple(_sig) + ("imm_last_error", "imm_result_destroy", "imm_pool_destroy")


def library_path() -> str:
    return str(_LIB_PATH)


def _check(st: int):
    if st != IMM_OK:
        raise ImmError(st, _lib.imm_last_error().decode(errors="replace"))


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream or None
    return int(getattr(stream, "cuda_stream"))


def _is_dev(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def _ptr(a, dtype):
    """(pointer, keepalive, is_device) for a numpy array or torch tensor."""
    if a is None:
        return None, None, False
    if _is_dev(a):
        if not a.is_contiguous():
            raise ValueError("device tensors must be contiguous")
        return a.data_ptr(), a, True
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data, arr, False


class Graph:
    """Owning handle of a resident imm_graph."""

    def __init__(self, handle, n, m, model):
        self._h = C.c_void_p(handle)
        self.n, self.m, self.model = n, m, model

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._h.value:
            _check(_lib.imm_graph_destroy(self._h))
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def imm_graph_create(n, m, col_off, row_src, weight, model, flags=0, stream=None) -> Graph:
    if isinstance(model, str):
        model = IMM_IC if model == "ic" else IMM_LT
    p0, k0, d0 = _ptr(col_off, np.uint64)
    p1, k1, d1 = _ptr(row_src, np.uint32)
    p2, k2, d2 = _ptr(weight, np.uint32)
    if d0 or d1 or d2:
        if not (d0 and d1 and d2):
            raise ValueError("either all arrays are device tensors or none")
        flags |= IMM_DEVICE_PTRS
    out = C.c_void_p()
    _check(_lib.imm_graph_create(n, m, p0, p1, p2, model, flags, _stream(stream), C.byref(out)))
    return Graph(out.value, n, m, model)


def imm_graph_destroy(g: Graph):
    g.close()


def imm_graph_info(g: Graph):
    n, m, mo, b = _u32(), _u64(), _int(), _u64()
    _check(_lib.imm_graph_info(g.handle, C.byref(n), C.byref(m), C.byref(mo), C.byref(b)))
    return dict(n=n.value, m=m.value, model=mo.value, device_bytes=b.value)


def imm_theta_plan(n, k, eps, ell):
    lp, ls, im = _dbl(), _dbl(), _u32()
    _check(_lib.imm_theta_plan(n, k, eps, ell, C.byref(lp), C.byref(ls), C.byref(im)))
    return lp.value, ls.value, im.value


class Result:
    """Owning handle of an imm_result, with its fields copied out."""

    def __init__(self, handle, k):
        self._h = C.c_void_p(handle)
        th, rd, lb, cv = _u64(), _u32(), _dbl(), _u64()
        _check(_lib.imm_result_info(self._h, C.byref(th), C.byref(rd), C.byref(lb), C.byref(cv)))
        self.theta, self.rounds, self.lb, self.covered = th.value, rd.value, lb.value, cv.value
        self.seeds = np.zeros(k, dtype=np.uint32)
        self.gains = np.zeros(k, dtype=np.uint64)
        _check(_lib.imm_result_seeds(self._h, self.seeds.ctypes.data, self.gains.ctypes.data))
        cnt = _u32()
        tg = np.zeros(64, dtype=np.uint64)
        rc = np.zeros(64, dtype=np.uint64)
        _check(_lib.imm_result_targets(self._h, C.byref(cnt), tg.ctypes.data, rc.ctypes.data))
        self.targets = [int(x) for x in tg[: cnt.value]]
        self.round_cov = [int(x) for x in rc[: self.rounds]]
        su, al = _dbl(), _dbl()
        rc2 = np.zeros(64, dtype=np.uint64)
        _check(_lib.imm_result_early(self._h, C.byref(su), C.byref(al), rc2.ctypes.data))
        self.sigma_up, self.alpha = su.value, al.value
        self.round_cov2 = [int(x) for x in rc2[: self.rounds]]
        st = imm_stats()
        _check(_lib.imm_result_stats(self._h, C.byref(st)))
        self.stats = st.as_dict()

    def pool(self):
        """Canonical pool (set_off uint64[n_sets+1], set_vtx uint32[P])."""
        ns, ne = _u64(), _u64()
        _check(_lib.imm_result_pool(self._h, C.byref(ns), C.byref(ne), None, None))
        so = np.zeros(ns.value + 1, dtype=np.uint64)
        sv = np.zeros(max(ne.value, 1), dtype=np.uint32)
        _check(_lib.imm_result_pool(self._h, C.byref(ns), C.byref(ne), so.ctypes.data,
                                    sv.ctypes.data))
        return so, sv[: ne.value]

    def close(self):
        if self._h and self._h.value:
            _lib.imm_result_destroy(self._h)
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def imm_run(g: Graph, k, epsilon, ell=1.0, seed=0, flags=0, max_device_bytes=0,
            stream=None) -> Result:
    p = imm_params(k=k, flags=flags, epsilon=epsilon, ell=ell, seed=seed,
                   max_device_bytes=max_device_bytes)
    out = C.c_void_p()
    _check(_lib.imm_run(g.handle, C.byref(p), _stream(stream), C.byref(out)))
    return Result(out.value, k)


def imm_run_batch(queries, stream=None) -> list:
    """Run several IMM queries together (imm_run_batch).

    queries: sequence of (Graph, dict) where the dict holds imm_run's keyword
    arguments k, epsilon and optionally ell, seed, flags, max_device_bytes.
    Returns one Result per query, in order."""
    cnt = len(queries)
    if cnt == 0:
        return []
    hs = (C.c_void_p * cnt)(*[g.handle.value for g, _ in queries])
    ps = (imm_params * cnt)()
    for j, (_, q) in enumerate(queries):
        ps[j] = imm_params(k=q["k"], flags=q.get("flags", 0), epsilon=q["epsilon"],
                           ell=q.get("ell", 1.0), seed=q.get("seed", 0),
                           max_device_bytes=q.get("max_device_bytes", 0))
    outs = (C.c_void_p * cnt)()
    _check(_lib.imm_run_batch(C.cast(hs, _vp), C.cast(ps, _vp), cnt, _stream(stream),
                              C.cast(outs, _vp)))
    return [Result(outs[j], queries[j][1]["k"]) for j in range(cnt)]


class Server:
    """Owning handle of an imm_server (continuous batching on the current
    device). Graphs passed to submit must stay open while the server runs."""

    def __init__(self, budget_bytes: int, max_slots: int = 8):
        h = C.c_void_p()
        _check(_lib.imm_server_create(budget_bytes, max_slots, C.byref(h)))
        self._h = h
        self._k = {}

    def submit(self, g: Graph, k, epsilon, ell=1.0, seed=0, flags=0, max_device_bytes=0) -> int:
        p = imm_params(k=k, flags=flags, epsilon=epsilon, ell=ell, seed=seed,
                       max_device_bytes=max_device_bytes)
        t = _u64()
        _check(_lib.imm_server_submit(self._h, g.handle, C.byref(p), C.byref(t)))
        self._k[t.value] = k
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """The query's Result; None while it runs (wait=False). Raises the
        query's error (IMM_ECANCELLED after cancel)."""
        out = C.c_void_p()
        st = _lib.imm_server_poll(self._h, ticket, 1 if wait else 0, C.byref(out))
        if st == IMM_EBUSY:
            return None
        k = self._k.pop(ticket, 1)
        _check(st)
        return Result(out.value, k)

    def cancel(self, ticket: int):
        _check(_lib.imm_server_cancel(self._h, ticket))

    def info(self):
        q, r, b = _u64(), _u32(), _u64()
        _check(_lib.imm_server_info(self._h, C.byref(q), C.byref(r), C.byref(b)))
        return {"queued": q.value, "running": r.value, "reserved_bytes": b.value}

    def close(self):
        if self._h and self._h.value:
            _check(_lib.imm_server_destroy(self._h))
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Owning handle of an imm_pool (sets resident in device memory)."""

    def __init__(self, handle, n):
        self._h = C.c_void_p(handle)
        self.n = n
        ns, ne, st = _u64(), _u64(), imm_stats()
        _check(_lib.imm_pool_info(self._h, C.byref(ns), C.byref(ne), C.byref(st)))
        self.n_sets, self.n_entries, self.stats = ns.value, ne.value, st.as_dict()

    def export(self):
        so = np.zeros(self.n_sets + 1, dtype=np.uint64)
        sv = np.zeros(max(self.n_entries, 1), dtype=np.uint32)
        cn = np.zeros(self.n, dtype=np.uint32)
        _check(_lib.imm_pool_export(self._h, so.ctypes.data, sv.ctypes.data, cn.ctypes.data))
        return so, sv[: self.n_entries], cn

    def close(self):
        if self._h and self._h.value:
            _lib.imm_pool_destroy(self._h)
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def imm_sample(g: Graph, seed, first_id, count, flags=0, stream=None) -> Pool:
    out = C.c_void_p()
    _check(_lib.imm_sample(g.handle, seed, first_id, count, flags, _stream(stream), C.byref(out)))
    return Pool(out.value, g.n)


def imm_greedy(n, set_off, set_vtx, k, flags=0, stream=None):
    """Greedy over a caller pool; returns (seeds uint32[k], gains uint64[k], covered)."""
    return _greedy(_lib.imm_greedy, n, set_off, set_vtx, k, flags, stream)


def imm_greedy_static(n, set_off, set_vtx, k, flags=0, stream=None):
    """imm_greedy without any allocation (scratch in the library's fixed
    per-device array); same arguments and results."""
    return _greedy(_lib.imm_greedy_static, n, set_off, set_vtx, k, flags, stream)


def _greedy(fn, n, set_off, set_vtx, k, flags, stream):
    p0, k0, d0 = _ptr(set_off, np.uint64)
    n_sets = (len(set_off) - 1)
    if set_vtx is None or len(set_vtx) == 0:
        set_vtx = np.zeros(1, dtype=np.uint32)
    p1, k1, d1 = _ptr(set_vtx, np.uint32)
    if d0 or d1:
        if not (d0 and d1):
            raise ValueError("either both arrays are device tensors or neither")
        flags |= IMM_DEVICE_PTRS
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    cov = _u64()
    _check(fn(n, p0, p1, n_sets, k, flags, _stream(stream), seeds.ctypes.data,
              gains.ctypes.data, C.byref(cov)))
    return seeds, gains, cov.value


def imm_philox4x32_10(ctr, key, stream=None):
    """Device Philox4x32-10 on counters ctr (uint32[count, 4]) -> uint32[count, 4]."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    _check(_lib.imm_philox4x32_10(c.ctypes.data, c.shape[0], key, 0, _stream(stream),
                                  out.ctypes.data))
    return out


def graph_from(g, stream=None) -> Graph:
    """Upload a graph object with n, m, col_off, row_src, weight, model fields."""
    return imm_graph_create(g.n, g.m, g.col_off, g.row_src, g.weight, g.model, stream=stream)
