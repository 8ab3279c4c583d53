"""Helpers shared by the GPU parity tests (no GPU work here)."""

import numpy as np


def canonical(set_off, set_vtx, n):
    """Sort every set ascending (sets stay in sample-id order)."""
    so = np.asarray(set_off, dtype=np.uint64)
    sv = np.asarray(set_vtx, dtype=np.uint64)
    sizes = np.diff(so).astype(np.int64)
    sid = np.repeat(np.arange(sizes.size, dtype=np.uint64), sizes)
    key = np.sort(sid * np.uint64(n) + sv)
    return so.copy(), (key % np.uint64(n)).astype(np.uint32)


def say(msg):
    print(msg, flush=True)
