"""Build libimm.so (HIP for gfx950) in-tree with hipcc.

Every translation unit under ``csrc/`` is compiled to an object file in
``_build/`` (in parallel) and linked into ``paper_2411_09473_amd/libimm.so``.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
BUILD = PKG.parent / "_build"
LIB = PKG / "libimm.so"
# a memory probe for bench.py (random-read chains), not part of the IMM path
PROBE = PKG / "libimm_probe.so"
PROBE_SOURCES = ["probe_chase.hip"]
ARCH = os.environ.get("IMM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["k_sample_ic.hip", "k_sample_lt.hip", "k_pool.hip", "k_select.hip",
           "greedy_static.hip", "workspace.cpp", "runner.cpp", "tune.cpp", "server.cpp", "api.cpp"]

COMMON = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    "-ffp-contract=off",
    # packed FP32 instructions stay disabled in every device compile
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{PKG.parent / 'include'}",
    "-pthread",
]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(h).exists():
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libimm")
    return h


def _compile(src: Path, obj: Path) -> None:
    cmd = [_hipcc(), *COMMON, "-x", "hip", "-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def _link(objs, lib: Path) -> None:
    tmp = lib.with_suffix(f".so.tmp{os.getpid()}")
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", str(tmp),
           *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> Path:
    BUILD.mkdir(exist_ok=True)
    objs, pobjs = [], []
    jobs = []
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        for names, out in ((SOURCES, objs), (PROBE_SOURCES, pobjs)):
            for s in names:
                src = CSRC / s
                obj = BUILD / (s + ".o")
                out.append(obj)
                jobs.append(ex.submit(_compile, src, obj))
        for j in jobs:
            j.result()
    _link(objs, LIB)
    _link(pobjs, PROBE)
    if verbose:
        print(f"built {LIB} and {PROBE}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
