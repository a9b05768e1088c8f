"""Builds the gfx950 engine library ``librdist.so`` in-tree with hipcc.

Usage: ``python -m paper_2308_07403_amd.build`` (or ``build()`` from Python).
Every call recompiles.  The library exports the C ABI of ``include/rdist.h``.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librdist.so")
SOURCES = ["rd_engine.hip", "rd_host.cpp", "rd_batch.hip", "rd_mixed.hip", "rd_server.hip", "rd_kernels.hip", "rd_update.hip", "rd_level.hip", "rd_paths.hip", "rd_dynamic.hip", "rd_rows.hip", "rd_gamma.hip", "rd_gemm.hip", "rd_chain.hip"]
# every kernel is this project's own: no vendor math library is linked
LINK = []
OBJDIR = os.path.join(HERE, "_build")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res.returncode


def build(verbose: bool = True) -> str:
    """Compiles every source to an object (in parallel), then links the library."""
    t0 = time.time()
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    objs, cmds = [], []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, s + f".{os.getpid()}.o")
        objs.append(obj)
        cmds.append([hipcc(), *flags, *inc, "-c", os.path.join(CSRC, s), "-o", obj])
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        rcs = list(ex.map(_run, cmds))
    if any(rcs):
        raise RuntimeError("hipcc failed to compile the engine")
    tmp = LIB + f".tmp{os.getpid()}"
    if _run([hipcc(), *HIPCC_FLAGS, *objs, *LINK, "-o", tmp]):
        raise RuntimeError("hipcc failed to link librdist.so")
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] {LIB} ({time.time() - t0:.1f}s)")
    return LIB


if __name__ == "__main__":
    build()
