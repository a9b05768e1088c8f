"""Host logic of the batched plans (rd_batch.hip, rd_host.cpp) on the CPU.

The two sources hold no device code, so they are built here with g++ against
a stand-in of the HIP runtime (tests/host/hip) and driven by
tests/host/plan_cache_harness.cpp under AddressSanitizer and UBSan: captured
plans matched, replayed and evicted across more batches than the cache holds,
eager and kept-Y transient plans, a tuning change (one new capture, then
replays), the autotuner, eviction of a plan whose caller stream was destroyed,
and every device byte returned at the end.  The kernel stand-ins check, when
a launch runs (also inside a graph replay), that every table, workspace and
caller buffer it names is live.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
CSRC = os.path.join(ROOT, "paper_2308_07403_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan_cache") / "harness")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I", HOST,
           "-x", "c++", os.path.join(CSRC, "rd_batch.hip"), "-x", "c++", os.path.join(CSRC, "rd_host.cpp"),
           "-x", "none", os.path.join(HOST, "hip_stub.cpp"), os.path.join(HOST, "plan_cache_harness.cpp"),
           "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


@pytest.mark.parametrize("scenario", ["1", "2", "3"])
def test_plan_cache_host_logic(harness, scenario):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    res = subprocess.run([harness, scenario], capture_output=True, text=True, env=env, timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0 and "[harness] OK" in res.stdout, out[-4000:]
