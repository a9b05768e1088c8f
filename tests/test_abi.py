"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments synchronously (no GPU needed)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "rdist.h")
LIB = os.path.join(ROOT, "paper_2308_07403_amd", "librdist.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rdist_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librdist.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "rdist_solve" in names and "rdist_next_hop" in names and "rdist_solve_batched" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in rdist.h but not exported"


def test_binding_uses_the_c_names():
    from paper_2308_07403_amd import rdist
    for name in declared_functions():
        assert hasattr(rdist, name), name
    assert rdist.INFO_SIZE == 72


def test_status_strings(lib):
    lib.rdist_status_string.restype = ctypes.c_char_p
    assert lib.rdist_status_string(0) == b"RDIST_OK"
    assert lib.rdist_status_string(3) == b"RDIST_E_NOT_DD"
    assert lib.rdist_status_string(99) == b"RDIST_E_UNKNOWN"


def test_synchronous_argument_errors_without_device(lib):
    from paper_2308_07403_amd import rdist as R
    # NULL context / pointers are refused before any device call
    assert R.rdist_solve(None, None, 4, 0.1, 0, None, None, None, None) == R.RDIST_E_ARG
    assert b"ctx" in R.rdist_last_error()
    assert R.rdist_solve_batched(None, 1, None, None, None, 0, None, None, None, None) == R.RDIST_E_ARG
    assert R.rdist_next_hop(None, None, None, None, 1, 1, None, None) == R.RDIST_E_ARG
    assert R.rdist_epilogue(None, None, 4, 4, 0.5, None, None, None) == R.RDIST_E_ARG
    assert R.rdist_create(None, 0, 0, None, 0) == R.RDIST_E_ARG
    assert R.rdist_hbm_in_use(None) == 0
    # the widened entry points refuse NULL handles the same way
    assert R.rdist_graph_update_edge(None, None, 0, 1, 1, None, None, None) == R.RDIST_E_ARG
    assert R.rdist_graph_update_edges(None, None, 1, None, None, None, None, None, None) == R.RDIST_E_ARG
    assert R.rdist_goal_rows(None, 4, None, None, 0, None, 0.1, None, 1, None, None, None, None, None) == R.RDIST_E_ARG
    assert R.rdist_goal_paths(None, 4, None, None, 0, None, None, None, 1, 1, None, None) == R.RDIST_E_ARG
    assert R.rdist_gain_bounds(None, None, 4, 0, 16, 0.0, None, None) == R.RDIST_E_ARG
    assert R.rdist_certify(None, None, None, None, None) == R.RDIST_E_ARG
    assert R.rdist_timing_hold(None, 1) == R.RDIST_E_ARG
    R.rdist_graph_release(None)
    R.rdist_destroy(None)


def test_oracle_and_engine_share_nothing():
    """The engine sources never mention the oracle and vice versa."""
    csrc = os.path.join(ROOT, "paper_2308_07403_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "oracle" not in text.lower(), f
    for f in ("rdist.py", "__init__.py"):
        p = os.path.join(ROOT, "paper_2308_07403_amd", f)
        if os.path.exists(p):
            assert "import oracle" not in open(p).read()
    otext = open(os.path.join(ROOT, "oracle", "rdist_oracle.c")).read()
    assert "rdist.h" not in otext and "rd_device" not in otext


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with a message before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
