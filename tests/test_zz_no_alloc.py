"""The allocation-free solve (rdist_solve_noalloc) against rdist_solve.

Both are called through the C ABI on the same device inputs; the
allocation-free call must give the same D (bit for bit) and the same info,
on two calls in a row with the second one smaller (the static scratch keeps
the first call's contents), on the single-workgroup and the blocked plans,
integer weights, both block widths and the largest order; it must refuse
orders above RDIST_NOALLOC_MAX_N and the flags that allocate, and leave the
context's device memory unchanged.
"""
import ctypes
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2308_07403_amd import rdist as R  # noqa: E402

NOALLOC_MAX_N = 1024


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = R.Context(0)
    yield c
    c.close()


def solve_both(ctx, A_np, gamma, flags=0):
    """D and info from rdist_solve and from rdist_solve_noalloc (C ABI, same stream)."""
    n = A_np.shape[0]
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    s = torch.cuda.current_stream()
    D1 = torch.full((n, n), 0x1234, dtype=torch.int16, device="cuda")
    D2 = torch.full((n, n), 0x4321, dtype=torch.int16, device="cuda")
    info = R.PinnedInfo(2)
    st = R.rdist_solve(ctx.handle, A.data_ptr(), n, float(gamma), flags, D1.data_ptr(), None, info.at(0),
                       s.cuda_stream)
    assert st == R.RDIST_OK, R.rdist_last_error()
    before = R.rdist_hbm_in_use(ctx.handle)
    st = R.rdist_solve_noalloc(ctx.handle, A.data_ptr(), n, float(gamma), flags, D2.data_ptr(), info.at(1),
                               s.cuda_stream)
    assert st == R.RDIST_OK, R.rdist_last_error()
    s.synchronize()
    assert R.rdist_hbm_in_use(ctx.handle) == before
    return D1.cpu().numpy(), D2.cpu().numpy(), info.get(0).as_dict(), info.get(1).as_dict()


def check(ctx, A_np, gamma, flags=0, label="", against_oracle=False):
    note(f"[noalloc] {label} n={A_np.shape[0]} flags={flags:#x}")
    D1, D2, i1, i2 = solve_both(ctx, A_np, gamma, flags)
    assert i1 == i2, (i1, i2)
    assert np.array_equal(D1, D2), f"{label}: {int((D1 != D2).sum())} entries differ"
    if against_oracle:
        sol = oracle.solve_weighted(A_np, gamma) if flags & R.RDIST_WEIGHTED else oracle.solve(A_np, gamma)
        assert i2["status"] == sol.status
        assert np.array_equal(D2, sol.D)
    return i2


def test_two_calls_second_smaller(ctx):
    rng = gg.rng_for("noalloc", 1)
    first = gg.erdos_renyi(1000, 0.02, rng)
    second = gg.erdos_renyi(300, 0.05, rng)
    i1 = check(ctx, first, -0.5, label="first", against_oracle=True)
    i2 = check(ctx, second, -0.5, label="second (smaller)", against_oracle=True)
    assert i1["status"] == 0 and i2["status"] == 0


def test_plans_and_shapes(ctx):
    rng = gg.rng_for("noalloc", 2)
    cases = [
        (gg.erdos_renyi(100, 0.05, rng), -0.5, 0, "single workgroup"),
        (gg.erdos_renyi(100, 0.05, rng), -0.5, R.RDIST_PLAN_BLOCKED, "blocked, one block"),
        (gg.grid_lattice_deleted(700, rng), -0.5, R.RDIST_UNFUSED_EPILOGUE, "lattice, unfused readout"),
        (gg.erdos_renyi(NOALLOC_MAX_N, 0.02, rng), -0.5, R.RDIST_BLOCK_256, "largest order, b = 256"),
        (gg.erdos_renyi(NOALLOC_MAX_N, 0.02, rng), -0.5, R.RDIST_BLOCK_128, "largest order, b = 128"),
        (gg.weighted(gg.erdos_renyi(500, 0.03, rng), rng, 1, 20), -0.5, R.RDIST_WEIGHTED, "weighted"),
        (gg.out_star(300), 0.25, 0, "gate refusal"),
        (gg.erdos_renyi(129, 0.04, rng), -0.5, 0, "ragged tail"),
    ]
    for A, g, f, label in cases:
        check(ctx, A, g, f, label)


def test_refusals(ctx):
    n = NOALLOC_MAX_N + 1
    A = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    D = torch.empty((n, n), dtype=torch.int16, device="cuda")
    assert R.rdist_solve_noalloc(ctx.handle, A.data_ptr(), n, -0.5, 0, D.data_ptr(), None, None) == R.RDIST_E_ARG
    assert b"static scratch" in R.rdist_last_error()
    for f in (R.RDIST_KEEP_Y, R.RDIST_MIXED_F32, R.RDIST_NO_GRAPH):
        assert R.rdist_solve_noalloc(ctx.handle, A.data_ptr(), 64, -0.5, f, D.data_ptr(), None, None) == \
            R.RDIST_E_ARG
    assert R.rdist_solve_noalloc(None, A.data_ptr(), 64, -0.5, 0, D.data_ptr(), None, None) == R.RDIST_E_ARG
