"""GPU parity of goal rows without an inversion (rdist_goal_rows /
rdist_goal_paths) against the oracle: its inversion's rows on small graphs,
its series row for successor lists on large sparse graphs.

Bars: D bit-exact, except entries whose oracle R - eta lies within 1e-10 of
an integer (there +-1); Y within 8 (Delta + 2) u (16 + 2 d) relative (d the
entry's distance: sums of up to Delta + 1 rounded terms per step along walks
of about d steps) for entries at or above 2^-1000, exact zeros where the
graph has no walk; entries the oracle puts below 2^-1000 (underflow) only
checked to be below it too.
"""
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

U = 2.0 ** -53
FLOOR = 2.0 ** -1000
AMBIG = 1e-10


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = R.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def check_rows(Yg, Dg, Yo, gamma, delta, label, Do=None):
    """Yg, Dg: GPU rows; Yo: oracle rows (same shape); Do: oracle D rows
    (else the readout of Yo).  Y tolerance per entry: 8 (Delta + 2) u
    (16 + 2 d), d the entry's distance (walks of length about d carry the
    rounding of about d steps of sums of up to Delta + 1 terms)."""
    if Do is None:
        Do = np.full(Yo.shape, R.RDIST_UNREACHABLE, dtype=np.int16)
        pos = Yo > 0
        Do[pos] = oracle.readout_entries(Yo[pos], gamma)
    big = Yo >= FLOOR
    assert np.all(Yg[Yo == 0] <= FLOOR), label
    assert np.all((Yg == 0) <= (Yo < FLOOR)), label          # a GPU zero only where the oracle underflows
    if big.any():
        d = np.where(Do == R.RDIST_UNREACHABLE, 0, np.abs(Do.astype(np.float64)))
        tol = 8.0 * (delta + 2) * U * (16.0 + 2.0 * d)
        rel = np.abs(Yg - Yo) / np.where(big, Yo, 1.0)
        worst = np.max(np.where(big, rel / tol, 0.0))
        assert worst <= 1.0, (label, worst, float(rel[big].max()))
    sel = big | ((Yo == 0) & (Yg == 0))
    bad = (Dg != Do) & sel
    if bad.any():
        with np.errstate(divide="ignore"):
            t = np.log(np.where(Yo > 0, Yo, 1.0)) / np.log(gamma) - oracle.ETA
        amb = (Yo > 0) & (np.abs(t - np.rint(t)) < AMBIG)
        hard = bad & ~amb
        assert not hard.any(), (label, int(hard.sum()), np.argwhere(hard)[:5].tolist())
        assert np.all(np.abs(Dg[bad].astype(np.int32) - Do[bad].astype(np.int32)) == 1), label


def families(rng):
    return [("er", gg.erdos_renyi(300, 0.03, rng), -0.5), ("lattice", gg.grid_lattice_deleted(400, rng), -0.5),
            ("tree", gg.random_tree(200, rng), -0.5), ("rgg", gg.random_geometric(250, rng), -0.5),
            ("path", gg.directed_path(150), 0.5), ("cycle", gg.directed_cycle(90), 0.7),
            ("edgeless", np.zeros((20, 20), np.uint8), -0.5)]


@pytest.mark.parametrize("q", [1, 3, 8, 64, 100])
def test_rows_against_inversion(ctx, q):
    rng = gg.rng_for("rows", q)
    for name, A, gam in families(rng):
        n = A.shape[0]
        sol = oracle.solve(A, gam)
        assert sol.status == oracle.OK
        ptr, idx, _ = gg.csr_from_dense(A)
        goals = rng.integers(0, n, size=q).astype(np.int32)
        Y, D, info, steps = ctx.goal_rows(dev(ptr), dev(idx), torch.from_numpy(goals), gam)
        note(f"[rows] {name} n={n} q={q}: {steps} steps")
        assert info["status"] == 0 and info["delta"] == sol.delta and info["gamma"] == sol.gamma, info
        Yg, Dg = Y.cpu().numpy(), D.cpu().numpy()
        check_rows(Yg, Dg, sol.Y[goals], sol.gamma, sol.delta, f"{name} q={q}", Do=sol.D[goals])
        assert info["n_unreachable"] == int((sol.Y[goals] == 0).sum())


def test_rows_weighted(ctx):
    rng = gg.rng_for("rows", 500)
    W = gg.weighted(gg.erdos_renyi(300, 0.04, rng), rng, 1, 30)
    sol = oracle.solve_weighted(W, -0.5)
    ptr, idx, w = gg.csr_from_dense(W)
    goals = rng.integers(0, 300, size=16).astype(np.int32)
    Y, D, info, steps = ctx.goal_rows(dev(ptr), dev(idx), torch.from_numpy(goals), -0.5, weights=dev(w))
    assert info["status"] == 0 and info["delta"] == sol.delta and info["gamma"] == sol.gamma
    check_rows(Y.cpu().numpy(), D.cpu().numpy(), sol.Y[goals], sol.gamma, sol.delta, "weighted", Do=sol.D[goals])


def test_goal_paths(ctx):
    from test_gpu_parity import check_paths
    rng = gg.rng_for("rows", 600)
    for A in (gg.erdos_renyi(200, 0.04, rng), gg.grid_lattice_deleted(300, rng)):
        n = A.shape[0]
        sol = oracle.solve(A, -0.5)
        ptr, idx, _ = gg.csr_from_dense(A)
        pairs = rng.integers(0, n, size=(48, 2)).astype(np.int32)
        pairs[0] = [4, 4]
        Y, _, info, _ = ctx.goal_rows(dev(ptr), dev(idx), torch.from_numpy(pairs[:, 1].copy()), -0.5, want_d=False)
        out = ctx.goal_paths(dev(ptr), dev(idx), Y, torch.from_numpy(pairs[:, 1].copy()),
                             torch.from_numpy(pairs[:, 0].copy()), n - 1).cpu().numpy()
        check_paths(A, sol.Y, pairs, out, n - 1)
        short = ctx.goal_paths(dev(ptr), dev(idx), Y, torch.from_numpy(pairs[:, 1].copy()),
                               torch.from_numpy(pairs[:, 0].copy()), 3).cpu().numpy()   # walks cut at 3 hops
        assert short.shape == (48, 4)
        check_paths(A, sol.Y, pairs, short, 3)
        one = ctx.goal_paths(dev(ptr), dev(idx), Y, torch.from_numpy(pairs[:, 1].copy()),
                             torch.from_numpy(pairs[:, 0].copy()), 1).cpu().numpy()   # single-hop form
        assert one.shape == (48,)
        assert np.array_equal(one, np.where(pairs[:, 0] == pairs[:, 1], pairs[:, 0], out[:, 1]))


def test_rows_refusals(ctx):
    """Malformed successor lists give RDIST_E_ADJ, a failed gate
    RDIST_E_NOT_DD (rows zero, D the sentinel); argument errors raise."""
    A = gg.erdos_renyi(50, 0.1, gg.rng_for("rows", 700))
    ptr, idx, _ = gg.csr_from_dense(A)
    goals = torch.tensor([0, 7], dtype=torch.int32)
    j = int(np.argmax(np.diff(ptr) >= 2))
    e0 = int(ptr[j])
    cases = []
    loop = idx.copy(); loop[e0] = j; cases.append(("self-loop", ptr, loop))
    uns = idx.copy(); uns[e0], uns[e0 + 1] = idx[e0 + 1], idx[e0]; cases.append(("unsorted", ptr, uns))
    rng_ = idx.copy(); rng_[e0] = 50; cases.append(("out of range", ptr, rng_))
    bp = ptr.copy(); bp[-1] = ptr[-1] + 5; cases.append(("bad offsets", bp, idx))
    for label, p, i in cases:
        Y, D, info, _ = ctx.goal_rows(dev(p), dev(i), goals, -0.5)
        assert info["status"] == R.RDIST_E_ADJ, label
        assert bool((D == R.RDIST_UNREACHABLE).all()) and bool((Y == 0).all()), label
    Y, D, info, _ = ctx.goal_rows(dev(ptr), dev(idx), goals, 0.9)          # gamma * Delta >= 1
    assert info["status"] == R.RDIST_E_NOT_DD
    assert bool((D == R.RDIST_UNREACHABLE).all())
    with pytest.raises(R.RdistError):
        ctx.goal_rows(dev(ptr), dev(idx), torch.zeros(0, dtype=torch.int32), -0.5)
    with pytest.raises(R.RdistError):
        ctx.goal_rows(dev(ptr), dev(idx), goals, 1.5)
    Y, D, info, _ = ctx.goal_rows(dev(ptr), dev(idx), torch.tensor([-1, 50], dtype=torch.int32), -0.5)
    assert info["status"] == 0 and bool((Y == 0).all()) and bool((D == R.RDIST_UNREACHABLE).all())


def test_rows_large_lattice(ctx):
    """A 512 x 512 lattice with 10% of its directed edges deleted
    (n = 262144), gamma = 0.5 / Delta: four goal rows against the oracle's
    series for successor lists (entries far from the goal underflow)."""
    n = 512 * 512
    ptr, idx = gg.grid_lattice_csr(n, gg.rng_for("rows", 800))
    goals = np.array([0, 1000, 131000, n - 1], dtype=np.int32)
    Y, D, info, steps = ctx.goal_rows(dev(ptr), dev(idx), torch.from_numpy(goals), -0.5)
    note(f"[rows] lattice n={n}: {steps} steps, delta {info['delta']}")
    assert info["status"] == 0
    gamma = info["gamma"]
    Yg, Dg = Y.cpu().numpy(), D.cpu().numpy()
    for k, g in enumerate(goals):
        yo = oracle.y_row_csr(ptr, idx, gamma, int(g))
        check_rows(Yg[k][None, :], Dg[k][None, :], yo[None, :], gamma, info["delta"], f"lattice goal {g}")


def test_rows_c2_graph(ctx):
    """ER(8192, 0.02) at gamma = 0.5 / Delta (the C2 graph's shape): goal
    rows against the oracle's series rows."""
    rng = gg.rng_for("rows", 8192)
    A = gg.erdos_renyi(8192, 0.02, rng)
    ptr, idx, _ = gg.csr_from_dense(A)
    goals = np.array([3, 4095, 8000, 17], dtype=np.int32)
    Y, D, info, steps = ctx.goal_rows(dev(ptr), dev(idx), torch.from_numpy(goals), -0.5)
    note(f"[rows] ER 8192: {steps} steps")
    assert info["status"] == 0
    gamma = info["gamma"]
    Yg, Dg = Y.cpu().numpy(), D.cpu().numpy()
    for k, g in enumerate(goals):
        yo = oracle.y_row_csr(ptr, idx, gamma, int(g))
        check_rows(Yg[k][None, :], Dg[k][None, :], yo[None, :], gamma, info["delta"], f"ER goal {g}")


def test_captured_chunks_replay(ctx):
    """The iteration's captured chunk is replayed across calls with other
    goal sets and other work in between; every call matches the eager
    launches (per-step timing on) bitwise, and the oracle."""
    rng = gg.rng_for("rows", 900)
    A = gg.grid_lattice_deleted(900, rng)
    ptr, idx, _ = gg.csr_from_dense(A)
    P, I = dev(ptr), dev(idx)
    sol = oracle.solve(A, -0.5)
    sets = [rng.integers(0, 900, size=q).astype(np.int32) for q in (5, 5, 64, 5)]
    graph_out = []
    for k, goals in enumerate(sets):
        Y, D, info, steps = ctx.goal_rows(P, I, torch.from_numpy(goals), -0.5)
        graph_out.append((Y.cpu().numpy(), D.cpu().numpy()))
        ctx.solve(dev(gg.erdos_renyi(200, 0.05, rng)), -0.5)          # other work between replays
        torch.cuda.synchronize()
        check_rows(graph_out[-1][0], graph_out[-1][1], sol.Y[goals], sol.gamma, sol.delta, f"replay {k}",
                   Do=sol.D[goals])
    ctx.set_timing(True, classes=[R.RDIST_K_ROWS_STEP])
    try:
        for k, goals in enumerate(sets):
            Y, D, info, steps = ctx.goal_rows(P, I, torch.from_numpy(goals), -0.5)
            assert np.array_equal(Y.cpu().numpy(), graph_out[k][0]), k
            assert np.array_equal(D.cpu().numpy(), graph_out[k][1]), k
    finally:
        ctx.set_timing(False)


def test_rows_state_over_2_31_words():
    """1088 goals on the 1024 x 1024 lattice (n = 2^20): the iteration state
    is two buffers of 8.5 GiB, more 32-bit words than an int counts, so its
    zeroing needs 64-bit counts.  Two calls with different goals (the second
    starts from the state buffers the first left at its fixed point); sampled
    rows of each equal, bitwise, the same goals' rows from a call with five
    goals (the same sums in edge order, another kernel), and one row equals
    the oracle's series row."""
    n = 1024 * 1024
    rng = gg.rng_for("rows", 1000)
    ptr, idx = gg.grid_lattice_csr(n, rng)
    P, I = dev(ptr), dev(idx)
    c = R.Context(0)
    try:
        for call in range(2):
            goals = rng.integers(0, n, size=17 * 64).astype(np.int32)
            Y, _, info, steps = c.goal_rows(P, I, torch.from_numpy(goals), -0.5, want_d=False)
            note(f"[rows] lattice n={n} q={goals.size} call {call}: {steps} steps")
            assert info["status"] == 0
            ks = np.array([0, 63, 64, 700, goals.size - 1])
            Ys, Ds, _, _ = c.goal_rows(P, I, torch.from_numpy(goals[ks].copy()), -0.5)
            for t, k in enumerate(ks):
                assert torch.equal(Y[int(k)], Ys[t]), (call, int(k))
            if call == 0:
                yo = oracle.y_row_csr(ptr, idx, info["gamma"], int(goals[700]))
                check_rows(Ys[3:4].cpu().numpy(), Ds[3:4].cpu().numpy(), yo[None, :], info["gamma"], info["delta"],
                           "lattice 2^20 goal row")
            del Y, Ys, Ds
            torch.cuda.empty_cache()
    finally:
        c.close()


def test_rows_max_goal_count(ctx):
    """q = 65535 (the largest accepted: 1024 chunks of 64, the last one
    ragged), goals repeating and covering every node, on an ER graph with
    n = 120: every row equals the oracle's inversion's row of its goal (D
    exactly, Y within the tolerance); q = 65536 is refused."""
    rng = gg.rng_for("rows", 1100)
    A = gg.erdos_renyi(120, 0.05, rng)
    sol = oracle.solve(A, -0.5)
    ptr, idx, _ = gg.csr_from_dense(A)
    q = 65535
    goals = (np.arange(q) * 7 + rng.integers(0, 120)) % 120
    goals = goals.astype(np.int32)
    Y, D, info, steps = ctx.goal_rows(dev(ptr), dev(idx), torch.from_numpy(goals), -0.5)
    note(f"[rows] n=120 q={q}: {steps} steps")
    assert info["status"] == 0 and info["gamma"] == sol.gamma
    Yg, Dg = Y.cpu().numpy(), D.cpu().numpy()
    for g in range(120):                       # rows of one goal are identical wherever they sit
        ks = np.flatnonzero(goals == g)
        assert np.array_equal(Yg[ks], np.broadcast_to(Yg[ks[0]], (ks.size, 120))), g
        assert np.array_equal(Dg[ks], np.broadcast_to(Dg[ks[0]], (ks.size, 120))), g
    first = np.array([np.flatnonzero(goals == g)[0] for g in range(120)])
    check_rows(Yg[first], Dg[first], sol.Y, sol.gamma, sol.delta, "q = 65535", Do=sol.D)
    with pytest.raises(R.RdistError):
        ctx.goal_rows(dev(ptr), dev(idx), torch.zeros(65536, dtype=torch.int32), -0.5)
