"""Pins for the CPU oracle: checks against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's own
formula: they use the paper's printed worked example, closed forms, exact
integer walk counts, theorems checked by brute force, a library inverse
(LAPACK through numpy) and a library shortest-path routine (scipy).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse.csgraph as csg

import graphgen as gg
import oracle
from conftest import read_golden

EPS = np.finfo(np.float64).eps
DBL_MIN = np.finfo(np.float64).tiny


def rdist_ungated(A, gamma):
    """Oracle arithmetic without the diagonal-dominance gate (for theorem checks)."""
    Y, _ = oracle.gj_inverse(oracle.build_m(A, gamma))
    return Y, oracle.readout(Y, gamma).D


def bfs_scipy(A):
    """Distance from j to i at [i, j] (-1 unreachable), via scipy's BFS."""
    d = csg.shortest_path(np.ascontiguousarray(A.T, dtype=np.float64), unweighted=True, directed=True)
    d = d.T
    out = np.where(np.isinf(d), -1, d).astype(np.int64)
    return out


def diameter(dist):
    return int(dist[dist >= 0].max())


# ---------------------------------------------------------------------------
# The paper's worked example (Sec. 4.1.1): undirected path on three vertices
# ---------------------------------------------------------------------------

def _p3_fixture():
    rows = read_golden("p3_worked_example.txt")
    cases, gamma = [], None
    for k, v in rows:
        if k == "gamma":
            gamma = Fraction(v)
        elif k == "Y":
            Y = [[Fraction(t) for t in r.split()] for r in v.split("|")]
            cases.append((gamma, Y))
    meta = dict((k, v) for k, v in rows if k in ("A", "critical_gain", "eigenvalues"))
    return cases, meta


def test_p3_printed_closed_form():
    cases, meta = _p3_fixture()
    A = np.array([[int(t) for t in r.split()] for r in meta["A"].split("|")], dtype=np.uint8)
    assert np.array_equal(A, gg.undirected_path3())
    assert len(cases) == 2
    for gamma, Yq in cases:
        sol = oracle.solve(A, float(gamma))
        assert sol.status == oracle.OK
        Yx = np.array([[float(q) for q in r] for r in Yq])
        assert np.max(np.abs(sol.Y - Yx) / Yx) < 4 * EPS
        # below gamma = 1/2 the rounded R-distance is the graph distance
        assert np.array_equal(sol.D, np.array([[0, 1, 2], [1, 0, 1], [2, 1, 0]]))


def test_p3_critical_gain_and_failure_above_half():
    _, meta = _p3_fixture()
    A = gg.undirected_path3()
    ev = np.sort(np.linalg.eigvalsh(A.astype(np.float64)))
    assert np.allclose(ev, [float(x) for x in meta["eigenvalues"].split()], atol=1e-14)
    assert abs(1.0 / ev.max() - float(meta["critical_gain"])) < 1e-15
    truth = bfs_scipy(A)
    # globally correct just below 1/2 ...
    _, D = rdist_ungated(A, 0.499)
    assert np.array_equal(D, truth)
    # ... but not between 1/2 and the critical gain (Y_12 = g/(1-2g^2) > 1)
    Y, D = rdist_ungated(A, 0.6)
    assert not np.array_equal(D, truth)
    assert Y[0, 1] > 1.0
    # the gate refuses gamma * Delta >= 1 (Delta = 2 here)
    assert oracle.solve(A, 0.5).status == oracle.E_NOT_DD
    # approaching the critical gain the R-distance of adjacent vertices diverges to -inf
    g = 0.7071
    Y, _ = rdist_ungated(A, g)
    assert math.log(Y[0, 1]) / math.log(g) < -10


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("gamma", [0.1, 0.5, 0.9])
def test_directed_path(gamma):
    n = 40
    A = gg.directed_path(n)          # j -> j+1, so A is sub-diagonal
    sol = oracle.solve(A, gamma)
    assert sol.status == oracle.OK and sol.delta == 1
    i, j = np.indices((n, n))
    d = i - j
    below = d >= 0
    expect = np.where(below, np.power(gamma, np.where(below, d, 0).astype(np.float64)), 0.0)
    assert np.all(sol.Y[~below] == 0.0)
    rel = np.abs(sol.Y[below] - expect[below]) / expect[below]
    assert rel.max() < 64 * EPS
    assert np.array_equal(sol.D[below], d[below])           # exact integers: the eta reading
    assert np.all(sol.D[~below] == oracle.UNREACHABLE)


def test_directed_cycle():
    n, gamma = 30, 0.3
    A = gg.directed_cycle(n)
    sol = oracle.solve(A, gamma)
    i, j = np.indices((n, n))
    d = (i - j) % n
    expect = gamma ** d / (1.0 - gamma ** n)
    assert np.max(np.abs(sol.Y - expect) / expect) < 128 * EPS
    assert np.array_equal(sol.D, d)


def test_complete_digraph_sherman_morrison():
    n = 50
    A = gg.complete_digraph(n)
    sol = oracle.solve(A, -0.5)
    assert sol.delta == n - 1
    g = sol.gamma
    assert g == 0.5 / (n - 1)
    expect = (np.eye(n) + g * np.ones((n, n)) / (1.0 - (n - 1) * g)) / (1.0 + g)
    assert np.max(np.abs(sol.Y - expect) / expect) < 64 * n * EPS
    assert np.array_equal(sol.D, 1 - np.eye(n, dtype=np.int16))


# ---------------------------------------------------------------------------
# Identities and invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_inverse_identities_and_theorem4_identity(seed):
    A = gg.erdos_renyi(150, 0.05, gg.rng_for("pin", seed))
    sol = oracle.solve(A, -0.5)
    Y, g = sol.Y, sol.gamma
    M = np.eye(A.shape[0]) - g * A
    n = A.shape[0]
    scale = np.abs(Y).max()
    assert np.abs(M @ Y - np.eye(n)).max() < 8 * n * EPS * scale
    assert np.abs(Y @ M - np.eye(n)).max() < 8 * n * EPS * scale
    # proof of Theorem 4: Y_gi = gamma * sum_j Y_gj A_ji for i != g
    R = g * (Y @ A)
    off = ~np.eye(n, dtype=bool)
    assert np.all(np.abs(Y[off] - R[off]) <= 8 * n * EPS * np.maximum(Y[off], 1e-300) + 1e-300)


@pytest.mark.parametrize("seed", range(4))
def test_truncated_neumann_series(seed):
    rng = gg.rng_for("pin", 100 + seed)
    n = int(rng.integers(4, 12))
    A = gg.erdos_renyi(n, 0.3, rng)
    prep = oracle.prepare(A, -0.5)
    g, delta = prep.gamma, max(prep.delta, 1)
    Y, _ = oracle.gj_inverse(oracle.build_m(A, g))
    K = 40
    # exact integer walk counts N^(k) = A^k (Sec. 3.1), summed with gamma^k
    Ak = np.eye(n, dtype=np.int64)
    S = np.zeros((n, n))
    for k in range(K + 1):
        S += (g ** k) * Ak
        Ak = Ak @ A.astype(np.int64)
    tail = (g * delta) ** (K + 1) / (delta * (1 - g * delta))      # from N^(k) <= Delta^(k-1)
    assert np.all(Y >= S - 1e-15)
    assert np.all(Y - S <= tail + 1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_invariants(seed):
    rng = gg.rng_for("pin", 200 + seed)
    A = gg.erdos_renyi(120, float(rng.uniform(0.005, 0.05)), rng)
    sol = oracle.solve(A, -0.5)
    dist = bfs_scipy(A)
    assert sol.would_swap == 0
    assert np.all(sol.Y >= 0.0)
    assert np.all(np.diag(sol.Y) >= 1.0)
    assert np.array_equal(sol.Y == 0.0, dist < 0)
    assert np.all(np.diag(sol.D) == 0)
    assert sol.unreachable == int((dist < 0).sum())


@pytest.mark.parametrize("n", [200, 500])
def test_library_inverse(n):
    A = gg.erdos_renyi(n, 0.03, gg.rng_for("pin", 300 + n))
    sol = oracle.solve(A, -0.5)
    M = np.eye(n) - sol.gamma * A
    Ylap = np.linalg.inv(M)
    nz = sol.Y >= DBL_MIN
    assert np.max(np.abs(sol.Y[nz] - Ylap[nz]) / sol.Y[nz]) < 1e-13
    assert np.all(np.abs(Ylap[sol.Y == 0.0]) < 1e-14)


# ---------------------------------------------------------------------------
# Theorems checked by brute force
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(25))
def test_theorem2_sufficient_bound(seed):
    rng = gg.rng_for("pin", 400 + seed)
    n = int(rng.integers(3, 11))
    A = gg.erdos_renyi(n, float(rng.uniform(0.15, 0.6)), rng)
    dist = bfs_scipy(A)
    delta = int(A.sum(axis=0).max())
    if delta == 0:
        return
    d = diameter(dist)
    gamma = 0.999 / (delta + delta ** (d - 1))
    sol = oracle.solve(A, gamma)
    assert sol.status == oracle.OK
    reach = dist >= 0
    assert np.array_equal(sol.D[reach], dist[reach])
    assert np.all(sol.D[~reach] == oracle.UNREACHABLE)


@pytest.mark.parametrize("seed", range(15))
def test_theorem3_tree_bound(seed):
    rng = gg.rng_for("pin", 500 + seed)
    n = int(rng.integers(2, 30))
    A = gg.random_tree(n, rng)
    dist = bfs_scipy(A)
    delta = int(A.sum(axis=0).max())
    d = diameter(dist)
    x = delta * (d + 2)
    gamma = 0.999 * (-1 + math.sqrt(1 + 4 * x)) / (2 * x)
    _, D = rdist_ungated(A, gamma)
    assert np.array_equal(D, dist)


def test_theorem1_necessary_bound_negative():
    M = 4
    A = gg.square_grid(M)
    dist, count = oracle.bfs(A)
    smax = count.max()
    assert smax == 20
    gamma = 1.2 / smax                 # violates gamma < 1 / max S
    sol = oracle.solve(A, gamma)
    assert sol.status == oracle.OK     # still passes the gate (gamma * 4 < 1)
    assert not np.array_equal(sol.D, dist)


def test_grid_corner_counts_and_walk_counts():
    rows = read_golden("grid_corner_counts.txt")
    for _, line in rows:
        M, dcorner, S = (int(t) for t in line.split())
        A = gg.square_grid(M)
        dist, count = oracle.bfs(A)
        corner_a, corner_b = 0, M * M - 1
        assert dist[corner_b, corner_a] == dcorner
        assert count[corner_b, corner_a] == S
        assert S > 2 ** (M - 1) if M >= 3 else S == 2 ** (M - 1)   # strict only from M = 3
        # Sec. 3.1: Y = gamma^D (S + C(gamma)) with C -> 0, so at small gamma
        # round(Y gamma^-D) recovers the number of shortest paths exactly
        gamma = 1e-4
        sol = oracle.solve(A, gamma)
        est = np.rint(sol.Y * gamma ** (-dist.astype(np.float64)))
        assert np.array_equal(est, count)


@pytest.mark.parametrize("c", [0.5, 0.95])
@pytest.mark.parametrize("seed", range(4))
def test_theorem4_greedy_reaches_goal(c, seed):
    rng = gg.rng_for("pin", 600 + seed)
    n = 60
    A = gg.erdos_renyi(n, 0.06, rng)
    sol = oracle.solve(A, -c)
    dist = bfs_scipy(A)
    Y = sol.Y
    for goal in range(0, n, 7):
        for cur in range(n):
            if dist[goal, cur] < 0:
                assert oracle.next_hop(A, Y, cur, goal) in (-1, cur) if cur == goal else True
                continue
            p = oracle.path(A, Y, cur, goal, n - 1)
            nodes = p[p >= 0]
            assert nodes[-1] == goal
            assert len(set(nodes.tolist())) == len(nodes)           # corollary: no cycles
            vals = Y[goal, nodes]
            assert np.all(np.diff(vals) > 0)                        # strict ascent on Y
            for a, b in zip(nodes[:-1], nodes[1:]):
                assert A[b, a] == 1                                 # every hop is an edge


@pytest.mark.parametrize("seed", range(5))
def test_corollary_tree_paths_are_shortest(seed):
    rng = gg.rng_for("pin", 700 + seed)
    A = gg.random_tree(40, rng)
    sol = oracle.solve(A, -0.9)
    dist = bfs_scipy(A)
    for goal in range(40):
        for cur in range(40):
            p = oracle.path(A, sol.Y, cur, goal, 39)
            nodes = p[p >= 0]
            assert nodes[-1] == goal
            assert len(nodes) - 1 == dist[goal, cur]


def test_next_hop_tie_break_and_unreachable():
    # 0 -> 1, 0 -> 2, 1 -> 3, 2 -> 3 : successors 1 and 2 tie exactly toward goal 3
    A = gg.from_edges(5, [0, 0, 1, 2], [1, 2, 3, 3])
    sol = oracle.solve(A, 0.25)
    assert sol.Y[3, 1] == sol.Y[3, 2]
    assert oracle.next_hop(A, sol.Y, 0, 3) == 1
    assert oracle.next_hop(A, sol.Y, 3, 3) == 3
    assert oracle.next_hop(A, sol.Y, 0, 4) == -1      # node 4 is isolated
    assert oracle.next_hop(A, sol.Y, 3, 0) == -1      # 3 has no successors
    p = oracle.path(A, sol.Y, 0, 3, 4)
    assert p.tolist() == [0, 1, 3, -1, -1]


def test_path_from_one_series_row_cycle_closed_form():
    """Greedy walk over one goal row (Sec. 4.2) on a directed 12-cycle: the row
    from the walk series must be the closed form gamma^((g - j) mod n) / (1 - gamma^n)
    up to the series' rounding, and the walk from c must run c, c+1, ..., g."""
    n, gam = 12, 0.3
    A = gg.directed_cycle(n)
    for g in (0, 5, 11):
        y = oracle.y_row(A, gam, g)
        closed = np.array([gam ** ((g - j) % n) / (1 - gam ** n) for j in range(n)])
        assert np.max(np.abs(y - closed) / closed) < 1e-14
        for c in range(n):
            p = oracle.path_row(A, y, c, g, n)
            hops = (g - c) % n
            assert p[:hops + 1].tolist() == [(c + h) % n for h in range(hops + 1)]
            assert (p[hops + 1:] == -1).all()
    # the tie rule and the unreachable cases on one row, as for the full-Y walk
    B = gg.from_edges(5, [0, 0, 1, 2], [1, 2, 3, 3])
    y3 = oracle.y_row(B, 0.25, 3)
    assert oracle.path_row(B, y3, 0, 3, 4).tolist() == [0, 1, 3, -1, -1]
    assert oracle.path_row(B, oracle.y_row(B, 0.25, 0), 3, 0, 2).tolist() == [3, -1, -1]


# ---------------------------------------------------------------------------
# Machine precision (Sec. 5.1)
# ---------------------------------------------------------------------------

def test_precision_limit_directed_path():
    fx = dict(read_golden("precision_limit.txt"))
    delta, gc, dlim = float(fx["delta"]), float(fx["gamma_c"]), int(fx["d_limit"])
    assert dlim < math.log(delta) / math.log(gc) < dlim + 1
    n = 340
    A = gg.directed_path(n)
    sol = oracle.solve(A, gc)
    i, j = np.indices((n, n))
    d = i - j
    Y, D = sol.Y, sol.D
    normal = (d >= 0) & (d <= 307)
    assert np.array_equal(D[normal], d[normal])
    assert np.all(Y[(d >= 0) & (d <= dlim - 1)] > 0.0)
    assert np.all(Y[d >= dlim + 2] == 0.0)
    assert np.all(D[d >= dlim + 2] == oracle.UNREACHABLE)
    sub = (Y > 0) & (Y < DBL_MIN)
    assert sol.subnormal == int(sub.sum()) > 0


# ---------------------------------------------------------------------------
# Readout reading (ceil at exact integers) and the int16 encoding
# ---------------------------------------------------------------------------

def test_readout_eta_reading():
    g = 0.1
    vals = [0.001, g ** 3, math.pow(g, 3), np.nextafter(0.001, 1.0), np.nextafter(0.001, 0.0)]
    Y = np.array([vals + [1.0], [g ** (3 + 2e-9), g ** (3 + 0.5e-9), 0.0, 1.0001, 1 / g ** 2, -1.0]])
    Yp = np.zeros((6, 6))
    Yp[:2] = Y
    Yp[2:] = 1.0
    r = oracle.readout(Yp, g)
    assert r.D[0, :5].tolist() == [3] * 5          # naive ceil would give 4 for some of these
    assert r.D[0, 5] == 0
    assert r.D[1].tolist() == [4, 3, oracle.UNREACHABLE, 0, -2, oracle.UNREACHABLE]
    assert r.unreachable == 1 and r.negative == 1


def test_readout_saturation_and_ambiguous():
    g = 0.999
    Y = np.full((2, 2), 1.0)
    Y[0, 1] = 1e-300
    Y[1, 0] = g ** (5 + 1e-9)
    r = oracle.readout(Y, g)
    assert r.D[0, 1] == 32766 and r.saturated == 1
    assert r.ambiguous >= 1


# ---------------------------------------------------------------------------
# Degrees, gate, validation
# ---------------------------------------------------------------------------

def test_degree_is_out_degree_column_sum():
    n = 9
    p = oracle.prepare(gg.out_star(n), -0.5)
    assert p.delta == n - 1 and p.outdeg[0] == n - 1 and p.gamma == 0.5 / (n - 1)
    p = oracle.prepare(gg.in_star(n), -0.5)
    assert p.delta == 1 and p.outdeg[0] == 0


def test_gate_and_validation():
    A = gg.directed_cycle(5)
    assert oracle.prepare(A, 0.99).status == oracle.OK
    assert oracle.prepare(A, 1.0).status == oracle.E_ARG
    assert oracle.prepare(gg.out_star(5), 0.25).status == oracle.E_NOT_DD
    bad = A.copy()
    bad[2, 2] = 1
    assert oracle.prepare(bad, 0.1).status == oracle.E_ADJ
    bad = A.copy()
    bad[0, 1] = 2
    assert oracle.prepare(bad, 0.1).status == oracle.E_ADJ
    assert oracle.prepare(np.zeros((0, 0), np.uint8), 0.1).status == oracle.E_ARG
    # an edgeless graph is not an error: gamma = c and Y = I
    sol = oracle.solve(np.zeros((4, 4), np.uint8), -0.5)
    assert sol.status == oracle.OK and sol.gamma == 0.5
    assert np.array_equal(sol.Y, np.eye(4))
    assert np.array_equal(sol.D, np.where(np.eye(4) > 0, 0, oracle.UNREACHABLE))
    # refused graphs leave the sentinel everywhere
    sol = oracle.solve(gg.out_star(5), 0.25)
    assert sol.status == oracle.E_NOT_DD and np.all(sol.D == oracle.UNREACHABLE)


# ---------------------------------------------------------------------------
# Brute-force companions against a library routine
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_bfs_and_floyd_warshall_against_scipy(seed):
    rng = gg.rng_for("pin", 800 + seed)
    A = gg.erdos_renyi(90, 0.03, rng)
    ref = bfs_scipy(A)
    dist, _ = oracle.bfs(A)
    assert np.array_equal(dist, ref)
    fw = oracle.floyd_warshall(A)
    assert np.array_equal(np.where(fw >= oracle.FW_INF, -1, fw), ref)


def test_gj_steps_compose():
    A = gg.erdos_renyi(64, 0.1, gg.rng_for("pin", 900))
    p = oracle.prepare(A, -0.5)
    M = oracle.build_m(A, p.gamma)
    Y, _ = oracle.gj_inverse(M)
    M2 = M.copy()
    assert oracle.gj_steps_inplace(M2, 0, 17) == oracle.OK
    assert oracle.gj_steps_inplace(M2, 17, 64) == oracle.OK
    assert np.array_equal(M2, Y)


# ---------------------------------------------------------------------------
# Series rows/columns (Eq. inverse-series) against the Gauss-Jordan oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_series_rows_and_columns_match_gauss_jordan(seed):
    rng = gg.rng_for("pin", 1000 + seed)
    A = [gg.erdos_renyi(150, 0.04, rng), gg.grid_lattice_deleted(150, rng), gg.random_geometric(150, rng)][seed]
    sol = oracle.solve(A, -0.5)
    for idx in (0, 17, 149):
        col = oracle.y_column(A, sol.gamma, idx)
        row = oracle.y_row(A, sol.gamma, idx)
        for got, ref in ((col, sol.Y[:, idx]), (row, sol.Y[idx, :])):
            assert np.array_equal(got == 0.0, ref == 0.0)
            nz = ref > 0
            assert np.max(np.abs(got[nz] - ref[nz]) / ref[nz]) < 1e-13


def test_series_directed_path_exact_powers():
    A = gg.directed_path(30)
    col = oracle.y_column(A, 0.5, 3)
    assert np.array_equal(col[3:], 0.5 ** np.arange(27))
    assert np.all(col[:3] == 0.0)


def test_readout_entries_is_the_matrix_readout():
    """The vector form used for full-size spot checks agrees with the matrix readout."""
    rng = np.random.default_rng(5)
    Y = np.exp(-rng.uniform(0, 40, size=(37, 37)))
    Y[3, 4] = 0.0
    g = 0.05
    full = oracle.readout(Y, g).D
    assert np.array_equal(oracle.readout_entries(Y[:, 4], g), full[:, 4])
    assert np.array_equal(oracle.readout_entries(Y[10], g), full[10])


# ---------------------------------------------------------------------------
# Positive integer weights (Sec. 3.2): X = gamma^W, Y = (I - X)^{-1},
# R = log_gamma Y -> weighted distance as gamma -> 0 (Eq. distance-function-integer)
# ---------------------------------------------------------------------------

def test_weighted_path_closed_form():
    """Weighted directed path: Y[i, j] = gamma^(w_j + ... + w_{i-1}) for i >= j
    (the one walk from j to i), 0 above the diagonal; D is that weight sum."""
    rng = np.random.default_rng(11)
    w = rng.integers(1, 10, size=11)
    W = gg.weighted_path(w)
    g = Fraction(1, 20)
    sol = oracle.solve_weighted(W, float(g))
    assert sol.status == oracle.OK and sol.delta == 1
    n = W.shape[0]
    for i in range(n):
        for j in range(n):
            if i < j:
                assert sol.Y[i, j] == 0.0 and sol.D[i, j] == oracle.UNREACHABLE
            else:
                s = int(w[j:i].sum())
                exact = float(g ** s)
                # a product of i - j rounded factors gamma^w
                assert abs(sol.Y[i, j] - exact) <= 4 * (i - j + 2) * EPS * exact
                assert sol.D[i, j] == s


def test_weighted_cycle_closed_form():
    """Weighted directed cycle of total weight L: Y[i, j] = gamma^d / (1 - gamma^L)
    with d the weight of the arc from j to i; D = d."""
    w = np.array([3, 1, 4, 1, 5, 9, 2, 6])
    W = gg.weighted_cycle(w)
    n = w.size
    g = Fraction(1, 7)
    L = int(w.sum())
    sol = oracle.solve_weighted(W, float(g))
    assert sol.status == oracle.OK
    for i in range(n):
        for j in range(n):
            d = int(sum(w[(j + k) % n] for k in range((i - j) % n)))
            exact = float(g ** d / (1 - g ** L))
            assert abs(sol.Y[i, j] - exact) <= 4 * (n + 4) * EPS * exact
            assert sol.D[i, j] == d


@pytest.mark.parametrize("seed", range(6))
def test_weighted_small_gamma_is_dijkstra(seed):
    """At small gamma the weighted R-distance rounds to the weighted shortest
    distance (Eq. distance-function-integer): against scipy's Dijkstra."""
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(5, 13))
    A = gg.erdos_renyi(n, 0.3, rng)
    W = gg.weighted(A, rng, 1, 6)
    sol = oracle.solve_weighted(W, 1e-7)
    assert sol.status == oracle.OK
    d = csg.dijkstra(np.ascontiguousarray(W.T, dtype=np.float64), directed=True).T   # [i, j]: from j to i
    reach = ~np.isinf(d)
    assert np.array_equal(sol.D[reach], d[reach].astype(np.int64))
    assert np.all(sol.D[~reach] == oracle.UNREACHABLE)
    assert np.array_equal(sol.Y == 0.0, ~reach)


def test_weighted_unit_weights_are_the_unweighted_method():
    """All weights 1: X = gamma A, so the weighted pipeline gives the unweighted
    result bit for bit (Sec. 3.2, the special case)."""
    rng = np.random.default_rng(31)
    A = gg.erdos_renyi(60, 0.08, rng)
    a = oracle.solve(A, -0.5)
    b = oracle.solve_weighted(A, -0.5)
    assert a.status == b.status == oracle.OK and a.gamma == b.gamma and a.delta == b.delta
    assert np.array_equal(a.Y, b.Y) and np.array_equal(a.D, b.D)


def test_weighted_inverse_against_lapack():
    """The Gauss-Jordan inverse of I - gamma^W against LAPACK (numpy) on a
    weighted graph with weights up to 100."""
    rng = np.random.default_rng(41)
    W = gg.weighted(gg.erdos_renyi(120, 0.1, rng), rng, 1, 100)
    sol = oracle.solve_weighted(W, -0.5)
    assert sol.status == oracle.OK
    M = oracle.build_m_weighted(W, sol.gamma)
    ref = np.linalg.inv(M)
    nz = np.abs(ref) > 1e-300
    assert np.max(np.abs(sol.Y[nz] - ref[nz]) / np.abs(ref[nz])) < 1e-11
    # structure of M: identity diagonal, -gamma^w on the edges, 0 elsewhere
    e = W != 0
    assert np.all(np.diag(M) == 1.0) and np.all(M[~e & ~np.eye(120, dtype=bool)] == 0.0)
    assert np.all(M[e] < 0.0) and np.all(-M[e] <= sol.gamma)


def test_weighted_gate_and_validation():
    """Delta counts out-edges (not weights); AUTO gamma = c / Delta; the gate
    gamma * Delta < 1; a self-loop of any weight is refused; weight 255 allowed."""
    W = gg.weighted_path([255, 7, 1])
    W[3, 0] = 2                                  # 0 -> 3: node 0 has two out-edges
    p = oracle.prepare_weighted(W, -0.5)
    assert p.status == oracle.OK and p.delta == 2 and p.gamma == 0.25
    assert list(p.outdeg) == [2, 1, 1, 0]
    assert oracle.prepare_weighted(W, 0.5).status == oracle.E_NOT_DD
    loop = W.copy()
    loop[1, 1] = 3
    assert oracle.prepare_weighted(loop, -0.5).status == oracle.E_ADJ
    assert oracle.prepare_weighted(W, 1.0).status == oracle.E_ARG


@pytest.mark.parametrize("seed", range(4))
def test_weighted_greedy_reaches_goal(seed):
    """Theorem 4's argument carries over (Y_gi = sum over successors j of
    Y_gj gamma^W_ji, and those weights sum to less than 1 under the gate):
    greedy ascent reaches the goal with Y strictly increasing."""
    rng = np.random.default_rng(300 + seed)
    n = 40
    A = gg.erdos_renyi(n, 0.1, rng)
    W = gg.weighted(A, rng, 1, 20)
    sol = oracle.solve_weighted(W, -0.5)
    assert sol.status == oracle.OK
    for cur, goal in rng.integers(0, n, size=(30, 2)):
        if sol.Y[goal, cur] == 0.0:
            continue
        out = oracle.path(W, sol.Y, int(cur), int(goal), n)
        hops = [int(x) for x in out if x >= 0]
        assert hops[-1] == goal
        ys = [sol.Y[goal, h] for h in hops]
        assert all(b > a for a, b in zip(ys, ys[1:]))
        assert all(W[b, a] != 0 for a, b in zip(hops, hops[1:]))


def test_rank_one_edge_change_identity():
    """An edge change src -> dst alters entry (dst, src) of X; Y of the changed
    graph is Y + f Y[:, dst] Y[src, :] with f = delta / (1 - delta Y[src, dst])
    (Sherman-Morrison on M' = M - delta e_dst e_src^T), checked against the
    oracle's inversion of the changed graph, for an addition, a removal and a
    weight change."""
    rng = gg.rng_for("pins", 4242)
    A = gg.erdos_renyi(80, 0.05, rng)
    W = gg.weighted(A, rng, 1, 9)
    sol = oracle.solve_weighted(W, -0.5)
    gamma, Y = sol.gamma, sol.Y
    dst, src = map(int, np.argwhere(W != 0)[3])
    add_dst, add_src = map(int, np.argwhere((W == 0) & ~np.eye(80, dtype=bool))[5])
    for s, d, w in [(src, dst, 0), (src, dst, int(W[dst, src]) % 9 + 1), (add_src, add_dst, 2)]:
        W2 = W.copy()
        W2[d, s] = w
        x_old = gamma ** float(W[d, s]) if W[d, s] else 0.0
        delta = (gamma ** float(w) if w else 0.0) - x_old
        f = delta / (1.0 - delta * Y[s, d])
        Y2 = Y + f * np.outer(Y[:, d], Y[s, :])
        ref = oracle.solve_weighted(W2, gamma)
        assert ref.status == oracle.OK
        np.testing.assert_allclose(Y2, ref.Y, rtol=1e-9, atol=1e-15)
        # a transposed orientation is not the changed graph's inverse
        wrong = Y + f * np.outer(Y[:, s], Y[d, :])
        assert np.abs(wrong - ref.Y).max() > 1e-6 * np.abs(ref.Y).max()


def test_row_series_on_successor_lists():
    """The series row for successor lists equals the (pinned) inversion's row
    on ER, lattice and tree graphs and on a weighted graph, and the directed
    path's closed form Y[g, j] = gamma^(g - j) at n = 3000; the lattice
    generator's lists equal those of its dense form."""
    rng = gg.rng_for("pins", 777)
    for A, gam in [(gg.erdos_renyi(90, 0.05, rng), -0.5), (gg.grid_lattice_deleted(100, rng), -0.5),
                   (gg.random_tree(70, rng), -0.6)]:
        sol = oracle.solve(A, gam)
        ptr, idx, _ = gg.csr_from_dense(A)
        for g in (0, 17, A.shape[0] - 1):
            row = oracle.y_row_csr(ptr, idx, sol.gamma, g)
            assert np.array_equal(row == 0, sol.Y[g] == 0)
            nz = sol.Y[g] > 0
            assert np.max(np.abs(row[nz] - sol.Y[g][nz]) / sol.Y[g][nz]) < 1e-13
    W = gg.weighted(gg.erdos_renyi(80, 0.06, rng), rng, 1, 9)
    sol = oracle.solve_weighted(W, -0.5)
    ptr, idx, w = gg.csr_from_dense(W)
    row = oracle.y_row_csr(ptr, idx, sol.gamma, 5, weights=w)
    nz = sol.Y[5] > 0
    assert np.array_equal(row == 0, sol.Y[5] == 0)
    assert np.max(np.abs(row[nz] - sol.Y[5][nz]) / sol.Y[5][nz]) < 1e-13
    n, gamma, g = 3000, 0.7, 1500                      # 0.7^1500 ~ 1e-232: no underflow
    ptr, idx = np.arange(n + 1, dtype=np.int64), np.arange(1, n + 1, dtype=np.int32)
    ptr[-1] = n - 1
    idx = idx[: n - 1]                                  # edge j -> j + 1
    row = oracle.y_row_csr(ptr, idx, gamma, g)
    j = np.arange(n)
    exact = np.where(j <= g, gamma ** np.maximum(g - j, 0).astype(np.float64), 0.0)
    nz = exact > 0
    assert np.array_equal(row == 0, exact == 0)
    assert np.max(np.abs(row[nz] - exact[nz]) / exact[nz]) < 1e-12
    p1, i1 = gg.grid_lattice_csr(500, gg.rng_for("pins", 778))
    p2, i2, _ = gg.csr_from_dense(gg.grid_lattice_deleted(500, gg.rng_for("pins", 778)))
    assert np.array_equal(p1, p2) and np.array_equal(i1, i2)


# ---------------------------------------------------------------------------
# Gain selection and the per-entry certificate
# ---------------------------------------------------------------------------

def test_spectral_radius_closed_forms():
    """rho(A) of the paper's three-vertex path (sqrt 2, its Example), a
    directed cycle (1), the complete digraph (n - 1) and an M x M grid
    (4 cos(pi / (M + 1)))."""
    assert abs(oracle.spectral_radius(gg.undirected_path3()) - math.sqrt(2.0)) < 1e-14
    assert abs(oracle.spectral_radius(gg.directed_cycle(40)) - 1.0) < 1e-12
    assert abs(oracle.spectral_radius(gg.complete_digraph(30)) - 29.0) < 1e-11
    for M in (3, 7, 12):
        assert abs(oracle.spectral_radius(gg.square_grid(M)) - 4.0 * math.cos(math.pi / (M + 1))) < 1e-12



def test_certificate_error_margin_on_both_sides():
    """The certificate must allow for Y's error on the lower side too: on a
    directed path every entry is one exact walk, Y = gamma^d.  Lowered by half
    the assumed relative error, an entry reads out as d + 1; without a margin
    the certificate would prove that wrong value, with the margin it refuses
    it, while the exact entries stay certified."""
    A = gg.directed_path(12)
    g, rel = 0.3, 1e-6
    sol = oracle.solve(A, g)
    low = np.tril(np.ones((12, 12), dtype=bool))
    assert oracle.certify(sol.Y, sol.D, g, 1, rel=rel)[low].all()
    Yp = sol.Y * (1.0 - 0.5 * rel)
    Dp = oracle.readout(Yp, g).D
    flipped = low & (Dp != sol.D)
    assert flipped.sum() > 0 and np.all(Dp[flipped] == sol.D[flipped] + 1)
    assert oracle.certify(Yp, Dp, g, 1)[flipped].all()                 # the failure the margin prevents
    assert not oracle.certify(Yp, Dp, g, 1, rel=rel)[flipped].any()

@pytest.mark.parametrize("seed", range(8))
def test_certificate_implies_bfs_distance(seed):
    """Every entry the certificate accepts has D equal to the BFS distance, at
    gains from tiny to the gate; below 1 / (Delta + Delta^d) every entry is
    accepted; the certificate is not vacuous at AUTO gain on trees."""
    rng = gg.rng_for("pin", 900 + seed)
    n = int(rng.integers(20, 60))
    for A in (gg.erdos_renyi(n, 0.08, rng), gg.random_tree(n, rng), gg.square_grid(5), gg.hanoi(3)):
        dist = bfs_scipy(A)
        delta = int(A.sum(axis=0).max())
        d = diameter(dist)
        for gamma in (1e-6, 0.05 / delta, 0.5 / delta, 0.95 / delta):
            sol = oracle.solve(A, gamma)
            ok = oracle.certify(sol.Y, sol.D, sol.gamma, delta)
            reach = dist >= 0
            assert np.all(sol.D[ok & reach] == dist[ok & reach])
            assert np.all(sol.D[ok & ~reach] == oracle.UNREACHABLE)
        g_all = 0.99 / (delta + float(delta) ** d)
        sol = oracle.solve(A, g_all)
        assert oracle.certify(sol.Y, sol.D, sol.gamma, delta).all()


def test_gain_bound_functions_against_bfs():
    """oracle.gain_bounds: below Theorem 2's bound D equals BFS on random
    graphs, below Theorem 3's on trees; the precision bound keeps gamma^d
    representable."""
    rng = gg.rng_for("pin", 950)
    for _ in range(6):
        A = gg.erdos_renyi(int(rng.integers(4, 10)), 0.4, rng)
        dist = bfs_scipy(A)
        delta = int(A.sum(axis=0).max())
        if delta == 0:
            continue
        b = oracle.gain_bounds(delta, diameter(dist))
        sol = oracle.solve(A, 0.999 * b["gamma_global"])
        assert oracle.global_fraction(sol.D, dist) == 1.0
        T = gg.random_tree(int(rng.integers(5, 25)), rng)
        dist = bfs_scipy(T)
        b = oracle.gain_bounds(int(T.sum(axis=0).max()), diameter(dist))
        _, D = rdist_ungated(T, 0.999 * b["gamma_tree"])
        assert oracle.global_fraction(D, dist) == 1.0
    b = oracle.gain_bounds(4, 300)
    assert b["gamma_precision"] ** 300 > 0.0 and (0.99 * b["gamma_precision"]) ** 300 == 0.0


def test_global_and_local_fractions():
    """global_fraction and local_fraction against direct counts on small
    graphs: the three-vertex path above gamma = 1/2 (the Example) is not
    globally correct but locally correct; a direct loop over oracle.next_hop
    gives the same local fraction on a grid at a large gain."""
    A = gg.undirected_path3()
    dist = bfs_scipy(A)
    Y, D = rdist_ungated(A, 0.6)
    assert oracle.global_fraction(D, dist) < 1.0
    assert oracle.local_fraction(A, Y, dist) == 1.0
    G = gg.square_grid(6)
    dist = bfs_scipy(G)
    sol = oracle.solve(G, 0.24)
    good = total = 0
    for g in range(G.shape[0]):
        for c in range(G.shape[0]):
            if dist[g, c] > 0:
                total += 1
                j = oracle.next_hop(G, sol.Y, c, g)
                good += int(j >= 0 and dist[g, j] == dist[g, c] - 1)
    assert oracle.local_fraction(G, sol.Y, dist) == good / total
    ok = np.where(dist >= 0, sol.D == dist, sol.D == oracle.UNREACHABLE)
    np.fill_diagonal(ok, False)
    assert oracle.global_fraction(sol.D, dist) == ok.sum() / (36 * 35)


def test_hanoi_and_power_law_generators():
    """Towers of Hanoi: 3^k states, 3 (3^k - 1) / 2 moves, diameter 2^k - 1,
    degree at most 3; preferential attachment: m edges per new node."""
    for k in (2, 3, 4):
        H = gg.hanoi(k)
        assert H.shape[0] == 3 ** k and int(H.sum()) == 3 * (3 ** k - 1)
        assert np.array_equal(H, H.T) and int(H.sum(axis=0).max()) == 3
        assert diameter(bfs_scipy(H)) == 2 ** k - 1
    B = gg.barabasi_albert(200, 2, gg.rng_for("pin", 960))
    assert np.array_equal(B, B.T) and int(B.sum()) == 2 * (3 + 2 * (200 - 3))


@pytest.mark.parametrize("seed", range(6))
def test_weighted_certificate_implies_dijkstra(seed):
    """The weighted certificate accepts only entries whose D is the weighted
    graph distance (Dijkstra, scipy), at gains from tiny to the gate, and
    accepts every entry above DBL_MIN once gamma (Delta^(d+1) - 1) / (Delta - 1)
    is small;
    on unit weights it accepts a subset of what the unweighted certificate
    accepts (its bound is at least as large)."""
    rng = gg.rng_for("pin", 980 + seed)
    n = int(rng.integers(15, 40))
    A = gg.erdos_renyi(n, 0.12, rng)
    W = gg.weighted(A, rng, 1, 9)
    dist = csg.shortest_path(np.ascontiguousarray(W.T, dtype=np.float64), directed=True).T
    delta = int((W != 0).sum(axis=0).max())
    if delta == 0:
        return
    reach = np.isfinite(dist)
    for gamma in (1e-9, 1e-4, 0.05 / delta, 0.5 / delta, 0.95 / delta):
        sol = oracle.solve_weighted(W, gamma)
        ok = oracle.certify_weighted(sol.Y, sol.D, sol.gamma, delta)
        assert np.all(sol.D[ok & reach] == dist[ok & reach].astype(np.int64))
        assert np.all(sol.D[ok & ~reach] == oracle.UNREACHABLE)
    dmax = int(dist[reach].max())
    g_all = 0.5 * (delta - 1) / (delta ** (dmax + 1) - 1) if delta > 1 else 0.5 / (dmax + 2)
    sol = oracle.solve_weighted(W, g_all)
    normal = sol.Y >= np.finfo(np.float64).tiny          # long weighted distances underflow at such gains
    assert normal[reach].any()
    assert oracle.certify_weighted(sol.Y, sol.D, sol.gamma, delta)[reach & normal].all()
    sol = oracle.solve(A, 0.3 / delta)
    assert not np.any(oracle.certify_weighted(sol.Y, sol.D, sol.gamma, delta)
                      & ~oracle.certify(sol.Y, sol.D, sol.gamma, delta))
