"""GPU checks of the gain bounds (rdist_gain_bounds) and the per-entry
certificate (rdist_certify) against the oracle.

Bars: the bracket [rho_lo, rho_hi] contains the oracle's spectral radius
(numpy's eigenvalues, within 1e-9 of their own rounding) and is narrower
than 1e-6 relative on strongly connected graphs; Delta exact; the gain
bounds equal the oracle's formulas to 1e-15 relative.  Certificate: the
mask equals the oracle's on the oracle's Y except entries within 1e-8 of the
bound in log space (Y differs by rounding and the kernel keeps a 2^-30
margin); every certified GPU entry has D equal to the BFS (or, with
weights, Dijkstra) distance.
"""
import math
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


def graphs():
    rng = gg.rng_for("gain", 1)
    return [("er", gg.erdos_renyi(200, 0.05, rng), True), ("cycle", gg.directed_cycle(100), True),
            ("K50", gg.complete_digraph(50), True), ("grid", gg.square_grid(10), True),
            ("hanoi4", gg.hanoi(4), True), ("ba", gg.barabasi_albert(300, 2, rng), True),
            ("tree", gg.random_tree(100, rng), True), ("path", gg.directed_path(8), False),
            ("dense", gg.erdos_renyi(120, 0.5, rng), True), ("odd", gg.erdos_renyi(77, 0.1, rng), False)]


def test_gain_bounds_bracket(ctx):
    for name, A, strong in graphs():
        rho = oracle.spectral_radius(A)
        dist, _ = oracle.bfs(A)
        d = int(dist.max())
        r = ctx.gain_bounds(dev(A), diameter=d)
        note(f"[gain] {name}: rho {rho:.12g} in [{r['rho_lo']:.12g}, {r['rho_hi']:.12g}], {r['steps']} steps")
        assert r["status"] == 0
        delta = int(A.sum(axis=0).max())
        assert r["delta"] == delta
        slack = 1e-9 * max(rho, 1.0)
        assert r["rho_lo"] - slack <= rho <= r["rho_hi"] + slack, (name, rho, r)
        if strong:
            assert r["rho_hi"] - r["rho_lo"] <= 1e-6 * r["rho_hi"], (name, r)
        b = oracle.gain_bounds(delta, d)
        for key in ("gamma_gate", "gamma_global", "gamma_tree", "gamma_precision"):
            assert math.isclose(r[key], b[key], rel_tol=1e-14), (name, key, r[key], b[key])
        assert r["gamma_c_lo"] == pytest.approx(1.0 / r["rho_hi"]) if r["rho_hi"] > 0 else True


def test_gain_bounds_refusals(ctx):
    A = gg.erdos_renyi(40, 0.1, gg.rng_for("gain", 2))
    B = A.copy()
    B[3, 3] = 1
    assert ctx.gain_bounds(dev(B))["status"] == R.RDIST_E_ADJ
    C = A.copy()
    C[1, 2] = 2
    assert ctx.gain_bounds(dev(C))["status"] == R.RDIST_E_ADJ
    with pytest.raises(R.RdistError):
        ctx.gain_bounds(dev(A), diameter=40)
    r = ctx.gain_bounds(dev(np.zeros((10, 10), np.uint8)))
    assert r["delta"] == 0 and r["rho_lo"] == 0.0 and r["rho_hi"] == 0.0


def near_lower(Y, D, gamma, tol):
    """Entries whose ln Y lies within tol of the certificate's lower boundary
    (k - 1 + eta) ln gamma: the GPU takes Y's error into account there and
    may refuse an entry the oracle (exact Y) accepts."""
    k = D.astype(np.float64)
    return np.abs(np.log(Y) - (k - 1.0 + oracle.ETA) * math.log(gamma)) < tol


def test_certificate_matches_oracle(ctx):
    rng = gg.rng_for("gain", 3)
    for name, A in [("er", gg.erdos_renyi(300, 0.03, rng)), ("tree", gg.random_tree(200, rng)),
                    ("grid", gg.square_grid(12)), ("hanoi", gg.hanoi(4)), ("path", gg.directed_path(130))]:
        dist, _ = oracle.bfs(A)
        delta = int(A.sum(axis=0).max())
        for gamma in (1e-6, 0.05 / delta, 0.5 / delta, 0.9 / delta):
            sol = oracle.solve(A, gamma)
            D, info, g = ctx.solve(dev(A), gamma, keep=True)
            cnt, mask = ctx.certify(g, want_mask=True)
            m = mask.cpu().numpy().astype(bool)
            want = oracle.certify(sol.Y, sol.D, sol.gamma, delta)
            assert cnt == int(m.sum())
            diff = m != want
            if diff.any():
                Yo = sol.Y[diff]
                k = sol.D[diff].astype(np.float64)
                lb = (k + 1) * math.log(gamma * delta) - math.log(delta * (1 - gamma * delta))
                ok = (np.abs(np.log(Yo) - lb) < 1e-8) | near_lower(Yo, sol.D[diff], gamma, 1e-8)
                assert np.all(ok), (name, gamma, int(diff.sum()))
            Dg = D.cpu().numpy()
            reach = dist >= 0
            assert np.all(Dg[m & reach] == dist[m & reach]), (name, gamma)
            assert np.all(Dg[m & ~reach] == R.RDIST_UNREACHABLE)
            note(f"[cert] {name} gamma={gamma:.3g}: {cnt} of {A.shape[0] ** 2} certified")
            g.release()


def test_certificate_weighted(ctx):
    """Weighted graphs: the mask equals the oracle's weighted certificate
    (except within 1e-8 of the bound in log space) and every certified GPU
    entry is the Dijkstra distance."""
    import scipy.sparse.csgraph as csg
    rng = gg.rng_for("gain", 4)
    for n, p, hi in ((150, 0.05, 9), (300, 0.02, 30)):
        W = gg.weighted(gg.erdos_renyi(n, p, rng), rng, 1, hi)
        dist = csg.shortest_path(np.ascontiguousarray(W.T, dtype=np.float64), directed=True).T
        reach = np.isfinite(dist)
        delta = int((W != 0).sum(axis=0).max())
        for gamma in (1e-9, 1e-5, 0.1 / delta, 0.6 / delta):
            sol = oracle.solve_weighted(W, gamma)
            D, info, g = ctx.solve(dev(W), gamma, flags=R.RDIST_WEIGHTED, keep=True)
            cnt, mask = ctx.certify(g, want_mask=True)
            m = mask.cpu().numpy().astype(bool)
            want = oracle.certify_weighted(sol.Y, sol.D, sol.gamma, delta)
            assert cnt == int(m.sum())
            diff = m != want
            if diff.any():
                k = sol.D[diff].astype(np.float64)
                d = float(max(delta, 1))
                first = (k + 1) * math.log(gamma) + (k + 1) * math.log(d) + np.log1p(-d ** (-(k + 1))) - math.log(d - 1)
                second = (k + 2) * math.log(gamma * d) - math.log(d * (1 - gamma * d))
                lb = np.logaddexp(first, second)
                ok = (np.abs(np.log(sol.Y[diff]) - lb) < 1e-8) | near_lower(sol.Y[diff], sol.D[diff], gamma, 1e-8)
                assert np.all(ok), (n, gamma, int(diff.sum()))
            Dg = D.cpu().numpy()
            assert np.all(Dg[m & reach] == dist[m & reach].astype(np.int64)), (n, gamma)
            assert np.all(Dg[m & ~reach] == R.RDIST_UNREACHABLE)
            note(f"[cert] weighted n={n} gamma={gamma:.3g}: {cnt} of {n * n} certified")
            g.release()


def test_gain_bounds_c2_size(ctx):
    """ER(8192, 0.02): the bracket is tight and lies below Delta; the
    spectral radius of G(n, p) is close to n p (the mean degree)."""
    A = gg.erdos_renyi(8192, 0.02, gg.rng_for("gain", 8192))
    r = ctx.gain_bounds(dev(A))
    note(f"[gain] ER 8192: rho in [{r['rho_lo']:.10g}, {r['rho_hi']:.10g}], {r['steps']} steps, delta {r['delta']}")
    assert r["status"] == 0 and r["rho_hi"] - r["rho_lo"] <= 1e-6 * r["rho_hi"]
    assert abs(r["rho_hi"] - 8191 * 0.02) < 0.02 * 8191 * 0.02
    assert r["rho_hi"] < r["delta"]


def test_certificate_after_changes(ctx):
    """A kept graph changed by edge additions (no re-inversion): the
    certificate allows for the 2^-20 relative error a changed Y may carry.
    The mask equals the oracle's certificate of the changed graph except
    entries within 4e-6 of the bound in log space (twice the margin), and
    every certified entry's D is the changed graph's BFS distance."""
    rng = gg.rng_for("gain", 5)
    n = 300
    A = gg.erdos_renyi(n, 0.03, rng)
    D, info, g = ctx.solve(dev(A), -0.5, keep=True)
    gamma = info["gamma"]
    outdeg = A.sum(axis=0)
    changes = []
    for src in np.argsort(outdeg, kind="stable")[:12]:       # low out-degree nodes gain an edge
        cand = np.flatnonzero((A[:, src] == 0) & (np.arange(n) != src))
        dst = int(rng.choice(cand))
        changes.append((int(src), dst, 1))
        A[dst, src] = 1
    inf = g.update_edges(changes, D=D)
    delta = int(A.sum(axis=0).max())
    assert inf["status"] == 0 and inf["fallback_fraction"] == 0.0 and inf["delta"] == delta
    cnt, mask = ctx.certify(g, want_mask=True)
    m = mask.cpu().numpy().astype(bool)
    assert cnt == int(m.sum())
    sol = oracle.solve(A, gamma)
    want = oracle.certify(sol.Y, sol.D, gamma, delta)
    diff = m != want
    if diff.any():
        k = sol.D[diff].astype(np.float64)
        lb = (k + 1) * math.log(gamma * delta) - math.log(delta * (1 - gamma * delta))
        ok = (np.abs(np.log(sol.Y[diff]) - lb) < 4e-6) | near_lower(sol.Y[diff], sol.D[diff], gamma, 4e-6)
        assert np.all(ok), int(diff.sum())
    dist, _ = oracle.bfs(A)
    Dg = D.cpu().numpy()
    reach = dist >= 0
    assert np.all(Dg[m & reach] == dist[m & reach])
    assert np.all(Dg[m & ~reach] == R.RDIST_UNREACHABLE)
    note(f"[cert] changed ER n={n}: {cnt} of {n * n} certified, {int(diff.sum())} differ from the oracle")
    g.release()
