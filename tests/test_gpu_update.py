"""GPU parity of edge changes on a kept graph (rank-one update of Y) against
the oracle's inversion of the changed graph at the same gain.

Bars: D bit-exact, except entries whose oracle R - eta lies within 1e-10 of
an integer (the readout's own ambiguity band), which may differ by one; Y
within 2^-20 relative (the largest error bound an update keeps before it
re-inverts; in practice far smaller, printed), zeros exactly where the
oracle has zeros.  Sampled columns at n = 8192 come from the oracle's series
for one column, or from closed forms.
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

DBL_MIN = np.finfo(np.float64).tiny
Y_TOL = 2.0 ** -20
AMBIG = 1e-10


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = R.Context(0)
    yield c
    c.close()


def dev(A):
    return torch.from_numpy(np.ascontiguousarray(A)).cuda()


def near_boundary(Yo, gamma):
    """Entries whose oracle R - eta lies within AMBIG of an integer."""
    with np.errstate(divide="ignore"):
        t = np.log(np.where(Yo > 0, Yo, 1.0)) / np.log(gamma) - oracle.ETA
    return (Yo > 0) & (np.abs(t - np.rint(t)) < AMBIG)


def check_d(Dg, Do, Yo, gamma, label):
    """D equal to the oracle's readout of the exact Y, except by one step near
    an integer and where the exact Y is subnormal: there FP64 keeps only a few
    significant digits (the precision limit of Sec. 5.1), so which side of the
    integer the computed Y lands on depends on rounding order (check_y skips
    those entries too)."""
    bad = Dg != Do
    if not bad.any():
        return
    amb = near_boundary(Yo, gamma) | ((Yo > 0) & (Yo < DBL_MIN))
    hard = bad & ~amb
    assert not hard.any(), (label, int(hard.sum()), np.argwhere(hard)[:5].tolist())
    assert np.all(np.abs(Dg[bad].astype(np.int32) - Do[bad].astype(np.int32)) == 1), label


def check_y(Yg, Yo, label):
    assert np.array_equal(Yg == 0.0, Yo == 0.0), label
    nz = Yo >= DBL_MIN
    rel = np.abs(Yg[nz] - Yo[nz]) / Yo[nz] if nz.any() else np.zeros(1)
    assert rel.max() <= Y_TOL, (label, rel.max())
    return float(rel.max())


def check_full(ctx, g, A, gamma, D, info, weighted, label):
    sol = (oracle.solve_weighted if weighted else oracle.solve)(A, gamma)
    assert sol.status == oracle.OK
    assert info["status"] == 0, (label, info)
    assert info["delta"] == sol.delta, (label, info["delta"], sol.delta)
    assert info["gamma"] == gamma
    Dg = D.cpu().numpy()
    check_d(Dg, sol.D, sol.Y, gamma, label)
    assert info["n_unreachable"] == sol.unreachable, label
    rel = check_y(g.y().cpu().numpy(), sol.Y, label)
    note(f"[update] {label}: ok, Y max rel {rel:.2e}, lost {info['n_uncertified']}, "
         f"re-inverted {info['fallback_fraction'] == 1.0}")
    return sol


def pick_change(rng, A, delta_cap, weighted):
    """A removal, an addition (keeping every out-degree <= delta_cap) or, on
    weighted graphs, a re-weighting; returns (src, dst, weight)."""
    n = A.shape[0]
    outdeg = (A != 0).sum(axis=0)
    kind = rng.integers(0, 3 if weighted else 2)
    if kind == 0:                                   # remove an edge
        dst, src = map(int, np.argwhere(A != 0)[rng.integers(0, int((A != 0).sum()))])
        return src, dst, 0
    if kind == 2:                                   # re-weight an edge
        dst, src = map(int, np.argwhere(A != 0)[rng.integers(0, int((A != 0).sum()))])
        return src, dst, int(rng.integers(1, 31))
    while True:                                     # add an edge
        src, dst = map(int, rng.integers(0, n, size=2))
        if src != dst and A[dst, src] == 0 and outdeg[src] < delta_cap:
            return src, dst, int(rng.integers(1, 31)) if weighted else 1


@pytest.mark.parametrize("weighted", [False, True])
def test_change_sequence(ctx, weighted):
    """Sixteen changes on a kept n = 600 graph, D and Y against the oracle's
    inversion of each changed graph."""
    rng = gg.rng_for("update", 600 + weighted)
    n = 600
    A = gg.erdos_renyi(n, 0.02, rng)
    if weighted:
        A = gg.weighted(A, rng, 1, 30)
    flags = R.RDIST_WEIGHTED if weighted else 0
    D, info, g = ctx.solve(dev(A), -0.5, flags=flags, keep=True)
    assert info["status"] == 0
    gamma = info["gamma"]
    delta0 = info["delta"]
    for step in range(16):
        src, dst, w = pick_change(rng, A, delta0, weighted)
        note(f"[update] weighted={weighted} step {step}: {src} -> {dst} weight {w}")
        inf = g.update_edge(src, dst, w, D=D)
        A[dst, src] = w
        if step % 4 == 3 or inf["fallback_fraction"] == 1.0:
            check_full(ctx, g, A, gamma, D, inf, weighted, f"step {step}")
        else:
            assert inf["status"] == 0
    g.release()


def test_removal_that_disconnects_reinverts(ctx):
    """Cutting a directed path: the entries it disconnects cancel to their
    rounding residue, so the call re-inverts; adding the edge back is exact."""
    n = 200
    A = gg.directed_path(n)
    D, info, g = ctx.solve(dev(A), 0.5, keep=True)
    inf = g.update_edge(99, 100, 0, D=D)     # edge 99 -> 100 is A[100, 99]
    A[100, 99] = 0
    assert inf["n_uncertified"] > 0 and inf["fallback_fraction"] == 1.0
    sol = check_full(ctx, g, A, 0.5, D, inf, False, "cut path")
    assert sol.unreachable == n * n - 2 * (100 * 101 // 2)
    inf = g.update_edge(99, 100, 1, D=D)
    A[100, 99] = 1
    assert inf["n_uncertified"] == 0 and inf["fallback_fraction"] == 0.0
    check_full(ctx, g, A, 0.5, D, inf, False, "path restored")
    i, j = np.indices(A.shape)
    Dh = D.cpu().numpy()
    assert np.array_equal(Dh[i >= j], (i - j)[i >= j])
    g.release()


def test_weighted_removal_that_disconnects_reinverts(ctx):
    """Cutting a weighted directed path (weights 1 .. 5, gamma = 0.5) re-inverts
    through the weighted blocked plan; restoring the edge with its weight is
    exact again.  D is the weighted distance (the sum of the weights)."""
    n = 150
    rng = gg.rng_for("update", 150)
    W = gg.directed_path(n).astype(np.uint8)
    W[W != 0] = rng.integers(1, 6, size=int((W != 0).sum()))
    D, info, g = ctx.solve(dev(W), 0.5, flags=R.RDIST_WEIGHTED, keep=True)
    w_cut = int(W[71, 70])
    inf = g.update_edge(70, 71, 0, D=D)          # edge 70 -> 71 is W[71, 70]
    W[71, 70] = 0
    assert inf["n_uncertified"] > 0 and inf["fallback_fraction"] == 1.0
    check_full(ctx, g, W, 0.5, D, inf, True, "weighted path cut")
    inf = g.update_edge(70, 71, w_cut, D=D)
    W[71, 70] = w_cut
    assert inf["n_uncertified"] == 0 and inf["fallback_fraction"] == 0.0
    check_full(ctx, g, W, 0.5, D, inf, True, "weighted path restored")
    w = np.diag(W, -1).astype(np.int64)          # w[k]: weight of k -> k + 1
    pre = np.concatenate([[0], np.cumsum(w)])
    i, j = np.indices(W.shape)
    Dh = D.cpu().numpy().astype(np.int64)
    assert np.array_equal(Dh[i >= j], (pre[i] - pre[j])[i >= j])
    g.release()


def test_refused_change_leaves_graph(ctx):
    """A change that breaks the gate gamma * Delta' < 1 is refused and leaves
    Y, D and the graph as they were; the next change applies."""
    n = 50
    A = gg.directed_cycle(n)
    D, info, g = ctx.solve(dev(A), 0.6, keep=True)
    Y0 = g.y().cpu().numpy()
    D0 = D.cpu().numpy().copy()
    inf = g.update_edge(3, 10, 1, D=D)          # node 3 would get 2 out-edges: 1.2 >= 1
    assert inf["status"] == R.RDIST_E_NOT_DD and inf["delta"] == 1
    assert np.array_equal(g.y().cpu().numpy(), Y0)
    assert np.array_equal(D.cpu().numpy(), D0)
    inf = g.update_edge(3, 4, 0, D=D)           # cut the cycle: a path
    A[4, 3] = 0
    check_full(ctx, g, A, 0.6, D, inf, False, "cycle cut")
    inf = g.update_edge(3, 10, 1, D=D)          # node 3 has no out-edge now
    A[10, 3] = 1
    check_full(ctx, g, A, 0.6, D, inf, False, "chord")
    g.release()


def test_delta_follows_changes(ctx):
    """Delta' after each change (the gate's input) is the changed graph's
    largest out-degree: removals from the single node of largest degree
    lower it, removals elsewhere and additions below it keep it, an
    addition above it raises it."""
    rng = gg.rng_for("update", 201)
    n = 200
    A = gg.erdos_renyi(n, 0.03, rng)
    hub = 7
    free = [i for i in range(n) if i != hub and not A[i, hub]]
    A[free[:20], hub] = 1                      # node 7: the one node of largest out-degree
    D, info, g = ctx.solve(dev(A), 0.02, keep=True)
    assert info["status"] == 0 and info["delta"] == int(A.sum(axis=0).max())
    outs = list(np.nonzero(A[:, hub])[0])
    for step in range(12):
        if step % 3 == 2:                      # an addition at a low-degree node
            src = int(np.argmin(A.sum(axis=0)))
            dst = next(i for i in range(n) if i != src and not A[i, src])
            w = 1
        else:                                   # a removal from the hub
            src, dst, w = hub, int(outs.pop()), 0
        inf = g.update_edge(src, dst, w, D=D)
        A[dst, src] = w
        assert inf["status"] == 0
        assert inf["delta"] == int(A.sum(axis=0).max()), (step, inf["delta"], int(A.sum(axis=0).max()))
    src = int(np.argmin(A.sum(axis=0)))
    top = int(A.sum(axis=0).max())
    for dst in [i for i in range(n) if i != src and not A[i, src]][: top + 1 - int(A[:, src].sum())]:
        inf = g.update_edge(src, dst, 1, D=D)
        A[dst, src] = 1
    assert inf["delta"] == top + 1 == int(A.sum(axis=0).max())
    check_full(ctx, g, A, 0.02, D, inf, False, "degree changes")
    g.release()


def test_next_hop_follows_changes(ctx):
    from test_gpu_parity import check_paths
    rng = gg.rng_for("update", 300)
    n = 300
    A = gg.erdos_renyi(n, 0.03, rng)
    D, info, g = ctx.solve(dev(A), -0.5, keep=True)
    gamma = info["gamma"]
    for _ in range(6):
        src, dst, w = pick_change(rng, A, info["delta"], False)
        g.update_edge(src, dst, w)
        A[dst, src] = w
    sol = oracle.solve(A, gamma)
    pairs = rng.integers(0, n, size=(64, 2)).astype(np.int32)
    out = ctx.next_hop(g, torch.from_numpy(pairs[:, 0].copy()), torch.from_numpy(pairs[:, 1].copy()),
                       max_hops=n).cpu().numpy()
    check_paths(A, sol.Y, pairs, out, n)
    g.release()


def test_noop_and_bad_arguments(ctx):
    rng = gg.rng_for("update", 77)
    A = gg.erdos_renyi(150, 0.05, rng)
    D, info, g = ctx.solve(dev(A), -0.5, keep=True)
    Y0 = g.y().cpu().numpy()
    D0 = D.cpu().numpy().copy()
    dst, src = map(int, np.argwhere(A != 0)[0])
    inf = g.update_edge(src, dst, 1, D=D)        # weight unchanged: f = 0
    assert inf["status"] == 0 and inf["n_uncertified"] == 0
    assert np.array_equal(g.y().cpu().numpy(), Y0)
    assert np.array_equal(D.cpu().numpy(), D0)
    inf = g.update_edges([], D=D)                # empty batch: nothing changes
    assert inf["status"] == 0 and inf["delta"] == info["delta"] and inf["gamma"] == info["gamma"]
    assert inf["n_uncertified"] == 0 and inf["n_unreachable"] == 0
    assert np.array_equal(g.y().cpu().numpy(), Y0)
    assert np.array_equal(D.cpu().numpy(), D0)
    for a in [(src, src, 1), (-1, 3, 1), (3, 150, 1), (src, dst, 2), (src, dst, -1)]:
        with pytest.raises(R.RdistError):
            g.update_edge(*a)
    g.release()
    W = gg.weighted(gg.erdos_renyi(100, 0.05, rng), rng, 1, 30)
    _, _, gw = ctx.solve(dev(W), -0.5, flags=R.RDIST_WEIGHTED, keep=True)
    with pytest.raises(R.RdistError):
        gw.update_edge(1, 2, 256)
    gw.release()


# ---------------------------------------------------------------------------
# Full size (n = 8192), sampled
# ---------------------------------------------------------------------------

def test_full_size_path_chord_closed_form(ctx):
    """A chord a -> b on a directed path of 8192 nodes, then its removal.
    With the chord, Y[i, j] = gamma^(i-j) + gamma^((i-j) - (b-a) + 1) for
    j <= a, b <= i, gamma^(i-j) elsewhere below the diagonal, 0 above."""
    n, gamma, a, b = 8192, 0.45, 1000, 1040
    A = gg.directed_path(n)
    D, info, g = ctx.solve(dev(A), gamma, keep=True)
    assert info["status"] == 0
    inf = g.update_edge(a, b, 1, D=D)
    assert inf["status"] == 0 and inf["delta"] == 2
    Y = g.y()
    i = np.arange(n)

    def expect(j, chord):
        d = np.maximum(i - j, 0).astype(np.float64)
        exact = np.where(i >= j, gamma ** d, 0.0)        # underflows to 0 far down the path
        if chord:
            via = (j <= a) & (i >= b)
            exact[via] += gamma ** (d[via] - (b - a) + 1)
        Do = np.full(n, R.RDIST_UNREACHABLE, dtype=np.int16)
        Do[exact > 0] = oracle.readout_entries(exact[exact > 0], gamma)
        return exact, Do

    for j in (0, 500, 999, 1000, 1001, 1039, 5000, 8191):
        exact, Do = expect(j, True)
        check_y(Y[:, j].cpu().numpy()[None, :], exact[None, :], f"chord column {j}")
        check_d(D[:, j].cpu().numpy(), Do, exact, gamma, f"chord column {j}")
    del Y
    inf = g.update_edge(a, b, 0, D=D)           # cancels: re-inverted
    assert inf["status"] == 0 and inf["fallback_fraction"] == 1.0 and inf["n_uncertified"] > 0
    Y = g.y()
    for j in (0, 999, 1000, 1040, 8191):
        exact, Do = expect(j, False)
        check_y(Y[:, j].cpu().numpy()[None, :], exact[None, :], f"path column {j}")
        check_d(D[:, j].cpu().numpy(), Do, exact, gamma, f"path column {j}")
    del Y
    g.release()


def test_full_size_er_sampled_columns(ctx):
    """Changes on ER(8192, 0.02) at gamma = 0.5 / Delta, the size and launch
    the benchmark times: sampled columns against the oracle's series."""
    rng = gg.rng_for("update", 8192)
    n = 8192
    A = gg.erdos_renyi(n, 0.02, rng)
    D, info, g = ctx.solve(dev(A), -0.5, keep=True)
    assert info["status"] == 0
    gamma = info["gamma"]
    changes = []
    for _ in range(4):
        src, dst, w = pick_change(rng, A, info["delta"], False)
        inf = g.update_edge(src, dst, w, D=D)
        assert inf["status"] == 0
        A[dst, src] = w
        changes.append((src, dst, w, inf["n_uncertified"], inf["fallback_fraction"]))
    note(f"[update] n=8192 changes {changes}")
    Y = g.y()
    cols = sorted({c[0] for c in changes} | {c[1] for c in changes} | {0, 4095, 8191})
    for j in cols:
        yo = oracle.y_column(A, gamma, j)
        check_y(Y[:, j].cpu().numpy()[None, :], yo[None, :], f"column {j}")
        Do = np.full(n, R.RDIST_UNREACHABLE, dtype=np.int16)
        Do[yo > 0] = oracle.readout_entries(yo[yo > 0], gamma)
        check_d(D[:, j].cpu().numpy(), Do, yo, gamma, f"column {j}")
    del Y
    g.release()


# ---------------------------------------------------------------------------
# Batched changes (up to 8 per pass over Y)
# ---------------------------------------------------------------------------

def plan_batch(rng, A, count, delta_cap, weighted):
    """count changes in order, applied to a copy of A as they are drawn (so
    repeated edges see the earlier change); a repeat of an earlier edge is
    planted every fifth change."""
    A = A.copy()
    out = []
    for t in range(count):
        if t % 5 == 4 and out:
            s, d, _ = out[int(rng.integers(0, len(out)))]
            w = 0 if A[d, s] else (int(rng.integers(1, 31)) if weighted else 1)
            outdeg = (A != 0).sum(axis=0)
            if w and outdeg[s] >= delta_cap:
                w = 0
        else:
            s, d, w = pick_change(rng, A, delta_cap, weighted)
        A[d, s] = w
        out.append((s, d, w))
    return out, A


@pytest.mark.parametrize("weighted", [False, True])
def test_batch_sequence(ctx, weighted):
    """Three batches of 13 changes (a chunk of 8 and one of 5, repeated edges
    inside a chunk) on a kept n = 600 graph against the oracle's inversion of
    each changed graph."""
    rng = gg.rng_for("update", 1600 + weighted)
    n = 600
    A = gg.erdos_renyi(n, 0.02, rng)
    if weighted:
        A = gg.weighted(A, rng, 1, 30)
    flags = R.RDIST_WEIGHTED if weighted else 0
    D, info, g = ctx.solve(dev(A), -0.5, flags=flags, keep=True)
    gamma, delta0 = info["gamma"], info["delta"]
    for step in range(3):
        changes, A = plan_batch(rng, A, 13, delta0, weighted)
        inf = g.update_edges(changes, D=D)
        check_full(ctx, g, A, gamma, D, inf, weighted, f"batch {step}")
    g.release()


def test_batch_equals_single_changes(ctx):
    """The same 16 changes as two batches and one by one give the same D
    (both checked against the oracle) and Y within the bounds."""
    rng = gg.rng_for("update", 1700)
    A = gg.erdos_renyi(500, 0.03, rng)
    changes, A2 = plan_batch(rng, A, 16, int((A != 0).sum(axis=0).max()), False)
    D1, info, g1 = ctx.solve(dev(A), -0.5, keep=True)
    D2, _, g2 = ctx.solve(dev(A), -0.5, keep=True)
    g1.update_edges(changes, D=D1)
    for s, d, w in changes:
        g2.update_edge(s, d, w, D=D2)
    Yo = oracle.solve(A2, info["gamma"])
    check_d(D1.cpu().numpy(), Yo.D, Yo.Y, info["gamma"], "batched")
    check_d(D2.cpu().numpy(), Yo.D, Yo.Y, info["gamma"], "one by one")
    check_y(g1.y().cpu().numpy(), Yo.Y, "batched")
    check_y(g2.y().cpu().numpy(), Yo.Y, "one by one")
    g1.release()
    g2.release()


def test_batch_refusal(ctx):
    """A chunk whose intermediate graph breaks the gate is refused with the
    rest of the list; earlier chunks stay applied."""
    n = 50
    A = gg.directed_cycle(n)
    D, info, g = ctx.solve(dev(A), 0.6, keep=True)
    Y0 = g.y().cpu().numpy()
    D0 = D.cpu().numpy().copy()
    inf = g.update_edges([(3, 10, 1), (3, 4, 0)], D=D)      # node 3 first gets 2 out-edges: 1.2 >= 1
    assert inf["status"] == R.RDIST_E_NOT_DD
    assert np.array_equal(g.y().cpu().numpy(), Y0) and np.array_equal(D.cpu().numpy(), D0)
    inf = g.update_edges([(3, 4, 0), (3, 10, 1)], D=D)      # the other order passes
    A[4, 3] = 0
    A[10, 3] = 1
    check_full(ctx, g, A, 0.6, D, inf, False, "cycle cut and chord")
    first = [(k, k + 1, 0) for k in range(20, 28)]          # a chunk of 8 removals: applied
    inf = g.update_edges(first + [(30, 35, 1), (30, 36, 1)], D=D)   # node 30 would get 2 out-edges
    assert inf["status"] == R.RDIST_E_NOT_DD
    for s, d, w in first:
        A[d, s] = w
    sol = oracle.solve(A, 0.6)
    check_y(g.y().cpu().numpy(), sol.Y, "first chunk kept")
    g.release()


def test_batch_full_size(ctx):
    """A batch of 8 changes on ER(8192, 0.02) at gamma = 0.5 / Delta (the
    benchmark's graph and launch): sampled columns against the oracle's
    series."""
    rng = gg.rng_for("update", 18192)
    n = 8192
    A = gg.erdos_renyi(n, 0.02, rng)
    D, info, g = ctx.solve(dev(A), -0.5, keep=True)
    gamma = info["gamma"]
    changes, A = plan_batch(rng, A, 8, info["delta"], False)
    inf = g.update_edges(changes, D=D)
    note(f"[update] batch n=8192: lost {inf['n_uncertified']}, re-inverted {inf['fallback_fraction']}")
    assert inf["status"] == 0
    Y = g.y()
    cols = sorted({c[0] for c in changes} | {c[1] for c in changes} | {1, 8190})
    for j in cols:
        yo = oracle.y_column(A, gamma, j)
        check_y(Y[:, j].cpu().numpy()[None, :], yo[None, :], f"column {j}")
        Do = np.full(n, R.RDIST_UNREACHABLE, dtype=np.int16)
        Do[yo > 0] = oracle.readout_entries(yo[yo > 0], gamma)
        check_d(D[:, j].cpu().numpy(), Do, yo, gamma, f"column {j}")
    del Y
    g.release()


def test_long_change_sequence_full_size(ctx):
    """256 changes (alternating removals and additions, one at a time and in
    batches) on ER(8192, 0.02): the bounds carried through every change keep
    D exact; sampled columns against the oracle's series at the end."""
    rng = gg.rng_for("update", 28192)
    n = 8192
    A = gg.erdos_renyi(n, 0.02, rng)
    D, info, g = ctx.solve(dev(A), -0.5, keep=True)
    gamma, delta = info["gamma"], info["delta"]
    outdeg = (A != 0).sum(axis=0).astype(np.int64)
    changes = []
    for k in range(256):
        while True:
            s, d = map(int, rng.integers(0, n, size=2))
            if s == d:
                continue
            if k % 2 == 0 and A[d, s]:
                w = 0
                break
            if k % 2 == 1 and not A[d, s] and outdeg[s] < delta:
                w = 1
                break
        outdeg[s] += 1 if w else -1
        A[d, s] = w
        changes.append((s, d, w))
    lost = reinv = 0
    for s, d, w in changes[:128]:
        inf = g.update_edge(s, d, w)
        assert inf["status"] == 0
        lost += inf["n_uncertified"]
        reinv += inf["fallback_fraction"] == 1.0
    for k in range(128, 256, 32):
        inf = g.update_edges(changes[k:k + 32], D=D if k == 224 else None)
        assert inf["status"] == 0
        lost += inf["n_uncertified"]
        reinv += inf["fallback_fraction"] == 1.0
    note(f"[update] 256 changes at n=8192: lost {lost}, re-inversions {reinv}")
    Y = g.y()
    touched = sorted({c[0] for c in changes[-8:]} | {c[1] for c in changes[-8:]} | {0, 8191})
    for j in touched:
        yo = oracle.y_column(A, gamma, j)
        rel = check_y(Y[:, j].cpu().numpy()[None, :], yo[None, :], f"column {j}")
        Do = np.full(n, R.RDIST_UNREACHABLE, dtype=np.int16)
        Do[yo > 0] = oracle.readout_entries(yo[yo > 0], gamma)
        check_d(D[:, j].cpu().numpy(), Do, yo, gamma, f"column {j}")
    note(f"[update] last column max rel {rel:.2e}")
    del Y
    g.release()
