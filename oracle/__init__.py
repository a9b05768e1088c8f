"""CPU oracle for the R-distance -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU engine never imports, links or
calls it, and the two share no code.

The arithmetic lives in ``rdist_oracle.c`` (plain IEEE double, no FMA
contraction, unblocked Gauss-Jordan without pivoting, libm ``log``).  This
wrapper only marshals numpy arrays through ctypes.

Paper: Jing & Meister, arXiv 2308.07403.  Convention (Sec. 2): ``A[i, j] = 1``
iff edge ``j -> i``; ``D[i, j]`` is the distance from ``j`` to ``i``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import math

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rdist_oracle.c")
_LIB = os.path.join(_HERE, "librdist_oracle.so")

OK, E_ARG, E_ADJ, E_NOT_DD, E_PIVOT, E_NOMEM = 0, 1, 2, 3, 4, 5
UNREACHABLE = 0x7FFF
ETA = 1e-9      # ceil(R - eta): the reading of the rounded distance at exact integers
BETA = 1e-10    # band around a threshold k + eta that is reported as ambiguous
FW_INF = 0x3FFFFFFF

_CFLAGS = ["-O2", "-ftree-vectorize", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE double, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i32, f64, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
        L.orc_prepare.argtypes = [P, i32, f64, P, P, P]
        L.orc_prepare.restype = i32
        L.orc_build_m.argtypes = [P, i32, f64, P]
        L.orc_gj_steps.argtypes = [P, i32, i32, i32, P]
        L.orc_gj_steps.restype = i32
        L.orc_gj_invert.argtypes = [P, i32, P]
        L.orc_gj_invert.restype = i32
        L.orc_readout.argtypes = [P, i32, f64, f64, f64, P, P]
        L.orc_solve.argtypes = [P, i32, f64, f64, f64, P, P, P, P, P, P]
        L.orc_solve.restype = i32
        L.orc_prepare_weighted.argtypes = [P, i32, f64, P, P, P]
        L.orc_prepare_weighted.restype = i32
        L.orc_build_m_weighted.argtypes = [P, i32, f64, P]
        L.orc_solve_weighted.argtypes = [P, i32, f64, f64, f64, P, P, P, P, P, P]
        L.orc_solve_weighted.restype = i32
        L.orc_next_hop.argtypes = [P, P, i32, i32, i32]
        L.orc_next_hop.restype = i32
        L.orc_path.argtypes = [P, P, i32, i32, i32, i32, P]
        L.orc_path_row.argtypes = [P, P, i32, i32, i32, i32, P]
        L.orc_bfs.argtypes = [P, i32, P, P]
        L.orc_floyd_warshall.argtypes = [P, i32, i32, i32, P]
        L.orc_num_threads.restype = i32
        L.orc_y_column_series.argtypes = [P, i32, f64, i32, f64, i32, P]
        L.orc_y_column_series.restype = i32
        L.orc_y_row_series.argtypes = [P, i32, f64, i32, f64, i32, P]
        L.orc_y_row_series.restype = i32
        L.orc_y_row_series_csr.argtypes = [P, P, P, i32, f64, i32, f64, i32, P]
        L.orc_y_row_series_csr.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _adj(A) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.uint8)
    assert A.ndim == 2 and A.shape[0] == A.shape[1]
    return A


@dataclass
class Prep:
    status: int
    delta: int
    gamma: float
    outdeg: np.ndarray


def prepare(A, gamma_arg: float) -> Prep:
    """Validation, out-degrees, Delta, gain and the gate (gamma * Delta < 1)."""
    A = _adj(A)
    n = A.shape[0]
    outdeg = np.zeros(max(n, 1), dtype=np.int32)
    delta = np.zeros(1, dtype=np.int32)
    gamma = np.zeros(1, dtype=np.float64)
    st = lib().orc_prepare(_p(A), n, float(gamma_arg), _p(outdeg), _p(delta), _p(gamma))
    return Prep(int(st), int(delta[0]), float(gamma[0]), outdeg[:n])


def build_m(A, gamma: float) -> np.ndarray:
    A = _adj(A)
    n = A.shape[0]
    M = np.empty((n, n), dtype=np.float64)
    lib().orc_build_m(_p(A), n, float(gamma), _p(M))
    return M


def gj_inverse(M, count_swaps: bool = False):
    """Unblocked Gauss-Jordan inverse, no pivoting.  Returns (Y, would_swap)."""
    Y = np.array(M, dtype=np.float64, order="C", copy=True)
    sw = np.zeros(1, dtype=np.int64)
    st = lib().orc_gj_invert(_p(Y), Y.shape[0], _p(sw) if count_swaps else None)
    if st != OK:
        raise ArithmeticError(f"oracle Gauss-Jordan failed with status {st}")
    return Y, int(sw[0])


def gj_steps_inplace(M: np.ndarray, k0: int, k1: int) -> int:
    """Run elimination steps k0..k1-1 in place (used to time a bounded sample)."""
    assert M.flags.c_contiguous and M.dtype == np.float64
    return int(lib().orc_gj_steps(_p(M), M.shape[0], int(k0), int(k1), None))


@dataclass
class Readout:
    D: np.ndarray
    unreachable: int
    subnormal: int
    saturated: int
    ambiguous: int
    negative: int


def readout(Y, gamma: float, eta: float = ETA, beta: float = BETA) -> Readout:
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    n = Y.shape[0]
    D = np.empty((n, n), dtype=np.int16)
    c = np.zeros(5, dtype=np.int64)
    lib().orc_readout(_p(Y), n, float(gamma), float(eta), float(beta), _p(D), _p(c))
    return Readout(D, *[int(x) for x in c])


def readout_entries(y, gamma: float, eta: float = ETA, beta: float = BETA) -> np.ndarray:
    """The readout of orc_readout applied to a vector of Y entries (e.g. one
    column from the series): the entries are laid into a square block (the
    rest filled with 1.0) and read out by the same routine."""
    y = np.asarray(y, dtype=np.float64).ravel()
    m = max(1, int(np.ceil(np.sqrt(y.size))))
    blk = np.ones(m * m, dtype=np.float64)
    blk[: y.size] = y
    return readout(blk.reshape(m, m), gamma, eta, beta).D.ravel()[: y.size]


@dataclass
class Solution:
    status: int
    delta: int
    gamma: float
    D: np.ndarray
    Y: np.ndarray | None
    unreachable: int = 0
    subnormal: int = 0
    saturated: int = 0
    ambiguous: int = 0
    negative: int = 0
    would_swap: int = 0


def solve(A, gamma_arg: float, keep_y: bool = True, eta: float = ETA, beta: float = BETA) -> Solution:
    """Full oracle pipeline: gate, M = I - gamma*A, Gauss-Jordan inverse, readout."""
    A = _adj(A)
    n = A.shape[0]
    D = np.empty((n, n), dtype=np.int16)
    Y = np.empty((n, n), dtype=np.float64) if keep_y else None
    delta = np.zeros(1, dtype=np.int32)
    gamma = np.zeros(1, dtype=np.float64)
    c = np.zeros(5, dtype=np.int64)
    sw = np.zeros(1, dtype=np.int64)
    st = lib().orc_solve(_p(A), n, float(gamma_arg), float(eta), float(beta), _p(D),
                         _p(Y) if keep_y else None, _p(delta), _p(gamma), _p(c), _p(sw))
    return Solution(int(st), int(delta[0]), float(gamma[0]), D, Y if st == OK else None,
                    *[int(x) for x in c], int(sw[0]))


def prepare_weighted(W, gamma_arg: float) -> Prep:
    """Sec. 3.2 weights (W[i, j] = weight of edge j -> i, 0 = no edge): no
    self-loops, out-edge counts, Delta, gain and the gate gamma * Delta < 1."""
    W = _adj(W)
    n = W.shape[0]
    outdeg = np.zeros(max(n, 1), dtype=np.int32)
    delta = np.zeros(1, dtype=np.int32)
    gamma = np.zeros(1, dtype=np.float64)
    st = lib().orc_prepare_weighted(_p(W), n, float(gamma_arg), _p(outdeg), _p(delta), _p(gamma))
    return Prep(int(st), int(delta[0]), float(gamma[0]), outdeg[:n])


def build_m_weighted(W, gamma: float) -> np.ndarray:
    """M = I - gamma^W elementwise (0 where there is no edge)."""
    W = _adj(W)
    n = W.shape[0]
    M = np.empty((n, n), dtype=np.float64)
    lib().orc_build_m_weighted(_p(W), n, float(gamma), _p(M))
    return M


def solve_weighted(W, gamma_arg: float, keep_y: bool = True, eta: float = ETA, beta: float = BETA) -> Solution:
    """Weighted pipeline (Sec. 3.2): gate, M = I - gamma^W, Gauss-Jordan inverse, readout."""
    W = _adj(W)
    n = W.shape[0]
    D = np.empty((n, n), dtype=np.int16)
    Y = np.empty((n, n), dtype=np.float64) if keep_y else None
    delta = np.zeros(1, dtype=np.int32)
    gamma = np.zeros(1, dtype=np.float64)
    c = np.zeros(5, dtype=np.int64)
    sw = np.zeros(1, dtype=np.int64)
    st = lib().orc_solve_weighted(_p(W), n, float(gamma_arg), float(eta), float(beta), _p(D),
                                  _p(Y) if keep_y else None, _p(delta), _p(gamma), _p(c), _p(sw))
    return Solution(int(st), int(delta[0]), float(gamma[0]), D, Y if st == OK else None,
                    *[int(x) for x in c], int(sw[0]))


def next_hop(A, Y, cur: int, goal: int) -> int:
    A = _adj(A)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    return int(lib().orc_next_hop(_p(A), _p(Y), A.shape[0], int(cur), int(goal)))


def path(A, Y, cur: int, goal: int, max_hops: int) -> np.ndarray:
    A = _adj(A)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    out = np.empty(max_hops + 1, dtype=np.int32)
    lib().orc_path(_p(A), _p(Y), A.shape[0], int(cur), int(goal), int(max_hops), _p(out))
    return out


def path_row(A, y_goal, cur: int, goal: int, max_hops: int) -> np.ndarray:
    """The greedy walk of ``path`` given only row ``goal`` of Y (e.g. from ``y_row``)."""
    A = _adj(A)
    y = np.ascontiguousarray(y_goal, dtype=np.float64)
    assert y.shape == (A.shape[0],)
    out = np.empty(max_hops + 1, dtype=np.int32)
    lib().orc_path_row(_p(A), _p(y), A.shape[0], int(cur), int(goal), int(max_hops), _p(out))
    return out


def paths(A, Y, pairs, max_hops: int) -> np.ndarray:
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return np.stack([path(A, Y, int(s), int(g), max_hops) for s, g in pairs]) if len(pairs) else \
        np.empty((0, max_hops + 1), dtype=np.int32)


def bfs(A):
    """(dist, count): shortest-path lengths j -> i (-1 unreachable) and path counts S_ij."""
    A = _adj(A)
    n = A.shape[0]
    dist = np.empty((n, n), dtype=np.int32)
    cnt = np.empty((n, n), dtype=np.float64)
    lib().orc_bfs(_p(A), n, _p(dist), _p(cnt))
    return dist, cnt


def floyd_warshall(A, k_steps: int | None = None) -> np.ndarray:
    """Min-plus APSP baseline; ``k_steps`` limits the relaxation to a bounded sample."""
    A = _adj(A)
    n = A.shape[0]
    dist = np.empty((n, n), dtype=np.int32)
    lib().orc_floyd_warshall(_p(A), n, 0, n if k_steps is None else int(k_steps), _p(dist))
    return dist


def y_column(A, gamma: float, j: int, rel_tol: float = 1e-17, max_terms: int = 100000) -> np.ndarray:
    """Column j of Y from the series sum_k (gamma A)^k e_j (needs gamma * Delta < 1)."""
    A = _adj(A)
    y = np.empty(A.shape[0], dtype=np.float64)
    k = lib().orc_y_column_series(_p(A), A.shape[0], float(gamma), int(j), float(rel_tol), int(max_terms), _p(y))
    if k < 0:
        raise ValueError("bad column index")
    return y


def y_row(A, gamma: float, g: int, rel_tol: float = 1e-17, max_terms: int = 100000) -> np.ndarray:
    """Row g of Y from the series e_g^T sum_k (gamma A)^k (needs gamma * Delta < 1)."""
    A = _adj(A)
    y = np.empty(A.shape[0], dtype=np.float64)
    k = lib().orc_y_row_series(_p(A), A.shape[0], float(gamma), int(g), float(rel_tol), int(max_terms), _p(y))
    if k < 0:
        raise ValueError("bad row index")
    return y


def y_row_csr(ptr, idx, gamma: float, g: int, weights=None, rel_tol: float = 1e-17,
              max_terms: int = 1000000) -> np.ndarray:
    """Row g of Y from the series, for a graph given as successor lists
    (successors of c: idx[ptr[c]:ptr[c+1]], optional integer weights)."""
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n = ptr.shape[0] - 1
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint8)
    y = np.empty(n, dtype=np.float64)
    k = lib().orc_y_row_series_csr(_p(ptr), _p(idx), _p(w) if w is not None else None, n, float(gamma), int(g),
                                   float(rel_tol), int(max_terms), _p(y))
    if k < 0:
        raise ValueError("bad row index")
    return y


def spectral_radius(A) -> float:
    """rho(A), the largest modulus of A's eigenvalues (numpy's eigenvalue routine);
    the critical gain is 1 / rho(A) (Eq. critical-gain)."""
    A = np.asarray(A, dtype=np.float64)
    if A.shape[0] == 0:
        return 0.0
    return float(np.max(np.abs(np.linalg.eigvals(A))))


def certify(Y, D, gamma: float, delta: int, rel: float = 0.0) -> np.ndarray:
    """Per-entry certificate (Eq. Y-bracket of Theorem 2's proof, from
    Eq. Y-series-trunc and Eq. Nijk-limit): with k = D, a true distance of
    k + 1 or more would give Y <= gamma^(k+1) Delta^k / (1 - gamma Delta); Y
    above that proves D exact, given that the true distance is at least k,
    i.e. that Y is below gamma^(k - 1 + eta) (a walk of length d gives
    Y >= gamma^d; the readout k = ceil(R - eta) of Y itself implies it).  With
    rel > 0, Y is taken to carry a relative error up to rel, and both sides
    must hold for every value in [Y (1 - rel), Y (1 + rel)].  Y == 0
    certifies unreachable when e gamma^(n-1) > DBL_MIN (no reachable entry can
    underflow); Y below DBL_MIN is not certified.  Returns a boolean mask."""
    Y = np.asarray(Y, dtype=np.float64)
    k = np.asarray(D, dtype=np.float64)
    dl = float(max(delta, 1))
    tiny = np.finfo(np.float64).tiny
    # a zero proves "no walk" only if no reachable entry (>= gamma^(n-1)) can underflow
    zero_ok = (Y.shape[0] - 1) * math.log(gamma) > math.log(tiny) + 1.0
    out = (Y == 0.0) & zero_ok
    pos = Y >= np.finfo(np.float64).tiny
    lb = (k + 1.0) * math.log(gamma * dl) - math.log(dl * (1.0 - gamma * dl))
    lny = np.log(Y[pos])
    above = lny + math.log1p(-rel) > lb[pos]
    below = lny + math.log1p(rel) < (k[pos] - 1.0 + ETA) * math.log(gamma)
    out[pos] = above & below
    return out


def certify_weighted(Y, D, gamma: float, delta: int, rel: float = 0.0) -> np.ndarray:
    """Per-entry certificate for positive integer weights (Sec. 3.2 with the
    walk-count bound Eq. Nijk-limit): with k = D, a true distance of k + 1 or
    more makes every walk of l edges weigh at least max(l, k + 1), so
    Y <= sum_l Delta^(l-1) gamma^max(l, k+1)
      = gamma^(k+1) (Delta^(k+1) - 1) / (Delta - 1) + (gamma Delta)^(k+2) / (Delta (1 - gamma Delta))
    ((k + 1) gamma^(k+1) + gamma^(k+2) / (1 - gamma) for Delta = 1); Y above
    that proves D exact.  The lower side (true distance at least k), rel,
    zeros and entries below DBL_MIN as in certify."""
    Y = np.asarray(Y, dtype=np.float64)
    k = np.asarray(D, dtype=np.float64)
    dl = float(max(delta, 1))
    tiny = np.finfo(np.float64).tiny
    zero_ok = (Y.shape[0] - 1) * math.log(gamma) > math.log(tiny) + 1.0
    out = (Y == 0.0) & zero_ok
    pos = Y >= tiny
    kp = k[pos]
    if dl == 1.0:
        first = np.log(kp + 1.0) + (kp + 1.0) * math.log(gamma)
        second = (kp + 2.0) * math.log(gamma) - math.log(1.0 - gamma)
    else:
        # ln((Delta^(k+1) - 1) / (Delta - 1)) = (k+1) ln Delta + ln(1 - Delta^-(k+1)) - ln(Delta - 1)
        first = ((kp + 1.0) * math.log(gamma) + (kp + 1.0) * math.log(dl) + np.log1p(-dl ** (-(kp + 1.0)))
                 - math.log(dl - 1.0))
        second = (kp + 2.0) * math.log(gamma * dl) - math.log(dl * (1.0 - gamma * dl))
    lb = np.logaddexp(first, second)
    lny = np.log(Y[pos])
    out[pos] = (lny + math.log1p(-rel) > lb) & (lny + math.log1p(rel) < (kp - 1.0 + ETA) * math.log(gamma))
    return out


def gain_bounds(delta: int, d: int) -> dict:
    """The paper's gain bounds for largest out-degree Delta and diameter d:
    Theorem 2 (1 / (Delta + Delta^(d-1))), Theorem 3 for trees, and the
    machine-precision bound Eq. gamma-precision (smallest double)^(1/d)."""
    x = delta * (d + 2)
    return {"gamma_gate": 1.0 / delta if delta else math.inf,
            "gamma_global": 1.0 / (delta + float(delta) ** (d - 1)) if delta else math.inf,
            "gamma_tree": (-1.0 + math.sqrt(1.0 + 4.0 * x)) / (2.0 * x) if delta else math.inf,
            "gamma_precision": math.exp(math.log(5e-324) / d)}


def global_fraction(D, dist) -> float:
    """Fraction of ordered pairs i != j whose D is the graph distance
    (Sec. 4.1's global performance; unreachable pairs count when D says so)."""
    D = np.asarray(D)
    dist = np.asarray(dist)
    n = D.shape[0]
    if n < 2:
        return 1.0
    ok = np.where(dist >= 0, D == dist, D == UNREACHABLE)
    np.fill_diagonal(ok, False)
    return float(ok.sum()) / (n * (n - 1))


def local_fraction(A, Y, dist) -> float:
    """Fraction of (current, goal) pairs, current != goal and the goal
    reachable, whose greedy successor (Eq. descent read as ascent on Y:
    the successor with the largest Y[goal, j], the lowest j on ties) lies one
    step closer to the goal (Sec. 4.2's local performance)."""
    A = np.asarray(A)
    Y = np.asarray(Y, dtype=np.float64)
    dist = np.asarray(dist)
    n = A.shape[0]
    succ = A.T != 0                                   # succ[c, j]: edge c -> j
    good = total = 0
    for g in range(n):
        vals = np.where(succ, Y[g][None, :], -np.inf)     # [cur, j]
        best = np.argmax(vals, axis=1)                    # first maximum: the lowest j on ties
        has = np.isfinite(vals.max(axis=1)) & (vals.max(axis=1) > 0)
        want = (dist[g] > 0)                              # cur != g, goal reachable from cur
        ok = has & (dist[g, best] == dist[g] - 1)
        good += int((ok & want).sum())
        total += int(want.sum())
    return good / total if total else 1.0


def num_threads() -> int:
    return int(lib().orc_num_threads())
