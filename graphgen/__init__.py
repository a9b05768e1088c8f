"""Seeded synthetic inputs for the R-distance engine and its oracle.

This module only draws graphs, query pairs and arrival times.  It holds none of
the R-distance arithmetic (no gain, no inversion, no logarithm), so the CPU
oracle and the GPU path can both consume exactly the same inputs without
sharing any code that computes a result.

Adjacency convention (paper, Sec. 2, the adjacency equation and its footnote):
``A[i, j] = 1`` iff there is a directed edge from node ``j`` to node ``i``.
This is the transpose of the usual graph-theory convention.  Every generator
returns a C-contiguous ``uint8`` array of shape ``(n, n)`` with a zero diagonal
and no multi-edges (the paper's standing assumptions, Sec. 3.1 footnote).

Graph families follow the paper's workloads: dense/sparse random directed
graphs (Fig. 2 D, Fig. 4 A), square grids (Fig. 2 B, the grid example after
Theorem 1), trees (Fig. 2 C, Theorem 3), plus the lattices, geometric graphs
and request streams of the benchmark configurations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 20230814

# Stable numeric keys for the per-configuration seed streams.
_CONFIG_KEYS = {
    "c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5,
    "test": 100, "pin": 101, "parity": 102, "bench": 103,
}


def rng_for(config: str, index: int = 0) -> np.random.Generator:
    """Independent, reproducible generator for ``(config, index)``.

    Streams come from ``SeedSequence(ROOT_SEED)`` with spawn key
    ``(config_key, index)``, i.e. the same stream ``spawn`` would produce.
    """
    key = _CONFIG_KEYS.get(config)
    if key is None:
        key = int.from_bytes(config.encode()[:6].ljust(6, b"\0"), "little")
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(key, int(index)))
    return np.random.default_rng(ss)


def _empty(n: int) -> np.ndarray:
    return np.zeros((n, n), dtype=np.uint8)


def from_edges(n: int, src, dst) -> np.ndarray:
    """Adjacency from directed edges ``src[k] -> dst[k]`` (self-loops dropped)."""
    A = _empty(n)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    A[dst[keep], src[keep]] = 1
    return A


# ---------------------------------------------------------------------------
# Random directed graphs
# ---------------------------------------------------------------------------

def erdos_renyi(n: int, p: float, rng: np.random.Generator, chunk: int = 1024) -> np.ndarray:
    """Directed G(n, p): each ordered pair i != j is an edge independently with prob. p."""
    A = _empty(n)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        block = rng.random((r1 - r0, n), dtype=np.float32) < np.float32(p)
        A[r0:r1] = block
    np.fill_diagonal(A, 0)
    return A


def weighted(A: np.ndarray, rng: np.random.Generator, w_lo: int = 1, w_hi: int = 100) -> np.ndarray:
    """Integer weights on the edges of A (W[i, j] = weight of edge j -> i, 0 = no
    edge), log-uniform in [w_lo, w_hi] (w_hi <= 255, uint8)."""
    assert 1 <= w_lo <= w_hi <= 255
    W = np.zeros_like(A)
    e = A != 0
    k = int(e.sum())
    w = np.exp(rng.uniform(np.log(w_lo), np.log(w_hi + 1.0), size=k)).astype(np.int64)
    W[e] = np.clip(w, w_lo, w_hi).astype(np.uint8)
    return W


def induced_subgraph(A: np.ndarray, nodes) -> np.ndarray:
    """Subgraph induced by ``nodes`` (order kept), same convention."""
    nodes = np.asarray(nodes, dtype=np.int64)
    return np.ascontiguousarray(A[np.ix_(nodes, nodes)])


def random_subsample(A: np.ndarray, m: int, rng: np.random.Generator) -> np.ndarray:
    """Induced subgraph on ``m`` nodes drawn uniformly without replacement."""
    nodes = np.sort(rng.choice(A.shape[0], size=m, replace=False))
    return induced_subgraph(A, nodes)


# ---------------------------------------------------------------------------
# Lattices and geometric graphs
# ---------------------------------------------------------------------------

def grid_lattice_deleted(n: int, rng: np.random.Generator, p_delete: float = 0.1) -> np.ndarray:
    """2-D grid with random directed-edge deletion.

    ``a = floor(sqrt(n))`` rows and ``w = ceil(n / a)`` columns, cells numbered
    row-major and only the first ``n`` kept.  4-neighbour edges in both
    directions; every *directed* edge is then deleted independently with
    probability ``p_delete``.
    """
    a = max(1, int(math.isqrt(n)))
    w = -(-n // a)
    ids = np.arange(n)
    r, c = ids // w, ids % w
    src, dst = [], []
    for dr, dc in ((0, 1), (1, 0), (0, -1), (-1, 0)):
        rr, cc = r + dr, c + dc
        tgt = rr * w + cc
        ok = (rr >= 0) & (rr < a) & (cc >= 0) & (cc < w) & (tgt < n)
        src.append(ids[ok])
        dst.append(tgt[ok])
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    keep = rng.random(src.shape[0]) >= p_delete
    return from_edges(n, src[keep], dst[keep])


def random_geometric(n: int, rng: np.random.Generator, mean_degree: float = 8.0) -> np.ndarray:
    """Random geometric graph in the unit square with a tuned radius.

    ``n`` points uniform in ``[0, 1)^2``; an undirected (bidirectional) edge
    joins two points closer than ``r``.  ``r`` is placed between the m-th and
    (m+1)-th smallest pair distance with ``m = round(mean_degree * n / 2)``, so
    the realised mean out-degree is ``2m / n`` (8 exactly for the default).
    """
    pts = rng.random((n, 2))
    d = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    iu = np.triu_indices(n, 1)
    dist = d[iu]
    m = int(round(mean_degree * n / 2.0))
    m = max(0, min(m, dist.shape[0]))
    if m == 0:
        return _empty(n)
    order = np.argsort(dist, kind="stable")
    chosen = order[:m]
    i, j = iu[0][chosen], iu[1][chosen]
    return from_edges(n, np.concatenate([i, j]), np.concatenate([j, i]))


def _torus_offsets(kind: str):
    if kind == "tri":          # 2-D triangular lattice, 6 neighbours (axial coords)
        return [(1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1)], 2
    if kind == "moore":        # 2-D Moore neighbourhood, 8 neighbours
        return [(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1) if (dx, dy) != (0, 0)], 2
    if kind == "manhattan2":   # 2-D Manhattan radius 2, 12 neighbours
        return [(dx, dy) for dx in range(-2, 3) for dy in range(-2, 3)
                if 0 < abs(dx) + abs(dy) <= 2], 2
    if kind == "cubic18":      # 3-D, faces + edges of the unit cube, 18 neighbours
        return [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
                if 0 < abs(dx) + abs(dy) + abs(dz) <= 2], 3
    raise ValueError(f"unknown lattice kind {kind!r}")


TORUS_KINDS = ("tri", "moore", "manhattan2", "cubic18")


def torus_lattice(n: int, kind: str) -> np.ndarray:
    """Periodic lattice on the first ``n`` cells of a near-cubic box.

    2-D kinds use an ``a x ceil(n/a)`` torus with ``a = round(sqrt(n))``; the
    3-D kind a ``c x c x ceil(n/c^2)`` torus with ``c = round(n^(1/3))``.  Edges
    whose wrapped target falls outside the first ``n`` cells are dropped.
    Every edge appears in both directions.
    """
    offs, dim = _torus_offsets(kind)
    ids = np.arange(n)
    if dim == 2:
        a = max(1, int(round(math.sqrt(n))))
        b = -(-n // a)
        shape = (a, b)
        coords = (ids // b, ids % b)
    else:
        c = max(1, int(round(n ** (1.0 / 3.0))))
        dz = -(-n // (c * c))
        shape = (c, c, dz)
        coords = (ids // (c * dz), (ids // dz) % c, ids % dz)
    src, dst = [], []
    for off in offs:
        wrapped = [(coords[k] + off[k]) % shape[k] for k in range(dim)]
        if dim == 2:
            tgt = wrapped[0] * shape[1] + wrapped[1]
        else:
            tgt = (wrapped[0] * shape[1] + wrapped[1]) * shape[2] + wrapped[2]
        ok = (tgt < n) & (tgt != ids)
        src.append(ids[ok])
        dst.append(tgt[ok])
    A = from_edges(n, np.concatenate(src), np.concatenate(dst))
    # make every edge bidirectional (dropped wrap targets break symmetry otherwise)
    A |= A.T
    np.fill_diagonal(A, 0)
    return np.ascontiguousarray(A)


# ---------------------------------------------------------------------------
# Small structured graphs with known answers
# ---------------------------------------------------------------------------

def directed_path(n: int) -> np.ndarray:
    """0 -> 1 -> ... -> n-1."""
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1)


def weighted_path(weights) -> np.ndarray:
    """0 -> 1 -> ... -> n-1 with the given edge weights (weights[k] on k -> k+1)."""
    w = np.asarray(weights, dtype=np.uint8)
    n = w.size + 1
    W = _empty(n)
    i = np.arange(n - 1)
    W[i + 1, i] = w
    return W


def weighted_cycle(weights) -> np.ndarray:
    """0 -> 1 -> ... -> n-1 -> 0 with weights[k] on k -> (k+1) mod n."""
    w = np.asarray(weights, dtype=np.uint8)
    n = w.size
    W = _empty(n)
    i = np.arange(n)
    W[(i + 1) % n, i] = w
    return W


def directed_cycle(n: int) -> np.ndarray:
    """0 -> 1 -> ... -> n-1 -> 0."""
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n)


def complete_digraph(n: int) -> np.ndarray:
    A = np.ones((n, n), dtype=np.uint8)
    np.fill_diagonal(A, 0)
    return A


def undirected_path3() -> np.ndarray:
    """The three-vertex undirected path of the paper's first worked example."""
    return np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=np.uint8)


def square_grid(M: int) -> np.ndarray:
    """Undirected M x M grid, 4 nearest neighbours (paper Fig. 2 B)."""
    n = M * M
    ids = np.arange(n)
    r, c = ids // M, ids % M
    src, dst = [], []
    for dr, dc in ((0, 1), (1, 0)):
        ok = (r + dr < M) & (c + dc < M)
        a = ids[ok]
        b = (r[ok] + dr) * M + (c[ok] + dc)
        src += [a, b]
        dst += [b, a]
    return from_edges(n, np.concatenate(src), np.concatenate(dst))


def random_tree(n: int, rng: np.random.Generator) -> np.ndarray:
    """Undirected random recursive tree: node k attaches to a uniform earlier node."""
    if n <= 1:
        return _empty(n)
    child = np.arange(1, n)
    parent = np.array([rng.integers(0, k) for k in range(1, n)], dtype=np.int64)
    return from_edges(n, np.concatenate([child, parent]), np.concatenate([parent, child]))


def binary_tree(levels: int) -> np.ndarray:
    """Undirected complete binary tree with ``levels`` levels (paper Fig. 2 C)."""
    n = (1 << levels) - 1
    child = np.arange(1, n)
    parent = (child - 1) // 2
    return from_edges(n, np.concatenate([child, parent]), np.concatenate([parent, child]))


def out_star(n: int) -> np.ndarray:
    """Node 0 points to every other node."""
    return from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n))


def in_star(n: int) -> np.ndarray:
    """Every other node points to node 0."""
    return from_edges(n, np.arange(1, n), np.zeros(n - 1, dtype=np.int64))


# ---------------------------------------------------------------------------
# Benchmark configurations
# ---------------------------------------------------------------------------

def c1_graph(seed_index: int) -> np.ndarray:
    """Single directed ER graph, n = 64, p = 0.1."""
    return erdos_renyi(64, 0.1, rng_for("c1", seed_index))


C1_GAMMA = 0.05


def c2_graph(seed_index: int = 0) -> np.ndarray:
    """Dense directed ER graph, n = 8192, p = 0.02."""
    return erdos_renyi(8192, 0.02, rng_for("c2", seed_index))


def c2_subsample(seed_index: int, m: int = 2048, fresh: bool = False) -> np.ndarray:
    """n = 2048 graph of the C2 density.

    ``fresh=False``: induced subgraph of the full C2 graph on ``m`` random nodes;
    ``fresh=True``: a new ER(m, 0.02) draw.  Both are ER(m, 0.02) in law.
    """
    rng = rng_for("c2", 1000 + seed_index)
    if fresh:
        return erdos_renyi(m, 0.02, rng)
    return random_subsample(c2_graph(seed_index), m, rng)


def c4_graph(seed_index: int = 0) -> np.ndarray:
    """ER graph, n = 16384, p = 0.01."""
    return erdos_renyi(16384, 0.01, rng_for("c4", seed_index))


def c4_subsample(seed_index: int, m: int = 2048) -> np.ndarray:
    return erdos_renyi(m, 0.01, rng_for("c4", 1000 + seed_index))


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


C3_FAMILIES = ("er", "lattice", "rgg")


@dataclass
class GraphSpec:
    """A reproducible description of one synthetic graph."""
    family: str
    n: int
    seed: tuple
    param: float = 0.0
    kind: str = ""

    def build(self) -> np.ndarray:
        rng = rng_for(self.seed[0], self.seed[1])
        if self.family == "er":
            return erdos_renyi(self.n, self.param, rng)
        if self.family == "lattice":
            return grid_lattice_deleted(self.n, rng, 0.1)
        if self.family == "rgg":
            return random_geometric(self.n, rng, 8.0)
        if self.family == "torus":
            return torus_lattice(self.n, self.kind)
        raise ValueError(self.family)


def c3_specs(count: int = 1024, batch_index: int = 0) -> list:
    """1024 graphs, n log-uniform in [32, 512], family uniform over ER/lattice/RGG."""
    rng = rng_for("c3", batch_index)
    specs = []
    for g in range(count):
        n = log_uniform_int(rng, 32, 512)
        fam = C3_FAMILIES[int(rng.integers(0, 3))]
        p = float(rng.uniform(0.05, 0.2)) if fam == "er" else 0.0
        specs.append(GraphSpec(fam, n, ("c3", 10_000 * (batch_index + 1) + g), p))
    return specs


@dataclass
class Request:
    """One serving request: a graph and what is asked about it."""
    rid: int
    arrival_s: float
    spec: GraphSpec
    query: str                      # "D" or "paths"
    pairs: np.ndarray = field(default=None)   # (64, 2) int32 (src, goal) when query == "paths"


def c5_requests(count: int, qps: float, stream_index: int = 0, n_lo: int = 64,
                n_hi: int = 4096, pairs_per_request: int = 64) -> list:
    """Poisson request stream of the serving configuration.

    Exponential inter-arrival times at rate ``qps``; ``n`` log-uniform in
    ``[n_lo, n_hi]``; family 50/50 ER (``p = k/(n-1)``, ``k ~ U[6, 20]``) or a
    torus lattice with a neighbourhood drawn from {triangular 6, Moore 8,
    Manhattan r=2 12, 3-D 18}; query 50/50 full distance matrix or next-hop paths
    for ``pairs_per_request`` uniform random (src, goal) pairs.
    """
    rng = rng_for("c5", stream_index)
    t = 0.0
    out = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / qps))
        n = log_uniform_int(rng, n_lo, n_hi)
        if rng.random() < 0.5:
            k = float(rng.uniform(6.0, 20.0))
            spec = GraphSpec("er", n, ("c5", 1_000_000 * (stream_index + 1) + rid), min(1.0, k / (n - 1)))
        else:
            kind = TORUS_KINDS[int(rng.integers(0, len(TORUS_KINDS)))]
            spec = GraphSpec("torus", n, ("c5", 1_000_000 * (stream_index + 1) + rid), 0.0, kind)
        query = "D" if rng.random() < 0.5 else "paths"
        pairs = None
        if query == "paths":
            pairs = rng.integers(0, n, size=(pairs_per_request, 2)).astype(np.int32)
        out.append(Request(rid, t, spec, query, pairs))
    return out


# ---------------------------------------------------------------------------
# Successor lists (CSR) for graphs too large for a dense adjacency
# ---------------------------------------------------------------------------

def csr_from_edges(n: int, src, dst, weights=None):
    """Successor lists from directed edges ``src[k] -> dst[k]`` (self-loops and
    repeated edges dropped, the first weight kept): ``ptr`` (n + 1, int64),
    ``idx`` (int32, increasing within a node) and the weights (uint8, or None)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    w = None if weights is None else np.asarray(weights, dtype=np.uint8)[keep]
    key = src * n + dst
    key, first = np.unique(key, return_index=True)
    s2, d2 = key // n, key % n
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(s2, minlength=n), out=ptr[1:])
    return ptr, d2.astype(np.int32), (None if w is None else w[first])


def csr_from_dense(A: np.ndarray):
    """Successor lists of a dense adjacency (``A[i, j] != 0`` iff edge j -> i);
    the nonzero values become the weights (uint8)."""
    At = np.ascontiguousarray(A.T)
    nz = At != 0
    ptr = np.zeros(A.shape[0] + 1, dtype=np.int64)
    np.cumsum(nz.sum(axis=1), out=ptr[1:])
    rows, cols = np.nonzero(nz)
    return ptr, cols.astype(np.int32), At[rows, cols].astype(np.uint8)


def dense_from_csr(n: int, ptr, idx, weights=None) -> np.ndarray:
    """The dense adjacency (or weight matrix) of successor lists."""
    A = _empty(n)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(ptr, dtype=np.int64)))
    A[np.asarray(idx, dtype=np.int64), src] = 1 if weights is None else np.asarray(weights, dtype=np.uint8)
    return A


def grid_lattice_csr(n: int, rng: np.random.Generator, p_delete: float = 0.1):
    """``grid_lattice_deleted`` as successor lists: the same grid, the same
    deletions for the same generator state."""
    a = max(1, int(math.isqrt(n)))
    w = -(-n // a)
    ids = np.arange(n)
    r, c = ids // w, ids % w
    src, dst = [], []
    for dr, dc in ((0, 1), (1, 0), (0, -1), (-1, 0)):
        rr, cc = r + dr, c + dc
        tgt = rr * w + cc
        ok = (rr >= 0) & (rr < a) & (cc >= 0) & (cc < w) & (tgt < n)
        src.append(ids[ok])
        dst.append(tgt[ok])
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    keep = rng.random(src.shape[0]) >= p_delete
    ptr, idx, _ = csr_from_edges(n, src[keep], dst[keep])
    return ptr, idx


def erdos_renyi_csr(n: int, mean_degree: float, rng: np.random.Generator):
    """Sparse random directed graph with the given mean out-degree: the number
    of edges m ~ Binomial(n (n - 1), p) with p = mean_degree / (n - 1), drawn
    as uniform ordered pairs (self-loops redrawn, repeats dropped)."""
    p = mean_degree / max(n - 1, 1)
    m = int(rng.binomial(n * (n - 1), p))
    src = rng.integers(0, n, size=m)
    off = rng.integers(1, n, size=m)          # dst != src
    dst = (src + off) % n
    ptr, idx, _ = csr_from_edges(n, src, dst)
    return ptr, idx


def weights_for(count: int, rng: np.random.Generator, w_lo: int = 1, w_hi: int = 100) -> np.ndarray:
    """``count`` integer edge weights, log-uniform in [w_lo, w_hi] (as ``weighted``)."""
    w = np.exp(rng.uniform(np.log(w_lo), np.log(w_hi + 1.0), size=count)).astype(np.int64)
    return np.clip(w, w_lo, w_hi).astype(np.uint8)


def hanoi(disks: int) -> np.ndarray:
    """State graph of the Towers of Hanoi with ``disks`` disks on 3 pegs (paper
    Fig. 2 A): 3^disks states (peg of each disk, digit k = disk k, disk 0 the
    smallest); an undirected edge for every legal move of one top disk."""
    n = 3 ** disks
    src, dst = [], []
    for s in range(n):
        pegs = [(s // 3 ** k) % 3 for k in range(disks)]
        top = {}
        for k in range(disks):                     # smallest disk on each peg
            top.setdefault(pegs[k], k)
        for a, k in top.items():
            for b in range(3):
                if b != a and (b not in top or top[b] > k):
                    src.append(s)
                    dst.append(s + (b - a) * 3 ** k)
    return from_edges(n, src, dst)


def barabasi_albert(n: int, m: int, rng: np.random.Generator) -> np.ndarray:
    """Undirected preferential-attachment graph (degree distribution with a
    power-law tail of exponent 3, paper Fig. 2 E): start from a clique of
    m + 1 nodes; each new node joins m distinct earlier nodes chosen with
    probability proportional to their degree."""
    src, dst = [], []
    ends = []
    for a in range(m + 1):
        for b in range(a + 1, m + 1):
            src += [a, b]
            dst += [b, a]
            ends += [a, b]
    for v in range(m + 1, n):
        chosen = set()
        while len(chosen) < m:
            chosen.add(int(ends[int(rng.integers(0, len(ends)))]))
        for u in chosen:
            src += [v, u]
            dst += [u, v]
            ends += [v, u]
    return from_edges(n, src, dst)

