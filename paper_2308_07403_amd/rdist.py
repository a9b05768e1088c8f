"""ctypes binding of the gfx950 R-distance engine (``include/rdist.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``librdist.so``.  torch supplies device memory and streams.  If the
library is missing this module raises at import time; there is no fallback.

Raw entry points keep the C names (``rdist_create``, ``rdist_solve``,
``rdist_solve_batched``, ``rdist_next_hop``, ...); ``Context`` wraps them for
torch tensors.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librdist.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP engine first "
        "(python -m paper_2308_07403_amd.build); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)
_hip = ctypes.CDLL("libamdhip64.so")
_hip.hipMemcpy2D.restype = ctypes.c_int

# ---- status codes and flags (include/rdist.h) ----
RDIST_OK, RDIST_E_ARG, RDIST_E_ADJ, RDIST_E_NOT_DD = 0, 1, 2, 3
RDIST_E_NOMEM, RDIST_E_AGAIN, RDIST_E_HIP, RDIST_E_STATE = 4, 5, 6, 7
RDIST_UNREACHABLE = 0x7FFF
RDIST_F64 = 0x0
RDIST_MIXED_F32 = 0x1
RDIST_KEEP_Y = 0x10
RDIST_PLAN_SMALL = 0x100
RDIST_PLAN_BLOCKED = 0x200
RDIST_UNFUSED_EPILOGUE = 0x400
RDIST_BLOCK_128 = 0x800
RDIST_BLOCK_256 = 0x1000
RDIST_NO_GRAPH = 0x2000
RDIST_WEIGHTED = 0x4000
RDIST_THREADSAFE = 0x1
(RDIST_K_UPDATE, RDIST_K_PANEL, RDIST_K_ROWCOL, RDIST_K_INGEST, RDIST_K_EPILOGUE, RDIST_K_SMALL,
 RDIST_K_BATCHED, RDIST_K_NEXTHOP, RDIST_K_CERTIFY, RDIST_K_UPDATE_EDGE, RDIST_K_MIXED_GEMM, RDIST_K_REFINE,
 RDIST_K_EDGE_UPDATE, RDIST_K_ROWS_STEP, RDIST_K_COUNT) = range(15)

def RDIST_TIMING_CLASS(k: int) -> int:
    return 2 << k


STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_ADJ", 3: "E_NOT_DD", 4: "E_NOMEM", 5: "E_AGAIN",
                6: "E_HIP", 7: "E_STATE"}


class rdist_info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("delta", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("n_unreachable", ctypes.c_int64),
        ("n_subnormal", ctypes.c_int64),
        ("n_saturated", ctypes.c_int64),
        ("n_ambiguous", ctypes.c_int64),
        ("n_negative", ctypes.c_int64),
        ("n_uncertified", ctypes.c_int64),
        ("fallback_fraction", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rdist_request(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("A_dev", ctypes.c_void_p), ("n", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("D_host", ctypes.c_void_p), ("cur_host", ctypes.c_void_p),
                ("goal_host", ctypes.c_void_p),
                ("q", ctypes.c_int32), ("max_hops", ctypes.c_int32), ("paths_host", ctypes.c_void_p),
                ("info_host", ctypes.c_void_p)]


class rdist_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("in_flight", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("batched_requests", ctypes.c_int64), ("max_in_flight", ctypes.c_int64),
                ("footprint_in_flight", ctypes.c_size_t), ("max_footprint_in_flight", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rdist_kernel_stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


INFO_SIZE = ctypes.sizeof(rdist_info)
assert INFO_SIZE == 72, INFO_SIZE

_P = ctypes.c_void_p
_lib.rdist_create.argtypes = [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_size_t, ctypes.c_char_p, ctypes.c_uint32]
_lib.rdist_create.restype = ctypes.c_int
_lib.rdist_destroy.argtypes = [_P]
_lib.rdist_destroy.restype = None
_lib.rdist_solve.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_uint32, _P, ctypes.POINTER(_P),
                             _P, _P]
_lib.rdist_solve.restype = ctypes.c_int
_lib.rdist_solve_noalloc.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_uint32, _P, _P, _P]
_lib.rdist_solve_noalloc.restype = ctypes.c_int
_lib.rdist_solve_batched.argtypes = [_P, ctypes.c_int32, _P, _P, _P, ctypes.c_uint32, _P, _P, _P, _P]
_lib.rdist_solve_batched.restype = ctypes.c_int
_lib.rdist_next_hop.argtypes = [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]
_lib.rdist_next_hop.restype = ctypes.c_int
_lib.rdist_goal_rows.argtypes = [_P, ctypes.c_int32, _P, _P, ctypes.c_int64, _P, ctypes.c_double, _P, ctypes.c_int32,
                                 _P, _P, _P, _P, _P]
_lib.rdist_goal_rows.restype = ctypes.c_int
_lib.rdist_goal_paths.argtypes = [_P, ctypes.c_int32, _P, _P, ctypes.c_int64, _P, _P, _P, ctypes.c_int32,
                                  ctypes.c_int32, _P, _P]
_lib.rdist_goal_paths.restype = ctypes.c_int
class rdist_gain_report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("delta", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("diameter", ctypes.c_int32), ("rho_lo", ctypes.c_double), ("rho_hi", ctypes.c_double),
                ("gamma_c_lo", ctypes.c_double), ("gamma_c_hi", ctypes.c_double), ("gamma_gate", ctypes.c_double),
                ("gamma_global", ctypes.c_double), ("gamma_tree", ctypes.c_double),
                ("gamma_precision", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib.rdist_gain_bounds.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _P, _P]
_lib.rdist_gain_bounds.restype = ctypes.c_int
_lib.rdist_certify.argtypes = [_P, _P, _P, _P, _P]
_lib.rdist_certify.restype = ctypes.c_int
_lib.rdist_graph_release.argtypes = [_P]
_lib.rdist_graph_release.restype = None
_lib.rdist_graph_y.argtypes = [_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
_lib.rdist_graph_y.restype = ctypes.c_int
_lib.rdist_graph_update_edge.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]
_lib.rdist_graph_update_edge.restype = ctypes.c_int
_lib.rdist_graph_update_edges.argtypes = [_P, _P, ctypes.c_int32, _P, _P, _P, _P, _P, _P]
_lib.rdist_graph_update_edges.restype = ctypes.c_int
_lib.rdist_epilogue.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _P, _P, _P]
_lib.rdist_epilogue.restype = ctypes.c_int
_lib.rdist_set_timing.argtypes = [_P, ctypes.c_int]
_lib.rdist_set_timing.restype = ctypes.c_int
_lib.rdist_timing_hold.argtypes = [_P, ctypes.c_int]
_lib.rdist_timing_hold.restype = ctypes.c_int
_lib.rdist_kernel_stats_get.argtypes = [_P, ctypes.c_int, ctypes.POINTER(rdist_kernel_stats)]
_lib.rdist_kernel_stats_get.restype = ctypes.c_int
_lib.rdist_hbm_in_use.argtypes = [_P]
_lib.rdist_hbm_in_use.restype = ctypes.c_size_t
_lib.rdist_last_error.argtypes = []
_lib.rdist_last_error.restype = ctypes.c_char_p
_lib.rdist_status_string.argtypes = [ctypes.c_int]
_lib.rdist_status_string.restype = ctypes.c_char_p
_lib.rdist_server_create.argtypes = [_P, ctypes.c_int32, ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(_P)]
_lib.rdist_server_create.restype = ctypes.c_int
_lib.rdist_server_submit.argtypes = [_P, ctypes.POINTER(rdist_request)]
_lib.rdist_server_submit.restype = ctypes.c_int
_lib.rdist_server_poll.argtypes = [_P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
_lib.rdist_server_poll.restype = ctypes.c_int
_lib.rdist_server_stats_get.argtypes = [_P, ctypes.POINTER(rdist_server_stats)]
_lib.rdist_server_stats_get.restype = ctypes.c_int
_lib.rdist_server_destroy.argtypes = [_P]
_lib.rdist_server_destroy.restype = None

# Raw C entry points under their C names.
rdist_create = _lib.rdist_create
rdist_destroy = _lib.rdist_destroy
rdist_solve = _lib.rdist_solve
rdist_solve_noalloc = _lib.rdist_solve_noalloc
rdist_solve_batched = _lib.rdist_solve_batched
rdist_next_hop = _lib.rdist_next_hop
rdist_graph_release = _lib.rdist_graph_release
rdist_goal_rows = _lib.rdist_goal_rows
rdist_gain_bounds = _lib.rdist_gain_bounds
rdist_certify = _lib.rdist_certify
rdist_goal_paths = _lib.rdist_goal_paths
rdist_graph_y = _lib.rdist_graph_y
rdist_graph_update_edge = _lib.rdist_graph_update_edge
rdist_graph_update_edges = _lib.rdist_graph_update_edges
rdist_epilogue = _lib.rdist_epilogue
rdist_set_timing = _lib.rdist_set_timing
rdist_timing_hold = _lib.rdist_timing_hold
rdist_kernel_stats_get = _lib.rdist_kernel_stats_get
rdist_hbm_in_use = _lib.rdist_hbm_in_use
rdist_last_error = _lib.rdist_last_error
rdist_status_string = _lib.rdist_status_string
rdist_server_create = _lib.rdist_server_create
rdist_server_submit = _lib.rdist_server_submit
rdist_server_poll = _lib.rdist_server_poll
rdist_server_stats_get = _lib.rdist_server_stats_get
rdist_server_destroy = _lib.rdist_server_destroy

EXPORTS = ("rdist_create", "rdist_destroy", "rdist_solve", "rdist_solve_noalloc", "rdist_solve_batched", "rdist_next_hop",
           "rdist_graph_release", "rdist_graph_y", "rdist_graph_update_edge", "rdist_graph_update_edges", "rdist_goal_rows", "rdist_goal_paths",
           "rdist_gain_bounds", "rdist_certify",
           "rdist_epilogue", "rdist_set_timing", "rdist_timing_hold",
           "rdist_kernel_stats_get", "rdist_hbm_in_use", "rdist_last_error", "rdist_status_string",
           "rdist_server_create", "rdist_server_submit", "rdist_server_poll", "rdist_server_stats_get",
           "rdist_server_destroy")
RDIST_QUERY_D = 0
RDIST_QUERY_PATHS = 1


class RdistError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = rdist_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} {msg}")
        self.status = status


def _check(st: int, where: str):
    if st != RDIST_OK:
        raise RdistError(st, where)


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def path_shape(q: int, max_hops: int) -> tuple:
    """Shape of a path output: (q,) next nodes for max_hops = 1, else (q, max_hops + 1) rows."""
    return (q,) if max_hops == 1 else (q, max_hops + 1)


class PinnedInfo:
    """rdist_info records in pinned host memory (written asynchronously by the device)."""

    def __init__(self, count: int = 1):
        self.count = count
        self.buf = torch.zeros(count * INFO_SIZE, dtype=torch.uint8, pin_memory=True)
        self.ptr = self.buf.data_ptr()

    def at(self, i: int = 0) -> int:
        return self.ptr + i * INFO_SIZE

    def get(self, i: int = 0) -> rdist_info:
        return rdist_info.from_address(self.at(i))


@dataclass
class Graph:
    """A kept graph: device-resident Y (+ successor bitmaps) owned by the engine."""
    ctx: "Context"
    handle: int
    n: int

    def update_edge(self, src: int, dst: int, weight: int, D: torch.Tensor | None = None, stream=None) -> dict:
        """Sets the weight of edge src -> dst (0 removes it) by a rank-one update of Y;
        D (optional, n x n int16) receives the new D.  Blocks until the change is
        complete; returns the call's info."""
        if D is not None:
            assert D.is_cuda and D.dtype == torch.int16 and D.numel() == self.n * self.n
        out = rdist_info()
        _check(rdist_graph_update_edge(self.ctx.handle, self.handle, int(src), int(dst), int(weight),
                                       D.data_ptr() if D is not None else None, ctypes.byref(out),
                                       _stream_ptr(stream)),
               "rdist_graph_update_edge")
        return out.as_dict()

    def update_edges(self, changes, D: torch.Tensor | None = None, stream=None) -> dict:
        """Applies [(src, dst, weight), ...] in order (chunks of up to 8 per pass over Y);
        D (optional) receives the final D.  Blocks; returns the call's info."""
        ch = np.asarray(changes, dtype=np.int32).reshape(-1, 3)
        if D is not None:
            assert D.is_cuda and D.dtype == torch.int16 and D.numel() == self.n * self.n
        srcs = np.ascontiguousarray(ch[:, 0])
        dsts = np.ascontiguousarray(ch[:, 1])
        ws = np.ascontiguousarray(ch[:, 2])
        out = rdist_info()
        _check(rdist_graph_update_edges(self.ctx.handle, self.handle, int(ch.shape[0]), srcs.ctypes.data,
                                        dsts.ctypes.data, ws.ctypes.data, D.data_ptr() if D is not None else None,
                                        ctypes.byref(out), _stream_ptr(stream)), "rdist_graph_update_edges")
        return out.as_dict()

    def y(self) -> torch.Tensor:
        """Copy of Y (n x n float64) on the device."""
        yp, n, ld = _P(), ctypes.c_int32(), ctypes.c_int32()
        _check(rdist_graph_y(self.handle, ctypes.byref(yp), ctypes.byref(n), ctypes.byref(ld)), "rdist_graph_y")
        out = torch.empty((n.value, n.value), dtype=torch.float64, device=self.ctx.device)
        torch.cuda.synchronize(self.ctx.device)
        err = _hip.hipMemcpy2D(_P(out.data_ptr()), ctypes.c_size_t(8 * n.value), yp,
                               ctypes.c_size_t(8 * ld.value), ctypes.c_size_t(8 * n.value),
                               ctypes.c_size_t(n.value), 3)   # hipMemcpyDeviceToDevice
        if err != 0:
            raise RuntimeError(f"hipMemcpy2D failed with {err}")
        return out

    def release(self):
        if self.handle:
            rdist_graph_release(self.handle)
            self.handle = 0


class Batch:
    """Argument arrays of one batch (sizes, adjacency and output pointers,
    gains) marshalled once, for repeated rdist_solve_batched calls."""

    def __init__(self, As, gamma, Ds=None):
        self.As = list(As)
        self.count = len(self.As)
        for a in self.As:
            assert a.is_cuda and a.dtype == torch.uint8 and a.dim() == 2 and a.shape[0] == a.shape[1]
            assert a.is_contiguous()
        if Ds is None:
            Ds = [torch.empty((int(a.shape[0]),) * 2, dtype=torch.int16, device=a.device) for a in self.As]
        self.Ds = list(Ds)
        for a, d in zip(self.As, self.Ds):
            assert d.is_cuda and d.dtype == torch.int16 and d.is_contiguous() and d.numel() == a.shape[0] ** 2
        gam = gamma if hasattr(gamma, "__len__") else [gamma] * self.count
        self.ns = (ctypes.c_int32 * self.count)(*[int(a.shape[0]) for a in self.As])
        self.aptr = (ctypes.c_void_p * self.count)(*[a.data_ptr() for a in self.As])
        self.dptr = (ctypes.c_void_p * self.count)(*[d.data_ptr() for d in self.Ds])
        self.gptr = (ctypes.c_double * self.count)(*[float(x) for x in gam])


class Context:
    """One engine context on a device (owns workspaces, budget, kept graphs)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, tile_cache: str | None = None,
                 threadsafe: bool = False):
        self.device = torch.device("cuda", device)
        h = _P()
        _check(rdist_create(ctypes.byref(h), device, hbm_budget,
                            tile_cache.encode() if tile_cache else None,
                            RDIST_THREADSAFE if threadsafe else 0), "rdist_create")
        self.handle = h.value
        self.info = PinnedInfo(1)

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            rdist_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- solves ----
    def solve_async(self, A: torch.Tensor, gamma: float, flags: int = RDIST_F64, D: torch.Tensor | None = None,
                    keep: bool = False, info: PinnedInfo | None = None, info_index: int = 0, stream=None):
        """Enqueues one solve; returns (D, Graph or None).  info is filled when the stream gets there."""
        assert A.is_cuda and A.dtype == torch.uint8 and A.dim() == 2 and A.shape[0] == A.shape[1]
        A = A.contiguous()
        n = A.shape[0]
        if D is None:
            D = torch.empty((n, n), dtype=torch.int16, device=A.device)
        assert D.is_cuda and D.dtype == torch.int16 and D.is_contiguous() and D.numel() == n * n
        if keep:
            flags |= RDIST_KEEP_Y
        g = _P()
        info = info or self.info
        st = rdist_solve(self.handle, A.data_ptr(), n, float(gamma), flags, D.data_ptr(),
                         ctypes.byref(g) if keep else None, info.at(info_index), _stream_ptr(stream))
        _check(st, "rdist_solve")
        graph = Graph(self, g.value, n) if keep else None
        return D, graph

    def solve(self, A: torch.Tensor, gamma: float, flags: int = RDIST_F64, D: torch.Tensor | None = None,
              keep: bool = False, stream=None):
        """Synchronous convenience: returns (D, info dict, Graph or None)."""
        D, graph = self.solve_async(A, gamma, flags, D, keep, self.info, 0, stream)
        (stream or torch.cuda.current_stream()).synchronize()
        return D, self.info.get(0).as_dict(), graph

    def solve_batched(self, As, gamma=None, flags: int = RDIST_F64, Ds=None, keep: bool = False, stream=None,
                      info: PinnedInfo | None = None, sync: bool = True):
        """Solves many graphs in one call.  As: list of uint8 adjacency tensors,
        or a Batch (its argument arrays are reused as they are)."""
        b = As if isinstance(As, Batch) else Batch(As, gamma, Ds)
        info = info or PinnedInfo(b.count)
        keeps = (ctypes.c_void_p * b.count)() if keep else None
        if keep:
            flags |= RDIST_KEEP_Y
        st = rdist_solve_batched(self.handle, b.count, b.ns, b.aptr, b.gptr, flags, b.dptr, keeps, info.ptr,
                                 _stream_ptr(stream))
        _check(st, "rdist_solve_batched")
        graphs = [Graph(self, keeps[i], int(b.ns[i])) for i in range(b.count)] if keep else None
        if sync:
            (stream or torch.cuda.current_stream()).synchronize()
        return b.Ds, info, graphs

    def next_hop(self, graph: Graph, cur: torch.Tensor, goal: torch.Tensor, max_hops: int = 1,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        q = int(cur.numel())
        cur = cur.to(device=self.device, dtype=torch.int32).contiguous()
        goal = goal.to(device=self.device, dtype=torch.int32).contiguous()
        if out is None:
            out = torch.empty(path_shape(q, max_hops), dtype=torch.int32, device=self.device)
        st = rdist_next_hop(self.handle, graph.handle, cur.data_ptr(), goal.data_ptr(), q, max_hops,
                            out.data_ptr(), _stream_ptr(stream))
        _check(st, "rdist_next_hop")
        return out

    def goal_rows(self, ptr: torch.Tensor, idx: torch.Tensor, goals: torch.Tensor, gamma: float,
                  weights: torch.Tensor | None = None, want_y: bool = True, want_d: bool = True, stream=None):
        """Rows Y[g, :] (and their D) for the goals of a graph given as successor lists
        (device tensors: ptr int64 (n + 1), idx int32); returns (Y or None, D or None, info, steps)."""
        assert ptr.is_cuda and ptr.dtype == torch.int64 and idx.is_cuda and idx.dtype == torch.int32
        n = int(ptr.numel()) - 1
        goals = goals.to(device=self.device, dtype=torch.int32).contiguous()
        q = int(goals.numel())
        Y = torch.empty((q, n), dtype=torch.float64, device=self.device) if want_y else None
        D = torch.empty((q, n), dtype=torch.int16, device=self.device) if want_d else None
        if weights is not None:
            assert weights.is_cuda and weights.dtype == torch.uint8 and weights.numel() == idx.numel()
        steps = ctypes.c_int32(0)
        st = rdist_goal_rows(self.handle, n, ptr.data_ptr(), idx.data_ptr() if idx.numel() else None,
                             int(idx.numel()), weights.data_ptr() if weights is not None else None, float(gamma),
                             goals.data_ptr(), q, Y.data_ptr() if Y is not None else None,
                             D.data_ptr() if D is not None else None, ctypes.byref(steps), self.info.at(0),
                             _stream_ptr(stream))
        _check(st, "rdist_goal_rows")
        (stream or torch.cuda.current_stream()).synchronize()
        return Y, D, self.info.get(0).as_dict(), int(steps.value)

    def gain_bounds(self, A: torch.Tensor, diameter: int = 0, max_steps: int = 4000, rel_tol: float = 1e-10,
                    stream=None) -> dict:
        """Bracket of rho(A), the critical gain and the paper's bounds on gamma (a dict)."""
        assert A.is_cuda and A.dtype == torch.uint8 and A.dim() == 2 and A.shape[0] == A.shape[1]
        A = A.contiguous()
        r = rdist_gain_report()
        _check(rdist_gain_bounds(self.handle, A.data_ptr(), A.shape[0], int(diameter), int(max_steps),
                                 float(rel_tol), ctypes.byref(r), _stream_ptr(stream)), "rdist_gain_bounds")
        return r.as_dict()

    def certify(self, graph: "Graph", want_mask: bool = False, stream=None):
        """Per-entry certificate of a kept graph's D: (count, n x n uint8 mask or None)."""
        mask = torch.empty((graph.n, graph.n), dtype=torch.uint8, device=self.device) if want_mask else None
        cnt = ctypes.c_int64(0)
        _check(rdist_certify(self.handle, graph.handle, mask.data_ptr() if mask is not None else None,
                             ctypes.byref(cnt), _stream_ptr(stream)), "rdist_certify")
        return int(cnt.value), mask

    def goal_paths(self, ptr: torch.Tensor, idx: torch.Tensor, Y_rows: torch.Tensor, goals: torch.Tensor,
                   starts: torch.Tensor, max_hops: int, stream=None) -> torch.Tensor:
        """Greedy paths over goal rows (query k: row k, goals[k], starts[k])."""
        n = int(ptr.numel()) - 1
        goals = goals.to(device=self.device, dtype=torch.int32).contiguous()
        starts = starts.to(device=self.device, dtype=torch.int32).contiguous()
        q = int(goals.numel())
        out = torch.empty(path_shape(q, max_hops), dtype=torch.int32, device=self.device)
        st = rdist_goal_paths(self.handle, n, ptr.data_ptr(), idx.data_ptr(), int(idx.numel()), Y_rows.data_ptr(),
                              goals.data_ptr(),
                              starts.data_ptr(), q, max_hops, out.data_ptr(), _stream_ptr(stream))
        _check(st, "rdist_goal_paths")
        return out

    def epilogue(self, Y: torch.Tensor, gamma: float, n: int | None = None, D: torch.Tensor | None = None,
                 stream=None):
        assert Y.is_cuda and Y.dtype == torch.float64 and Y.stride(1) == 1
        n = n or Y.shape[0]
        if D is None:
            D = torch.empty((n, n), dtype=torch.int16, device=Y.device)
        st = rdist_epilogue(self.handle, Y.data_ptr(), n, Y.stride(0), float(gamma), D.data_ptr(),
                            self.info.at(0), _stream_ptr(stream))
        _check(st, "rdist_epilogue")
        return D

    # ---- timing ----
    def set_timing(self, on: bool, classes=None):
        """Event timing of every kernel class, or of the RDIST_K_* classes listed."""
        mask = (1 if on else 0) if classes is None else sum(RDIST_TIMING_CLASS(k) for k in classes)
        _check(rdist_set_timing(self.handle, mask), "rdist_set_timing")

    def timing_hold(self, hold: bool):
        """Launches enqueued while held are not timed; counters and pending timings are kept."""
        _check(rdist_timing_hold(self.handle, 1 if hold else 0), "rdist_timing_hold")

    def kernel_stats(self, which: int) -> dict:
        s = rdist_kernel_stats()
        _check(rdist_kernel_stats_get(self.handle, which, ctypes.byref(s)), "rdist_kernel_stats_get")
        return {"launches": s.launches, "total_ms": s.total_ms, "flops": s.flops, "bytes": s.bytes}

    def hbm_in_use(self) -> int:
        return int(rdist_hbm_in_use(self.handle))


class Server:
    """The engine's request loop (continuous batching, HBM-footprint admission).

    submit() queues a request (A on the device, results into pinned host
    buffers the caller keeps alive until the request is reported done);
    poll() returns the ids finished since the last call and dispatches more.
    """

    def __init__(self, ctx: Context, slots: int = 8, hbm_budget: int = 0, max_batch: int = 64):
        self.ctx = ctx
        h = _P()
        _check(rdist_server_create(ctx.handle, slots, hbm_budget, max_batch, ctypes.byref(h)), "rdist_server_create")
        self.handle = h.value
        self._ids = (ctypes.c_int64 * 4096)()
        self._req = rdist_request()

    def submit(self, rid: int, A: torch.Tensor, gamma: float, kind: int = RDIST_QUERY_D, D_host=None,
               cur_host=None, goal_host=None, max_hops: int = 64, paths_host=None, info_ptr: int = 0):
        r = self._req
        r.id = rid
        r.A_dev = A.data_ptr()
        r.n = int(A.shape[0])
        r.kind = kind
        r.gamma = float(gamma)
        r.D_host = D_host.data_ptr() if D_host is not None else None
        r.cur_host = cur_host.data_ptr() if cur_host is not None else None
        r.goal_host = goal_host.data_ptr() if goal_host is not None else None
        r.q = int(cur_host.numel()) if cur_host is not None else 0
        r.max_hops = max_hops
        r.paths_host = paths_host.data_ptr() if paths_host is not None else None
        r.info_host = info_ptr or None
        return rdist_server_submit(self.handle, ctypes.byref(r))

    def poll(self) -> list:
        n = ctypes.c_int32()
        _check(rdist_server_poll(self.handle, self._ids, 4096, ctypes.byref(n)), "rdist_server_poll")
        return [self._ids[i] for i in range(n.value)]

    def stats(self) -> dict:
        s = rdist_server_stats()
        _check(rdist_server_stats_get(self.handle, ctypes.byref(s)), "rdist_server_stats_get")
        return s.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            rdist_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
