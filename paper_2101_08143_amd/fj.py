"""Thin ctypes binding of libfjgpu (include/fj.h). Argument marshalling only:
every step of the computation runs in the library's HIP kernels.

PyTorch provides device memory (plan, workspace, vectors) and the stream
(torch.cuda.current_stream()). The binding raises if the library has not been
built; there is no fallback of any kind.

Entry points keep the C names: fj_plan_bytes, fj_prepare, fj_workspace_bytes,
fj_apply, fj_solve, fj_indices, fj_status_string, fj_default_opts. The Graph
class and indices()/solve() wrap them for tensors.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FJGPU_LIB selects another build of the same library (for tuning experiments).
LIB_PATH = os.environ.get("FJGPU_LIB", os.path.join(_HERE, "libfjgpu.so"))

FJ_OK = 0
FJ_ERR_INVALID_ARG = 1
FJ_ERR_INVALID_GRAPH = 2
FJ_ERR_OPINION_RANGE = 3
FJ_ERR_WORKSPACE = 4
FJ_ERR_NOT_CONVERGED = 5
FJ_ERR_BREAKDOWN = 6
FJ_ERR_UNCERTIFIABLE = 7
FJ_ERR_HIP = 8
FJ_ERR_CANCELLED = 9
FJ_ERR_HOST_MEMORY = 10
FJ_ERR_INTERNAL = 11

FJ_VAL_UNIT, FJ_VAL_F32, FJ_VAL_F64 = 0, 1, 2
FJ_FP64, FJ_MIXED = 0, 1
FJ_TWO_SOLVE, FJ_NO_RANGE_CHECK, FJ_VALIDATE_GRAPH, FJ_PROFILE, FJ_NO_TUNE, FJ_WARM_START, FJ_ZERO_START = \
    1, 2, 4, 8, 16, 32, 64
FJ_DIAG_PRECOND = 128
FJ_BLOCK_CG = 256
FJ_MULTILEVEL = 512
FJ_WINDOW_SPMV = 1024
FJ_PHASED_SPMV = 2048

INDEX_NAMES = ("internal_conflict", "disagreement", "polarization", "controversy", "dc_index")

# Every function declared in include/fj.h, in declaration order.
EXPORTS = ("fj_default_opts", "fj_status_string", "fj_last_error", "fj_plan_bytes", "fj_prepare",
           "fj_workspace_bytes", "fj_apply", "fj_apply_phased", "fj_solve", "fj_apriori_delta", "fj_spmm_choice",
           "fj_spmm_set_choice", "fj_reorder_by_degree", "fj_permute", "fj_hierarchy_create", "fj_hierarchy_shape",
           "fj_hierarchy_destroy",
           "fj_gather_bound", "fj_gather_bound_sliced", "fj_dynamics", "fj_indices", "fj_indices_noalloc",
           "fj_server_block_bytes",
           "fj_server_create", "fj_server_destroy", "fj_server_add_graph", "fj_server_submit",
           "fj_server_step", "fj_server_poll", "fj_server_cancel")


class fj_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p), ("val_type", ctypes.c_int32)]


class fj_opts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32),
                ("hierarchy", ctypes.c_void_p)]


class fj_indices_t(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in INDEX_NAMES]


class fj_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("bound", ctypes.c_double * 5), ("ms_spmv", ctypes.c_double),
                ("n_spmv", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("residual_norm", ctypes.c_double), ("abs_bound", ctypes.c_double * 5)]


class fj_server_opts(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t), ("block_columns", ctypes.c_int32),
                ("iters_per_replay", ctypes.c_int32), ("eps", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("large_lanes", ctypes.c_int32),
                ("large_iters_per_replay", ctypes.c_int32), ("large_blocks", ctypes.c_int32),
                ("large_entries", ctypes.c_int64)]


class fj_server_done(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("graph_id", ctypes.c_int32), ("status", ctypes.c_int32),
                ("latency_ms", ctypes.c_double)]


class FJError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = fj_status_string(status)
        extra = last_error()
        super().__init__(f"{where}: {msg} (status {status})" + (f" [{extra}]" if extra else ""))


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2101_08143_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.fj_default_opts.argtypes = [P(fj_opts)]
        L.fj_default_opts.restype = None
        L.fj_status_string.argtypes = [ctypes.c_int]
        L.fj_status_string.restype = ctypes.c_char_p
        L.fj_last_error.argtypes = []
        L.fj_last_error.restype = ctypes.c_char_p
        L.fj_plan_bytes.argtypes = [P(fj_csr)]
        L.fj_plan_bytes.restype = sz
        L.fj_prepare.argtypes = [P(fj_csr), P(fj_opts), vp, sz, vp]
        L.fj_workspace_bytes.argtypes = [P(fj_csr), i32, P(fj_opts)]
        L.fj_workspace_bytes.restype = sz
        L.fj_apply.argtypes = [P(fj_csr), vp, vp, vp, vp]
        L.fj_apply_phased.argtypes = [P(fj_csr), vp, vp, vp, vp]
        L.fj_apriori_delta.argtypes = [i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.fj_apriori_delta.restype = ctypes.c_double
        L.fj_spmm_choice.argtypes = [P(fj_csr), i32, i32, P(i32), P(i32), P(i32), P(i32)]
        L.fj_spmm_set_choice.argtypes = [P(fj_csr), i32, i32, i32, i32, i32, i32]
        L.fj_gather_bound.argtypes = [P(fj_csr), vp, vp, vp]
        L.fj_reorder_by_degree.argtypes = [P(fj_csr), vp, vp, vp, vp, vp]
        L.fj_permute.argtypes = [i32, i32, vp, vp, i64, vp, i64, i32, vp]
        L.fj_hierarchy_create.argtypes = [P(fj_csr), i32, P(vp), vp]
        L.fj_hierarchy_shape.argtypes = [vp, P(i32), P(i32), P(i64), P(i32)]
        L.fj_hierarchy_destroy.argtypes = [vp]
        L.fj_gather_bound_sliced.argtypes = [P(fj_csr), vp, i32, vp, i32, i32, vp, P(i64), vp]
        L.fj_dynamics.argtypes = [P(fj_csr), vp, vp, vp, vp, i32, ctypes.c_double, vp, sz, vp, P(fj_info)]
        L.fj_solve.argtypes = [P(fj_csr), vp, i32, vp, i64, vp, i64, P(fj_opts), vp, sz, vp, P(fj_info)]
        L.fj_indices.argtypes = [P(fj_csr), vp, i32, vp, i64, P(fj_opts), vp, sz, vp, P(fj_indices_t),
                                 P(fj_info)]
        L.fj_indices_noalloc.argtypes = [P(fj_csr), vp, i32, vp, i64, P(fj_opts), vp, P(fj_indices_t), P(fj_info)]
        L.fj_server_block_bytes.argtypes = [i32, i32, i32]
        L.fj_server_block_bytes.restype = sz
        L.fj_server_create.argtypes = [P(fj_server_opts), P(vp)]
        L.fj_server_destroy.argtypes = [vp]
        L.fj_server_add_graph.argtypes = [vp, P(fj_csr), vp, P(i32), vp]
        L.fj_server_submit.argtypes = [vp, i32, i32, vp, i64, P(fj_indices_t), P(fj_info), P(ctypes.c_uint64), vp]
        L.fj_server_step.argtypes = [vp, P(i32)]
        L.fj_server_poll.argtypes = [vp, P(fj_server_done), i32, P(i32)]
        L.fj_server_cancel.argtypes = [vp, ctypes.c_uint64]
        for name in ("fj_prepare", "fj_apply", "fj_apply_phased", "fj_spmm_choice", "fj_spmm_set_choice", "fj_gather_bound",
                     "fj_gather_bound_sliced", "fj_hierarchy_create", "fj_hierarchy_shape", "fj_hierarchy_destroy",
                     "fj_reorder_by_degree", "fj_permute",
                     "fj_dynamics", "fj_solve", "fj_indices", "fj_indices_noalloc", "fj_server_create",
                     "fj_server_destroy",
                     "fj_server_add_graph", "fj_server_submit", "fj_server_step", "fj_server_poll",
                     "fj_server_cancel"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def fj_status_string(status: int) -> str:
    return lib().fj_status_string(int(status)).decode()


def last_error() -> str:
    return lib().fj_last_error().decode()


def fj_default_opts() -> fj_opts:
    o = fj_opts()
    lib().fj_default_opts(ctypes.byref(o))
    return o


def make_opts(eps=1e-6, rtol=0.0, max_iter=0, precision=FJ_FP64, flags=0, hierarchy=None) -> fj_opts:
    """Solve options. hierarchy: a Hierarchy; passing one sets FJ_MULTILEVEL."""
    o = fj_default_opts()
    o.eps, o.rtol, o.max_iter, o.precision, o.flags = eps, rtol, max_iter, precision, flags
    if hierarchy is not None:
        o.flags |= FJ_MULTILEVEL
        o.hierarchy = hierarchy.handle
    return o


def _stream_handle(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _aligned_empty(torch, nbytes, device):
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


@dataclass
class Graph:
    """A graph resident in HBM with its prepared plan (fj_prepare)."""

    n: int
    nnz: int
    row_ptr: object
    col: object
    val: object
    val_type: int
    plan: object
    csr: fj_csr
    device: object

    @classmethod
    def from_csr(cls, g, device="cuda", validate=True, stream=None) -> "Graph":
        """g: a workloads.CSRGraph (numpy arrays). Copies to the device and prepares."""
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int32)).to(device)
        col = torch.from_numpy(np.ascontiguousarray(g.col, dtype=np.int32)).to(device)
        if g.val is None:
            val, vt = None, FJ_VAL_UNIT
        elif g.val.dtype == np.float32:
            val, vt = torch.from_numpy(np.ascontiguousarray(g.val)).to(device), FJ_VAL_F32
        else:
            val, vt = torch.from_numpy(np.ascontiguousarray(g.val, dtype=np.float64)).to(device), FJ_VAL_F64
        return cls.from_tensors(g.n, rp, col, val, vt, validate=validate, stream=stream)

    @classmethod
    def from_tensors(cls, n, row_ptr, col, val, val_type, validate=True, stream=None) -> "Graph":
        import torch
        nnz = int(col.numel())
        csr = fj_csr(n=int(n), nnz=nnz, row_ptr=_ptr(row_ptr), col_idx=_ptr(col) if nnz else None,
                     val=_ptr(val) if val is not None else None, val_type=val_type)
        device = row_ptr.device
        nbytes = lib().fj_plan_bytes(ctypes.byref(csr))
        plan = _aligned_empty(torch, nbytes, device)
        o = make_opts(flags=FJ_VALIDATE_GRAPH if validate else 0)
        rc = lib().fj_prepare(ctypes.byref(csr), ctypes.byref(o), _ptr(plan), nbytes,
                              _stream_handle(torch, stream))
        if rc != FJ_OK:
            raise FJError(rc, "fj_prepare")
        return cls(n=int(n), nnz=nnz, row_ptr=row_ptr, col=col, val=val, val_type=val_type, plan=plan,
                   csr=csr, device=device)

    def workspace(self, k=1, opts: Optional[fj_opts] = None):
        import torch
        o = opts or fj_default_opts()
        nbytes = lib().fj_workspace_bytes(ctypes.byref(self.csr), int(k), ctypes.byref(o))
        return _aligned_empty(torch, nbytes, self.device)


def fj_apply(graph: Graph, x, y=None, stream=None, phased=False):
    """y = (I + L) x for a device float64 vector x; phased=True runs
    fj_apply_phased (the time-phased layout of the plan)."""
    import torch
    assert x.dtype == torch.float64 and x.is_contiguous() and x.numel() == graph.n
    if y is None:
        y = torch.empty_like(x)
    fn = lib().fj_apply_phased if phased else lib().fj_apply
    rc = fn(ctypes.byref(graph.csr), _ptr(graph.plan), _ptr(x), _ptr(y), _stream_handle(torch, stream))
    if rc != FJ_OK:
        raise FJError(rc, "fj_apply_phased" if phased else "fj_apply")
    return y


def _check_block(graph, S, name):
    import torch
    if S.dtype != torch.float64 or S.device != graph.device:
        raise ValueError(f"{name} must be float64 on {graph.device}")
    if S.dim() == 1:
        S = S.view(-1, 1)
    if S.dim() != 2 or S.shape[0] != graph.n or S.stride(1) != 1:
        raise ValueError(f"{name} must be n x k with unit column stride")
    return S, S.shape[1], S.stride(0)


def fj_apriori_delta(n: int, w_min: float, w_max: float, sbar_norm: float, eps: float) -> float:
    """Algorithm 1's a-priori solver accuracy delta (for reports)."""
    return lib().fj_apriori_delta(int(n), float(w_min), float(w_max), float(sbar_norm), float(eps))


def fj_spmm_choice(graph: Graph, kb: int, precision: int = 0):
    """(columns per lane, grid, split, passes) the SpMM autotuner chose for this
    graph, block width and precision, or None if nothing is tuned yet."""
    cpl, grid, split, passes = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    rc = lib().fj_spmm_choice(ctypes.byref(graph.csr), int(kb), int(precision), ctypes.byref(cpl),
                              ctypes.byref(grid), ctypes.byref(split), ctypes.byref(passes))
    return (cpl.value, grid.value, split.value, passes.value) if rc == FJ_OK else None


def fj_spmm_set_choice(graph: Graph, kb: int, cpl: int, grid: int, precision: int = 0, split: int = 1,
                       passes: int = 1):
    """Pin the SpMM launch shape (columns per lane, grid, split, column passes)
    instead of tuning it."""
    rc = lib().fj_spmm_set_choice(ctypes.byref(graph.csr), int(kb), int(precision), int(cpl), int(grid),
                                  int(split), int(passes))
    if rc != FJ_OK:
        raise FJError(rc, "fj_spmm_set_choice")


def reorder_by_degree(graph: "Graph", validate=True, stream=None):
    """fj_reorder_by_degree: the graph relabelled by non-increasing degree,
    prepared, and perm (device int32[n], new node i = old node perm[i])."""
    import torch
    dev = graph.device
    perm = torch.empty(graph.n, dtype=torch.int32, device=dev)
    rp = torch.empty(graph.n + 1, dtype=torch.int32, device=dev)
    col = torch.empty(graph.nnz, dtype=torch.int32, device=dev)
    val = None if graph.val is None else torch.empty_like(graph.val)
    rc = lib().fj_reorder_by_degree(ctypes.byref(graph.csr), _ptr(perm), _ptr(rp), _ptr(col) if graph.nnz else None,
                                    _ptr(val), _stream_handle(torch, stream))
    if rc != FJ_OK:
        raise FJError(rc, "fj_reorder_by_degree")
    return Graph.from_tensors(graph.n, rp, col, val, graph.val_type, validate=validate), perm


def permute(perm, x, inverse=False, stream=None):
    """fj_permute: x (float64, n or n x k, device) from the old labels to the
    new ones (or back with inverse=True) for perm[new] = old."""
    import torch
    assert x.dtype == torch.float64 and x.is_contiguous()
    n = x.shape[0]
    k = 1 if x.dim() == 1 else x.shape[1]
    y = torch.empty_like(x)
    rc = lib().fj_permute(int(n), int(k), _ptr(perm), _ptr(x), k, _ptr(y), k, 1 if inverse else 0,
                          _stream_handle(torch, stream))
    if rc != FJ_OK:
        raise FJError(rc, "fj_permute")
    return y


class Hierarchy:
    """The aggregation hierarchy of FJ_MULTILEVEL for one graph (see
    include/fj.h, fj_hierarchy_create). It keeps the graph alive; pass it to
    make_opts(hierarchy=...). One solve at a time per hierarchy."""

    def __init__(self, graph: "Graph", coarse_max: int = 0, stream=None):
        import torch
        self.graph = graph
        self.handle = None
        h = ctypes.c_void_p()
        rc = lib().fj_hierarchy_create(ctypes.byref(graph.csr), int(coarse_max), ctypes.byref(h),
                                       _stream_handle(torch, stream))
        if rc != FJ_OK:
            raise FJError(rc, "fj_hierarchy_create")
        self.handle = h.value

    def shape(self):
        """(levels, [n per level], [stored entries per level], dense last level)"""
        lv, dense = ctypes.c_int32(0), ctypes.c_int32(0)
        n, nnz = (ctypes.c_int32 * 16)(), (ctypes.c_int64 * 16)()
        rc = lib().fj_hierarchy_shape(self.handle, ctypes.byref(lv), n, nnz, ctypes.byref(dense))
        if rc != FJ_OK:
            raise FJError(rc, "fj_hierarchy_shape")
        k = lv.value
        return k, list(n[:k]), list(nnz[:k]), bool(dense.value)

    def close(self):
        if self.handle is not None:
            lib().fj_hierarchy_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fj_gather_bound(graph: Graph, x, y=None, stream=None):
    """Measurement aid: the bare CSR-order gather (see include/fj.h). Returns y."""
    import torch
    assert x.dtype == torch.float64 and x.is_contiguous() and x.numel() == graph.n
    if y is None:
        y = torch.empty((graph.csr.nnz + 7) // 8, dtype=torch.float64, device=x.device)
    rc = lib().fj_gather_bound(ctypes.byref(graph.csr), _ptr(x), _ptr(y), _stream_handle(torch, stream))
    if rc != FJ_OK:
        raise FJError(rc, "fj_gather_bound")
    return y


def fj_gather_bound_sliced(graph: Graph, x, slices: int = 8, hub_cols: int = 0, y=None, check=None, stream=None):
    """Measurement aid: the gather over XCD-aligned entry streams (see
    include/fj.h). x is float64 or float32. Returns (y, bounds)."""
    import torch
    assert x.dtype in (torch.float64, torch.float32) and x.is_contiguous() and x.numel() == graph.n
    if y is None:
        y = torch.empty((graph.csr.nnz + 7) // 8 + 8, dtype=torch.float64, device=x.device)
    bounds = (ctypes.c_int64 * 9)()
    rc = lib().fj_gather_bound_sliced(ctypes.byref(graph.csr), _ptr(x), 8 if x.dtype == torch.float64 else 4,
                                      _ptr(y), int(slices), int(hub_cols), _ptr(check) if check is not None else None,
                                      bounds, _stream_handle(torch, stream))
    if rc != FJ_OK:
        raise FJError(rc, "fj_gather_bound_sliced")
    return y, list(bounds)


def fj_dynamics(graph: Graph, s, steps: int, tol: float = -1.0, z0=None, z=None, ws=None, stream=None):
    """Up to `steps` synchronous FJ updates (Eq. FJmodel) from z0 (default s);
    stops early once a step changes no z_i by more than tol (tol < 0: never).
    Returns (z, info dict); FJ_ERR_NOT_CONVERGED is reported in info, not raised."""
    import torch
    assert s.dtype == torch.float64 and s.is_contiguous() and s.numel() == graph.n
    if z0 is not None:
        assert z0.dtype == torch.float64 and z0.is_contiguous() and z0.numel() == graph.n
    if z is None:
        z = torch.empty_like(s)
    if ws is None:
        ws = graph.workspace(1)
    inf = fj_info()
    rc = lib().fj_dynamics(ctypes.byref(graph.csr), _ptr(graph.plan), _ptr(s),
                           _ptr(z0) if z0 is not None else None, _ptr(z), int(steps), float(tol),
                           _ptr(ws), ws.numel(), _stream_handle(torch, stream), ctypes.byref(inf))
    if rc not in (FJ_OK, FJ_ERR_NOT_CONVERGED):
        raise FJError(rc, "fj_dynamics")
    return z, info_dict(inf)


def fj_solve(graph: Graph, S, opts: Optional[fj_opts] = None, ws=None, Z=None, stream=None,
             check=True):
    """Z ~= (I+L)^{-1} S. Returns (Z, [fj_info]*k, status)."""
    import torch
    S2, k, lds = _check_block(graph, S, "S")
    o = opts or fj_default_opts()
    if Z is None:
        Z = torch.empty((graph.n, k), dtype=torch.float64, device=graph.device)
    Z2, kz, ldz = _check_block(graph, Z, "Z")
    assert kz == k
    if ws is None:
        ws = graph.workspace(k, o)
    info = (fj_info * k)()
    rc = lib().fj_solve(ctypes.byref(graph.csr), _ptr(graph.plan), k, _ptr(S2), lds, _ptr(Z2), ldz,
                        ctypes.byref(o), _ptr(ws), ws.numel(), _stream_handle(torch, stream), info)
    if check and rc not in (FJ_OK,):
        raise FJError(rc, "fj_solve")
    return (Z.view(-1) if S.dim() == 1 else Z), list(info), rc


def fj_indices(graph: Graph, S, opts: Optional[fj_opts] = None, ws=None, stream=None, check=True):
    """Algorithm 1: the five indices per column. Returns (list of dicts, [fj_info]*k, status)."""
    import torch
    S2, k, lds = _check_block(graph, S, "S")
    o = opts or fj_default_opts()
    if ws is None:
        ws = graph.workspace(k, o)
    out = (fj_indices_t * k)()
    info = (fj_info * k)()
    rc = lib().fj_indices(ctypes.byref(graph.csr), _ptr(graph.plan), k, _ptr(S2), lds, ctypes.byref(o),
                          _ptr(ws), ws.numel(), _stream_handle(torch, stream), out, info)
    if check and rc != FJ_OK:
        raise FJError(rc, "fj_indices")
    vals = [{name: getattr(out[c], name) for name in INDEX_NAMES} for c in range(k)]
    return vals, list(info), rc


def fj_indices_noalloc(graph: Graph, S, opts: Optional[fj_opts] = None, stream=None, check=True):
    """fj_indices with the library's static scratch instead of a workspace
    (allocates no device memory). Returns (list of dicts, [fj_info]*k, status)."""
    import torch
    S2, k, lds = _check_block(graph, S, "S")
    o = opts or fj_default_opts()
    out = (fj_indices_t * k)()
    info = (fj_info * k)()
    rc = lib().fj_indices_noalloc(ctypes.byref(graph.csr), _ptr(graph.plan), k, _ptr(S2), lds, ctypes.byref(o),
                                  _stream_handle(torch, stream), out, info)
    if check and rc != FJ_OK:
        raise FJError(rc, "fj_indices_noalloc")
    vals = [{name: getattr(out[c], name) for name in INDEX_NAMES} for c in range(k)]
    return vals, list(info), rc


def info_dict(inf: fj_info) -> dict:
    return dict(status=inf.status, iters=inf.iters, passes=inf.passes, outer_iters=inf.outer_iters,
                rel_residual=inf.rel_residual, bound=list(inf.bound), ms_spmv=inf.ms_spmv,
                n_spmv=inf.n_spmv, residual_norm=inf.residual_norm, abs_bound=list(inf.abs_bound))


class Server:
    """Continuous-batching server (fj_server_* in include/fj.h). The arena is
    one torch allocation; requests keep their opinion tensors alive here
    until they complete."""

    def __init__(self, arena_bytes, block_columns=16, iters_per_replay=8, eps=1e-6, max_iter=0, device="cuda",
                 precision=FJ_FP64, large_lanes=0, large_entries=0, large_iters_per_replay=0, large_blocks=0):
        import torch
        self.arena = _aligned_empty(torch, arena_bytes, device)
        self.opts = fj_server_opts(arena=self.arena.data_ptr(), arena_bytes=int(arena_bytes),
                                   block_columns=block_columns, iters_per_replay=iters_per_replay, eps=eps,
                                   max_iter=max_iter, precision=precision, large_lanes=large_lanes,
                                   large_iters_per_replay=large_iters_per_replay, large_entries=large_entries,
                                   large_blocks=large_blocks)
        self.handle = ctypes.c_void_p()
        rc = lib().fj_server_create(ctypes.byref(self.opts), ctypes.byref(self.handle))
        if rc != FJ_OK:
            raise FJError(rc, "fj_server_create")
        self.graphs = []
        self.pending = {}

    @staticmethod
    def block_bytes(n, block_columns=16, precision=0):
        return lib().fj_server_block_bytes(int(n), int(block_columns), int(precision))

    def add_graph(self, graph: Graph, stream=None) -> int:
        """stream: where the graph and plan were produced (default: torch's current stream)."""
        import torch
        gid = ctypes.c_int32()
        rc = lib().fj_server_add_graph(self.handle, ctypes.byref(graph.csr), _ptr(graph.plan), ctypes.byref(gid),
                                       _stream_handle(torch, stream))
        if rc != FJ_OK:
            raise FJError(rc, "fj_server_add_graph")
        self.graphs.append(graph)
        return gid.value

    def submit(self, gid, S, stream=None) -> int:
        """S: device float64 tensor, n or n x k (k <= block_columns), produced on
        `stream` (default: torch's current stream)."""
        import torch
        S2, k, lds = _check_block(self.graphs[gid], S, "S")
        out = (fj_indices_t * k)()
        info = (fj_info * k)()
        rid = ctypes.c_uint64()
        rc = lib().fj_server_submit(self.handle, gid, k, _ptr(S2), lds, out, info, ctypes.byref(rid),
                                    _stream_handle(torch, stream))
        if rc != FJ_OK:
            raise FJError(rc, "fj_server_submit")
        self.pending[rid.value] = (S2, out, info, k)
        return rid.value

    def step(self) -> int:
        busy = ctypes.c_int32()
        rc = lib().fj_server_step(self.handle, ctypes.byref(busy))
        if rc != FJ_OK:
            raise FJError(rc, "fj_server_step")
        return busy.value

    def poll(self, max_items=256):
        """Completed requests: list of dicts with id, graph, status, latency_ms, values, infos."""
        done = (fj_server_done * max_items)()
        cnt = ctypes.c_int32()
        rc = lib().fj_server_poll(self.handle, done, max_items, ctypes.byref(cnt))
        if rc != FJ_OK:
            raise FJError(rc, "fj_server_poll")
        res = []
        for d in done[:cnt.value]:
            S2, out, info, k = self.pending.pop(d.request_id)
            res.append(dict(id=d.request_id, graph=d.graph_id, status=d.status, latency_ms=d.latency_ms,
                            values=[{nm: getattr(out[c], nm) for nm in INDEX_NAMES} for c in range(k)],
                            infos=[info_dict(info[c]) for c in range(k)]))
        return res

    def cancel(self, rid: int):
        """Withdraw a request; poll() then reports it with FJ_ERR_CANCELLED."""
        rc = lib().fj_server_cancel(self.handle, ctypes.c_uint64(rid))
        if rc != FJ_OK:
            raise FJError(rc, "fj_server_cancel")

    def drain(self, timeout_s=300.0):
        """Step until every submitted request has completed; returns their results."""
        import time
        t0 = time.perf_counter()
        results = []
        while self.pending:
            self.step()
            results.extend(self.poll())
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"{len(self.pending)} requests still pending")
        return results

    def close(self):
        if self.handle:
            rc = lib().fj_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            if rc != FJ_OK:
                raise FJError(rc, "fj_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
