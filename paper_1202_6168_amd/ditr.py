"""Thin Python binding of the ditr C-ABI (include/ditr.h).

Argument marshalling only: every step of a solve runs in the HIP kernels of
libditr.so. PyTorch supplies device memory (tensors) and the stream. There is
no CPU fallback: if the library is missing, importing the binding raises.

Functions keep the C names without the ``ditr_`` prefix.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
import weakref

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libditr.so")

OK, NOT_CONVERGED, ABORTED, NOT_FOUND = 0, 1, 2, 3
EINVAL, EGRAPH, ENOMEM, EHIP, ENONFINITE = -1, -2, -3, -4, -5
PART_CB, PART_UNIFORM, PART_CB_INOUT, PART_PMASS, PART_MINCUT = 0, 1, 2, 3, 4
MODE_AUTO, MODE_ASYNC, MODE_SWEEP, MODE_PARTITION = 0, 1, 2, 3
FLAG_TIME_KERNELS = 1
FLAG_NO_RESIDENT = 2
FLAG_PRIORITY = 4
TRACE_FIELDS = 6  # doubles per per-partition trace record (DITR_TRACE_FIELDS)
GNN_PARAMS = 9409
GNN_ACT_X, GNN_ACT_PX, GNN_ACT_H1, GNN_ACT_PH1, GNN_ACT_H2 = 0, 1, 2, 3, 4

_STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "ABORTED", 3: "NOT_FOUND", -1: "EINVAL", -2: "EGRAPH",
                 -3: "ENOMEM", -4: "EHIP", -5: "ENONFINITE"}


class DitrError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (_STATUS_NAMES.get(status, "?"), status, message))
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double),
        ("refresh_at", ctypes.c_double),
        ("park_ratio", ctypes.c_double),
        ("rescale_cap", ctypes.c_double),
        ("mode", ctypes.c_int32),
        ("part_type", ctypes.c_int32),
        ("part_nodes", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("wg_per_cu", ctypes.c_int32),
        ("sweeps_per_claim", ctypes.c_int32),
        ("max_rounds", ctypes.c_int32),
        ("max_sweeps", ctypes.c_int32),
        ("xcd_remap", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [
        ("edges", ctypes.c_int64),
        ("diffusions", ctypes.c_int64),
        ("sweeps", ctypes.c_int64),
        ("launches", ctypes.c_int64),
        ("refreshes", ctypes.c_int64),
        ("idle_polls", ctypes.c_int64),
        ("resid_l1", ctypes.c_double),
        ("b_l1", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("kernel_seconds", ctypes.c_double),
        ("timed_launches", ctypes.c_int64),
        ("rounds", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AdaptInfo(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int32),
        ("kept", ctypes.c_int32),
        ("seconds_before", ctypes.c_double),
        ("seconds_after", ctypes.c_double),
        ("spread_before", ctypes.c_double),
        ("spread_after", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneInfo(ctypes.Structure):
    _fields_ = [
        ("key", ctypes.c_uint64),
        ("from_cache", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("default_seconds", ctypes.c_double),
        ("best_seconds", ctypes.c_double),
        ("default_edges", ctypes.c_int64),
        ("best_edges", ctypes.c_int64),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GnnStart(ctypes.Structure):
    _fields_ = [
        ("b_l1", ctypes.c_double),
        ("scale_c", ctypes.c_double),
        ("f0_l1", ctypes.c_double),
        ("fell_back", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


_lib = None
_lock = threading.Lock()

_vp, _i64, _i32, _dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
_SIGNATURES = {
    "ditr_version": ([], _i32),
    "ditr_last_error": ([], ctypes.c_char_p),
    "ditr_opts_default": ([ctypes.POINTER(Opts)], _i32),
    "ditr_create": ([ctypes.POINTER(_vp), _i32, _vp], _i32),
    "ditr_destroy": ([_vp], _i32),
    "ditr_abort": ([_vp], _i32),
    "ditr_graph_create": ([_vp, ctypes.POINTER(_vp), _i64, _i64, _vp, _vp, _dbl,
                           ctypes.POINTER(Opts)], _i32),
    "ditr_graph_create_weighted": ([_vp, ctypes.POINTER(_vp), _i64, _i64, _vp, _vp, _vp,
                                    ctypes.POINTER(Opts)], _i32),
    "ditr_graph_contraction": ([_vp, ctypes.POINTER(_dbl)], _i32),
    "ditr_graph_destroy": ([_vp], _i32),
    "ditr_graph_set_partitions": ([_vp, _vp, _vp, _i64], _i32),
    "ditr_graph_adapt": ([_vp, _vp, _vp, _vp, _vp, _dbl, _i32, _dbl, ctypes.POINTER(AdaptInfo)], _i32),
    "ditr_graph_partitions": ([_vp, ctypes.POINTER(_i64), _vp, _i64], _i32),
    "ditr_partition": ([_vp, _i64, _i64, _vp, _vp, _i32, _i64, _vp], _i32),
    "ditr_partition_pmass": ([_vp, _i64, _i64, _vp, _vp, _vp, _dbl, _i64, _vp], _i32),
    "ditr_residual": ([_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_dbl)], _i32),
    "ditr_solve": ([_vp, _vp, _vp, _vp, _vp, _i32, _dbl, ctypes.POINTER(Opts),
                    ctypes.POINTER(Stats)], _i32),
    "ditr_solve_noalloc": ([_vp, _vp, _vp, _vp, _vp, _i32, _dbl, ctypes.POINTER(Opts),
                            ctypes.POINTER(Stats)], _i32),
    "ditr_noalloc_scratch_bytes": ([], ctypes.c_size_t),
    "ditr_set_trace": ([_vp, _vp, _i64], _i32),
    "ditr_solve_batched": ([_vp, _vp, _i32, _vp, _vp, _vp, _dbl, ctypes.POINTER(Opts),
                            _vp, ctypes.c_size_t, _vp, ctypes.POINTER(Stats)], _i32),
    "ditr_workspace_bytes": ([_vp, _i64, _i64, _i32, ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_size_t)],
                             _i32),
    "ditr_graph_upload_csc": ([_vp, ctypes.POINTER(_vp), _i64, _i64, _vp, _vp, _dbl, _vp, ctypes.c_size_t,
                               ctypes.POINTER(Opts)], _i32),
    "ditr_graph_workspace_used": ([_vp, ctypes.POINTER(ctypes.c_size_t)], _i32),
    "ditr_tune": ([_vp, _i64, _i64, _vp, _vp, _dbl, _vp, _vp, _vp, _dbl, _i32, ctypes.c_char_p,
                   ctypes.POINTER(Opts), ctypes.POINTER(TuneInfo)], _i32),
    "ditr_tune_batched": ([_vp, _vp, _i32, _vp, _vp, _vp, _dbl, _vp, ctypes.c_size_t, _i32,
                           ctypes.POINTER(Opts), ctypes.POINTER(TuneInfo)], _i32),
    "ditr_tune_key": ([_vp, _i64, _i64, _vp, _vp, _dbl, _vp, _dbl,
                       ctypes.POINTER(ctypes.c_uint64)], _i32),
    "ditr_tune_cache_get": ([ctypes.c_char_p, ctypes.c_uint64, ctypes.POINTER(Opts)], _i32),
    "ditr_tune_cache_put": ([ctypes.c_char_p, ctypes.c_uint64, ctypes.POINTER(Opts), _dbl, _dbl],
                            _i32),
    "ditr_gnn_create": ([_vp, ctypes.POINTER(_vp), _i32, _i32, ctypes.c_uint64], _i32),
    "ditr_gnn_destroy": ([_vp], _i32),
    "ditr_gnn_get_params": ([_vp, _vp], _i32),
    "ditr_gnn_set_params": ([_vp, _vp], _i32),
    "ditr_gnn_forward": ([_vp, _vp, _vp, _vp], _i32),
    "ditr_gnn_activation": ([_vp, _vp, _i32, _i64, _vp], _i32),
    "ditr_gnn_targets": ([_vp, _vp, _vp, _dbl, _vp, _vp], _i32),
    "ditr_gnn_grad": ([_vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_dbl)], _i32),
    "ditr_gnn_train_step": ([_vp, _vp, _vp, _vp, _vp, _dbl, ctypes.POINTER(_dbl)], _i32),
    "ditr_gnn_predict_h0": ([_vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(GnnStart)], _i32),
}


def lib():
    """Load libditr.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libditr.so is not built: run __graft_entry__.build() "
                                   "(no CPU fallback exists)")
            L = ctypes.CDLL(LIB_PATH)
            for name, (args, res) in _SIGNATURES.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = res
            _lib = L
    return _lib


def last_error() -> str:
    m = lib().ditr_last_error()
    return m.decode(errors="replace") if m else ""


def check(status: int, allow=(OK,)) -> int:
    if status not in allow:
        raise DitrError(status, last_error())
    return status


def version() -> int:
    return lib().ditr_version()


def opts_default(**overrides) -> Opts:
    o = Opts()
    check(lib().ditr_opts_default(ctypes.byref(o)))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# Contexts still open when the interpreter exits are closed by an exit handler
# registered after torch was imported, so it runs before torch and the HIP
# runtime are torn down: every handle (graphs, networks, the context's stream
# and pinned words) is released in a defined order, never from a finalizer
# during interpreter shutdown.
_live_contexts = weakref.WeakSet()
_exit_hook = False


def _close_all():
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """ditr_ctx on one device, issuing work on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        global _exit_hook
        import torch

        self.device = device
        self.torch = torch
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(torch, device)
        h = ctypes.c_void_p()
        check(lib().ditr_create(ctypes.byref(h), device, s))
        self.handle = h
        self._children = weakref.WeakSet()  # graphs and networks, closed first
        with _lock:
            _live_contexts.add(self)
            if not _exit_hook:
                atexit.register(_close_all)
                _exit_hook = True

    def abort(self):
        check(lib().ditr_abort(self.handle))

    def set_trace(self, trace=None):
        """Register a float64 CUDA tensor of TRACE_FIELDS * records elements as
        the per-partition trace of the partitioned sweep (ditr_set_trace; the
        tensor must stay alive while tracing is on), or switch it off (None).
        Record l * K + k holds partition k at level l of a solve."""
        if trace is None:
            check(lib().ditr_set_trace(self.handle, None, 0))
            self._trace = None
            return
        if trace.dtype != self.torch.float64 or not trace.is_cuda or not trace.is_contiguous():
            raise ValueError("trace must be a contiguous float64 CUDA tensor")
        check(lib().ditr_set_trace(self.handle, _ptr(trace), trace.numel() // TRACE_FIELDS))
        self._trace = trace  # kept alive while registered

    def close(self):
        if self.handle:
            for child in list(self._children):
                child.close()
            lib().ditr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(ctx: Context, n: int, nnz: int, nrhs: int = 0, opts: Opts = None) -> int:
    """ditr_workspace_bytes: device bytes of a graph upload (nrhs = 0) or of a
    batched solve with nrhs right-hand sides."""
    b = ctypes.c_size_t()
    check(lib().ditr_workspace_bytes(ctx.handle, n, nnz, nrhs, ctypes.byref(opts) if opts else None,
                                     ctypes.byref(b)))
    return b.value


class Graph:
    """ditr_graph: borrows the CSC tensors (int32, on the context's device).

    val (optional, float64, one weight per CSC entry): a general matrix
    (ditr_graph_create_weighted); damping is then unused.
    workspace (optional, uint8 device tensor of at least workspace_bytes(ctx,
    n, nnz) bytes): every device table of the graph lives in it
    (ditr_graph_upload_csc) and the library allocates nothing for the graph.

    Batched solves on this graph keep their workspace in a tensor cached on
    the graph per right-hand-side count, so repeated solves allocate nothing."""

    def __init__(self, ctx: Context, col_ptr, row_idx, damping: float = 0.85, opts: Opts = None,
                 val=None, workspace=None):
        torch = ctx.torch
        if col_ptr.dtype != torch.int32 or row_idx.dtype != torch.int32:
            raise TypeError("CSC arrays must be int32")
        if not (col_ptr.is_cuda and row_idx.is_cuda):
            raise TypeError("CSC arrays must be device tensors")
        self.ctx = ctx
        self.col_ptr = col_ptr.contiguous()
        self.row_idx = row_idx.contiguous()
        self.n = self.col_ptr.numel() - 1
        self.nnz = self.row_idx.numel()
        self.val = None
        self.workspace = None
        self._batch_ws = {}
        h = ctypes.c_void_p()
        o = opts if opts is not None else opts_default()
        if workspace is not None:
            if val is not None:
                raise ValueError("a workspace upload takes PageRank graphs")
            if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
                raise TypeError("workspace must be a contiguous uint8 device tensor")
            self.workspace = workspace
            check(lib().ditr_graph_upload_csc(ctx.handle, ctypes.byref(h), self.n, self.nnz,
                                              _ptr(self.col_ptr),
                                              _ptr(self.row_idx) if self.nnz else None, damping,
                                              _ptr(workspace), workspace.numel(), ctypes.byref(o)))
        elif val is not None:
            if val.dtype != torch.float64 or not val.is_cuda or val.numel() != self.nnz:
                raise TypeError("val must be a float64 device tensor with one entry per link")
            self.val = val.contiguous()
            check(lib().ditr_graph_create_weighted(ctx.handle, ctypes.byref(h), self.n, self.nnz,
                                                   _ptr(self.col_ptr),
                                                   _ptr(self.row_idx) if self.nnz else None,
                                                   _ptr(self.val) if self.nnz else None,
                                                   ctypes.byref(o)))
        else:
            check(lib().ditr_graph_create(ctx.handle, ctypes.byref(h), self.n, self.nnz,
                                          _ptr(self.col_ptr), _ptr(self.row_idx) if self.nnz else None,
                                          damping, ctypes.byref(o)))
        self.handle = h
        ctx._children.add(self)

    def workspace_used(self) -> int:
        u = ctypes.c_size_t()
        check(lib().ditr_graph_workspace_used(self.handle, ctypes.byref(u)))
        return u.value

    def batch_workspace(self, R: int):
        """The uint8 device tensor ditr_solve_batched works in for R right-hand sides."""
        ws = self._batch_ws.get(R)
        if ws is None:
            nb = workspace_bytes(self.ctx, self.n, self.nnz, R)
            ws = self.ctx.torch.empty(nb, dtype=self.ctx.torch.uint8, device=self.col_ptr.device)
            self._batch_ws = {R: ws}  # one cached size at a time
        return ws

    def contraction(self) -> float:
        c = ctypes.c_double()
        check(lib().ditr_graph_contraction(self.handle, ctypes.byref(c)))
        return c.value

    def partitions(self):
        import numpy as np

        K = ctypes.c_int64()
        check(lib().ditr_graph_partitions(self.handle, ctypes.byref(K), None, 0))
        out = np.empty(K.value + 1, np.int64)
        check(lib().ditr_graph_partitions(self.handle, ctypes.byref(K),
                                          ctypes.c_void_p(out.ctypes.data), out.size))
        return out

    def set_partitions(self, ptr):
        """ditr_graph_set_partitions: new boundaries (K + 1 host int64 values) and tables."""
        import numpy as np

        p = np.ascontiguousarray(ptr, np.int64)
        check(lib().ditr_graph_set_partitions(self.ctx.handle, self.handle, ctypes.c_void_p(p.ctypes.data),
                                              p.size - 1))

    def close(self):
        if self.handle:
            lib().ditr_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def partition(ctx: Context, col_ptr, part_type: int, K: int, out, row_idx=None):
    """ditr_partition: K+1 boundaries (int64 device tensor `out`)."""
    nnz = row_idx.numel() if row_idx is not None else 0
    check(lib().ditr_partition(ctx.handle, col_ptr.numel() - 1, nnz, _ptr(col_ptr),
                               _ptr(row_idx) if row_idx is not None else None, part_type, K,
                               _ptr(out)))
    return out


def partition_pmass(ctx: Context, col_ptr, row_idx, K: int, out, val=None, damping: float = 0.85):
    """ditr_partition_pmass: K+1 boundaries of equal internal p mass (int64 device tensor `out`)."""
    nnz = row_idx.numel()
    check(lib().ditr_partition_pmass(ctx.handle, col_ptr.numel() - 1, nnz, _ptr(col_ptr),
                                     _ptr(row_idx) if nnz else None,
                                     _ptr(val) if val is not None else None, damping, K, _ptr(out)))
    return out


def residual(ctx: Context, g: Graph, b, h, f, want_norm: bool = True):
    """ditr_residual: F = B + P H - H (FP64 arithmetic, FP32 store); returns ||F||_1."""
    r = ctypes.c_double()
    check(lib().ditr_residual(ctx.handle, g.handle, _ptr(b), _ptr(h), _ptr(f),
                              ctypes.byref(r) if want_norm else None))
    return r.value if want_norm else None


def solve(ctx: Context, g: Graph, b, h, f, warm: bool = False, rel_tol: float = 1e-9,
          opts: Opts = None, allow=(OK, NOT_CONVERGED, ABORTED)) -> Stats:
    """ditr_solve: diffuse until the exact ||F||_1 <= rel_tol ||B||_1."""
    torch = ctx.torch
    if b.dtype != torch.float64 or h.dtype != torch.float64 or f.dtype != torch.float32:
        raise TypeError("b, h must be float64 and f float32")
    for t in (b, h, f):
        if t.numel() != g.n or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("b, h, f must be contiguous device vectors of length n")
    st = Stats()
    o = opts if opts is not None else opts_default()
    if int(warm) not in (0, 1, 2):
        raise ValueError("warm must be 0 (cold), 1 (H_0 given) or 2 (H_0 and its F_0 given)")
    rc = lib().ditr_solve(ctx.handle, g.handle, _ptr(b), _ptr(h), _ptr(f), int(warm),
                          rel_tol, ctypes.byref(o), ctypes.byref(st))
    check(rc, allow)
    return st


def solve_noalloc(ctx: Context, g: Graph, b, h, f, warm: bool = False, rel_tol: float = 1e-9,
                  opts: Opts = None, allow=(OK, NOT_CONVERGED, ABORTED)) -> Stats:
    """ditr_solve_noalloc: ditr_solve with its per-solve buffers in the library's
    static device scratch (no allocation inside the call; partitioned sweep only)."""
    torch = ctx.torch
    if b.dtype != torch.float64 or h.dtype != torch.float64 or f.dtype != torch.float32:
        raise TypeError("b, h must be float64 and f float32")
    for t in (b, h, f):
        if t.numel() != g.n or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("b, h, f must be contiguous device vectors of length n")
    st = Stats()
    o = opts if opts is not None else opts_default()
    rc = lib().ditr_solve_noalloc(ctx.handle, g.handle, _ptr(b), _ptr(h), _ptr(f), int(bool(warm)),
                                  rel_tol, ctypes.byref(o), ctypes.byref(st))
    check(rc, allow)
    return st


def noalloc_scratch_bytes() -> int:
    """Size of the static device scratch behind solve_noalloc."""
    return int(lib().ditr_noalloc_scratch_bytes())


def solve_batched(ctx: Context, g: Graph, b, h, f, rel_tol: float = 1e-8, opts: Opts = None,
                  allow=(OK, NOT_CONVERGED, ABORTED), workspace=None):
    """ditr_solve_batched: node-major [n, R] right-hand sides; returns (total, per_rhs).
    The solve works in `workspace` (uint8 device tensor) or in the graph's cached one."""
    torch = ctx.torch
    if b.dtype != torch.float64 or h.dtype != torch.float64 or f.dtype != torch.float32:
        raise TypeError("b, h must be float64 and f float32")
    if b.dim() != 2 or b.shape[0] != g.n or h.shape != b.shape or f.shape != b.shape:
        raise ValueError("b, h, f must be [n, R] with the same shape")
    for t in (b, h, f):
        if not (t.is_contiguous() and t.is_cuda):
            raise ValueError("b, h, f must be contiguous device tensors")
    R = b.shape[1]
    per = (Stats * R)()
    tot = Stats()
    o = opts if opts is not None else opts_default()
    ws = workspace if workspace is not None else g.batch_workspace(R)
    rc = lib().ditr_solve_batched(ctx.handle, g.handle, R, _ptr(b), _ptr(h), _ptr(f), rel_tol,
                                  ctypes.byref(o), _ptr(ws), ws.numel(),
                                  ctypes.cast(per, ctypes.c_void_p), ctypes.byref(tot))
    check(rc, allow)
    return tot, list(per)


def _check_problem(ctx, col_ptr, row_idx, b, h, f):
    torch = ctx.torch
    if col_ptr.dtype != torch.int32 or row_idx.dtype != torch.int32:
        raise TypeError("CSC arrays must be int32")
    n = col_ptr.numel() - 1
    if b.dtype != torch.float64 or h.dtype != torch.float64 or f.dtype != torch.float32:
        raise TypeError("b, h must be float64 and f float32")
    for t in (col_ptr, row_idx, b, h, f):
        if not (t.is_contiguous() and t.is_cuda):
            raise ValueError("arrays must be contiguous device tensors")
    for t in (b, h, f):
        if t.numel() != n:
            raise ValueError("b, h, f must have length n")
    return n, row_idx.numel()


def tune_key(ctx: Context, col_ptr, row_idx, b, rel_tol: float, damping: float = 0.85) -> int:
    """ditr_tune_key: cache key of (CSC, damping, B, rel_tol, device)."""
    n, nnz = col_ptr.numel() - 1, row_idx.numel()
    k = ctypes.c_uint64()
    check(lib().ditr_tune_key(ctx.handle, n, nnz, _ptr(col_ptr), _ptr(row_idx) if nnz else None,
                              damping, _ptr(b), rel_tol, ctypes.byref(k)))
    return k.value


def tune(ctx: Context, col_ptr, row_idx, b, h, f, rel_tol: float = 1e-9, effort: int = 1,
         cache_path: str = None, damping: float = 0.85):
    """ditr_tune: options of the fastest plain solve of this problem; returns (opts, info).
    h and f are work buffers (overwritten)."""
    n, nnz = _check_problem(ctx, col_ptr, row_idx, b, h, f)
    o, info = Opts(), TuneInfo()
    check(lib().ditr_tune(ctx.handle, n, nnz, _ptr(col_ptr), _ptr(row_idx) if nnz else None,
                          damping, _ptr(b), _ptr(h), _ptr(f), rel_tol, effort,
                          cache_path.encode() if cache_path else None, ctypes.byref(o),
                          ctypes.byref(info)))
    return o, info


def adapt(ctx: Context, g: Graph, b, h, f, rel_tol: float = 1e-9, rounds: int = 4, omega: float = 0.5):
    """ditr_graph_adapt: move g's partition boundaries towards equal measured work per
    partition (Section 3.4) while the solve gets faster; returns AdaptInfo. h and f are
    work buffers (overwritten)."""
    info = AdaptInfo()
    check(lib().ditr_graph_adapt(ctx.handle, g.handle, _ptr(b), _ptr(h), _ptr(f), rel_tol, rounds, omega,
                                 ctypes.byref(info)))
    return info


def tune_batched(ctx: Context, g: Graph, b, h, f, rel_tol: float = 1e-8, effort: int = 1,
                 workspace=None):
    """ditr_tune_batched: options (alpha, first refresh point) of the fastest batched
    solve of these [n, R] right-hand sides on g; returns (opts, info). h and f are
    work buffers (overwritten)."""
    torch = ctx.torch
    if b.dtype != torch.float64 or h.dtype != torch.float64 or f.dtype != torch.float32:
        raise TypeError("b, h must be float64 and f float32")
    if b.dim() != 2 or b.shape[0] != g.n or h.shape != b.shape or f.shape != b.shape:
        raise ValueError("b, h, f must be [n, R] with the same shape")
    R = b.shape[1]
    ws = workspace if workspace is not None else g.batch_workspace(R)
    o, info = Opts(), TuneInfo()
    check(lib().ditr_tune_batched(ctx.handle, g.handle, R, _ptr(b), _ptr(h), _ptr(f), rel_tol,
                                  _ptr(ws), ws.numel(), effort, ctypes.byref(o), ctypes.byref(info)))
    return o, info


def tune_cache_get(path: str, key: int, base: Opts = None):
    """ditr_tune_cache_get: the cached options under `key` over `base`, or None."""
    o = Opts()
    if base is not None:
        ctypes.memmove(ctypes.byref(o), ctypes.byref(base), ctypes.sizeof(Opts))
    else:
        check(lib().ditr_opts_default(ctypes.byref(o)))
    rc = check(lib().ditr_tune_cache_get(path.encode(), key, ctypes.byref(o)), (OK, NOT_FOUND))
    return o if rc == OK else None


def tune_cache_put(path: str, key: int, o: Opts, seconds: float = 0.0,
                   default_seconds: float = 0.0):
    """ditr_tune_cache_put: add or replace the entry under `key`."""
    check(lib().ditr_tune_cache_put(path.encode(), key, ctypes.byref(o), seconds, default_seconds))


def gnn_targets(ctx: Context, g: Graph, h, b_l1: float, y=None, w=None):
    """ditr_gnn_targets: (y, w) FP32 device vectors from a solved H."""
    torch = ctx.torch
    if h.dtype != torch.float64 or h.numel() != g.n or not (h.is_cuda and h.is_contiguous()):
        raise ValueError("h must be a contiguous float64 device vector of length n")
    y = torch.empty(g.n, dtype=torch.float32, device=h.device) if y is None else y
    w = torch.empty(g.n, dtype=torch.float32, device=h.device) if w is None else w
    check(lib().ditr_gnn_targets(ctx.handle, g.handle, _ptr(h), b_l1, _ptr(y), _ptr(w)))
    return y, w


class Gnn:
    """ditr_gnn: the warm-start network (hidden width 64)."""

    def __init__(self, ctx: Context, block: int = 1000, seed: int = 7, hidden: int = 64):
        self.ctx = ctx
        h = ctypes.c_void_p()
        check(lib().ditr_gnn_create(ctx.handle, ctypes.byref(h), hidden, block, seed))
        self.handle = h
        ctx._children.add(self)

    def get_params(self):
        import numpy as np

        out = np.empty(GNN_PARAMS, np.float32)
        check(lib().ditr_gnn_get_params(self.handle, ctypes.c_void_p(out.ctypes.data)))
        return out

    def set_params(self, theta):
        import numpy as np

        t = np.ascontiguousarray(theta, dtype=np.float32)
        if t.size != GNN_PARAMS:
            raise ValueError("expected %d parameters" % GNN_PARAMS)
        check(lib().ditr_gnn_set_params(self.handle, ctypes.c_void_p(t.ctypes.data)))

    def forward(self, g: Graph, yhat=None):
        torch = self.ctx.torch
        dev = g.col_ptr.device
        yhat = torch.empty(g.n, dtype=torch.float32, device=dev) if yhat is None else yhat
        check(lib().ditr_gnn_forward(self.ctx.handle, self.handle, g.handle, _ptr(yhat)))
        return yhat

    def activation(self, which: int, n: int):
        """A BF16 activation of the last forward pass as a [n, width] tensor."""
        torch = self.ctx.torch
        width = 16 if which in (GNN_ACT_X, GNN_ACT_PX) else 64
        out = torch.empty((n, width), dtype=torch.bfloat16, device="cuda:%d" % self.ctx.device)
        check(lib().ditr_gnn_activation(self.ctx.handle, self.handle, which, n, _ptr(out)))
        return out

    def grad(self, g: Graph, y, w):
        """(loss, gradient) at the current weights; gradient is an FP32 device vector."""
        torch = self.ctx.torch
        gr = torch.empty(GNN_PARAMS, dtype=torch.float32, device=y.device)
        loss = ctypes.c_double()
        check(lib().ditr_gnn_grad(self.ctx.handle, self.handle, g.handle, _ptr(y), _ptr(w),
                                  _ptr(gr), ctypes.byref(loss)))
        return loss.value, gr

    def train_step(self, g: Graph, y, w, lr: float, want_loss: bool = True):
        loss = ctypes.c_double()
        check(lib().ditr_gnn_train_step(self.ctx.handle, self.handle, g.handle, _ptr(y), _ptr(w),
                                        lr, ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def predict_h0(self, g: Graph, b, h0, f0) -> GnnStart:
        """ditr_gnn_predict_h0: H_0 into h0 (FP64) and its exact fluid into f0 (FP32)."""
        torch = self.ctx.torch
        if b.dtype != torch.float64 or h0.dtype != torch.float64 or f0.dtype != torch.float32:
            raise TypeError("b, h0 must be float64 and f0 float32")
        for t in (b, h0, f0):
            if t.numel() != g.n or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("b, h0, f0 must be contiguous device vectors of length n")
        info = GnnStart()
        check(lib().ditr_gnn_predict_h0(self.ctx.handle, self.handle, g.handle, _ptr(b), _ptr(h0),
                                        _ptr(f0), ctypes.byref(info)))
        return info

    def close(self):
        if self.handle:
            lib().ditr_gnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
