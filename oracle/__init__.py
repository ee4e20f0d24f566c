"""Oracle: plain sequential FP64 D-iteration (C, gcc -O2, no fast-math).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
imports it and shares no code with it.

See dref.c for what is computed and which passage of the paper each part
follows (Section 2 equations defF/defH, the Section 2.1 pseudo-code, the
Section 2.4 cyclic threshold, the Section 2.3 partitions).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdref.so")
_lib = None

OK, NOT_CONVERGED, EINVAL, EGRAPH = 0, 1, -1, -2


class _Stats(ctypes.Structure):
    _fields_ = [
        ("edges", ctypes.c_int64),
        ("diffusions", ctypes.c_int64),
        ("sweeps", ctypes.c_int64),
        ("increases", ctypes.c_int64),
        ("resid_l1", ctypes.c_double),
        ("b_l1", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("converged", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


@dataclass
class Result:
    h: np.ndarray
    f: np.ndarray
    edges: int
    diffusions: int
    sweeps: int
    increases: int
    resid_l1: float
    b_l1: float
    seconds: float
    converged: bool
    status: int
    r_hist: np.ndarray


def build(force: bool = True) -> str:
    """Compile libdref.so (single-threaded FP64, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall",
                           "-fno-fast-math", "-ffp-contract=off",
                           os.path.join(_HERE, "dref.c"), "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _open(path):
    lib = ctypes.CDLL(path)
    vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    lib.dref_check_csc.argtypes = [i64, i64, vp, vp]
    lib.dref_fluid_from_history.argtypes = [i64, i64, vp, vp, dbl, vp, vp, vp]
    lib.dref_solve.argtypes = [i64, i64, vp, vp, dbl, vp, vp, dbl, dbl, i64, vp, vp,
                               ctypes.POINTER(_Stats), vp, i64]
    lib.dref_solve_ex.argtypes = [i64, i64, vp, vp, dbl, vp, ctypes.c_int, vp, vp, dbl, dbl, i64, vp,
                                  vp, ctypes.POINTER(_Stats), vp, i64]
    lib.dref_fluid_from_history_w.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
    lib.dref_col_norm.argtypes = [i64, vp, vp]
    lib.dref_col_norm.restype = dbl
    lib.dref_partition_pmass.argtypes = [i64, i64, vp, vp, vp, dbl, i64, vp]
    for f in (lib.dref_solve_ex, lib.dref_fluid_from_history_w, lib.dref_partition_pmass):
        f.restype = ctypes.c_int
    lib.dref_partition_uniform.argtypes = [i64, i64, vp]
    lib.dref_partition_cb.argtypes = [i64, vp, i64, vp]
    lib.dref_partition_cb_inout.argtypes = [i64, i64, vp, vp, i64, vp]
    lib.dref_partition_mincut.argtypes = [i64, i64, vp, vp, i64, vp]
    for f in (lib.dref_check_csc, lib.dref_fluid_from_history, lib.dref_solve,
              lib.dref_partition_uniform, lib.dref_partition_cb, lib.dref_partition_cb_inout,
              lib.dref_partition_mincut):
        f.restype = ctypes.c_int
    return lib


def _load(lib=None):
    global _lib
    if lib is not None:
        return lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _open(_LIB_PATH)
    return _lib


def load_variant(path):
    """Open another build of dref.c (the tests compile planted mistakes this way)."""
    return _open(path)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def check_csc(n, col_ptr, row_idx, lib=None) -> int:
    col_ptr, row_idx = _i32(col_ptr), _i32(row_idx)
    return _load(lib).dref_check_csc(n, row_idx.size, col_ptr.ctypes.data, row_idx.ctypes.data)


def fluid_from_history(col_ptr, row_idx, b, h, d: float = 0.85, lib=None) -> np.ndarray:
    """F = B + P H - H in FP64 (the D-iteration identity)."""
    col_ptr, row_idx, b, h = _i32(col_ptr), _i32(row_idx), _f64(b), _f64(h)
    n = b.size
    f = np.empty(n, np.float64)
    _load(lib).dref_fluid_from_history(n, row_idx.size, col_ptr.ctypes.data, row_idx.ctypes.data,
                                    d, b.ctypes.data, h.ctypes.data, f.ctypes.data)
    return f


def solve(col_ptr, row_idx, b, rel_tol: float = 1e-12, d: float = 0.85, alpha: float = 1.5,
          h0=None, max_sweeps: int = 100000, hist_cap: int = 4096, lib=None, val=None,
          priority: bool = False) -> Result:
    """Sequential FP64 D-iteration to ||F||_1 <= rel_tol * ||B||_1.

    val: per-entry weights of a general matrix (None: PageRank d / #out_i);
    priority: threshold test on |F_i| / ((#in_i + 1)(#out_i + 1)) (Section 2.4)."""
    col_ptr, row_idx, b = _i32(col_ptr), _i32(row_idx), _f64(b)
    if val is not None:
        val = _f64(val)
        if val.size != row_idx.size:
            raise ValueError("val must have one entry per link")
    n = b.size
    if col_ptr.size != n + 1:
        raise ValueError("col_ptr must have n+1 entries")
    h = np.empty(n, np.float64)
    f = np.empty(n, np.float64)
    hist = np.zeros(hist_cap, np.float64)
    st = _Stats()
    h0p = None
    if h0 is not None:
        h0 = _f64(h0)
        h0p = h0.ctypes.data
    if val is None and not priority:
        rc = _load(lib).dref_solve(n, row_idx.size, col_ptr.ctypes.data, row_idx.ctypes.data, d,
                                   b.ctypes.data, h0p, rel_tol, alpha, max_sweeps, h.ctypes.data,
                                   f.ctypes.data, ctypes.byref(st), hist.ctypes.data, hist_cap)
    else:
        rc = _load(lib).dref_solve_ex(n, row_idx.size, col_ptr.ctypes.data, row_idx.ctypes.data, d,
                                      val.ctypes.data if val is not None else None, int(bool(priority)),
                                      b.ctypes.data, h0p, rel_tol, alpha, max_sweeps, h.ctypes.data,
                                      f.ctypes.data, ctypes.byref(st), hist.ctypes.data, hist_cap)
    if rc < 0:
        raise ValueError("dref_solve rejected its input (%d)" % rc)
    return Result(h=h, f=f, edges=st.edges, diffusions=st.diffusions, sweeps=st.sweeps,
                  increases=st.increases, resid_l1=st.resid_l1, b_l1=st.b_l1,
                  seconds=st.seconds, converged=bool(st.converged), status=rc,
                  r_hist=hist[:min(st.sweeps, hist_cap)].copy())


def fluid_from_history_w(col_ptr, row_idx, val, b, h, lib=None) -> np.ndarray:
    """F = B + P H - H in FP64 for the general matrix with entry weights val."""
    col_ptr, row_idx, val, b, h = _i32(col_ptr), _i32(row_idx), _f64(val), _f64(b), _f64(h)
    n = b.size
    f = np.empty(n, np.float64)
    _load(lib).dref_fluid_from_history_w(n, row_idx.size, col_ptr.ctypes.data, row_idx.ctypes.data,
                                         val.ctypes.data, b.ctypes.data, h.ctypes.data, f.ctypes.data)
    return f


def col_norm(col_ptr, val, lib=None) -> float:
    """max over columns of sum |p_ji| (the contraction factor of the bound)."""
    col_ptr, val = _i32(col_ptr), _f64(val)
    return _load(lib).dref_col_norm(col_ptr.size - 1, col_ptr.ctypes.data, val.ctypes.data)


def partition_pmass(col_ptr, row_idx, K: int, val=None, d: float = 0.85, lib=None) -> np.ndarray:
    """Contiguous K-block partition of equal internal p mass (min-max, greedy)."""
    col_ptr, row_idx = _i32(col_ptr), _i32(row_idx)
    vp = None
    if val is not None:
        val = _f64(val)
        vp = val.ctypes.data
    ptr = np.empty(K + 1, np.int64)
    if _load(lib).dref_partition_pmass(col_ptr.size - 1, row_idx.size, col_ptr.ctypes.data,
                                       row_idx.ctypes.data, vp, d, K, ptr.ctypes.data):
        raise ValueError("bad partition count")
    return ptr


def partition_uniform(n: int, K: int) -> np.ndarray:
    ptr = np.empty(K + 1, np.int64)
    if _load().dref_partition_uniform(n, K, ptr.ctypes.data):
        raise ValueError("bad partition count")
    return ptr


def partition_cb(col_ptr, K: int, lib=None) -> np.ndarray:
    col_ptr = _i32(col_ptr)
    ptr = np.empty(K + 1, np.int64)
    if _load(lib).dref_partition_cb(col_ptr.size - 1, col_ptr.ctypes.data, K, ptr.ctypes.data):
        raise ValueError("bad partition count")
    return ptr


def partition_cb_inout(col_ptr, row_idx, K: int, lib=None) -> np.ndarray:
    """CB partition with the cost of a prefix = its out-links + its in-links."""
    col_ptr, row_idx = _i32(col_ptr), _i32(row_idx)
    ptr = np.empty(K + 1, np.int64)
    if _load(lib).dref_partition_cb_inout(col_ptr.size - 1, row_idx.size, col_ptr.ctypes.data,
                                          row_idx.ctypes.data, K, ptr.ctypes.data):
        raise ValueError("bad partition count")
    return ptr


def partition_mincut(col_ptr, row_idx, K: int, lib=None) -> np.ndarray:
    """CB boundaries moved, within windows and a 5% balance slack, to where the
    fewest short links cross (least sum over the inner boundaries)."""
    col_ptr, row_idx = _i32(col_ptr), _i32(row_idx)
    ptr = np.empty(K + 1, np.int64)
    if _load(lib).dref_partition_mincut(col_ptr.size - 1, row_idx.size, col_ptr.ctypes.data,
                                        row_idx.ctypes.data, K, ptr.ctypes.data):
        raise ValueError("bad partition count")
    return ptr
