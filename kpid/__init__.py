"""K-PID simulator: the time-stepped model of the paper's asynchronous
distributed D-iteration (Sections 2.3-2.6 and 3), run on one CPU core.

CPU only, a context tool: its outputs are operation counts on synthetic
graphs (normalized iterations, idle proportion, messages), as in the paper's
own evaluation; nothing in it runs on the GPU or feeds the GPU path. See
kpid.c for the model and the readings it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libkpid.so")
_lib = None


class _Stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64),
        ("ops", ctypes.c_int64),
        ("idle", ctypes.c_int64),
        ("messages", ctypes.c_int64),
        ("adaptations", ctypes.c_int64),
        ("norm_iters", ctypes.c_double),
        ("idle_frac", ctypes.c_double),
        ("resid_l1", ctypes.c_double),
        ("converged", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


@dataclass
class SimResult:
    h: np.ndarray
    f: np.ndarray
    omega: np.ndarray       # final boundaries (moved by the K = 2 adaptation)
    steps: int
    ops: int
    idle: int
    messages: int
    adaptations: int
    norm_iters: float       # steps * speed / L: the slowest PID's clock in matrix-vector products
    idle_frac: float        # idle / (elementary + idle), Section 3.3
    resid_l1: float
    converged: bool
    trace: np.ndarray       # [steps, K, 2]: r_k and s_k after each step (when requested)


def build(force: bool = True) -> str:
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-fno-fast-math",
                           os.path.join(_HERE, "kpid.c"), "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.kpid_simulate.argtypes = [i64, vp, vp, dbl, vp, ctypes.c_int, vp, i64, dbl, dbl, dbl,
                                    ctypes.c_int, ctypes.c_uint64, i64, vp, vp, ctypes.POINTER(_Stats),
                                    vp, i64]
        L.kpid_simulate.restype = ctypes.c_int
        _lib = L
    return _lib


def simulate(col_ptr, row_idx, b, omega, d: float = 0.85, speed: int = None, alpha: float = 1.5,
             target_error: float = None, delay_proba: float = 0.0, adapt_every: int = 0,
             seed: int = 1, max_steps: int = 1_000_000, trace_steps: int = 0) -> SimResult:
    """Simulate K = len(omega) - 1 PIDs on the PageRank matrix of the CSC graph.

    speed: operations per PID per step (default L / K, the paper's PID_Speed);
    target_error: stop once ||F||_1 / (1 - d) <= target_error (default 1/N)."""
    cp = np.ascontiguousarray(col_ptr, np.int32)
    ri = np.ascontiguousarray(row_idx, np.int32)
    b = np.ascontiguousarray(b, np.float64)
    om = np.ascontiguousarray(omega, np.int64).copy()
    n, K = b.size, om.size - 1
    L = int(cp[-1])
    speed = max(1, L // K) if speed is None else int(speed)
    target_error = 1.0 / n if target_error is None else target_error
    h, f = np.empty(n), np.empty(n)
    tr = np.zeros((max(trace_steps, 0), K, 2))
    st = _Stats()
    rc = _load().kpid_simulate(n, cp.ctypes.data, ri.ctypes.data, d, b.ctypes.data, K, om.ctypes.data,
                               speed, alpha, target_error, delay_proba, adapt_every, seed, max_steps,
                               h.ctypes.data, f.ctypes.data, ctypes.byref(st),
                               tr.ctypes.data if trace_steps > 0 else None, trace_steps)
    if rc < 0:
        raise ValueError("kpid_simulate rejected its input (%d)" % rc)
    return SimResult(h=h, f=f, omega=om, steps=st.steps, ops=st.ops, idle=st.idle, messages=st.messages,
                     adaptations=st.adaptations, norm_iters=st.norm_iters, idle_frac=st.idle_frac,
                     resid_l1=st.resid_l1, converged=bool(st.converged),
                     trace=tr[:min(st.steps, trace_steps)])
