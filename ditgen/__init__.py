"""Seeded synthetic inputs for the D-iteration solvers.

This module holds no D-iteration arithmetic. It produces
  * web-like directed graphs in CSC form (column j = out-links of node j),
  * right-hand sides: the uniform PageRank vector and personalized seed sets.
Both the FP64 oracle and the GPU library consume these arrays.

The graph model stands in for the web crawl used in the paper's evaluation
(Section 3, Table 1): power-law out-degrees, 10% dangling nodes, 80% of links
inside a block of consecutive ids and 20% preferential on in-degree.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libditgen.so")
_lib = None


class _Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("block", ctypes.c_int32),
        ("deg_min", ctypes.c_int32),
        ("deg_max", ctypes.c_int32),
        ("zipf_exponent", ctypes.c_double),
        ("mean_outdeg", ctypes.c_double),
        ("p_dangling", ctypes.c_double),
        ("p_local", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


def build(force: bool = True) -> str:
    """Compile libditgen.so with gcc (OpenMP, no fast-math)."""
    import subprocess

    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    src = os.path.join(_HERE, "ditgen.c")
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wno-unused-function",
         src, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_Params)
        lib.ditgen_zipf_offset.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
        lib.ditgen_zipf_offset.restype = ctypes.c_int
        lib.ditgen_count_edges.argtypes = [P]
        lib.ditgen_count_edges.restype = ctypes.c_int64
        lib.ditgen_build.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        lib.ditgen_build.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class GraphSpec:
    """Parameters of the synthetic web-like graph."""

    n: int
    block: int = 1000
    seed: int = 2
    deg_min: int = 1
    deg_max: int = 200
    zipf_exponent: float = 2.0
    mean_outdeg: float = 8.0
    p_dangling: float = 0.10
    p_local: float = 0.80
    gamma: float = 2.1

    def _c(self) -> _Params:
        return _Params(self.n, self.block, self.deg_min, self.deg_max, self.zipf_exponent,
                       self.mean_outdeg, self.p_dangling, self.p_local, self.gamma,
                       self.seed & 0xFFFFFFFFFFFFFFFF)


# The workloads the benchmarks and parity tests use.
SMALL = GraphSpec(n=10_000, block=100, seed=1)           # 1e4 nodes, FP64 reference case
HEADLINE = GraphSpec(n=1_000_000, block=1000, seed=2)    # 1e6 nodes, ~8e6 edges
LARGE = GraphSpec(n=50_000_000, block=1000, seed=3)      # 5e7 nodes, ~4e8 edges


def zipf_offset(spec: GraphSpec) -> float:
    s = ctypes.c_double()
    rc = _load().ditgen_zipf_offset(ctypes.byref(spec._c()), ctypes.byref(s))
    if rc:
        raise ValueError("invalid generator parameters (%d)" % rc)
    return s.value


def generate(spec: GraphSpec):
    """Return (col_ptr int32[n+1], row_idx int32[nnz]) for `spec`."""
    lib = _load()
    p = spec._c()
    nnz = lib.ditgen_count_edges(ctypes.byref(p))
    if nnz < 0:
        raise ValueError("invalid generator parameters (%d)" % nnz)
    col_ptr = np.empty(spec.n + 1, dtype=np.int32)
    row_idx = np.empty(max(nnz, 1), dtype=np.int32)[:nnz]
    rc = lib.ditgen_build(ctypes.byref(p), col_ptr.ctypes.data, row_idx.ctypes.data, nnz)
    if rc:
        raise RuntimeError("ditgen_build failed (%d)" % rc)
    return col_ptr, row_idx


def graph_stats(spec: GraphSpec, col_ptr: np.ndarray, row_idx: np.ndarray) -> dict:
    """Shape statistics of a generated graph (counts only, no solver arithmetic)."""
    n = spec.n
    outdeg = np.diff(col_ptr.astype(np.int64))
    indeg = np.bincount(row_idx, minlength=n) if n else np.zeros(0, np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), outdeg)
    local = (src // spec.block) == (row_idx.astype(np.int64) // spec.block)
    # Hill estimator of the in-degree tail exponent over the top 1% (at least 10 values)
    tail_exp = None
    pos = np.sort(indeg[indeg > 0])[::-1].astype(np.float64)
    k = max(10, len(pos) // 100)
    if len(pos) > k + 1:
        xk = pos[k]
        tail_exp = 1.0 + k / float(np.sum(np.log(pos[:k] / xk)))
    return {
        "n": int(n),
        "nnz": int(row_idx.size),
        "mean_outdeg": float(row_idx.size / n) if n else 0.0,
        "dangling_frac": float(np.mean(outdeg == 0)) if n else 0.0,
        "local_frac": float(np.mean(local)) if row_idx.size else 0.0,
        "max_outdeg": int(outdeg.max()) if n else 0,
        "max_indeg": int(indeg.max()) if n else 0,
        "indeg_tail_exponent": tail_exp,
        "self_loops": int(np.sum(src == row_idx)),
        "zipf_offset": zipf_offset(spec),
        "spec": asdict(spec),
    }


def uniform_b(n: int, mass: float = 0.15) -> np.ndarray:
    """PageRank right-hand side B_i = (1-d)/N with 1-d = mass (FP64)."""
    return np.full(n, mass / n if n else 0.0, dtype=np.float64)


def ppr_seed_sets(n: int, nrhs: int, seed: int = 42, max_size: int = 1000):
    """Seed sets for personalized right-hand sides.

    Set sizes are floor(exp(U[0, ln(max_size+1)))), i.e. log-uniform in
    [1, max_size]; seeds are uniform without replacement. Returns a list of
    int64 arrays.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sets = []
    for _ in range(nrhs):
        size = int(np.floor(np.exp(rng.uniform(0.0, np.log(max_size + 1)))))
        size = max(1, min(size, max_size, n))
        sets.append(np.sort(rng.choice(n, size=size, replace=False)).astype(np.int64))
    return sets


def ppr_rhs_dense(n: int, seed_sets, mass: float = 0.15) -> np.ndarray:
    """Node-major FP64 [n, R] right-hand sides: mass spread evenly on each seed set."""
    b = np.zeros((n, len(seed_sets)), dtype=np.float64)
    for r, s in enumerate(seed_sets):
        b[s, r] = mass / len(s)
    return b


def signed_weights(col_ptr, c: float = 0.85, seed: int = 17) -> np.ndarray:
    """One weight per CSC entry for a general matrix of the same graph: values
    uniform in [-1, 1) with a seeded generator, each non-empty column scaled to
    l1 norm c (so the matrix is contractive with factor c)."""
    col_ptr = np.asarray(col_ptr, np.int64)
    rng = np.random.default_rng(seed)
    val = rng.uniform(-1.0, 1.0, int(col_ptr[-1]))
    deg = np.diff(col_ptr)
    col = np.repeat(np.arange(deg.size), deg)
    norm = np.bincount(col, weights=np.abs(val), minlength=deg.size)
    scale = np.where(norm > 0, c / np.where(norm > 0, norm, 1.0), 0.0)
    return val * scale[col]
