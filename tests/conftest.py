import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


# ---------------------------------------------------------------------------
# Helpers used by the tests only. They restate the problem definition (P from
# a CSC graph) with library routines, independently of the oracle's C code.
# ---------------------------------------------------------------------------

D = 0.85


def csc_from_edges(n, edges):
    """CSC (col_ptr, row_idx) from a list of (source, target) out-links, in order."""
    cols = [[] for _ in range(n)]
    for s, t in edges:
        cols[s].append(t)
    col_ptr = np.zeros(n + 1, np.int32)
    for i in range(n):
        col_ptr[i + 1] = col_ptr[i] + len(cols[i])
    row_idx = np.array([t for c in cols for t in c], dtype=np.int32)
    return col_ptr, row_idx


def sparse_p(col_ptr, row_idx, d=D):
    """scipy CSC matrix P with P[j, i] = d / #out_i for every entry (duplicates summed)."""
    import scipy.sparse as sp

    n = col_ptr.size - 1
    outdeg = np.diff(col_ptr.astype(np.int64))
    vals = np.repeat(np.where(outdeg > 0, d / np.maximum(outdeg, 1), 0.0), outdeg)
    return sp.csc_matrix((vals, row_idx.astype(np.int64), col_ptr.astype(np.int64)), shape=(n, n))


def dense_p(col_ptr, row_idx, d=D):
    return sparse_p(col_ptr, row_idx, d).toarray()


def random_graph(n, rng, p_edge=0.05, self_loops=False, multi=False, dangling_frac=0.1):
    edges = []
    for s in range(n):
        if rng.random() < dangling_frac:
            continue
        for t in range(n):
            if t == s and not self_loops:
                continue
            if rng.random() < p_edge:
                edges.append((s, t))
                if multi and rng.random() < 0.3:
                    edges.append((s, t))
    return csc_from_edges(n, edges)


@pytest.fixture
def rng():
    return np.random.default_rng(12345)
