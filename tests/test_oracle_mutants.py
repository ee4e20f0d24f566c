"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle/dref.c to a temporary directory, applies one plausible
mistake (wrong index, dropped term, wrong sign, reordered step, off-by-one),
compiles it with the same flags and runs a compact pin suite (exact rational
solutions, dense LAPACK solves, the identity, warm start, partition
definition). The committed oracle passes the suite; every mutant must fail it.
"""
import json
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import ditgen
import oracle
from conftest import D, csc_from_edges, dense_p, random_graph, sparse_p

SRC = os.path.join(os.path.dirname(os.path.abspath(oracle.__file__)), "dref.c")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_small.json")

MUTANTS = {
    "push_to_self": ("f[row_idx[e]] += sent * p;", "f[i] += sent * p;"),
    "degree_off_by_one": ("double p = d / (double)k; /* p_ji", "double p = d / (double)(k + 1); /* p_ji"),
    "damping_dropped": ("double p = d / (double)k; /* p_ji", "double p = 1.0 / (double)k; /* p_ji"),
    "history_overwritten": ("h[i] += sent;", "h[i] = sent;"),
    "zero_after_push": ("      f[i] = 0.0;\n      int64_t k", "      int64_t k"),
    "signed_threshold": ("if (!(fabs(f[i]) > T)) continue;", "if (!(f[i] > T)) continue;"),
    "identity_sign": ("f[i] = b[i] - h[i];", "f[i] = b[i] + h[i];"),
    "transposed_identity": ("for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[row_idx[e]] += p * h[i];",
                            "for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[i] += p * h[row_idx[e]];"),
    "cb_off_by_one": ("(int64_t)col_ptr[j] * K < k * L", "(int64_t)col_ptr[j] * K <= k * L"),
    "inout_drops_in_links": ("for (int64_t e = 0; e < nnz; ++e) cost[row_idx[e] + 1] += 1;",
                             "for (int64_t e = 0; e < 0; ++e) cost[row_idx[e] + 1] += 1;"),
    "inout_in_links_shifted": ("cost[row_idx[e] + 1] += 1;", "cost[row_idx[e]] += 1;"),
}


def _zero_after_push_fixup(src):
    # the mutant zeroes F_i after the pushes, which drops a self-loop's share
    return src.replace("        for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[row_idx[e]] += sent * p;\n      }",
                       "        for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[row_idx[e]] += sent * p;\n      }\n      f[i] = 0.0;")


def build_variant(tmp_path, name):
    src = open(SRC).read()
    if name is not None:
        old, new = MUTANTS[name]
        assert src.count(old) == 1, name
        src = src.replace(old, new)
        if name == "zero_after_push":
            src = _zero_after_push_fixup(src)
    c = tmp_path / ("dref_%s.c" % (name or "orig"))
    so = tmp_path / ("libdref_%s.so" % (name or "orig"))
    c.write_text(src)
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-fno-fast-math",
                           "-ffp-contract=off", str(c), "-o", str(so), "-lm"])
    return oracle.load_variant(str(so))


def pin_suite(lib):
    """Return the names of the pins that fail for this build."""
    fails = []
    try:
        for c in json.load(open(GOLDEN))["cases"]:
            cp, ri = csc_from_edges(c["n"], [tuple(e) for e in c["edges"]])
            b = np.array([float(Fraction(v)) for v in c["b"]])
            x = np.array([float(Fraction(v)) for v in c["x"]])
            r = oracle.solve(cp, ri, b, rel_tol=1e-15, max_sweeps=5000, lib=lib)
            if not (r.converged and np.abs(r.h - x).max() < 1e-14):
                fails.append("golden")
                break
    except ValueError:
        fails.append("golden")
    rng = np.random.default_rng(1)
    for _ in range(3):
        n = 60
        cp, ri = random_graph(n, rng, p_edge=0.08, self_loops=True, multi=True)
        b = rng.uniform(0, 1, n)
        x = np.linalg.solve(np.eye(n) - dense_p(cp, ri), b)
        r = oracle.solve(cp, ri, b, rel_tol=1e-13, max_sweeps=5000, lib=lib)
        if not (r.converged and np.abs(r.h - x).sum() <= r.resid_l1 / (1 - D) + 1e-13):
            fails.append("dense")
            break
    h = rng.normal(size=60)
    f = oracle.fluid_from_history(cp, ri, b, h, lib=lib)
    if np.abs(f - (b + sparse_p(cp, ri) @ h - h)).max() > 1e-13:
        fails.append("identity")
    spec = ditgen.GraphSpec(n=3000, block=100, seed=4)
    gcp, gri = ditgen.generate(spec)
    gb = ditgen.uniform_b(spec.n)
    ref = np.linalg.solve(np.eye(spec.n) - dense_p(gcp, gri), gb) if spec.n <= 3000 else None
    h0 = ref * np.random.default_rng(2).uniform(0.5, 1.5, spec.n)
    w = oracle.solve(gcp, gri, gb, rel_tol=1e-12, h0=h0, max_sweeps=400, lib=lib)
    if not (w.converged and np.abs(w.h - ref).sum() <= w.resid_l1 / (1 - D) + 1e-14):
        fails.append("warm_start")
    # on a 1-regular graph every prefix hits k L / K exactly: CB = uniform
    ccp, _ = csc_from_edges(16, [(i, (i + 1) % 16) for i in range(16)])
    if oracle.partition_cb(ccp, 4, lib=lib).tolist() != [0, 4, 8, 12, 16]:
        fails.append("cb_regular")
    # in+out balance against the definition (in-links counted independently)
    indeg = np.bincount(gri, minlength=spec.n)
    cost = np.concatenate([[0], np.cumsum(np.diff(gcp) + indeg)])
    pio = oracle.partition_cb_inout(gcp, gri, 8, lib=lib)
    for k in range(1, 8):
        j = int(pio[k])
        if not (8 * int(cost[j]) >= k * int(cost[-1]) and (j == 0 or 8 * int(cost[j - 1]) < k * int(cost[-1]))):
            fails.append("cb_inout")
            break
    K, L = 8, int(gcp[-1])
    ptr = oracle.partition_cb(gcp, K, lib=lib)
    for k in range(1, K):
        j = int(ptr[k])
        if not (K * int(gcp[j]) >= k * L and (j == 0 or K * int(gcp[j - 1]) < k * L)):
            fails.append("cb_partition")
            break
    return fails


def test_committed_oracle_passes(tmp_path):
    assert pin_suite(build_variant(tmp_path, None)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    fails = pin_suite(build_variant(tmp_path, name))
    assert fails, "planted mistake %r went unnoticed" % name
