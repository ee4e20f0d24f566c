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

import sys
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

SRC = os.path.join(os.path.dirname(os.path.abspath(oracle.__file__)), "dref.c")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_small.json")

MUTANTS = {
    "push_to_self": ("f[row_idx[e]] += sent * p;", "f[i] += sent * p;"),
    "degree_off_by_one": ("double p = d / (double)k; /* p_ji", "double p = d / (double)(k + 1); /* p_ji"),
    "damping_dropped": ("double p = d / (double)k; /* p_ji", "double p = 1.0 / (double)k; /* p_ji"),
    "history_overwritten": ("h[i] += sent;", "h[i] = sent;"),
    "zero_after_push": ("      f[i] = 0.0;\n      int64_t k", "      int64_t k"),
    "signed_threshold": ("if (!(fabs(f[i]) > Ti)) continue;", "if (!(f[i] > Ti)) continue;"),
    "identity_sign": ("f[i] = b[i] - h[i];\n  for (int64_t i = 0; i < n; ++i) {",
                      "f[i] = b[i] + h[i];\n  for (int64_t i = 0; i < n; ++i) {"),
    "weighted_identity_sign": ("f[i] = b[i] - h[i];\n  for (int64_t i = 0; i < n; ++i)\n",
                               "f[i] = b[i] + h[i];\n  for (int64_t i = 0; i < n; ++i)\n"),
    "transposed_identity": ("for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[row_idx[e]] += p * h[i];",
                            "for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[i] += p * h[row_idx[e]];"),
    "cb_off_by_one": ("(int64_t)col_ptr[j] * K < k * L", "(int64_t)col_ptr[j] * K <= k * L"),
    "inout_drops_in_links": ("for (int64_t e = 0; e < nnz; ++e) cost[row_idx[e] + 1] += 1;",
                             "for (int64_t e = 0; e < 0; ++e) cost[row_idx[e] + 1] += 1;"),
    "inout_in_links_shifted": ("cost[row_idx[e] + 1] += 1;", "cost[row_idx[e]] += 1;"),
    # general matrix, priority test, internal-mass partition
    "weight_of_first_entry": ("f[row_idx[e]] += sent * val[e];", "f[row_idx[e]] += sent * val[col_ptr[i]];"),
    "weighted_identity_transposed": ("f[row_idx[e]] += val[e] * h[i];", "f[i] += val[e] * h[row_idx[e]];"),
    "priority_without_plus_one": ("c[i] = (c[i] + 1.0) * (double)(col_ptr[i + 1] - col_ptr[i] + 1);",
                                  "c[i] = c[i] * (double)(col_ptr[i + 1] - col_ptr[i]);"),
    "priority_in_links_only": ("c[i] = (c[i] + 1.0) * (double)(col_ptr[i + 1] - col_ptr[i] + 1);",
                               "c[i] = (c[i] + 1.0);"),
    "pmass_in_links_dropped": ("if (in_src[q] >= a && in_src[q] < j) inc += win[q];", ""),
    "pmass_self_links_twice": ("if (in_src[q] >= a && in_src[q] < j) inc += win[q];",
                               "if (in_src[q] >= a && in_src[q] <= j) inc += win[q];"),
    "pmass_first_fit_not_min_max": ("if (pmass_greedy(n, col_ptr, row_idx, wout, in_ptr, in_src, win, mid, K, NULL) <= K) hi = mid;",
                                    "if (pmass_greedy(n, col_ptr, row_idx, wout, in_ptr, in_src, win, mid, K, NULL) <= K + 1) hi = mid;"),
    # cut-minimizing partition
    "mincut_tie_takes_last": ("if (v < best) best = v, arg = q;", "if (v <= best) best = v, arg = q;"),
    "mincut_long_links_counted": ("if (a == z || z - a >= span) continue;", "if (a == z) continue;"),
    "mincut_unweighted": ("const int64_t u = link_units(NULL, 0.85, col_ptr, i, e);", "const int64_t u = 1;"),
    "mincut_in_cost_uncapped": ("C[i + 1] = C[i] + 1 + out + (indeg[i] < h ? indeg[i] : h);",
                                "C[i + 1] = C[i] + 1 + out + indeg[i];"),
    "mincut_no_slack": ("const int64_t cmax = cstar + cstar / 10, smax = sstar + sstar / 10;",
                        "const int64_t cmax = cstar, smax = sstar;"),
    "mincut_window_one_wider": ("lo[k] = t[k] - w;\n    hi[k] = t[k] + w;", "lo[k] = t[k] - w - 1;\n    hi[k] = t[k] + w + 1;"),
    "mincut_crossing_off_by_one": ("cross[a + 1] += u; /* the link", "cross[a] += u; /* the link"),
    "mincut_crossing_end_kept": ("      cross[z + 1] -= u;\n", "      cross[z] -= u;\n"),
    "mincut_tight_cycles_ignored": ("if (pass == 0 && k < K && tight[b] > 0) best = INF;",
                                    "if (pass == 0 && k < K && tight[b] < 0) best = INF;"),
    "mincut_three_cycles_ignored": ("if (k <= i || k == j || oi * oj * ok > 2) continue;", "if (1) continue;"),
    "mincut_tight_span_from_min": ("if (j - i < span) tight[i + 1] += 1, tight[j + 1] -= 1;",
                                   "if (j - i < span) tight[i] += 1, tight[j + 1] -= 1;"),
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
    """Return the names of the pins that fail for this oracle library."""
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


def general_pin_suite(lib):
    """Pins of the general-matrix solve, the priority test and the internal-mass
    partition (tests/test_oracle_general.py restated compactly)."""
    import test_oracle_general as tg

    fails = []
    rng = np.random.default_rng(21)
    n = 60
    cp, ri = random_graph(n, rng, p_edge=0.08, self_loops=True, multi=True)
    val = tg.signed_weights(cp, rng, 0.9)
    b = rng.normal(size=n)
    x = np.linalg.solve(np.eye(n) - tg.dense_w(cp, ri, val), b)
    try:
        r = oracle.solve(cp, ri, b, rel_tol=1e-14, val=val, d=0.9, max_sweeps=5000, lib=lib)
        if not (r.converged and np.abs(r.h - x).sum() <= r.resid_l1 / (1 - 0.9) + 1e-12):
            fails.append("general_dense")
    except ValueError:
        fails.append("general_dense")
    h = rng.normal(size=n)
    if np.abs(oracle.fluid_from_history_w(cp, ri, val, b, h, lib=lib)
              - (b + tg.dense_w(cp, ri, val) @ h - h)).max() > 1e-13:
        fails.append("general_identity")
    fcp, fri = csc_from_edges(5, [(i, 0) for i in range(1, 5)])
    r = oracle.solve(fcp, fri, np.array([1.0, .9, .9, .9, .9]), rel_tol=0.0, max_sweeps=1,
                     priority=True, lib=lib)
    if not np.array_equal(r.h, [0, .9, .9, .9, .9]):
        fails.append("priority_fan_in")
    ocp, ori = csc_from_edges(4, [(0, 1), (0, 2), (0, 3)])
    r = oracle.solve(ocp, ori, np.array([1.0, .3, .3, .3]), rel_tol=0.0, max_sweeps=1,
                     priority=True, lib=lib)
    if not (r.h[0] == 1.0 and np.all(r.f == 0)):
        fails.append("priority_fan_out")
    for seed, K in [(0, 2), (1, 3), (3, 4)]:
        g = np.random.default_rng(seed)
        scp, sri = random_graph(9, g, p_edge=0.3, self_loops=True, multi=True)
        w = tg.unit_weights(scp)
        ptr = oracle.partition_pmass(scp, sri, K, lib=lib)
        masses = [tg.block_mass(scp, sri, w, ptr[k], ptr[k + 1]) for k in range(K)]
        if max(masses) != tg.brute_min_max(scp, sri, w, K):
            fails.append("pmass_brute")
            break
    import test_oracle_mincut as tm
    cases = [(seed, n, K) for seed, n, K in [(0, 30, 2), (1, 30, 3), (3, 40, 4), (5, 25, 5), (6, 33, 3)]]
    for seed, n, K in cases:
        g = np.random.default_rng(seed)
        mcp, mri = tm.local_graph(n, g, p_out=0.25 if seed % 2 else 0.5)
        try:
            got = oracle.partition_mincut(mcp, mri, K, lib=lib).tolist()
        except ValueError:
            got = None
        if got != tm.brute_plan(mcp, mri, K)[0]:
            fails.append("mincut_brute")
            break
    for seed, K in [(0, 3), (1, 4), (2, 3)]:
        hcp, hri = tm.hub_graph(38, np.random.default_rng(50 + seed))
        try:
            got = oracle.partition_mincut(hcp, hri, K, lib=lib).tolist()
        except ValueError:
            got = None
        if got != tm.brute_plan(hcp, hri, K)[0]:
            fails.append("mincut_hubs")
            break
    for seed in (13, 17):
        xcp, xri, K = tm.mixed_case(seed)
        try:
            got = oracle.partition_mincut(xcp, xri, K, lib=lib).tolist()
        except ValueError:
            got = None
        if got != tm.brute_plan(xcp, xri, K)[0]:
            fails.append("mincut_mixed")
            break
    for seed in (23, 76, 103, 184):
        (pcp, pri), K = tm.planted_cycle(seed)
        try:
            got = oracle.partition_mincut(pcp, pri, K, lib=lib).tolist()
        except ValueError:
            got = None
        if got != tm.brute_plan(pcp, pri, K)[0]:
            fails.append("mincut_tight")
            break
    ecp, eri = csc_from_edges(40, [])
    try:
        got = oracle.partition_mincut(ecp, eri, 4, lib=lib).tolist()
    except ValueError:
        got = None
    if got != tm.brute_plan(ecp, eri, 4)[0]:
        fails.append("mincut_ties")
    return fails


def test_committed_oracle_passes(tmp_path):
    lib = build_variant(tmp_path, None)
    assert pin_suite(lib) == [] and general_pin_suite(lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    lib = build_variant(tmp_path, name)
    fails = pin_suite(lib) + general_pin_suite(lib)
    assert fails, "planted mistake %r went unnoticed" % name
