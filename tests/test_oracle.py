"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check compares the oracle with something other than itself: exact
rational solutions, LAPACK dense solves, power iteration, closed forms, the
bound ||X - H||_1 <= ||F||_1 / (1 - d) (Section 2), the identity
F = B + P H - H (equations defF and defH) recomputed with scipy, and the
partition definitions of Section 2.3.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import ditgen
import oracle
from conftest import D, csc_from_edges, dense_p, random_graph, sparse_p

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_small.json")


def bound(res):
    return res.resid_l1 / (1 - D)


# ---------------- exact and dense references ---------------------------------

def test_exact_rational_golden():
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        cp, ri = csc_from_edges(c["n"], [tuple(e) for e in c["edges"]])
        b = np.array([float(Fraction(v)) for v in c["b"]])
        x = np.array([float(Fraction(v)) for v in c["x"]])
        res = oracle.solve(cp, ri, b, rel_tol=1e-15)
        assert res.converged
        assert np.abs(res.h - x).sum() <= bound(res) + 1e-15, c["name"]
        assert np.abs(res.h - x).max() < 1e-14, c["name"]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("kind", ["plain", "loops_multi"])
def test_dense_solve(seed, kind):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 120))
    cp, ri = random_graph(n, rng, p_edge=float(rng.uniform(0.01, 0.2)),
                          self_loops=kind != "plain", multi=kind != "plain")
    b = rng.uniform(0, 1, n) * (rng.random(n) < 0.7)
    x = np.linalg.solve(np.eye(n) - dense_p(cp, ri), b)
    res = oracle.solve(cp, ri, b, rel_tol=1e-13)
    assert res.converged and res.increases == 0
    err = np.abs(res.h - x).sum()
    assert err <= bound(res) + 1e-13
    assert err <= 1e-12 * max(np.abs(x).sum(), 1e-300) + 1e-15


def test_power_iteration_headline_shape():
    spec = ditgen.GraphSpec(n=20_000, block=1000, seed=5)
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    P = sparse_p(cp, ri)
    x = b.copy()
    for _ in range(400):  # ||P||_1 <= 0.85 -> error 0.85^400 ~ 1e-28
        x = P @ x + b
    res = oracle.solve(cp, ri, b, rel_tol=1e-13)
    assert res.converged
    assert np.abs(res.h - x).sum() <= bound(res) + 1e-15
    # D-iteration spends fewer elementary diffusions than the ~213 L of power
    # iteration to the same 1e-13 (Section 2.4 normalized iterations)
    assert res.edges < 213 * ri.size


# ---------------- closed forms -------------------------------------------------

def test_no_edges():
    n = 7
    cp = np.zeros(n + 1, np.int32)
    ri = np.zeros(0, np.int32)
    b = np.arange(1, n + 1, dtype=np.float64)
    res = oracle.solve(cp, ri, b, rel_tol=0)
    assert np.array_equal(res.h, b) and np.all(res.f == 0)
    assert res.edges == 0 and res.diffusions == n


def test_single_edge():
    cp, ri = csc_from_edges(2, [(0, 1)])
    b = np.array([0.3, 0.5])
    res = oracle.solve(cp, ri, b, rel_tol=1e-15)
    assert np.allclose(res.h, [0.3, 0.5 + D * 0.3], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 5, 64])
def test_cycle_uniform(n):
    cp, ri = csc_from_edges(n, [(i, (i + 1) % n) for i in range(n)]) if n > 1 else \
        csc_from_edges(1, [(0, 0)])
    b = np.full(n, 0.2)
    res = oracle.solve(cp, ri, b, rel_tol=1e-14)
    assert np.abs(res.h - 0.2 / (1 - D)).sum() <= bound(res) + 1e-13


def test_complete_digraph():
    n = 9
    cp, ri = csc_from_edges(n, [(i, j) for i in range(n) for j in range(n) if i != j])
    b = np.full(n, 0.01)
    res = oracle.solve(cp, ri, b, rel_tol=1e-14)
    assert np.abs(res.h - 0.01 / (1 - D)).max() < 1e-13


def test_star():
    k = 6
    cp, ri = csc_from_edges(k + 1, [(0, j) for j in range(1, k + 1)])
    b = np.linspace(0.1, 0.7, k + 1)
    res = oracle.solve(cp, ri, b, rel_tol=1e-15)
    want = b.copy()
    want[1:] += D * b[0] / k
    assert np.abs(res.h - want).max() < 1e-15


def test_probability_vector_distance():
    """Dangling-free graph, B = (1-d)/N: X is a probability vector and
    ||X - H||_1 = 1 - ||H||_1 (Section 2, after the bound)."""
    rng = np.random.default_rng(3)
    n = 80
    cp, ri = random_graph(n, rng, p_edge=0.08, dangling_frac=0.0)
    assert np.all(np.diff(cp) > 0)
    b = np.full(n, (1 - D) / n)
    x = np.linalg.solve(np.eye(n) - dense_p(cp, ri), b)
    assert abs(x.sum() - 1) < 1e-13
    for tol in [1e-2, 1e-5, 1e-9]:
        res = oracle.solve(cp, ri, b, rel_tol=tol)
        assert abs(np.abs(x - res.h).sum() - (1 - res.h.sum())) < 1e-13
        # and the distance is within the fluid bound
        assert 1 - res.h.sum() <= bound(res) + 1e-14


# ---------------- invariants -------------------------------------------------

def test_identity_monotone_mass_balance():
    spec = ditgen.GraphSpec(n=5000, block=100, seed=9)
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    P = sparse_p(cp, ri)
    dangling = np.diff(cp) == 0
    prev_h = np.zeros(spec.n)
    prev_r = np.inf
    for sweeps in [1, 3, 10, 30]:
        res = oracle.solve(cp, ri, b, rel_tol=0, max_sweeps=sweeps)
        assert res.sweeps == sweeps
        ident = b + P @ res.h - res.h
        assert np.abs(res.f - ident).sum() <= 1e-12 * b.sum()
        assert np.all(res.h >= prev_h)           # H non-decreasing for P, B >= 0
        assert np.all(np.diff(res.r_hist) <= 0)  # ||F||_1 never grows
        assert res.resid_l1 <= prev_r
        lhs = b.sum() - res.f.sum()
        rhs = (1 - D) * res.h[~dangling].sum() + res.h[dangling].sum()
        assert abs(lhs - rhs) <= 1e-13 * b.sum()
        prev_h, prev_r = res.h, res.resid_l1


def test_fluid_from_history_matches_scipy():
    rng = np.random.default_rng(4)
    cp, ri = random_graph(150, rng, p_edge=0.05, self_loops=True, multi=True)
    b = rng.uniform(0, 1, 150)
    h = rng.normal(size=150)
    f = oracle.fluid_from_history(cp, ri, b, h)
    P = sparse_p(cp, ri)
    assert np.abs(f - (b + P @ h - h)).max() < 1e-13


# ---------------- warm start and schedule independence -----------------------

def test_warm_start_same_limit():
    spec = ditgen.GraphSpec(n=8000, block=100, seed=21)
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    cold = oracle.solve(cp, ri, b, rel_tol=1e-13)
    rng = np.random.default_rng(0)
    h0 = cold.h * rng.uniform(0.5, 1.5, spec.n)   # signed residual
    warm = oracle.solve(cp, ri, b, rel_tol=1e-13, h0=h0)
    assert warm.converged
    assert np.abs(warm.h - cold.h).sum() <= bound(warm) + bound(cold) + 1e-16
    # a close H_0 leaves ||F_0||_1 ~ 1e-5 ||B||_1: the remaining work shrinks
    # roughly like log(||F_0||_1 / tol) / log(1 / tol), here to about half
    good = oracle.solve(cp, ri, b, rel_tol=1e-13, h0=cold.h * (1 + 1e-6))
    assert good.edges < 0.6 * cold.edges


@pytest.mark.parametrize("alpha", [1.2, 1.5, 2.0])
def test_alpha_insensitive(alpha):
    spec = ditgen.GraphSpec(n=6000, block=100, seed=13)
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    ref = oracle.solve(cp, ri, b, rel_tol=1e-13, alpha=1.5)
    res = oracle.solve(cp, ri, b, rel_tol=1e-13, alpha=alpha)
    assert np.abs(res.h - ref.h).sum() <= bound(res) + bound(ref)
    # Section 2.4: the cost is not sensitive to alpha in [1.2, 2]
    assert res.edges < 1.5 * ref.edges


# ---------------- partitions (Section 2.3) -----------------------------------

def test_partition_uniform():
    assert oracle.partition_uniform(10, 3).tolist() == [0, 3, 6, 10]
    assert oracle.partition_uniform(8, 8).tolist() == list(range(9))
    with pytest.raises(ValueError):
        oracle.partition_uniform(4, 5)


@pytest.mark.parametrize("K", [1, 2, 4, 7, 64])
def test_partition_cb_balance(K):
    spec = ditgen.GraphSpec(n=30_000, block=1000, seed=2)
    cp, ri = ditgen.generate(spec)
    ptr = oracle.partition_cb(cp, K)
    assert ptr[0] == 0 and ptr[-1] == spec.n and np.all(np.diff(ptr) >= 0)
    L = int(cp[-1])
    maxdeg = int(np.diff(cp).max())
    cost = cp[ptr[1:]].astype(np.int64) - cp[ptr[:-1]]
    assert np.all(np.abs(cost - L / K) <= maxdeg)
    # brute force: each omega_k is the first id whose out-link prefix reaches k L / K
    for k in range(1, K):
        j = int(ptr[k])
        assert K * int(cp[j]) >= k * L and (j == 0 or K * int(cp[j - 1]) < k * L)


def test_partition_cb_regular_is_uniform():
    """With equal out-degrees, equal cost means equal size: CB = uniform."""
    for n, K in [(16, 4), (30, 5), (12, 12)]:
        cp, _ = csc_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
        assert oracle.partition_cb(cp, K).tolist() == oracle.partition_uniform(n, K).tolist()


def test_partition_cb_nested():
    """The K = 2 split reappears among the K = 4 boundaries (Section 3.2)."""
    spec = ditgen.GraphSpec(n=100_000, block=1000, seed=2)
    cp, _ = ditgen.generate(spec)
    p2, p4 = oracle.partition_cb(cp, 2), oracle.partition_cb(cp, 4)
    assert p2[1] == p4[2]
    p8 = oracle.partition_cb(cp, 8)
    assert set(p4.tolist()) <= set(p8.tolist())


@pytest.mark.parametrize("K", [1, 3, 16, 100])
def test_partition_cb_inout_balance(K):
    """In+out cost per block within the largest in+out degree of 2L/K, and each
    boundary is the first id whose in+out prefix reaches k 2L/K."""
    spec = ditgen.GraphSpec(n=20_000, block=1000, seed=6)
    cp, ri = ditgen.generate(spec)
    ptr = oracle.partition_cb_inout(cp, ri, K)
    indeg = np.bincount(ri, minlength=spec.n)
    cost = np.concatenate([[0], np.cumsum(np.diff(cp) + indeg)])
    L2 = int(cost[-1])
    maxdeg = int((np.diff(cp) + indeg).max())
    blocks = cost[ptr[1:]] - cost[ptr[:-1]]
    assert np.all(np.abs(blocks - L2 / K) <= maxdeg)
    for k in range(1, K):
        j = int(ptr[k])
        assert K * int(cost[j]) >= k * L2 and (j == 0 or K * int(cost[j - 1]) < k * L2)
    # hubs have large in-degree: the first block holds fewer ids than under CB
    if K >= 16:
        assert ptr[1] < oracle.partition_cb(cp, K)[1]


def test_partition_cb_inout_special_cases():
    # 1-regular both ways: in+out balance is the uniform split
    n = 24
    cp, ri = csc_from_edges(n, [(i, (i + 5) % n) for i in range(n)])
    assert oracle.partition_cb_inout(cp, ri, 6).tolist() == oracle.partition_uniform(n, 6).tolist()
    # symmetric graph: in-link prefix = out-link prefix, so CB_INOUT = CB
    rng = np.random.default_rng(8)
    und = set()
    for _ in range(300):
        a, b = rng.integers(0, 60, 2)
        if a != b:
            und.add((int(a), int(b)))
            und.add((int(b), int(a)))
    cp, ri = csc_from_edges(60, sorted(und))
    for K in (2, 5, 9):
        assert oracle.partition_cb_inout(cp, ri, K).tolist() == oracle.partition_cb(cp, K).tolist()


def test_rejects_bad_input():
    cp = np.array([0, 1], np.int32)
    ri = np.array([3], np.int32)
    with pytest.raises(ValueError):
        oracle.solve(cp, ri, np.ones(1))
    assert oracle.check_csc(1, cp, ri) == oracle.EGRAPH
    with pytest.raises(ValueError):
        oracle.solve(np.array([0, 0], np.int32), np.zeros(0, np.int32), np.ones(1), d=1.0)
