"""Pins of the oracle's general-matrix solve, priority test and internal-mass
partition (CPU only; nothing here uses the GPU library).

General matrix (Section 2: p_ij is the weight of the link j -> i, of either
sign; Section 1: the series converges when P is contractive):
  * LAPACK solves of (I - P) X = B with signed weights and signed B;
  * a two-node closed form;
  * power (Jacobi) iteration;
  * the PageRank weights d / #out_i given explicitly reproduce the PageRank
    solve bit for bit;
  * the identity F = B + P H - H against scipy, and ||F||_1 never growing.
Priority test (Section 2.4, F_i / ((#in_i + 1)(#out_i + 1))):
  * hand-computed first sweeps on a fan-in and a fan-out star that the plain
    |F_i| test would diffuse differently;
  * the converged H within the Section 2 bound of LAPACK.
Internal-mass partition (Section 2.3, the alternative balance):
  * brute force over every contiguous partition of small graphs (link weights
    in the same integer units, masses recomputed here from the definition);
  * equal blocks on a cycle.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from conftest import D, csc_from_edges, dense_p, random_graph


def signed_weights(cp, rng, c=0.9):
    """Random signed weights, each column's l1 norm equal to c (empty columns stay empty)."""
    n = cp.size - 1
    val = rng.uniform(-1.0, 1.0, int(cp[-1]))
    for i in range(n):
        s = np.abs(val[cp[i]:cp[i + 1]]).sum()
        if s > 0:
            val[cp[i]:cp[i + 1]] *= c / s
    return val


def dense_w(cp, ri, val):
    n = cp.size - 1
    rows = ri.astype(np.int64)
    cols = np.repeat(np.arange(n), np.diff(cp))
    return sp.csc_matrix((val, (rows, cols)), shape=(n, n)).toarray()  # duplicates summed


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_general_matrix_matches_lapack(seed):
    rng = np.random.default_rng(seed)
    n = 80
    cp, ri = random_graph(n, rng, p_edge=0.07, self_loops=True, multi=True)
    val = signed_weights(cp, rng, 0.9)
    assert abs(oracle.col_norm(cp, val) - 0.9) < 1e-12
    b = rng.normal(size=n)
    x = np.linalg.solve(np.eye(n) - dense_w(cp, ri, val), b)
    r = oracle.solve(cp, ri, b, rel_tol=1e-14, val=val, d=0.9)
    assert r.converged and r.increases == 0
    assert np.abs(r.h - x).sum() <= r.resid_l1 / (1 - 0.9) + 1e-12


def test_general_two_node_closed_form():
    # 0 -> 1 with weight -0.5, 1 -> 0 with weight 0.4:
    # x0 = b0 + 0.4 x1, x1 = b1 - 0.5 x0  =>  x0 = (b0 + 0.4 b1) / 1.2
    cp, ri = csc_from_edges(2, [(0, 1), (1, 0)])
    val = np.array([-0.5, 0.4])
    b = np.array([0.7, -0.2])
    x0 = (0.7 + 0.4 * -0.2) / 1.2
    x1 = -0.2 - 0.5 * x0
    r = oracle.solve(cp, ri, b, rel_tol=1e-15, val=val, d=0.5)
    assert r.converged
    assert abs(r.h[0] - x0) < 1e-14 and abs(r.h[1] - x1) < 1e-14


def test_general_matches_power_iteration():
    rng = np.random.default_rng(5)
    n = 120
    cp, ri = random_graph(n, rng, p_edge=0.05)
    val = signed_weights(cp, rng, 0.8)
    P = dense_w(cp, ri, val)
    b = rng.uniform(-1, 1, n)
    x = np.zeros(n)
    for _ in range(400):  # ||P||_1 <= 0.8: 0.8^400 is far below FP64 rounding
        x = P @ x + b
    r = oracle.solve(cp, ri, b, rel_tol=1e-14, val=val, d=0.8)
    assert np.abs(r.h - x).sum() <= r.resid_l1 / (1 - 0.8) + 1e-11


def test_pagerank_weights_given_explicitly_are_the_pagerank_solve():
    rng = np.random.default_rng(9)
    cp, ri = random_graph(150, rng, p_edge=0.04, self_loops=True, multi=True)
    deg = np.diff(cp)
    val = np.repeat(np.where(deg > 0, D / np.maximum(deg, 1), 0.0), deg)
    b = rng.uniform(0, 1, 150)
    a = oracle.solve(cp, ri, b, rel_tol=1e-13)
    w = oracle.solve(cp, ri, b, rel_tol=1e-13, val=val)
    assert np.array_equal(a.h, w.h) and np.array_equal(a.f, w.f) and a.edges == w.edges


def test_general_identity_against_scipy():
    rng = np.random.default_rng(11)
    n = 200
    cp, ri = random_graph(n, rng, p_edge=0.03, self_loops=True, multi=True)
    val = signed_weights(cp, rng, 0.95)
    b, h = rng.normal(size=n), rng.normal(size=n)
    want = b + dense_w(cp, ri, val) @ h - h
    got = oracle.fluid_from_history_w(cp, ri, val, b, h)
    assert np.abs(got - want).max() < 1e-13


def test_general_warm_start_reaches_the_same_limit():
    rng = np.random.default_rng(12)
    n = 90
    cp, ri = random_graph(n, rng, p_edge=0.06)
    val = signed_weights(cp, rng, 0.85)
    b = rng.normal(size=n)
    x = np.linalg.solve(np.eye(n) - dense_w(cp, ri, val), b)
    h0 = x + rng.normal(scale=0.1, size=n)
    r = oracle.solve(cp, ri, b, rel_tol=1e-14, val=val, h0=h0)
    assert r.converged
    assert np.abs(r.h - x).sum() <= r.resid_l1 / (1 - 0.85) + 1e-12


# --------------------------------------------------------------------- priority

def test_priority_first_sweep_fan_in():
    # leaves 1..4 -> hub 0 (dangling): c_0 = (4+1)(0+1) = 5, c_leaf = (0+1)(1+1) = 2.
    # B = [1, .9, .9, .9, .9]: scaled fluid [0.2, 0.45, ...], T_0 = 0.45 / 1.5 = 0.3.
    # Sweep 1: hub 1 > 0.3 * 5 fails; each leaf 0.9 > 0.3 * 2 passes and sends
    # 0.85 * 0.9 to the hub. The plain test (T_0 = 1 / 1.5) diffuses all five.
    cp, ri = csc_from_edges(5, [(i, 0) for i in range(1, 5)])
    b = np.array([1.0, 0.9, 0.9, 0.9, 0.9])
    r = oracle.solve(cp, ri, b, rel_tol=0.0, max_sweeps=1, priority=True)
    assert np.allclose(r.h, [0, 0.9, 0.9, 0.9, 0.9], atol=0, rtol=0)
    assert abs(r.f[0] - (1 + 4 * 0.85 * 0.9)) < 1e-15 and r.diffusions == 4
    plain = oracle.solve(cp, ri, b, rel_tol=0.0, max_sweeps=1)
    assert np.array_equal(plain.h, b)


def test_priority_first_sweep_fan_out():
    # hub 0 -> 1, 2, 3 (dangling): c_0 = (0+1)(3+1) = 4, c_leaf = (1+1)(0+1) = 2.
    # B = [1, .3, .3, .3]: T_0 = (1/4) / 1.5; the hub passes (1 > 2/3) and sends
    # 0.85/3 to each leaf, which then holds 0.3 + 0.85/3 > 2 T_0 = 1/3 and passes.
    cp, ri = csc_from_edges(4, [(0, 1), (0, 2), (0, 3)])
    b = np.array([1.0, 0.3, 0.3, 0.3])
    r = oracle.solve(cp, ri, b, rel_tol=0.0, max_sweeps=1, priority=True)
    leaf = 0.3 + 0.85 / 3
    assert r.h[0] == 1.0 and np.allclose(r.h[1:], leaf, rtol=1e-15, atol=0)
    assert np.all(r.f == 0)


@pytest.mark.parametrize("seed", [3, 4])
def test_priority_converges_to_lapack(seed):
    rng = np.random.default_rng(seed)
    n = 70
    cp, ri = random_graph(n, rng, p_edge=0.08, self_loops=True, multi=True)
    b = rng.uniform(0, 1, n)
    x = np.linalg.solve(np.eye(n) - dense_p(cp, ri), b)
    r = oracle.solve(cp, ri, b, rel_tol=1e-14, priority=True)
    assert r.converged and r.increases == 0
    assert np.abs(r.h - x).sum() <= r.resid_l1 / (1 - D) + 1e-13
    # with weights as well
    val = signed_weights(cp, rng, 0.9)
    x = np.linalg.solve(np.eye(n) - dense_w(cp, ri, val), b)
    r = oracle.solve(cp, ri, b, rel_tol=1e-14, priority=True, val=val)
    assert np.abs(r.h - x).sum() <= r.resid_l1 / (1 - 0.9) + 1e-12


# ----------------------------------------------------- internal-mass partition

def unit_weights(cp, val=None, d=D):
    deg = np.diff(cp)
    if val is None:  # the PageRank weight d / #out_i in FP64
        p = np.repeat(np.where(deg > 0, d / np.maximum(deg, 1), 0.0), deg)
    else:
        p = np.abs(val)
    return [int(np.floor(v * 4294967296.0)) for v in p]


def block_mass(cp, ri, w, a, b):
    """sum of the unit weights of links i -> t with a <= i < b and a <= t < b"""
    m = 0
    for i in range(a, b):
        for e in range(cp[i], cp[i + 1]):
            if a <= ri[e] < b:
                m += w[e]
    return m


def brute_min_max(cp, ri, w, K):
    n = cp.size - 1
    best = None
    for cuts in itertools.combinations_with_replacement(range(n + 1), K - 1):
        bounds = (0,) + cuts + (n,)
        worst = max(block_mass(cp, ri, w, bounds[k], bounds[k + 1]) for k in range(K))
        best = worst if best is None else min(best, worst)
    return best


@pytest.mark.parametrize("seed,K", [(0, 2), (1, 3), (2, 3), (3, 4), (4, 2)])
def test_pmass_partition_brute_force(seed, K):
    rng = np.random.default_rng(seed)
    n = 9
    cp, ri = random_graph(n, rng, p_edge=0.3, self_loops=True, multi=True)
    val = signed_weights(cp, rng, 0.9) if seed % 2 else None
    w = unit_weights(cp, val)
    ptr = oracle.partition_pmass(cp, ri, K, val=val)
    assert ptr[0] == 0 and ptr[K] == n and np.all(np.diff(ptr) >= 0)
    t_star = brute_min_max(cp, ri, w, K)
    masses = [block_mass(cp, ri, w, ptr[k], ptr[k + 1]) for k in range(K)]
    assert max(masses) == t_star
    # each block took as many nodes as the bound allows
    for k in range(K):
        a, b = int(ptr[k]), int(ptr[k + 1])
        if b < n and b > a:
            assert block_mass(cp, ri, w, a, b + 1) > t_star


def test_pmass_partition_equal_blocks_on_a_cycle():
    n = 16
    cp, ri = csc_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    assert oracle.partition_pmass(cp, ri, 4).tolist() == [0, 4, 8, 12, 16]
