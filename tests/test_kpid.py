"""The K-PID simulator (CPU): the paper's time-stepped model of K PIDs
(Sections 2.3-2.6, 3) on synthetic graphs.

Its outputs are context (operation counts), but its bookkeeping is pinned:
  * every run, with any K, delay or adaptation, ends with the D-iteration
    identity F = B + P H - H (fluid in flight counted in F), checked against
    the oracle's definition, so no message loses or duplicates fluid;
  * the converged H lies within the Section 2 bound of the oracle's solution;
  * the qualitative claims of Section 3: near-linear gain in K at large N/K,
    idle proportion growing with K, limited impact of delays, and the
    Section 3.4 adaptation moving omega_1 on an unbalanced 2-PID split.
"""
import numpy as np
import pytest

import ditgen
import kpid
import oracle
from conftest import D, dense_p, random_graph


@pytest.fixture(scope="module")
def web():
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=10_000, block=100, seed=1))
    b = ditgen.uniform_b(cp.size - 1)
    return cp, ri, b, oracle.solve(cp, ri, b, rel_tol=1e-13)


def check_run(cp, ri, b, r, ref=None):
    f_def = oracle.fluid_from_history(cp, ri, b, r.h)
    assert np.abs(r.f - f_def).sum() <= 1e-12 * np.abs(b).sum()
    assert abs(np.abs(r.f).sum() - r.resid_l1) <= 1e-12 * np.abs(b).sum()
    if ref is not None:
        assert np.abs(r.h - ref.h).sum() <= (r.resid_l1 + ref.resid_l1) / (1 - D) * (1 + 1e-9) + 1e-15


@pytest.mark.parametrize("K", [1, 2, 3, 8, 32])
def test_converges_within_the_bound(web, K):
    cp, ri, b, ref = web
    n = cp.size - 1
    r = kpid.simulate(cp, ri, b, oracle.partition_cb(cp, K), target_error=1e-9)
    assert r.converged and r.resid_l1 / (1 - D) <= 1e-9
    check_run(cp, ri, b, r, ref)
    assert (r.messages == 0) == (K == 1)


def test_small_graphs_against_lapack():
    rng = np.random.default_rng(4)
    for _ in range(3):
        n = 60
        cp, ri = random_graph(n, rng, p_edge=0.08, self_loops=True, multi=True)
        b = rng.uniform(0, 1, n)
        x = np.linalg.solve(np.eye(n) - dense_p(cp, ri), b)
        r = kpid.simulate(cp, ri, b, oracle.partition_uniform(n, 4), target_error=1e-12, speed=7)
        assert r.converged
        check_run(cp, ri, b, r)
        assert np.abs(r.h - x).sum() <= r.resid_l1 / (1 - D) + 1e-12


def test_gain_and_idle_grow_with_K(web):
    cp, ri, b, _ = web
    n = cp.size - 1
    runs = {K: kpid.simulate(cp, ri, b, oracle.partition_uniform(n, K)) for K in (1, 4, 64)}
    # target error 1/N (Section 3.1): the slowest PID's clock shrinks with K
    assert runs[4].norm_iters < runs[1].norm_iters / 2.5
    assert runs[64].norm_iters < runs[4].norm_iters
    assert runs[64].idle_frac > runs[4].idle_frac
    for r in runs.values():
        check_run(cp, ri, b, r)


@pytest.mark.parametrize("p", [0.2, 0.5, 0.8])
def test_delayed_exchange(web, p):
    cp, ri, b, ref = web
    n = cp.size - 1
    om = oracle.partition_cb(cp, 8)
    base = kpid.simulate(cp, ri, b, om, target_error=1e-9)
    r = kpid.simulate(cp, ri, b, om, target_error=1e-9, delay_proba=p, seed=11)
    assert r.converged
    check_run(cp, ri, b, r, ref)
    # Section 3.3: the impact is limited unless the delay probability is large
    if p <= 0.5:
        assert r.norm_iters <= 2.0 * base.norm_iters


def test_adaptation_moves_the_boundary():
    # Section 3.4: a uniform 2-PID split that is badly balanced: the first half
    # is a web graph, the second a ring of single out-links
    cp1, ri1 = ditgen.generate(ditgen.GraphSpec(n=10_000, block=100, seed=3))
    m = 10_000
    cp = np.concatenate([cp1, cp1[-1] + np.arange(1, m + 1)]).astype(np.int32)
    ri = np.concatenate([ri1, m + (np.arange(m) + 1) % m]).astype(np.int32)
    n = cp.size - 1
    b = ditgen.uniform_b(n)
    om = np.array([0, n // 2, n], np.int64)
    fixed = kpid.simulate(cp, ri, b, om, target_error=1e-9)
    r = kpid.simulate(cp, ri, b, om, target_error=1e-9, adapt_every=5, trace_steps=400)
    assert fixed.adaptations == 0 and r.adaptations > 0
    assert r.omega[1] < n // 2  # the loaded first PID gave nodes away
    assert r.converged and fixed.converged
    check_run(cp, ri, b, r)
    assert r.trace.shape[1:] == (2, 2) and np.all(r.trace[..., 0] >= 0)
