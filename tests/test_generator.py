"""Seeded input generator: determinism and the workload shape (no solver arithmetic)."""
import numpy as np
import pytest

import ditgen


def test_deterministic_by_seed():
    s = ditgen.GraphSpec(n=5000, block=100, seed=7)
    a = ditgen.generate(s)
    b = ditgen.generate(s)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c = ditgen.generate(ditgen.GraphSpec(n=5000, block=100, seed=8))
    assert not np.array_equal(a[1][:1000], c[1][:1000])


@pytest.mark.parametrize("spec", [ditgen.SMALL, ditgen.GraphSpec(n=200_000, block=1000, seed=2)])
def test_shape_statistics(spec):
    cp, ri = ditgen.generate(spec)
    st = ditgen.graph_stats(spec, cp, ri)
    assert abs(st["mean_outdeg"] - 8.0) / 8.0 < 0.03
    assert abs(st["dangling_frac"] - 0.10) < 0.01
    # block 100 caps local links of high-degree nodes, so allow a little less locality there
    assert 0.75 < st["local_frac"] < 0.82
    assert st["max_outdeg"] <= 200
    assert st["self_loops"] == 0
    assert abs(st["zipf_offset"] - 1.853) < 0.01


def test_csc_valid_sorted_distinct():
    spec = ditgen.GraphSpec(n=3000, block=100, seed=11)
    cp, ri = ditgen.generate(spec)
    assert cp[0] == 0 and cp[-1] == ri.size and np.all(np.diff(cp) >= 0)
    assert ri.min() >= 0 and ri.max() < spec.n
    for i in range(spec.n):
        col = ri[cp[i]:cp[i + 1]]
        assert np.all(np.diff(col) > 0), "targets of a column must be sorted and distinct"
        assert not np.any(col == i)


@pytest.mark.parametrize("n", [1, 2, 3, 17])
def test_tiny_graphs(n):
    spec = ditgen.GraphSpec(n=n, block=4, seed=3)
    cp, ri = ditgen.generate(spec)
    assert cp.size == n + 1
    outdeg = np.diff(cp)
    assert np.all(outdeg <= max(n - 1, 0))
    for i in range(n):
        col = ri[cp[i]:cp[i + 1]]
        assert len(set(col.tolist())) == len(col) and i not in col


def test_ppr_seed_sets():
    sets = ditgen.ppr_seed_sets(100_000, 256, seed=42)
    sizes = np.array([len(s) for s in sets])
    assert sizes.min() >= 1 and sizes.max() <= 1000
    # log-uniform sizes: the median sits near sqrt(1001) ~ 32
    assert 10 < np.median(sizes) < 100
    for s in sets:
        assert len(np.unique(s)) == len(s)
    b = ditgen.ppr_rhs_dense(100_000, sets[:4])
    assert np.allclose(b.sum(axis=0), 0.15)
