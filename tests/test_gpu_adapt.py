"""Partition plans set by the caller and the adaptation of Section 3.4
(ditr_graph_set_partitions, ditr_graph_adapt).

Any node-set partition is valid for the D-iteration (Section 2.3): the
solution does not depend on it, only the work does. So after every change of
the plan the solve must keep oracle parity, and the adaptation may only keep
a plan that made the solve faster.
"""
import numpy as np
import pytest

import ditgen
import oracle
from conftest import D, sparse_p

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1202_6168_amd import ditr  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ditr.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def problem():
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=60_000, block=300, seed=12))
    b = ditgen.uniform_b(cp.size - 1)
    return cp, ri, b, oracle.solve(cp, ri, b, rel_tol=1e-12)


def tensors(problem):
    cp, ri, b, _ = problem
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(cp).to(dev), torch.from_numpy(ri).to(dev), torch.from_numpy(b).to(dev),
            torch.empty(b.size, dtype=torch.float64, device=dev), torch.empty(b.size, dtype=torch.float32, device=dev))


def solve_and_check(ctx, g, problem, bt, ht, ft, flags=0, tol=1e-9):
    cp, ri, b, ref = problem
    st = ditr.solve(ctx, g, bt, ht, ft, rel_tol=tol, opts=ditr.opts_default(mode=ditr.MODE_PARTITION, flags=flags))
    torch.cuda.synchronize()
    h, f = ht.cpu().numpy(), ft.cpu().numpy().astype(np.float64)
    assert st.status == ditr.OK
    err = np.abs(h - ref.h).sum()
    assert err <= (st.resid_l1 + ref.resid_l1) / (1 - D) * (1 + 1e-6)
    assert err <= 1e-6 * np.abs(ref.h).sum()
    ident = b + sparse_p(cp, ri) @ h - h
    assert np.abs(f - ident).sum() <= 1e-7 * np.abs(ident).sum() + 1e-14 * np.abs(h).sum()
    return st


@pytest.mark.parametrize("flags", [0, ditr.FLAG_NO_RESIDENT], ids=["resident", "relaunch"])
def test_set_partitions_keeps_parity(ctx, problem, flags):
    cpt, rit, bt, ht, ft = tensors(problem)
    n = bt.numel()
    g = ditr.Graph(ctx, cpt, rit, opts=ditr.opts_default(part_nodes=2000))
    ptr = g.partitions()
    K = ptr.size - 1
    solve_and_check(ctx, g, problem, bt, ht, ft, flags)
    # shift every inner boundary by a pseudo-random amount, keeping the parts valid
    rng = np.random.default_rng(3)
    new = ptr.copy()
    new[1:-1] += rng.integers(-400, 401, size=K - 1)
    new[1:-1] = np.clip(new[1:-1], 1, n - 1)
    new = np.maximum.accumulate(new)
    g.set_partitions(new)
    assert np.array_equal(g.partitions(), new)
    solve_and_check(ctx, g, problem, bt, ht, ft, flags)
    # a different number of parts, uniform
    K2 = K + 5
    uni = (np.arange(K2 + 1) * n) // K2
    g.set_partitions(uni)
    assert len(g.partitions()) == K2 + 1
    solve_and_check(ctx, g, problem, bt, ht, ft, flags)
    g.close()


def test_set_partitions_rejects_bad_plans(ctx, problem):
    cpt, rit, bt, ht, ft = tensors(problem)
    n = bt.numel()
    g = ditr.Graph(ctx, cpt, rit, opts=ditr.opts_default(part_nodes=2000))
    good = g.partitions()
    for bad in (np.array([1, n]), np.array([0, n - 1]), np.array([0, n // 2, n // 4, n]),
                np.array([0, n])):  # the last: one part of n nodes does not fit one workgroup's LDS
        with pytest.raises(ditr.DitrError):
            g.set_partitions(bad)
        g.set_partitions(good)  # a failed call may leave no plan: a valid one restores it
    solve_and_check(ctx, g, problem, bt, ht, ft)
    g.close()
    # a graph in a caller workspace keeps its plan
    ws = torch.empty(ditr.workspace_bytes(ctx, n, rit.numel()), dtype=torch.uint8, device=bt.device)
    gw = ditr.Graph(ctx, cpt, rit, workspace=ws)
    with pytest.raises(ditr.DitrError):
        gw.set_partitions(gw.partitions())
    with pytest.raises(ditr.DitrError):
        ditr.adapt(ctx, gw, bt, ht, ft)
    gw.close()


def test_adapt_keeps_parity_and_never_slows(ctx, problem):
    cpt, rit, bt, ht, ft = tensors(problem)
    g = ditr.Graph(ctx, cpt, rit, opts=ditr.opts_default(part_nodes=2000))
    before = g.partitions()
    info = ditr.adapt(ctx, g, bt, ht, ft, rel_tol=1e-9, rounds=3, omega=0.5)
    assert 1 <= info.rounds <= 3 and 0 <= info.kept <= info.rounds
    assert info.seconds_after <= info.seconds_before
    assert info.spread_before >= 1 and info.spread_after >= 1
    after = g.partitions()
    assert after[0] == 0 and after[-1] == bt.numel() and (np.diff(after) >= 1).all()
    if info.kept == 0:
        assert np.array_equal(after, before)
    solve_and_check(ctx, g, problem, bt, ht, ft)
    with pytest.raises(ditr.DitrError):
        ditr.adapt(ctx, g, bt, ht, ft, omega=0.0)
    g.close()
