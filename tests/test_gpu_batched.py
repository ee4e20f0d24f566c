"""GPU parity of the batched personalized solve (many right-hand sides).

Each right-hand side B_r is a personalization vector (Section 2.2: V in
X = d Q X + (1-d) V) with mass 0.15 on a seed set. Every column of the
batched H must satisfy the same bound-based parity as a plain solve against an
independent oracle run with B_r alone, and the returned F must be the exact
residual of its column.
"""
import numpy as np
import pytest

import ditgen
import oracle
from conftest import D, csc_from_edges, sparse_p

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


def run_batched(ctx, cp, ri, B, tol, **opt):
    dev = torch.device("cuda", 0)
    g = ditr.Graph(ctx, torch.from_numpy(cp).to(dev), torch.from_numpy(ri).to(dev))
    bt = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
    ht = torch.empty_like(bt)
    ft = torch.empty(B.shape, dtype=torch.float32, device=dev)
    tot, per = ditr.solve_batched(ctx, g, bt, ht, ft, rel_tol=tol, opts=ditr.opts_default(**opt))
    torch.cuda.synchronize()
    out = ht.cpu().numpy(), ft.cpu().numpy().astype(np.float64), tot, per
    g.close()
    return out


def check_columns(cp, ri, B, H, F, per, tol, cols):
    P = sparse_p(cp, ri)
    for r in cols:
        b = B[:, r]
        ref = oracle.solve(cp, ri, b, rel_tol=1e-12)
        assert per[r].status == ditr.OK
        assert per[r].resid_l1 <= tol * np.abs(b).sum() * (1 + 1e-12)
        err = np.abs(H[:, r] - ref.h).sum()
        assert err <= (per[r].resid_l1 + ref.resid_l1) / (1 - D) * (1 + 1e-6), (r, err)
        assert err <= 1e-6 * ref.h.sum()
        ident = b + P @ H[:, r] - H[:, r]
        assert np.abs(F[:, r] - ident).sum() <= 1e-7 * np.abs(ident).sum() + 1e-14 * np.abs(H[:, r]).sum()


@pytest.mark.parametrize("R", [4, 16, 64])
def test_batched_parity_small(ctx, R):
    spec = ditgen.GraphSpec(n=20_000, block=1000, seed=5)
    cp, ri = ditgen.generate(spec)
    sets = ditgen.ppr_seed_sets(spec.n, R, seed=42)
    B = ditgen.ppr_rhs_dense(spec.n, sets)
    H, F, tot, per = run_batched(ctx, cp, ri, B, 1e-8)
    assert tot.status == ditr.OK
    check_columns(cp, ri, B, H, F, per, 1e-8, range(R) if R <= 16 else [0, 1, R // 2, R - 1])


def test_batched_uneven_and_uniform_columns(ctx):
    """Seed sets of very different sizes and a uniform column in one batch."""
    spec = ditgen.GraphSpec(n=30_000, block=1000, seed=8)
    cp, ri = ditgen.generate(spec)
    sets = [np.array([0]), np.arange(1000), np.array([spec.n - 1]), np.arange(0, spec.n, 7)]
    B = ditgen.ppr_rhs_dense(spec.n, sets)
    B = np.concatenate([B, ditgen.uniform_b(spec.n)[:, None], np.zeros((spec.n, 3))], axis=1)
    B[5, 6] = 0.3  # one seed, other mass
    H, F, tot, per = run_batched(ctx, cp, ri, B, 1e-9)
    check_columns(cp, ri, B, H, F, per, 1e-9, [0, 1, 2, 3, 4, 6])
    # an all-zero right-hand side stays at H = 0 with nothing diffused
    assert np.all(H[:, 5] == 0) and np.all(F[:, 5] == 0) and per[5].edges == 0


def _inlink_boundary_graph(n=3000, seed=11):
    """Rows with exactly 63, 64 and 65 in-links (64 is the most a row sums one
    link per lane; 65 goes to the heavy-row chunks), one with 200, rows with a
    single in-link, a self-loop, a repeated link and dangling nodes; the rest
    random with out-degree 1..8."""
    rng = np.random.default_rng(seed)
    edges = []
    special = {10: 63, 11: 64, 12: 65, 13: 200, 14: 64}
    for row, k in special.items():
        srcs = rng.choice(np.arange(100, n), size=k, replace=False)
        edges += [(int(s), row) for s in srcs]
    edges += [(20, 21), (21, 20), (22, 22), (23, 24), (23, 24)]  # self-loop, repeated link
    for s in range(100, n):
        if rng.random() < 0.1:
            continue  # many stay dangling (some also feed the special rows)
        for t in rng.integers(100, n, size=rng.integers(1, 9)):  # rows below 100 keep their counts
            edges.append((s, int(t)))
    return csc_from_edges(n, edges)


@pytest.mark.parametrize("R", [4, 256])
def test_batched_inlink_boundaries(ctx, R):
    """The in-link gathers of the batched sweep at their limits: rows of 63,
    64 and 65 in-links with every lane on (R = 256) and with most lanes off
    (R = 4); seed sets on the special rows and their sources."""
    cp, ri = _inlink_boundary_graph()
    n = cp.size - 1
    sets = [np.array([10, 11, 12, 13, 14]), np.arange(100, 400), np.array([20, 22, 23])]
    sets += list(ditgen.ppr_seed_sets(n, R - len(sets), seed=3))
    B = ditgen.ppr_rhs_dense(n, sets)
    H, F, tot, per = run_batched(ctx, cp, ri, B, 1e-9)
    assert tot.status == ditr.OK
    check_columns(cp, ri, B, H, F, per, 1e-9, sorted({0, 1, 2, R // 2, R - 1}))


def test_batched_matches_plain_solves(ctx):
    spec = ditgen.GraphSpec(n=50_000, block=1000, seed=9)
    cp, ri = ditgen.generate(spec)
    sets = ditgen.ppr_seed_sets(spec.n, 8, seed=7)
    B = ditgen.ppr_rhs_dense(spec.n, sets)
    H, F, tot, per = run_batched(ctx, cp, ri, B, 1e-9)
    dev = torch.device("cuda", 0)
    g = ditr.Graph(ctx, torch.from_numpy(cp).to(dev), torch.from_numpy(ri).to(dev))
    for r in range(8):
        bt = torch.from_numpy(np.ascontiguousarray(B[:, r])).to(dev)
        ht = torch.empty(spec.n, dtype=torch.float64, device=dev)
        ft = torch.empty(spec.n, dtype=torch.float32, device=dev)
        st = ditr.solve(ctx, g, bt, ht, ft, rel_tol=1e-9, allow=(ditr.OK,))
        h = ht.cpu().numpy()
        assert np.abs(h - H[:, r]).sum() <= (st.resid_l1 + per[r].resid_l1) / (1 - D) * (1 + 1e-6)
    g.close()


def test_batched_rejects_bad_shapes(ctx):
    dev = torch.device("cuda", 0)
    cp = torch.tensor([0, 1, 1], dtype=torch.int32, device=dev)
    ri = torch.tensor([1], dtype=torch.int32, device=dev)
    g = ditr.Graph(ctx, cp, ri)
    b = torch.zeros((2, 6), dtype=torch.float64, device=dev)
    with pytest.raises(ditr.DitrError) as e:
        ditr.solve_batched(ctx, g, b, torch.empty_like(b), torch.empty((2, 6), dtype=torch.float32, device=dev))
    assert e.value.status == ditr.EINVAL
    b = torch.full((2, 4), float("nan"), dtype=torch.float64, device=dev)
    with pytest.raises(ditr.DitrError) as e:
        ditr.solve_batched(ctx, g, b, torch.empty_like(b), torch.empty((2, 4), dtype=torch.float32, device=dev))
    assert e.value.status == ditr.ENONFINITE
    g.close()


def test_batched_headline_size_256(ctx):
    """The batched configuration at its own size: the 1e6-node headline graph
    with the benchmark's 256 seed sets (log-uniform sizes 1..1000, seed 42) at
    1e-8 per right-hand side. Its hub rows carry up to ~49K in-links, so their
    inflow is summed in many 2048-link chunks with all 256 lanes on, which the
    smaller batched cases never reach. Checked columns: the largest seed set,
    a single seed, and the sets that hold a seed on a row with more than 2048
    in-links (node 0, the largest hub, among them)."""
    spec = ditgen.HEADLINE
    cp, ri = ditgen.generate(spec)
    n, R, tol = spec.n, 256, 1e-8
    sets = ditgen.ppr_seed_sets(n, R, seed=42)
    indeg = np.bincount(ri, minlength=n)
    hubs = set(np.nonzero(indeg > 2048)[0].tolist())
    sizes = [len(s) for s in sets]
    largest = int(np.argmax(sizes))
    single = sizes.index(1)
    on_hub = [r for r, s in enumerate(sets) if hubs.intersection(s.tolist())]
    assert on_hub and max(indeg[list(hubs)]) > 2048 * 8, "workload lost its multi-chunk hub rows"
    cols = sorted({0, largest, single, *on_hub})
    print("c4 columns", cols, "sizes", [sizes[r] for r in cols], flush=True)
    dev = torch.device("cuda", 0)
    g = ditr.Graph(ctx, torch.from_numpy(cp).to(dev), torch.from_numpy(ri).to(dev))
    B = ditgen.ppr_rhs_dense(n, sets)
    bt = torch.from_numpy(B).to(dev)
    ht = torch.empty_like(bt)
    ft = torch.empty((n, R), dtype=torch.float32, device=dev)
    tot, per = ditr.solve_batched(ctx, g, bt, ht, ft, rel_tol=tol)
    torch.cuda.synchronize()
    assert tot.status == ditr.OK
    assert all(p.status == ditr.OK and p.resid_l1 <= tol * p.b_l1 * (1 + 1e-12) for p in per)
    idx = torch.tensor(cols, device=dev)
    H = np.zeros((n, R))
    F = np.zeros((n, R))
    H[:, cols] = ht.index_select(1, idx).cpu().numpy()
    F[:, cols] = ft.index_select(1, idx).cpu().numpy().astype(np.float64)
    del bt, ht, ft
    g.close()
    check_columns(cp, ri, B, H, F, per, tol, cols)


def test_batched_tuner_keeps_parity(ctx):
    """ditr_tune_batched picks alpha and the first refresh point by time; the
    options it returns still give oracle parity on every checked column, and
    it never returns options slower than the defaults at its final re-timing."""
    spec = ditgen.GraphSpec(n=20_000, block=1000, seed=6)
    cp, ri = ditgen.generate(spec)
    R = 16
    B = ditgen.ppr_rhs_dense(spec.n, ditgen.ppr_seed_sets(spec.n, R, seed=9))
    dev = torch.device("cuda", 0)
    g = ditr.Graph(ctx, torch.from_numpy(cp).to(dev), torch.from_numpy(ri).to(dev))
    bt = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
    ht = torch.empty_like(bt)
    ft = torch.empty(B.shape, dtype=torch.float32, device=dev)
    o, info = ditr.tune_batched(ctx, g, bt, ht, ft, rel_tol=1e-8, effort=1)
    assert info.candidates >= 8
    assert info.best_seconds <= info.default_seconds
    assert o.alpha in (1.25, 1.5, 2.0, 3.0, 4.0)
    assert o.refresh_at in (0.0, 1e-5, 1e-6, 1e-7)
    tot, per = ditr.solve_batched(ctx, g, bt, ht, ft, rel_tol=1e-8, opts=o)
    torch.cuda.synchronize()
    H, F = ht.cpu().numpy(), ft.cpu().numpy().astype(np.float64)
    g.close()
    assert tot.status == ditr.OK
    check_columns(cp, ri, B, H, F, per, 1e-8, [0, 5, R - 1])
    with pytest.raises(ditr.DitrError):
        ditr.tune_batched(ctx, ditr.Graph(ctx, torch.from_numpy(cp).to(dev), torch.from_numpy(ri).to(dev)),
                          bt, ht, ft, rel_tol=-1.0)
