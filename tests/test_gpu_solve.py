"""GPU parity of the plain solve against the FP64 oracle (through the C-ABI).

Several H are correct (the diffusion order is free, Section 2), so H is not
compared bit for bit: every valid run satisfies ||X - H||_1 <= ||F||_1/(1-d)
(Section 2, the bound after defH), hence
    ||H_gpu - H_oracle||_1 <= (tol_gpu + tol_oracle) ||B||_1 / (1 - d),
and the headline requirement ||H_gpu - H_oracle||_1 <= 1e-6 ||H_oracle||_1.
The returned F must be the exact residual B + P H - H (rounded to FP32).
"""
import threading
import time

import numpy as np
import pytest

import ditgen
import oracle
from conftest import D, csc_from_edges, random_graph, sparse_p

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


def upload(cp, ri):
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(np.ascontiguousarray(cp, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(ri, np.int32)).to(dev) if ri.size else
            torch.zeros(1, dtype=torch.int32, device=dev)[:0])


def gpu_solve(ctx, cp, ri, b, tol, h0=None, **opt):
    g = ditr.Graph(ctx, *upload(cp, ri), opts=ditr.opts_default(**{k: v for k, v in opt.items()
                                                                    if k in ("part_nodes", "part_type", "block", "wg_per_cu")}))
    dev = torch.device("cuda", 0)
    bt = torch.from_numpy(np.ascontiguousarray(b, np.float64)).to(dev)
    ht = (torch.from_numpy(np.ascontiguousarray(h0, np.float64)).to(dev) if h0 is not None
          else torch.empty(len(b), dtype=torch.float64, device=dev))
    ft = torch.empty(len(b), dtype=torch.float32, device=dev)
    st = ditr.solve(ctx, g, bt, ht, ft, warm=h0 is not None, rel_tol=tol,
                    opts=ditr.opts_default(**opt))
    torch.cuda.synchronize()
    out = ht.cpu().numpy(), ft.cpu().numpy().astype(np.float64), st
    g.close()
    return out


def resid_rounding(cp, ri, b, h):
    """Bound on the FP64 rounding of a computed ||B + P H - H||_1: per row j,
    (#in_j + 2) u (|B_j| + (P|H|)_j + |H_j|) (recursive summation, u = 2^-53)."""
    n = cp.size - 1
    indeg = np.bincount(ri, minlength=n)
    mag = np.abs(b) + sparse_p(cp, ri) @ np.abs(h) + np.abs(h)
    return float(((indeg + 2) * 2.0 ** -53 * mag).sum())


def check_parity(cp, ri, b, h, f, st, tol, ref=None, ref_tol=1e-13):
    """Bound-based parity with the oracle + the identity on the returned F.

    ||H - X||_1 <= ||F||_1 / (1 - d) (Section 2) holds for the exact residual;
    the reported ones are FP64 sums, so each side gets its rounding bound. The
    bound is attained on graphs whose leftover fluid circulates without loss
    (a cycle through a hub), where that rounding decides the comparison."""
    ref = ref if ref is not None else oracle.solve(cp, ri, b, rel_tol=ref_tol)
    b1 = np.abs(b).sum()
    assert st.status == ditr.OK, ditr.last_error()
    assert st.resid_l1 <= tol * b1 * (1 + 1e-12)
    err = np.abs(h - ref.h).sum()
    slack = resid_rounding(cp, ri, b, h) + resid_rounding(cp, ri, b, ref.h)
    assert err <= (st.resid_l1 + ref.resid_l1 + slack) / (1 - D) * (1 + 1e-6) + 1e-300
    assert err <= 1e-6 * np.abs(ref.h).sum() + 1e-300
    ident = b + sparse_p(cp, ri) @ h - h
    scale = np.abs(b).sum() + np.abs(h).sum()
    assert np.abs(f - ident).sum() <= 1e-7 * np.abs(ident).sum() + 1e-14 * scale
    assert abs(np.abs(f).sum() - st.resid_l1) <= 1e-6 * st.resid_l1 + 1e-14 * scale
    return ref


# ---------------------------------------------------------------------------
# adversarial small graphs, every kernel mode and forced tiny partitions

def _adversarial():
    cases = []
    n = 257
    cases.append(("hub_in", *csc_from_edges(n, [(i, 0) for i in range(1, n)] + [(0, 5)])))
    cases.append(("hub_out", *csc_from_edges(n, [(0, j) for j in range(1, n)])))
    cases.append(("loops_multi", *random_graph(150, np.random.default_rng(7), 0.05, True, True)))
    cases.append(("all_dangling", np.zeros(101, np.int32), np.zeros(0, np.int32)))
    cases.append(("single_node", np.zeros(2, np.int32), np.zeros(0, np.int32)))
    cases.append(("single_loop", *csc_from_edges(1, [(0, 0)])))
    edges = [(i, (i + 1) % 999) for i in range(3, 990)]  # empty columns at both ends
    cases.append(("empty_ends", *csc_from_edges(999, edges)))
    cases.append(("cycle", *csc_from_edges(1000, [(i, (i + 1) % 1000) for i in range(1000)])))
    return cases


ADV = _adversarial()


@pytest.mark.parametrize("case", ADV, ids=[c[0] for c in ADV])
@pytest.mark.parametrize("mode,part_nodes,block,flags", [
    (ditr.MODE_PARTITION, 0, 1024, 0),
    (ditr.MODE_PARTITION, 3, 1024, 0),  # tiny partitions: nearly every link crosses
    (ditr.MODE_PARTITION, 64, 1024, 0),
    (ditr.MODE_PARTITION, 3, 1024, ditr.FLAG_NO_RESIDENT),  # one launch per threshold level
    (ditr.MODE_PARTITION, 64, 1024, ditr.FLAG_NO_RESIDENT),
    (ditr.MODE_ASYNC, 0, 1024, 0),
    (ditr.MODE_ASYNC, 3, 256, 0),
    (ditr.MODE_ASYNC, 16, 512, 0),
    (ditr.MODE_SWEEP, 0, 1024, 0),
])
def test_adversarial_parity(ctx, case, mode, part_nodes, block, flags):
    name, cp, ri = case
    n = cp.size - 1
    rng = np.random.default_rng(n)
    b = rng.uniform(0.1, 1.0, n) / n
    tol = 1e-10
    h, f, st = gpu_solve(ctx, cp, ri, b, tol, mode=mode, part_nodes=part_nodes, block=block,
                         flags=flags)
    check_parity(cp, ri, b, h, f, st, tol)


def test_closed_forms(ctx):
    # one edge 0 -> 1
    cp, ri = csc_from_edges(2, [(0, 1)])
    b = np.array([0.3, 0.5])
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-12)
    assert np.abs(h - [0.3, 0.5 + D * 0.3]).max() < 1e-12
    # star: hub -> k dangling leaves
    k = 40
    cp, ri = csc_from_edges(k + 1, [(0, j) for j in range(1, k + 1)])
    b = np.linspace(0.1, 0.7, k + 1)
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-12, part_nodes=4)
    want = b.copy()
    want[1:] += D * b[0] / k
    assert np.abs(h - want).max() < 1e-12
    # directed cycle, uniform B: x = b / (1 - d)
    n = 5000
    cp, ri = csc_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    h, f, st = gpu_solve(ctx, cp, ri, np.full(n, 0.2), 1e-11)
    assert np.abs(h - 0.2 / (1 - D)).sum() <= st.resid_l1 / (1 - D) * (1 + 1e-6) + 1e-12


# ---------------------------------------------------------------------------
# the workload graphs

@pytest.mark.parametrize("mode", [ditr.MODE_PARTITION, ditr.MODE_ASYNC, ditr.MODE_SWEEP])
def test_small_workload_parity(ctx, mode):
    """1e4 nodes, block-100 locality, tolerance 1e-12 ||B||_1."""
    spec = ditgen.SMALL
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-12, mode=mode)
    check_parity(cp, ri, b, h, f, st, 1e-12, ref_tol=1e-14)
    assert st.edges > 0 and st.diffusions > 0


@pytest.fixture(scope="module")
def headline():
    spec = ditgen.HEADLINE
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    ref = oracle.solve(cp, ri, b, rel_tol=1e-12)
    return cp, ri, b, ref


@pytest.mark.parametrize("mode", [ditr.MODE_PARTITION, ditr.MODE_ASYNC, ditr.MODE_SWEEP])
def test_headline_parity(ctx, headline, mode):
    """1e6 nodes, ~8e6 edges, tolerance 1e-9 ||B||_1; H within 1e-6 relative L1."""
    cp, ri, b, ref = headline
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-9, mode=mode)
    check_parity(cp, ri, b, h, f, st, 1e-9, ref=ref)
    # D-iteration's cost stays well below power iteration's 128 L at 1e-9
    assert st.edges < 128 * ri.size


@pytest.mark.parametrize("flags", [0, ditr.FLAG_NO_RESIDENT])
def test_headline_resident_and_relaunch(ctx, headline, flags):
    """The partitioned sweep with its partitions resident across threshold
    levels (one cooperative launch per stage) and relaunched per level."""
    cp, ri, b, ref = headline
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-9, mode=ditr.MODE_PARTITION, flags=flags)
    check_parity(cp, ri, b, h, f, st, 1e-9, ref=ref)
    # one launch per stage when resident, one per level otherwise
    assert (st.launches <= st.rounds) if flags == 0 else (st.launches >= st.sweeps)


def uniform_graph(n, outdeg, seed, dangling=0.1):
    """Seeded graph: every non-dangling node has `outdeg` targets drawn
    uniformly (repeated links and self-loops allowed)."""
    rng = np.random.default_rng(seed)
    deg = np.where(rng.random(n) < dangling, 0, outdeg).astype(np.int64)
    cp = np.zeros(n + 1, np.int64)
    cp[1:] = np.cumsum(deg)
    ri = rng.integers(0, n, int(cp[-1]))
    return cp.astype(np.int32), ri.astype(np.int32)


def plan_counts(cp, ri, omega, heavy=4, item=512):
    """Per partition, the light outside in-links (rows with at most `heavy` of
    them) and, overall, the one-wave work units of the heavy items (a row's
    outside in-links cut in items of at most `item`; an item takes 2^l lanes of
    eight links; 64 lanes per unit, packed without gaps largest first)."""
    n = cp.size - 1
    pid = np.searchsorted(omega, np.arange(n), side="right") - 1
    src = np.repeat(np.arange(n), np.diff(cp))
    ext = pid[src] != pid[ri]
    extin = np.bincount(ri[ext], minlength=n)
    light = extin <= heavy
    light_per_part = np.bincount(pid[light], weights=extin[light], minlength=omega.size - 1)
    c = extin[~light].astype(np.int64)
    full = (c - 1) // item                      # items of `item` links: 64 lanes each
    last = c - full * item                      # the last item of each row
    lanes = full * 64 + 2 ** np.ceil(np.log2(np.ceil(last / 8))).astype(np.int64)
    return light_per_part, int(np.ceil(lanes.sum() / 64))


def partitions_of(ctx, cp, ri, **opt):
    g = ditr.Graph(ctx, *upload(cp, ri), opts=ditr.opts_default(**opt))
    omega = np.asarray(g.partitions(), np.int64)
    g.close()
    return omega


@pytest.mark.parametrize("flags", [0, ditr.FLAG_NO_RESIDENT])
def test_more_item_units_than_waves(ctx, flags):
    """Nearly every row of a uniform random graph has more than four outside
    in-links, so the heavy items fill more one-wave work units than the
    resident grid has waves: each wave then sums several units per level."""
    n, pn = 300_000, 4700
    cp, ri = uniform_graph(n, 10, seed=5)
    omega = partitions_of(ctx, cp, ri, part_nodes=pn)
    K = omega.size - 1
    _, units = plan_counts(cp, ri, omega)
    assert units > 3 * K * 16  # 16 waves per 1024-thread workgroup
    b = np.full(n, 0.15 / n)
    ref = oracle.solve(cp, ri, b, rel_tol=1e-13)
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-10, mode=ditr.MODE_PARTITION, part_nodes=pn, flags=flags)
    check_parity(cp, ri, b, h, f, st, 1e-10, ref=ref)
    assert (st.launches <= st.rounds) if flags == 0 else (st.launches >= st.sweeps)


@pytest.mark.parametrize("flags", [0, ditr.FLAG_NO_RESIDENT])
def test_light_links_beyond_the_register_batch(ctx, flags):
    """Two partitions of 6000 nodes with ~2 light outside in-links per row:
    over 8192 light links per partition, more than the eight per thread the
    resident sweep gathers during its first local sweep; the rest take the
    plain loop after it."""
    n, pn = 12_000, 6000
    cp, ri = uniform_graph(n, 4, seed=8)
    omega = partitions_of(ctx, cp, ri, part_nodes=pn)
    light, _ = plan_counts(cp, ri, omega)
    assert omega.size - 1 == 2 and light.min() > 8 * 1024
    b = np.random.default_rng(3).uniform(0.1, 1.0, n) / n
    ref = oracle.solve(cp, ri, b, rel_tol=1e-14)
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-11, mode=ditr.MODE_PARTITION, part_nodes=pn, flags=flags)
    check_parity(cp, ri, b, h, f, st, 1e-11, ref=ref, ref_tol=1e-14)


def test_repeat_runs_within_parity(ctx, headline):
    """Runs may differ (float atomics); every run must stay within parity."""
    cp, ri, b, ref = headline
    hs = []
    for _ in range(3):
        h, f, st = gpu_solve(ctx, cp, ri, b, 1e-9)
        check_parity(cp, ri, b, h, f, st, 1e-9, ref=ref)
        hs.append(h)
    assert np.abs(hs[0] - hs[1]).sum() <= 2 * 1e-9 * b.sum() / (1 - D) * 1.01


@pytest.mark.parametrize("ptype", [ditr.PART_CB, ditr.PART_UNIFORM, ditr.PART_CB_INOUT])
@pytest.mark.parametrize("part_nodes,m", [(500, 1), (2000, 2), (6000, 8)])
def test_partition_mode_settings(ctx, ptype, part_nodes, m):
    spec = ditgen.GraphSpec(n=60_000, block=1000, seed=31)
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-10, mode=ditr.MODE_PARTITION, part_type=ptype,
                         part_nodes=part_nodes, sweeps_per_claim=m)
    check_parity(cp, ri, b, h, f, st, 1e-10)


def test_warm_start_parity(ctx):
    spec = ditgen.GraphSpec(n=50_000, block=1000, seed=17)
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    ref = oracle.solve(cp, ri, b, rel_tol=1e-13)
    h0 = ref.h * np.random.default_rng(1).uniform(0.7, 1.3, spec.n)  # signed F_0
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-10, h0=h0)
    check_parity(cp, ri, b, h, f, st, 1e-10, ref=ref)
    # resume: a finished H restarts with nothing to do
    h2, f2, st2 = gpu_solve(ctx, cp, ri, b, 1e-10, h0=h)
    assert st2.edges == 0 and np.array_equal(h2, h)


# ---------------------------------------------------------------------------
# partition plan and exact residual kernels

@pytest.mark.parametrize("K", [1, 2, 3, 4, 64, 256, 1000])
@pytest.mark.parametrize("ptype", [ditr.PART_CB, ditr.PART_UNIFORM, ditr.PART_CB_INOUT])
def test_partition_bit_exact(ctx, K, ptype):
    spec = ditgen.GraphSpec(n=100_000, block=1000, seed=2)
    cp, ri = ditgen.generate(spec)
    out = torch.empty(K + 1, dtype=torch.int64, device="cuda")
    cpt, rit = upload(cp, ri)
    ditr.partition(ctx, cpt, ptype, K, out, row_idx=rit)
    want = {ditr.PART_CB: lambda: oracle.partition_cb(cp, K),
            ditr.PART_UNIFORM: lambda: oracle.partition_uniform(spec.n, K),
            ditr.PART_CB_INOUT: lambda: oracle.partition_cb_inout(cp, ri, K)}[ptype]()
    assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("ptype", [ditr.PART_CB, ditr.PART_CB_INOUT, ditr.PART_UNIFORM])
def test_graph_plan_matches_oracle(ctx, ptype):
    spec = ditgen.GraphSpec(n=200_000, block=1000, seed=4)
    cp, ri = ditgen.generate(spec)
    g = ditr.Graph(ctx, *upload(cp, ri), opts=ditr.opts_default(part_type=ptype))
    ptr = g.partitions()
    K = len(ptr) - 1
    want = {ditr.PART_CB: lambda: oracle.partition_cb(cp, K),
            ditr.PART_UNIFORM: lambda: oracle.partition_uniform(spec.n, K),
            ditr.PART_CB_INOUT: lambda: oracle.partition_cb_inout(cp, ri, K)}[ptype]()
    assert np.array_equal(ptr, want)
    g.close()


def test_residual_matches_oracle(ctx):
    rng = np.random.default_rng(9)
    spec = ditgen.GraphSpec(n=30_000, block=1000, seed=9)
    cp, ri = ditgen.generate(spec)
    # add a heavy in-degree row to exercise the per-row workgroup path
    cp2, ri2 = csc_from_edges(spec.n, [(s, t) for s in range(spec.n)
                                       for t in ri[cp[s]:cp[s + 1]]] + [(s, 7) for s in range(0, spec.n, 10) if s != 7])
    for (c, r) in [(cp, ri), (cp2, ri2)]:
        b = rng.uniform(0, 1e-4, spec.n)
        h = rng.uniform(0, 1e-3, spec.n) * (rng.random(spec.n) < 0.9)
        g = ditr.Graph(ctx, *upload(c, r))
        dev = torch.device("cuda", 0)
        bt, ht = torch.from_numpy(b).to(dev), torch.from_numpy(h).to(dev)
        ft = torch.empty(spec.n, dtype=torch.float32, device=dev)
        r1 = ditr.residual(ctx, g, bt, ht, ft)
        want = oracle.fluid_from_history(c, r, b, h)
        got = ft.cpu().numpy().astype(np.float64)
        scale = np.abs(b) + np.abs(h) + np.abs(sparse_p(c, r)) @ np.abs(h)
        assert np.all(np.abs(got - want) <= 2.0 ** -24 * np.abs(want) + 1e-15 * scale)
        assert abs(r1 - np.abs(want).sum()) <= 1e-12 * scale.sum()
        g.close()


# ---------------------------------------------------------------------------
# errors and abort

def test_errors(ctx):
    dev = torch.device("cuda", 0)
    cp = torch.tensor([0, 1, 1], dtype=torch.int32, device=dev)
    bad = torch.tensor([5], dtype=torch.int32, device=dev)
    with pytest.raises(ditr.DitrError) as e:
        ditr.Graph(ctx, cp, bad)
    assert e.value.status == ditr.EGRAPH
    with pytest.raises(ditr.DitrError) as e:
        ditr.Graph(ctx, torch.tensor([0, 2, 1], dtype=torch.int32, device=dev),
                   torch.tensor([0, 1], dtype=torch.int32, device=dev))
    assert e.value.status == ditr.EGRAPH
    ok = torch.tensor([0], dtype=torch.int32, device=dev)
    with pytest.raises(ditr.DitrError) as e:
        ditr.Graph(ctx, cp, ok, damping=1.0)
    assert e.value.status == ditr.EINVAL
    g = ditr.Graph(ctx, cp, ok)
    b = torch.tensor([1.0, float("nan")], dtype=torch.float64, device=dev)
    h = torch.empty(2, dtype=torch.float64, device=dev)
    f = torch.empty(2, dtype=torch.float32, device=dev)
    with pytest.raises(ditr.DitrError) as e:
        ditr.solve(ctx, g, b, h, f)
    assert e.value.status == ditr.ENONFINITE
    b = torch.tensor([1.0, 2.0], dtype=torch.float64, device=dev)
    for bad_refresh in (-1e-7, float("nan")):
        with pytest.raises(ditr.DitrError) as e:
            ditr.solve(ctx, g, b, h, f, opts=ditr.opts_default(refresh_at=bad_refresh))
        assert e.value.status == ditr.EINVAL
    g.close()


def test_resident_wait_timeout_is_an_error(ctx, monkeypatch):
    """The resident sweep's waits are bounded: with a spin limit of zero every
    barrier or item wait that is not already satisfied times out at its first
    poll, the workgroups leave the kernel, the solve returns DITR_EHIP, and the
    next solve on the same context is unaffected."""
    spec = ditgen.SMALL
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    # 157 partitions of 64 nodes: the first workgroups at a barrier poll it
    # long before the last one arrives
    monkeypatch.setenv("DITR_SPIN_LIMIT", "0")
    with pytest.raises(ditr.DitrError) as e:
        gpu_solve(ctx, cp, ri, b, 1e-12, mode=ditr.MODE_PARTITION, part_nodes=64)
    assert e.value.status == ditr.EHIP and "timed out" in str(e.value)
    monkeypatch.delenv("DITR_SPIN_LIMIT")
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-12, mode=ditr.MODE_PARTITION, part_nodes=64)
    check_parity(cp, ri, b, h, f, st, 1e-12, ref_tol=1e-14)
    assert st.launches <= st.rounds  # resident again


def test_abort_keeps_identity(ctx, headline):
    cp, ri, b, ref = headline
    g = ditr.Graph(ctx, *upload(cp, ri))
    dev = torch.device("cuda", 0)
    bt = torch.from_numpy(b).to(dev)
    ht = torch.empty(len(b), dtype=torch.float64, device=dev)
    ft = torch.empty(len(b), dtype=torch.float32, device=dev)
    t = threading.Timer(0.0005, ctx.abort)
    t.start()
    st = ditr.solve(ctx, g, bt, ht, ft, rel_tol=1e-14, opts=ditr.opts_default(max_rounds=64))
    t.join()
    assert st.status in (ditr.OK, ditr.ABORTED, ditr.NOT_CONVERGED)
    h, f = ht.cpu().numpy(), ft.cpu().numpy().astype(np.float64)
    ident = b + sparse_p(cp, ri) @ h - h
    assert np.abs(f - ident).sum() <= 1e-7 * np.abs(ident).sum() + 1e-14 * np.abs(h).sum()
    g.close()


def test_warm_given_fluid_is_certified(ctx):
    """warm = 2 takes the caller's F_0 for the first stage only: with the right
    F_0 and with a wrong one (zeros), the result is certified on the exact
    residual of its H and keeps parity with the oracle."""
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=30_000, block=1000, seed=12))
    n = cp.size - 1
    b = ditgen.uniform_b(n)
    ref = oracle.solve(cp, ri, b, rel_tol=1e-13)
    dev = torch.device("cuda", 0)
    g = ditr.Graph(ctx, *upload(cp, ri))
    bt = torch.from_numpy(b).to(dev)
    h0 = ref.h * np.random.default_rng(3).uniform(0.7, 1.0, n)
    for given in ("exact", "zeros"):
        ht = torch.from_numpy(h0).to(dev)
        ft = torch.empty(n, dtype=torch.float32, device=dev)
        if given == "exact":
            ditr.residual(ctx, g, bt, ht, ft)
        else:
            ft.zero_()
        st = ditr.solve(ctx, g, bt, ht, ft, warm=2, rel_tol=1e-10, allow=(ditr.OK,))
        torch.cuda.synchronize()
        assert st.refreshes >= 1
        check_parity(cp, ri, b, ht.cpu().numpy(), ft.cpu().numpy().astype(np.float64), st, 1e-10, ref=ref)
    with pytest.raises(ValueError):
        ditr.solve(ctx, g, bt, ht, ft, warm=3)
    g.close()


def test_plain_launch_parity(ctx, monkeypatch):
    """DITR_PLAIN_LAUNCH dispatches the resident sweep with an ordinary launch
    (for profiler runs); the result must keep parity like the cooperative one."""
    monkeypatch.setenv("DITR_PLAIN_LAUNCH", "1")
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=50_000, block=1000, seed=13))
    b = ditgen.uniform_b(cp.size - 1)
    h, f, st = gpu_solve(ctx, cp, ri, b, 1e-10)
    assert st.launches == st.rounds  # one resident launch per stage
    check_parity(cp, ri, b, h, f, st, 1e-10)
