"""GPU parity of the two Section 2.3 / 2.4 options against the oracle.

Equal internal p mass partition (Section 2.3, the alternative balance): the
device plan (ditr_partition_pmass and the DITR_PART_PMASS graph plan) must give
the oracle's boundaries bit for bit: both sides weigh links in the same integer
units, so the rule leaves no room for rounding differences.

Normalized priority test (Section 2.4, |F_i| / ((#in_i + 1)(#out_i + 1)) > T):
the node order changes, not the limit, so parity is the Section 2 bound against
the oracle, as for the plain test, in the resident and the per-level kernels.
"""
import numpy as np
import pytest

import ditgen
import oracle
from conftest import csc_from_edges, random_graph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1202_6168_amd import ditr  # noqa: E402
from test_gpu_solve import ADV, check_parity, gpu_solve, upload  # noqa: E402
from test_oracle_general import signed_weights  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ditr.Context(0)
    yield c
    c.close()


def _graphs():
    rng = np.random.default_rng(3)
    out = [("loops_multi", *random_graph(200, rng, 0.04, True, True), None)]
    cp, ri = random_graph(300, rng, 0.03, True, True)
    out.append(("signed", cp, ri, signed_weights(cp, rng, 0.9)))
    out.append(("web_1e4", *ditgen.generate(ditgen.GraphSpec(n=10_000, block=100, seed=1)), None))
    out.append(("web_5e4", *ditgen.generate(ditgen.GraphSpec(n=50_000, block=1000, seed=2)), None))
    out.append(("cycle", *csc_from_edges(1000, [(i, (i + 1) % 1000) for i in range(1000)]), None))
    out.append(("no_links", np.zeros(51, np.int32), np.zeros(0, np.int32), None))
    return out


GRAPHS = _graphs()


@pytest.mark.parametrize("case", GRAPHS, ids=[g[0] for g in GRAPHS])
@pytest.mark.parametrize("K", [1, 2, 7, 64, 256])
def test_pmass_partition_bit_exact(ctx, case, K):
    name, cp, ri, val = case
    n = cp.size - 1
    if K > n:
        pytest.skip("K > n")
    want = oracle.partition_pmass(cp, ri, K, val=val)
    cpt, rit = upload(cp, ri)
    vt = torch.from_numpy(val).cuda() if val is not None else None
    out = torch.empty(K + 1, dtype=torch.int64, device="cuda")
    ditr.partition_pmass(ctx, cpt, rit, K, out, val=vt)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want), (name, K)


def test_pmass_graph_plan_matches_oracle(ctx):
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=50_000, block=1000, seed=2))
    g = ditr.Graph(ctx, *upload(cp, ri), opts=ditr.opts_default(part_type=ditr.PART_PMASS))
    ptr = g.partitions()
    K = ptr.size - 1
    assert np.array_equal(ptr, oracle.partition_pmass(cp, ri, K))
    g.close()


def test_pmass_plan_solve_parity(ctx):
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=50_000, block=1000, seed=9))
    b = ditgen.uniform_b(cp.size - 1)
    tol = 1e-10
    for flags in (0, ditr.FLAG_NO_RESIDENT):
        h, f, st = gpu_solve(ctx, cp, ri, b, tol, part_type=ditr.PART_PMASS, flags=flags)
        check_parity(cp, ri, b, h, f, st, tol)


@pytest.mark.parametrize("case", ADV, ids=[c[0] for c in ADV])
@pytest.mark.parametrize("part_nodes,flags", [
    (0, 0), (3, 0), (64, 0), (3, ditr.FLAG_NO_RESIDENT), (64, ditr.FLAG_NO_RESIDENT)])
def test_priority_adversarial_parity(ctx, case, part_nodes, flags):
    name, cp, ri = case
    n = cp.size - 1
    b = np.random.default_rng(n).uniform(0.1, 1.0, n) / n
    tol = 1e-10
    h, f, st = gpu_solve(ctx, cp, ri, b, tol, mode=ditr.MODE_PARTITION, part_nodes=part_nodes,
                         flags=flags | ditr.FLAG_PRIORITY)
    check_parity(cp, ri, b, h, f, st, tol)


@pytest.mark.parametrize("n,block,seed,tol", [(10_000, 100, 1, 1e-12), (100_000, 1000, 4, 1e-10)])
def test_priority_web_graph_parity(ctx, n, block, seed, tol):
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=n, block=block, seed=seed))
    b = ditgen.uniform_b(n)
    ref = oracle.solve(cp, ri, b, rel_tol=1e-14, priority=True)
    for flags in (ditr.FLAG_PRIORITY, ditr.FLAG_PRIORITY | ditr.FLAG_NO_RESIDENT):
        h, f, st = gpu_solve(ctx, cp, ri, b, tol, flags=flags)
        check_parity(cp, ri, b, h, f, st, tol, ref=ref)


def test_priority_rejections(ctx):
    dev = torch.device("cuda", 0)
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=2_000, block=100, seed=3))
    g = ditr.Graph(ctx, *upload(cp, ri))
    b = torch.full((2000,), 0.15 / 2000, dtype=torch.float64, device=dev)
    h = torch.empty_like(b)
    f = torch.empty(2000, dtype=torch.float32, device=dev)
    for mode in (ditr.MODE_SWEEP, ditr.MODE_ASYNC):
        with pytest.raises(ditr.DitrError) as e:
            ditr.solve(ctx, g, b, h, f, opts=ditr.opts_default(mode=mode, flags=ditr.FLAG_PRIORITY))
        assert e.value.status == ditr.EINVAL
    out = torch.empty(3, dtype=torch.int64, device=dev)
    with pytest.raises(ditr.DitrError) as e:
        ditr.partition(ctx, g.col_ptr, ditr.PART_PMASS, 2, out, row_idx=g.row_idx)
    assert e.value.status == ditr.EINVAL
    g.close()
    # complete digraph on 700 nodes: sum (#in + 1)(#out + 1) = 700^3 > 2^28
    n = 700
    cp = (np.arange(n + 1) * (n - 1)).astype(np.int32)
    ri = np.array([t for s in range(n) for t in range(n) if t != s], np.int32)
    g = ditr.Graph(ctx, *upload(cp, ri))
    b = torch.full((n,), 0.15 / n, dtype=torch.float64, device=dev)
    h = torch.empty_like(b)
    f = torch.empty(n, dtype=torch.float32, device=dev)
    with pytest.raises(ditr.DitrError) as e:
        ditr.solve(ctx, g, b, h, f, opts=ditr.opts_default(flags=ditr.FLAG_PRIORITY))
    assert e.value.status == ditr.EINVAL and "2^28" in str(e.value)
    g.close()
