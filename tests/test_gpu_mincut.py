"""GPU parity of the cut-minimizing partition (DITR_PART_MINCUT).

The device plan (ditr_partition with DITR_PART_MINCUT and the graph plan of
that type) must give the oracle's boundaries bit for bit: costs, crossing
masses and the dynamic programme are integer arithmetic on both sides, and
both break ties the same way. A solve on such a plan keeps oracle parity (the
Section 2 bound), in the resident and the per-level kernels.
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
from test_oracle_mincut import hub_graph, local_graph, mixed_case, planted_cycle  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ditr.Context(0)
    yield c
    c.close()


def _graphs():
    rng = np.random.default_rng(7)
    out = [("loops_multi", *random_graph(200, rng, 0.04, True, True))]
    out.append(("local_44", *local_graph(44, np.random.default_rng(3))))
    out.append(("hubs_38", *hub_graph(38, np.random.default_rng(51))))
    cp, ri, _ = mixed_case(17)
    out.append(("mixed_17", cp, ri))
    for seed in (23, 76):
        (pcp, pri), _ = planted_cycle(seed)
        out.append(("tight_%d" % seed, pcp, pri))
    out.append(("web_1e4", *ditgen.generate(ditgen.GraphSpec(n=10_000, block=100, seed=1))))
    out.append(("web_5e4", *ditgen.generate(ditgen.GraphSpec(n=50_000, block=1000, seed=2))))
    out.append(("web_2e5_ragged", *ditgen.generate(ditgen.GraphSpec(n=200_003, block=700, seed=6))))
    out.append(("cycle", *csc_from_edges(1000, [(i, (i + 1) % 1000) for i in range(1000)])))
    out.append(("no_links", np.zeros(51, np.int32), np.zeros(0, np.int32)))
    return out


GRAPHS = _graphs()


@pytest.mark.parametrize("case", GRAPHS, ids=[g[0] for g in GRAPHS])
@pytest.mark.parametrize("K", [1, 2, 3, 5, 64, 256])
def test_mincut_partition_bit_exact(ctx, case, K):
    name, cp, ri = case
    n = cp.size - 1
    if K > n:
        pytest.skip("K > n")
    want = oracle.partition_mincut(cp, ri, K)
    cpt, rit = upload(cp, ri)
    out = torch.empty(K + 1, dtype=torch.int64, device="cuda")
    ditr.partition(ctx, cpt, ditr.PART_MINCUT, K, out, row_idx=rit)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want), (name, K)


def test_mincut_one_node_per_set(ctx):
    cp, ri = local_graph(40, np.random.default_rng(9))
    cpt, rit = upload(cp, ri)
    out = torch.empty(41, dtype=torch.int64, device="cuda")
    ditr.partition(ctx, cpt, ditr.PART_MINCUT, 40, out, row_idx=rit)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.partition_mincut(cp, ri, 40))


def test_mincut_headline_plan_bit_exact(ctx):
    # the benchmark's graph and partition count (the oracle takes ~10 s here)
    cp, ri = ditgen.generate(ditgen.HEADLINE)
    g = ditr.Graph(ctx, *upload(cp, ri), opts=ditr.opts_default(part_type=ditr.PART_MINCUT))
    ptr = g.partitions()
    K = ptr.size - 1
    assert K == 256
    assert np.array_equal(ptr, oracle.partition_mincut(cp, ri, K))
    g.close()


def test_mincut_plan_solve_parity(ctx):
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=100_000, block=1000, seed=9))
    b = ditgen.uniform_b(cp.size - 1)
    tol = 1e-10
    ref = oracle.solve(cp, ri, b, rel_tol=1e-13)
    for flags in (0, ditr.FLAG_NO_RESIDENT):
        h, f, st = gpu_solve(ctx, cp, ri, b, tol, part_type=ditr.PART_MINCUT, flags=flags)
        check_parity(cp, ri, b, h, f, st, tol, ref=ref)


@pytest.mark.parametrize("case", ADV, ids=[c[0] for c in ADV])
@pytest.mark.parametrize("part_nodes,flags", [(0, 0), (3, 0), (3, ditr.FLAG_NO_RESIDENT)])
def test_mincut_adversarial_parity(ctx, case, part_nodes, flags):
    name, cp, ri = case
    n = cp.size - 1
    b = np.random.default_rng(n + 1).uniform(0.1, 1.0, n) / n
    tol = 1e-10
    h, f, st = gpu_solve(ctx, cp, ri, b, tol, mode=ditr.MODE_PARTITION, part_nodes=part_nodes,
                         part_type=ditr.PART_MINCUT, flags=flags)
    check_parity(cp, ri, b, h, f, st, tol)


def test_mincut_rejections(ctx):
    cp, ri = local_graph(30, np.random.default_rng(2))
    cpt, rit = upload(cp, ri)
    out = torch.empty(32, dtype=torch.int64, device="cuda")
    for K in (0, 31):
        with pytest.raises(ditr.DitrError) as e:
            ditr.partition(ctx, cpt, ditr.PART_MINCUT, K, out, row_idx=rit)
        assert e.value.status == ditr.EINVAL
