"""Caller-owned workspaces: graph upload into a workspace, batched solves in
one, and the sizes ditr_workspace_bytes reports.

A graph uploaded with ditr_graph_upload_csc keeps every device table in the
caller's workspace; a batched solve given a workspace keeps its buffers there.
The results must be those of the allocating calls (parity with the oracle by
the Section 2 bound), and free device memory must not change across an upload,
a plain solve and a batched solve (hipMemGetInfo through torch).
"""
import numpy as np
import pytest

import ditgen
import oracle
from conftest import D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1202_6168_amd import ditr  # noqa: E402
from test_gpu_batched import check_columns  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ditr.Context(0)
    yield c
    c.close()


def _problem(n, seed, block=1000):
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=n, block=block, seed=seed))
    dev = torch.device("cuda", 0)
    return cp, ri, torch.from_numpy(cp).to(dev), torch.from_numpy(ri).to(dev)


@pytest.mark.parametrize("part_type,n", [(ditr.PART_CB_INOUT, 60_000), (ditr.PART_PMASS, 60_000),
                                         (ditr.PART_MINCUT, 60_000), (ditr.PART_MINCUT, 1_000_000)])
def test_upload_into_workspace_and_solve(ctx, part_type, n):
    # at 1e6 nodes the cut-minimizing plan's windows (~3900 positions) are the
    # widest its workspace bound has to cover
    cp, ri, cpt, rit = _problem(n, 41)
    n, nnz = cp.size - 1, ri.size
    opts = ditr.opts_default(part_type=part_type)
    nbytes = ditr.workspace_bytes(ctx, n, nnz, 0, opts)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.from_numpy(ditgen.uniform_b(n)).cuda()
    h = torch.empty(n, dtype=torch.float64, device="cuda")
    f = torch.empty(n, dtype=torch.float32, device="cuda")
    # an allocating upload and solve first, so that every kernel's code is
    # loaded before free memory is read
    g2 = ditr.Graph(ctx, cpt, rit, opts=opts)
    ditr.solve(ctx, g2, b, h, f, rel_tol=1e-10, allow=(ditr.OK,))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info(0)
    g = ditr.Graph(ctx, cpt, rit, opts=opts, workspace=ws)
    st = ditr.solve(ctx, g, b, h, f, rel_tol=1e-10, allow=(ditr.OK,))
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info(0)
    assert free1 == free0, (free0, free1)
    used = g.workspace_used()
    assert 0 < used <= nbytes
    # the same plan as the allocating upload
    assert np.array_equal(g.partitions(), g2.partitions())
    g2.close()
    ref = oracle.solve(cp, ri, ditgen.uniform_b(n), rel_tol=1e-13)
    H = h.cpu().numpy()
    assert np.abs(H - ref.h).sum() <= (st.resid_l1 + ref.resid_l1) / (1 - D) * (1 + 1e-6) + 1e-15
    g.close()
    # a workspace one byte short of what the graph used is refused
    small = torch.empty(used - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(ditr.DitrError) as e:
        ditr.Graph(ctx, cpt, rit, opts=opts, workspace=small)
    assert e.value.status == ditr.ENOMEM


def test_batched_in_workspace_allocates_nothing(ctx):
    cp, ri, cpt, rit = _problem(30_000, 42)
    n, nnz = cp.size - 1, ri.size
    ws = torch.empty(ditr.workspace_bytes(ctx, n, nnz, 0), dtype=torch.uint8, device="cuda")
    g = ditr.Graph(ctx, cpt, rit, workspace=ws)
    R = 16
    sets = ditgen.ppr_seed_sets(n, R, seed=7)
    B = torch.from_numpy(ditgen.ppr_rhs_dense(n, sets)).cuda()
    H = torch.empty_like(B)
    F = torch.empty((n, R), dtype=torch.float32, device="cuda")
    bws = torch.empty(ditr.workspace_bytes(ctx, n, nnz, R), dtype=torch.uint8, device="cuda")
    ditr.solve_batched(ctx, g, B, H, F, rel_tol=1e-8, workspace=bws, allow=(ditr.OK,))  # first call
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info(0)
    tot, per = ditr.solve_batched(ctx, g, B, H, F, rel_tol=1e-8, workspace=bws, allow=(ditr.OK,))
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info(0)
    assert free1 == free0, (free0, free1)
    check_columns(cp, ri, B.cpu().numpy(), H.cpu().numpy(), F.cpu().numpy(), per, 1e-8, [0, 5, 15])
    with pytest.raises(ditr.DitrError) as e:
        ditr.solve_batched(ctx, g, B, H, F, workspace=bws[:1024])
    assert e.value.status == ditr.EINVAL
    g.close()


def test_workspace_bytes_arguments(ctx):
    assert ditr.workspace_bytes(ctx, 1000, 8000, 0) > 0
    assert ditr.workspace_bytes(ctx, 1000, 8000, 256) > ditr.workspace_bytes(ctx, 1000, 8000, 4)
    for bad in (3, 260, 6):
        with pytest.raises(ditr.DitrError):
            ditr.workspace_bytes(ctx, 1000, 8000, bad)
