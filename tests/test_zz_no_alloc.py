"""The allocation-free solve (ditr_solve_noalloc) against ditr_solve.

ditr_solve_noalloc runs the same partitioned sweep with its per-solve buffers
in the library's static device scratch. Both results are valid D-iteration
runs of the same problem, so each satisfies ||X - H||_1 <= ||F||_1 / (1 - d)
(Section 2, the bound after defH); the two H must therefore agree within the
sum of their bounds, and each must meet the 1e-6 relative L1 bar against the
FP64 oracle. Two calls in a row, the second on a smaller graph, check that
what the first call left in the shared scratch does not leak into the second.
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


def _problem(ctx, n, seed):
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=n, block=1000, seed=seed))
    dev = torch.device("cuda", 0)
    keep = (torch.from_numpy(cp).to(dev), torch.from_numpy(ri).to(dev))
    g = ditr.Graph(ctx, *keep)
    b = ditgen.uniform_b(n)
    return cp, ri, b, keep, g


def _check_identity(cp, ri, b, h, f):
    ident = b + sparse_p(cp, ri) @ h - h
    scale = np.abs(b).sum() + np.abs(h).sum()
    assert np.abs(f - ident).sum() <= 1e-7 * np.abs(ident).sum() + 1e-14 * scale


def test_noalloc_matches_solve_twice_second_smaller(ctx):
    dev = torch.device("cuda", 0)
    tol = 1e-10
    for n, seed in [(60_000, 31), (20_000, 32)]:
        print("noalloc case n=%d seed=%d" % (n, seed), flush=True)
        cp, ri, b, keep, g = _problem(ctx, n, seed)
        bt = torch.from_numpy(b).to(dev)
        h1 = torch.empty(n, dtype=torch.float64, device=dev)
        f1 = torch.empty(n, dtype=torch.float32, device=dev)
        h2 = torch.empty_like(h1)
        f2 = torch.empty_like(f1)
        st1 = ditr.solve(ctx, g, bt, h1, f1, rel_tol=tol, allow=(ditr.OK,))
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info(0)
        st2 = ditr.solve_noalloc(ctx, g, bt, h2, f2, rel_tol=tol, allow=(ditr.OK,))
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info(0)
        assert free1 == free0, (free0, free1)
        assert st2.status == ditr.OK and st2.resid_l1 <= tol * st2.b_l1 * (1 + 1e-12)
        H1, H2 = h1.cpu().numpy(), h2.cpu().numpy()
        F2 = f2.cpu().numpy().astype(np.float64)
        # the two valid runs agree within the sum of their Section 2 bounds
        assert np.abs(H1 - H2).sum() <= (st1.resid_l1 + st2.resid_l1) / (1 - D) * (1 + 1e-6)
        ref = oracle.solve(cp, ri, b, rel_tol=1e-13)
        err = np.abs(H2 - ref.h).sum()
        assert err <= (st2.resid_l1 + ref.resid_l1) / (1 - D) * (1 + 1e-6) + 1e-15
        assert err <= 1e-6 * np.abs(ref.h).sum()
        _check_identity(cp, ri, b, H2, F2)
        assert abs(np.abs(F2).sum() - st2.resid_l1) <= 1e-6 * st2.resid_l1 + 1e-15
        g.close()


def test_noalloc_warm_resume(ctx):
    # resume from the H of a loose solve (warm start, F_0 = B + P H_0 - H_0)
    dev = torch.device("cuda", 0)
    n = 30_000
    cp, ri, b, keep, g = _problem(ctx, n, 33)
    bt = torch.from_numpy(b).to(dev)
    h = torch.empty(n, dtype=torch.float64, device=dev)
    f = torch.empty(n, dtype=torch.float32, device=dev)
    ditr.solve_noalloc(ctx, g, bt, h, f, rel_tol=1e-4, allow=(ditr.OK,))
    st = ditr.solve_noalloc(ctx, g, bt, h, f, warm=True, rel_tol=1e-11, allow=(ditr.OK,))
    torch.cuda.synchronize()
    ref = oracle.solve(cp, ri, b, rel_tol=1e-13)
    H = h.cpu().numpy()
    assert np.abs(H - ref.h).sum() <= (st.resid_l1 + ref.resid_l1) / (1 - D) * (1 + 1e-6) + 1e-15
    g.close()


def test_noalloc_rejects_what_it_cannot_serve(ctx):
    dev = torch.device("cuda", 0)
    n = 5_000
    cp, ri, b, keep, g = _problem(ctx, n, 34)
    bt = torch.from_numpy(b).to(dev)
    h = torch.empty(n, dtype=torch.float64, device=dev)
    f = torch.empty(n, dtype=torch.float32, device=dev)
    for o in (ditr.opts_default(mode=ditr.MODE_SWEEP), ditr.opts_default(mode=ditr.MODE_ASYNC),
              ditr.opts_default(flags=ditr.FLAG_TIME_KERNELS)):
        with pytest.raises(ditr.DitrError) as e:
            ditr.solve_noalloc(ctx, g, bt, h, f, rel_tol=1e-9, opts=o)
        assert e.value.status == ditr.EINVAL
    g.close()
    # a graph whose solve buffers exceed the static scratch is refused
    cap = ditr.noalloc_scratch_bytes()
    big = cap // 16 + 100_000
    print("noalloc oversize case n=%d (scratch %d bytes)" % (big, cap), flush=True)
    cp, ri, b, keep, g = _problem(ctx, big, 35)
    bt = torch.from_numpy(b).to(dev)
    h = torch.empty(big, dtype=torch.float64, device=dev)
    f = torch.empty(big, dtype=torch.float32, device=dev)
    with pytest.raises(ditr.DitrError) as e:
        ditr.solve_noalloc(ctx, g, bt, h, f, rel_tol=1e-9)
    assert e.value.status == ditr.EINVAL and "static scratch" in str(e.value)
    g.close()
