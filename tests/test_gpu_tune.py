"""GPU tests of the autotuner: search, cache reuse, keys, and that its
options keep parity with the oracle."""
import json

import numpy as np
import pytest

import ditgen
import oracle
from conftest import D

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
def problem(ctx):
    spec = ditgen.GraphSpec(n=100_000, block=1000, seed=11)
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    dev = torch.device("cuda", 0)
    t = dict(cp=torch.from_numpy(cp).to(dev), ri=torch.from_numpy(ri).to(dev),
             b=torch.from_numpy(b).to(dev), h=torch.empty(spec.n, dtype=torch.float64, device=dev),
             f=torch.empty(spec.n, dtype=torch.float32, device=dev))
    return cp, ri, b, t


def test_tune_search_cache_and_parity(ctx, problem, tmp_path):
    cp, ri, b, t = problem
    cache = str(tmp_path / "tune.json")
    o, info = ditr.tune(ctx, t["cp"], t["ri"], t["b"], t["h"], t["f"], rel_tol=1e-9, effort=1,
                        cache_path=cache)
    assert info.from_cache == 0 and info.candidates >= 15
    assert 0 < info.best_seconds <= info.default_seconds
    assert info.best_edges > 0 and info.default_edges > 0
    assert 1.2 <= o.alpha <= 3.0 and o.part_type in (ditr.PART_CB, ditr.PART_UNIFORM, ditr.PART_CB_INOUT,
                                                   ditr.PART_PMASS, ditr.PART_MINCUT)
    doc = json.load(open(cache))
    assert [e["key"] for e in doc["entries"]] == ["%016x" % info.key]

    # the second call reads the cache and times nothing
    o2, info2 = ditr.tune(ctx, t["cp"], t["ri"], t["b"], t["h"], t["f"], rel_tol=1e-9,
                          cache_path=cache)
    assert info2.from_cache == 1 and info2.candidates == 0 and info2.key == info.key
    assert o2.as_dict() == o.as_dict()

    # a solve with the tuned options keeps parity with the oracle
    g = ditr.Graph(ctx, t["cp"], t["ri"], opts=o)
    st = ditr.solve(ctx, g, t["b"], t["h"], t["f"], rel_tol=1e-9, opts=o, allow=(ditr.OK,))
    h = t["h"].cpu().numpy()
    g.close()
    ref = oracle.solve(cp, ri, b, rel_tol=1e-12)
    err = np.abs(h - ref.h).sum()
    assert st.resid_l1 <= 1e-9 * st.b_l1
    assert err <= (st.resid_l1 + ref.resid_l1) / (1 - D) * (1 + 1e-6)
    assert err <= 1e-6 * ref.h.sum()


def test_tune_key_tracks_the_problem(ctx, problem):
    cp, ri, b, t = problem
    k1 = ditr.tune_key(ctx, t["cp"], t["ri"], t["b"], 1e-9)
    assert k1 == ditr.tune_key(ctx, t["cp"], t["ri"], t["b"], 1e-9)
    assert k1 != ditr.tune_key(ctx, t["cp"], t["ri"], t["b"], 1e-8)
    assert k1 != ditr.tune_key(ctx, t["cp"], t["ri"], t["b"], 1e-9, damping=0.8)
    b2 = t["b"].clone()
    b2[17] *= 2
    assert k1 != ditr.tune_key(ctx, t["cp"], t["ri"], b2, 1e-9)
    ri2 = t["ri"].clone()
    # move one link to another target: same sizes, different graph
    ri2[5] = (ri2[5] + 1) % (t["cp"].numel() - 1)
    assert k1 != ditr.tune_key(ctx, t["cp"], ri2, t["b"], 1e-9)


def test_tune_quick_effort_without_cache(ctx, problem):
    cp, ri, b, t = problem
    o, info = ditr.tune(ctx, t["cp"], t["ri"], t["b"], t["h"], t["f"], rel_tol=1e-8, effort=0)
    assert info.from_cache == 0 and 5 <= info.candidates <= 16
    assert info.best_seconds <= info.default_seconds


def test_tune_rejects_bad_arguments(ctx, problem):
    cp, ri, b, t = problem
    for kw in (dict(effort=3), dict(rel_tol=0.0), dict(rel_tol=float("nan"))):
        args = dict(rel_tol=1e-9, effort=1)
        args.update(kw)
        with pytest.raises(ditr.DitrError) as e:
            ditr.tune(ctx, t["cp"], t["ri"], t["b"], t["h"], t["f"], **args)
        assert e.value.status == ditr.EINVAL
