"""Pins of the warm-start network oracle (oracle/gnn.py), CPU only.

- SplitMix64 against its published first outputs from state 0;
- features against brute-force counts over an edge list;
- the graph operator against the D-iteration: the solved X satisfies
  P X = X - B (Section 1, equation affine), with X from the separately pinned
  D-iteration oracle;
- every gradient component against central finite differences (FP64);
- planted mistakes in the backward pass, each caught by that check;
- Adam against torch.optim.Adam;
- the warm start: the scale minimizes ||B + c (P - I) xhat||_1 over its grid,
  an exact prediction leaves (almost) no fluid, a bad one falls back to
  H_0 = 0.
"""
import inspect
import textwrap

import numpy as np
import pytest

import oracle
from oracle import gnn
from conftest import csc_from_edges

D = 0.85


def small_graph(n=40, seed=3):
    rng = np.random.default_rng(seed)
    edges = []
    for s in range(n):
        if s % 7 == 3:
            continue  # dangling
        k = int(rng.integers(1, 6))
        for _ in range(k):
            edges.append((s, int(rng.integers(0, n))))  # self-loops and repeats allowed
    edges.append((0, 0))
    return csc_from_edges(n, edges)


def random_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return gnn.unflatten(rng.normal(0, scale, gnn.N_PARAMS))


def test_splitmix64_published_outputs():
    # first three outputs of SplitMix64 seeded with 0 (state advances by the increment)
    gold = 0x9E3779B97F4A7C15
    outs = [gnn.splitmix64((k * gold) & gnn.MASK64) for k in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_features_brute_force():
    n, block = 23, 5
    edges = [(0, 1), (0, 2), (0, 2), (1, 1), (3, 0), (4, 22), (22, 0), (10, 11)]
    cp, ri = csc_from_edges(n, edges)
    X = gnn.features(cp, ri, block)
    for i in range(n):
        nin = sum(1 for s, t in edges if t == i)
        nout = sum(1 for s, t in edges if s == i)
        assert X[i, 0] == np.log1p(nin) and X[i, 1] == np.log1p(nout)
        assert X[i, 2] == (1.0 if nout == 0 else 0.0) and X[i, 3] == 1.0
        assert np.all(X[i, 4:] == X[(i // block) * block, 4:])
        assert np.all((X[i, 4:] >= -1) & (X[i, 4:] < 1))
    # different blocks get different codes
    codes = {tuple(X[b * block, 4:]) for b in range(5)}
    assert len(codes) == 5
    s = gnn.splitmix64(2)
    assert X[12, 4] == (s & 0xFFFF) / 32768.0 - 1 and X[12, 7] == (s >> 48) / 32768.0 - 1


def test_operator_against_the_solved_iteration():
    cp, ri = small_graph(60, seed=9)
    b = np.full(60, 0.15 / 60)
    ref = oracle.solve(cp, ri, b, rel_tol=1e-15)
    P = gnn.p_matrix(cp, ri, D)
    # X solves X = P X + B; H is within ||F||_1/(1-d) of X
    err = np.abs(P @ ref.h - (ref.h - b)).sum()
    assert err <= (1 + D) * ref.resid_l1 / (1 - D) + 1e-15
    # and P is not its transpose here (the check above would fail for P.T)
    assert np.abs(P.T @ ref.h - (ref.h - b)).sum() > 1e3 * (err + 1e-16)


def fd_check(loss_and_grad, params, X, P, y, w, h=1e-6, tol=1e-6):
    """Max over all parameters of |analytic - central difference| / max |grad|."""
    _, g = loss_and_grad(params, X, P, y, w)
    theta = gnn.flatten(params)
    ga = gnn.flatten(g)
    fd = np.empty_like(theta)
    for k in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (gnn.loss(gnn.unflatten(tp), X, P, y, w) -
                 gnn.loss(gnn.unflatten(tm), X, P, y, w)) / (2 * h)
    return np.abs(ga - fd).max() / np.abs(fd).max()


@pytest.fixture(scope="module")
def fd_case():
    cp, ri = small_graph(40, seed=3)
    X = gnn.features(cp, ri, block=8)
    P = gnn.p_matrix(cp, ri, D)
    rng = np.random.default_rng(5)
    y = rng.normal(0, 1, 40)
    w = rng.random(40)
    w /= w.sum()
    # a seed whose pre-activations keep away from the relu kink by far more than
    # the difference step moves them
    for seed in range(100):
        params = random_params(seed)
        fw = gnn.forward(params, X, P)
        if min(np.abs(fw["z1"]).min(), np.abs(fw["z2"]).min()) > 1e-3:
            break
    else:
        pytest.fail("no parameter seed away from the relu kink")
    return params, X, P, y, w


@pytest.mark.slow
def test_gradient_matches_central_differences(fd_case):
    params, X, P, y, w = fd_case
    fw = gnn.forward(params, X, P)
    # both relu regimes are exercised
    for z in (fw["z1"], fw["z2"]):
        assert 0.2 < (z > 0).mean() < 0.8
    assert fd_check(gnn.loss_and_grad, params, X, P, y, w) <= 1e-6


MUTANTS = {
    "forward_operator_in_backward": ("P.T @ (gz2 @ params[\"W2n\"].T)", "P @ (gz2 @ params[\"W2n\"].T)"),
    "no_relu_mask_layer1": ("gz1 = gh1 * (fw[\"z1\"] > 0)", "gz1 = gh1"),
    "self_input_for_neighbour_weights": ("g[\"W1n\"] = fw[\"AX\"].T @ gz1", "g[\"W1n\"] = X.T @ gz1"),
    "dropped_bias_gradient": ("g[\"b2\"] = gz2.sum(axis=0)", "g[\"b2\"] = 0 * gz2.sum(axis=0)"),
    "missing_factor_two": ("dy = 2.0 * w * r", "dy = w * r"),
    "transposed_layer2_weights": ("gz2 @ params[\"W2s\"].T", "gz2 @ params[\"W2s\"]"),
    "link_derivative_without_sigmoid": ("dz = dy / fw[\"sp\"] / (1.0 + np.exp(-fw[\"z\"]))",
                                        "dz = dy / fw[\"sp\"]"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_backward_mistakes_are_caught(fd_case, name):
    old, new = MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(gnn.loss_and_grad))
    assert src.count(old) == 1, name
    ns = dict(vars(gnn))
    exec(src.replace(old, new), ns)
    params, X, P, y, w = fd_case
    assert fd_check(ns["loss_and_grad"], params, X, P, y, w) > 1e-3


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    theta = rng.normal(size=50)
    p = torch.nn.Parameter(torch.from_numpy(theta.copy()))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 6):
        g = rng.normal(size=50) * 10 ** rng.uniform(-6, 1)
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        theta, m, v = gnn.adam(theta, g, m, v, t, 3e-3)
        assert np.allclose(theta, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_flat_layout():
    assert gnn.N_PARAMS == 9409
    theta = np.arange(gnn.N_PARAMS, dtype=np.float64)
    p = gnn.unflatten(theta)
    assert p["W1s"][1, 0] == 64 and p["W1n"][0, 0] == 512 and p["b1"][0] == 1024
    assert p["W2s"][0, 1] == 1089 and p["W2n"][0, 0] == 5184 and p["b2"][0] == 9280
    assert p["w3"][0] == 9344 and p["b3"][0] == 9408
    assert np.array_equal(gnn.flatten(p), theta)


def test_targets_invert_to_h():
    h = np.array([0.2, 0.5, 1.0, 3.0]) * 0.15 / 4
    y, w = gnn.targets(h, b_l1=0.15)
    assert np.allclose(np.exp(y) * 0.15 / 4, h, rtol=1e-15) and np.isclose(w.sum(), 1.0)
    # scaling B scales H: the target of a scaled solve is unchanged
    y2, _ = gnn.targets(3 * h, b_l1=0.45)
    assert np.allclose(y, y2, rtol=0, atol=1e-15)


def test_head_link_values():
    # yhat = log(softplus(z)): a large z gives log z, a very negative z gives z
    p = gnn.unflatten(np.zeros(gnn.N_PARAMS))
    X = np.zeros((3, 8))
    P = gnn.p_matrix(np.array([0, 0, 0, 0]), np.array([], dtype=np.int32))
    for b3, want in ((0.0, np.log(np.log(2.0))), (50.0, np.log(50.0)), (-40.0, -40.0)):
        p["b3"][0] = b3
        assert np.allclose(gnn.forward(p, X, P)["yhat"], want, rtol=1e-12, atol=1e-12)


def test_warm_start_scale_and_fallback():
    cp, ri = small_graph(60, seed=9)
    n = 60
    b = np.full(n, 0.15 / n)
    P = gnn.p_matrix(cp, ri, D)
    ref = oracle.solve(cp, ri, b, rel_tol=1e-15)
    # exact prediction: c = 1 and no fluid left beyond the oracle's own residual
    y, _ = gnn.targets(ref.h, 0.15)
    h0, f0, c, fb = gnn.warm_start(y, P, b)
    assert not fb and c == 1.0 and np.abs(f0).sum() <= 1e-9 * 0.15
    # a prediction 25% too large is scaled back by the grid point 0.8
    h0, f0, c, fb = gnn.warm_start(y + np.log(1.25), P, b)
    assert not fb and c == 0.8 and np.abs(f0).sum() <= 1e-9 * 0.15
    # the chosen scale minimizes the L1 fluid over the grid, never above ||B||_1
    rng = np.random.default_rng(2)
    y_noisy = y + rng.normal(0, 0.3, n)
    h0, f0, c, fb = gnn.warm_start(y_noisy, P, b)
    xhat = np.exp(y_noisy) * 0.15 / n
    r = P @ xhat - xhat
    best = min(np.abs(b + s * r).sum() for s in gnn.SCALES)
    assert np.isclose(np.abs(f0).sum(), best, rtol=1e-12)
    assert np.abs(f0).sum() <= np.abs(b).sum()
    assert np.allclose(f0, b + P @ h0 - h0, rtol=0, atol=1e-15)
    # a personalized B (one seed node) with an unrelated prediction: every
    # scale leaves more L1 fluid than B itself, so the start falls back to cold
    b1 = np.zeros(n)
    b1[7] = 0.15
    h0, f0, c, fb = gnn.warm_start(rng.normal(0, 3, n), P, b1)
    assert fb and c == 0.0 and np.all(h0 == 0) and np.array_equal(f0, b1)
