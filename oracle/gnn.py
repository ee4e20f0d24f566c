"""Oracle of the learned warm start: a plain FP64 numpy model.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module. The GPU library never
imports it and shares no code with it.

What is computed. A two-layer message-passing network predicts, per node,
y = log(N x_i / ||B||_1) of the solution x of X = P X + B (Section 1, equation
affine; P of Section 2.2: p_ji = d / #out_i on each out-link i -> j, dangling
columns zero). Its one graph operator is P itself, applied to node features:
(P Z)_j = sum over in-links i -> j of d / #out_i * Z_i. The prediction gives
a start H_0 for the D-iteration; the exact fluid of that start is
F_0 = B + P H_0 - H_0 (identity of equations defF and defH), and the iteration
then diffuses only F_0, so the bound ||X - H||_1 <= ||F||_1 / (1 - d)
(Section 2) judges the final error whatever the prediction was.

Model (hidden width 64, all FP64 here):
    features  X_i = [log1p(#in_i), log1p(#out_i), [#out_i = 0], 1, u_0..u_3]
              u_k = ((s >> 16k) & 0xffff) / 32768 - 1, s = SplitMix64 output
              for state i // block (a fixed code of the node's id block)
    layer 1   h1 = relu(X W1s + (P X) W1n + b1)
    layer 2   h2 = relu(h1 W2s + (P h1) W2n + b2)
    head      z = h2 w3 + b3,  yhat = log(softplus(z))
    loss      L = sum_i w_i (yhat_i - y_i)^2
The log link lets the network form y as the log of a positive combination of
aggregates: the solution is the series B + P B + P^2 B + ... (Section 1), whose
first terms two aggregation layers can carry linearly.
Training targets from a solved H: y_i = log(N H_i / ||B||_1), w_i = H_i / sum H
(the first-order weight of node i in the L1 error of the start, which is the
fluid the D-iteration then has to diffuse). Optimizer: Adam (Kingma and Ba,
2015, Algorithm 1).

Warm start: xhat = exp(yhat) ||B||_1 / N, H_0 = c xhat with c taken from
{0} and {0.50, 0.55, ..., 1.50} to minimize ||B + c (P - I) xhat||_1, the L1
fluid of the start (Section 2: the error bound and the remaining work are in
that norm); c = 0 is the cold start H_0 = 0, F_0 = B, so the start never holds
more fluid than B.

Flat parameter order (the C-ABI uses the same): W1s [8][64], W1n [8][64],
b1 [64], W2s [64][64], W2n [64][64], b2 [64], w3 [64], b3 [1]; matrices are
[input][output], row-major.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 8
HIDDEN = 64
MASK64 = (1 << 64) - 1

_SHAPES = [("W1s", (N_FEAT, HIDDEN)), ("W1n", (N_FEAT, HIDDEN)), ("b1", (HIDDEN,)),
           ("W2s", (HIDDEN, HIDDEN)), ("W2n", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
           ("w3", (HIDDEN,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in _SHAPES)


def unflatten(theta):
    """Flat vector -> dict of named FP64 arrays (copies)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAMS
    out, k = {}, 0
    for name, shape in _SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[k:k + size].reshape(shape).copy()
        k += size
    return out


def flatten(params):
    return np.concatenate([np.asarray(params[name], np.float64).ravel() for name, _ in _SHAPES])


def splitmix64(state: int) -> int:
    """One output of SplitMix64 (Steele, Lea and Flood, 2014) for a given state:
    add the golden-ratio increment, then the two xor-shift-multiply rounds."""
    z = (state + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def p_matrix(col_ptr, row_idx, d=0.85):
    """P as a scipy CSC matrix: entry (j, i) = d / #out_i per out-link i -> j."""
    import scipy.sparse as sp

    n = col_ptr.size - 1
    outdeg = np.diff(col_ptr.astype(np.int64))
    vals = np.repeat(np.where(outdeg > 0, d / np.maximum(outdeg, 1), 0.0), outdeg)
    return sp.csc_matrix((vals, row_idx.astype(np.int64), col_ptr.astype(np.int64)), shape=(n, n))


def features(col_ptr, row_idx, block):
    """Node features X [n, 8] (FP64)."""
    n = col_ptr.size - 1
    outdeg = np.diff(col_ptr.astype(np.int64))
    indeg = np.bincount(row_idx, minlength=n).astype(np.int64)
    X = np.zeros((n, N_FEAT))
    X[:, 0] = np.log1p(indeg)
    X[:, 1] = np.log1p(outdeg)
    X[:, 2] = (outdeg == 0)
    X[:, 3] = 1.0
    codes = {}
    for i in range(n):
        blk = i // block
        if blk not in codes:
            s = splitmix64(blk)
            codes[blk] = [((s >> (16 * k)) & 0xFFFF) / 32768.0 - 1.0 for k in range(4)]
        X[i, 4:8] = codes[blk]
    return X


def forward(params, X, P):
    """All intermediates of the forward pass."""
    AX = P @ X
    z1 = X @ params["W1s"] + AX @ params["W1n"] + params["b1"]
    h1 = np.maximum(z1, 0.0)
    A1 = P @ h1
    z2 = h1 @ params["W2s"] + A1 @ params["W2n"] + params["b2"]
    h2 = np.maximum(z2, 0.0)
    z = h2 @ params["w3"] + params["b3"][0]
    sp = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))  # softplus, overflow-free
    yhat = np.log(sp)
    return dict(AX=AX, z1=z1, h1=h1, A1=A1, z2=z2, h2=h2, z=z, sp=sp, yhat=yhat)


def loss(params, X, P, y, w):
    yhat = forward(params, X, P)["yhat"]
    return float(np.sum(w * (yhat - y) ** 2))


def loss_and_grad(params, X, P, y, w):
    """L and dL/dparams by the chain rule, layer by layer (reverse order)."""
    fw = forward(params, X, P)
    r = fw["yhat"] - y
    L = float(np.sum(w * r * r))
    dy = 2.0 * w * r                                   # dL/dyhat
    dz = dy / fw["sp"] / (1.0 + np.exp(-fw["z"]))      # d log softplus(z)/dz = sigmoid(z)/softplus(z)
    g = {"w3": fw["h2"].T @ dz, "b3": np.array([dz.sum()])}
    gz2 = np.outer(dz, params["w3"]) * (fw["z2"] > 0)  # through relu of layer 2
    g["W2s"] = fw["h1"].T @ gz2
    g["W2n"] = fw["A1"].T @ gz2
    g["b2"] = gz2.sum(axis=0)
    # h1 feeds layer 2 directly and through P: the adjoint of P carries the second path
    gh1 = gz2 @ params["W2s"].T + P.T @ (gz2 @ params["W2n"].T)
    gz1 = gh1 * (fw["z1"] > 0)
    g["W1s"] = X.T @ gz1
    g["W1n"] = fw["AX"].T @ gz1
    g["b1"] = gz1.sum(axis=0)
    return L, g


def targets(h, b_l1):
    """Training targets from a solved history H: y = log(N H / ||B||_1),
    w = H / sum H."""
    h = np.asarray(h, np.float64)
    n = h.size
    y = np.log(n * h / b_l1)
    w = h / h.sum()
    return y, w


SCALES = np.concatenate([[0.0], 0.5 + 0.05 * np.arange(21)])


def adam(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015, Algorithm 1); t counts from 1.
    Returns the new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def warm_start(yhat, P, b):
    """H_0 from a prediction: xhat = exp(yhat) ||B||_1 / N, H_0 = c xhat with c
    the first of SCALES that minimizes ||B + c (P - I) xhat||_1 (c = 0: cold
    start). Returns (H_0, F_0 = B + P H_0 - H_0, c, fell_back = (c == 0))."""
    n = b.size
    b1 = np.abs(b).sum()
    xhat = np.exp(yhat) * (b1 / n)
    r = P @ xhat - xhat
    l1 = [np.abs(b + c * r).sum() for c in SCALES]
    c = float(SCALES[int(np.argmin(l1))])
    if c == 0.0:
        return np.zeros(n), b.copy(), c, True
    h0 = c * xhat
    return h0, b + P @ h0 - h0, c, False
