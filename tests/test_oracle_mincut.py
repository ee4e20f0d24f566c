"""Pins of the oracle's cut-minimizing partition (CPU only).

The plan keeps the cost-balanced (CB) sets of Section 2.3 but slides each
boundary, inside a window and a balance slack, to where the least p mass of
short links crosses. The pins:
  * exhaustive search: every feasible plan of small graphs is enumerated, its
    crossing mass recomputed here link by link, and the oracle's plan must be
    the optimum (and, among optima, the one with the smallest last boundary,
    then the one before, and so on);
  * disjoint blocks: on a graph whose links never leave a block, the plan cuts
    nothing whenever block edges are reachable;
  * invariants on web-like graphs: the plan is feasible and never crosses more
    mass than the CB targets it starts from;
  * degenerate sizes: one set, one node per set, a graph without links.
"""
import itertools

import numpy as np
import pytest

import ditgen
import oracle
from conftest import csc_from_edges, random_graph


def reference_parts(cp, ri, K):
    """Targets, windows, limits and the crossing mass of every position,
    recomputed from the definition (plain loops over the links)."""
    n = cp.size - 1
    nnz = ri.size
    outd = np.diff(cp.astype(np.int64))
    indeg = np.bincount(ri, minlength=n).astype(np.int64)
    h = max(1, (3 * nnz) // n)
    cost = 1 + outd + np.minimum(indeg, h)
    C = np.concatenate([[0], np.cumsum(cost)])
    t = [0]
    for k in range(1, K):
        t.append(min(j for j in range(n + 1) if K * C[j] >= k * C[n]))
    t.append(n)
    cB = max(C[t[k + 1]] - C[t[k]] for k in range(K))
    sB = max(t[k + 1] - t[k] for k in range(K))
    cmax, smax = cB + cB // 10, sB + sB // 10
    mean = -(-n // K)
    span, W = 2 * mean, mean // 2
    cross = [0] * (n + 1)
    for i in range(n):
        for e in range(cp[i], cp[i + 1]):
            r = int(ri[e])
            if r == i or abs(r - i) >= span:
                continue
            u = int(np.floor(0.85 / float(outd[i]) * 4294967296.0))
            for b in range(n + 1):
                if min(i, r) < b <= max(i, r):
                    cross[b] += u
    wins = []
    for k in range(1, K):
        w = max(0, min(W, (t[k] - t[k - 1] - 1) // 2, (t[k + 1] - t[k] - 1) // 2))
        wins.append(range(t[k] - w, t[k] + w + 1))
    # positions inside a short tight cycle: every directed cycle of 2 or 3
    # distinct nodes, found from the adjacency sets, whose out-degrees multiply
    # to at most 2
    succ = [set(int(x) for x in ri[cp[i]:cp[i + 1]]) for i in range(n)]
    forbidden = set()
    for i in range(n):
        for j in succ[i]:
            if j == i:
                continue
            cyc = []
            if i in succ[j]:
                cyc.append((i, j))
            for k in succ[j]:
                if k not in (i, j) and i in succ[k]:
                    cyc.append((i, j, k))
            for c in cyc:
                if np.prod([outd[x] for x in c]) <= 2 and max(c) - min(c) < span:
                    forbidden.update(range(min(c) + 1, max(c) + 1))
    return dict(C=C, t=t, cmax=cmax, smax=smax, cross=cross, wins=wins, forbidden=forbidden)


def feasible(ptr, ref):
    C = ref["C"]
    return all(0 <= ptr[k + 1] - ptr[k] <= ref["smax"] and C[ptr[k + 1]] - C[ptr[k]] <= ref["cmax"]
               for k in range(len(ptr) - 1))


def brute_plan(cp, ri, K):
    """The optimum over every feasible plan; plans with no boundary inside a
    tight cycle first, all plans only when there is none such."""
    n = cp.size - 1
    ref = reference_parts(cp, ri, K)
    best = [None, None]
    for inner in itertools.product(*ref["wins"]):
        ptr = [0, *inner, n]
        if not feasible(ptr, ref):
            continue
        key = (sum(ref["cross"][b] for b in inner), tuple(reversed(inner)))
        clean = not any(b in ref["forbidden"] for b in inner)
        for slot in ((0, 1) if clean else (1,)):
            if best[slot] is None or key < best[slot][0]:
                best[slot] = (key, ptr)
    b = best[0] if best[0] is not None else best[1]
    return b[1], b[0][0], ref


def local_graph(n, rng, reach=4, p_out=0.5, dangling_frac=0.1):
    """Links mostly to nearby ids, with a few long ones and some self-loops and
    repeats: windows then hold positions of very different crossing mass."""
    edges = []
    for s in range(n):
        if rng.random() < dangling_frac:
            continue
        k = 1 + rng.integers(0, 4)
        for _ in range(k):
            if rng.random() < p_out:
                t = int(rng.integers(0, n))
            else:
                t = int(np.clip(s + rng.integers(-reach, reach + 1), 0, n - 1))
            edges.append((s, t))
    return csc_from_edges(n, edges)


@pytest.mark.parametrize("seed,n,K", [(0, 30, 2), (1, 30, 3), (2, 36, 3), (3, 40, 4), (4, 41, 4),
                                      (5, 25, 5), (6, 33, 3), (7, 44, 4)])
def test_mincut_is_the_exhaustive_optimum(seed, n, K):
    rng = np.random.default_rng(seed)
    cp, ri = local_graph(n, rng, p_out=0.25 if seed % 2 else 0.5)
    want, val, ref = brute_plan(cp, ri, K)
    got = oracle.partition_mincut(cp, ri, K)
    assert got.tolist() == want
    assert feasible(got.tolist(), ref)


def hub_graph(n, rng, hubs=(0, 1)):
    """A local graph plus two hubs that most nodes link to: their in-degree
    is far above the cap h of the inflow cost, which moves the CB targets."""
    cp, ri = local_graph(n, rng, p_out=0.2)
    edges = [(s, int(t)) for s in range(n) for t in ri[cp[s]:cp[s + 1]]]
    edges += [(s, hubs[s % len(hubs)]) for s in range(2, n) if rng.random() < 0.8]
    return csc_from_edges(n, edges)


@pytest.mark.parametrize("seed,K", [(0, 3), (1, 4), (2, 3)])
def test_mincut_optimum_with_hubs(seed, K):
    rng = np.random.default_rng(50 + seed)
    cp, ri = hub_graph(38, rng)
    ref = reference_parts(cp, ri, K)
    indeg = np.bincount(ri, minlength=38)
    assert indeg.max() > max(1, 3 * ri.size // 38)  # the cap binds
    want, _, _ = brute_plan(cp, ri, K)
    assert oracle.partition_mincut(cp, ri, K).tolist() == want


def mixed_case(seed):
    """A graph of random size and kind (local, hubs, or sparse local with many
    dangling nodes) and a random K, drawn from one seed."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(20, 46))
    K = int(rng.integers(2, 6))
    kind = seed % 3
    if kind == 0:
        cp, ri = local_graph(n, rng, p_out=float(rng.uniform(0.05, 0.6)))
    elif kind == 1:
        cp, ri = hub_graph(n, rng)
    else:
        cp, ri = local_graph(n, rng, reach=int(rng.integers(2, 12)), p_out=0.1, dangling_frac=0.4)
    return cp, ri, K


@pytest.mark.parametrize("seed", [1, 13, 17, 29, 30, 31, 32, 33])
def test_mincut_optimum_on_mixed_graphs(seed):
    cp, ri, K = mixed_case(seed)
    want, _, ref = brute_plan(cp, ri, K)
    got = oracle.partition_mincut(cp, ri, K).tolist()
    assert got == want and feasible(got, ref)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mincut_optimum_on_dense_random_graphs(seed):
    rng = np.random.default_rng(100 + seed)
    cp, ri = random_graph(28, rng, p_edge=0.15, self_loops=True, multi=True)
    want, _, _ = brute_plan(cp, ri, 3)
    assert oracle.partition_mincut(cp, ri, 3).tolist() == want


def test_mincut_ties_take_the_smallest_boundaries():
    # no links at all: every position crosses nothing, so every feasible plan
    # ties and the rule alone picks the plan
    n, K = 40, 4
    cp, ri = csc_from_edges(n, [])
    want, val, ref = brute_plan(cp, ri, K)
    assert val == 0
    got = oracle.partition_mincut(cp, ri, K).tolist()
    assert got == want
    # the last boundary is as small as the balance of the last set allows
    C = ref["C"]
    assert got[K - 1] == min(b for b in ref["wins"][K - 2]
                             if n - b <= ref["smax"] and C[n] - C[b] <= ref["cmax"])


def cycle_blocks(sizes):
    """Directed cycles over consecutive ids, one per block: every position
    inside a block is crossed by a link, a block edge by none."""
    edges, a = [], 0
    for s in sizes:
        for i in range(s):
            edges.append((a + i, a + (i + 1) % s))
            edges.append((a + i, a + (i + 2) % s))
        a += s
    return csc_from_edges(a, edges), np.cumsum([0] + list(sizes))


def planted_cycle(seed):
    """A sparse local graph with a 2-cycle (odd seeds) or a 3-cycle (even
    seeds) of out-degree-1 nodes planted around the first CB target."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(24, 40))
    K = int(rng.integers(2, 4))
    cp, ri = local_graph(n, rng, reach=3, p_out=0.15, dangling_frac=0.05)
    edges = [(s_, int(t)) for s_ in range(n) for t in ri[cp[s_]:cp[s_ + 1]]]
    m = n // K
    cyc = [m - 1, m + 1] if seed % 2 else [m - 2, m, m + 1]
    edges = [(s_, t) for (s_, t) in edges if s_ not in cyc]
    edges += list(zip(cyc, cyc[1:] + cyc[:1]))
    return csc_from_edges(n, edges), K


@pytest.mark.parametrize("seed", [23, 76, 103, 184])
def test_mincut_keeps_tight_cycles_whole(seed):
    # on these graphs the least crossing mass alone would split the cycle
    (cp, ri), K = planted_cycle(seed)
    n = cp.size - 1
    ref = reference_parts(cp, ri, K)
    got = oracle.partition_mincut(cp, ri, K).tolist()
    assert got == brute_plan(cp, ri, K)[0]
    assert ref["forbidden"] and not any(b in ref["forbidden"] for b in got[1:-1])
    plain = min(([0, *inner, n] for inner in itertools.product(*ref["wins"])
                 if feasible([0, *inner, n], ref)),
                key=lambda p: (sum(ref["cross"][b] for b in p[1:-1]), tuple(reversed(p[1:-1]))))
    assert plain != got and any(b in ref["forbidden"] for b in plain[1:-1])


@pytest.mark.parametrize("degrees,tight", [((1, 1), True), ((1, 2), True), ((2, 2), False),
                                           ((1, 1, 1), True), ((1, 1, 2), True), ((1, 2, 2), False)])
def test_tight_cycle_definition(degrees, tight):
    # a cycle over ids 10, 13 (, 16) of a 30-node graph; extra out-links of a
    # cycle node go to a far dangling node, so only the cycle's own degrees count
    ids = [10, 13, 16][:len(degrees)]
    edges = list(zip(ids, ids[1:] + ids[:1]))
    for x, dg in zip(ids, degrees):
        edges += [(x, 29)] * (dg - 1)
    cp, ri = csc_from_edges(30, edges)
    ref = reference_parts(cp, ri, 2)
    assert (ref["forbidden"] == set(range(11, ids[-1] + 1))) == tight
    assert (not ref["forbidden"]) == (not tight)


def test_mincut_cuts_nothing_between_disjoint_blocks():
    (cp, ri), edges = cycle_blocks([9, 11, 10, 12, 8, 10, 11, 9, 10, 10, 12, 8])
    n = cp.size - 1
    K = 6
    ptr = oracle.partition_mincut(cp, ri, K)
    ref = reference_parts(cp, ri, K)
    assert sum(ref["cross"][b] for b in ptr[1:-1]) == 0
    assert set(ptr.tolist()) <= set(edges.tolist())
    # the CB targets themselves sit inside blocks here
    assert any(t not in set(edges.tolist()) for t in ref["t"])
    assert feasible(ptr.tolist(), ref) and ptr[0] == 0 and ptr[-1] == n


def test_mincut_never_worse_than_its_cb_targets():
    cp, ri = ditgen.generate(ditgen.GraphSpec(n=6000, block=100, seed=4))
    n = cp.size - 1
    K = 16
    ptr = oracle.partition_mincut(cp, ri, K)
    # crossing mass of a position, counted from the link list with numpy
    src = np.repeat(np.arange(n), np.diff(cp))
    dst = ri.astype(np.int64)
    outd = np.diff(cp.astype(np.int64))
    u = np.floor(0.85 / outd[src] * 4294967296.0).astype(np.int64)
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    mean = -(-n // K)
    short = (lo != hi) & (hi - lo < 2 * mean)

    def mass(b):
        return int(u[short & (lo < b) & (b <= hi)].sum())

    indeg = np.bincount(ri, minlength=n)
    C = np.concatenate([[0], np.cumsum(1 + outd + np.minimum(indeg, max(1, 3 * ri.size // n)))])
    t = [0] + [int(np.searchsorted(C * K, k * C[n], side="left")) for k in range(1, K)] + [n]
    for k in range(1, K):  # first-j definition of the targets, checked directly
        assert K * C[t[k]] >= k * C[n] and (t[k] == 0 or K * C[t[k] - 1] < k * C[n])
    cut_plan = sum(mass(b) for b in ptr[1:-1])
    cut_cb = sum(mass(b) for b in t[1:-1])
    assert cut_plan <= cut_cb
    # the generator's links stay in blocks of 100 ids 80% of the time, so a
    # plan can put most boundaries on block edges and cross far less
    assert cut_plan < 0.5 * cut_cb
    cB = max(C[t[k + 1]] - C[t[k]] for k in range(K))
    sB = max(t[k + 1] - t[k] for k in range(K))
    sizes, costs = np.diff(ptr), np.diff(C[ptr])
    assert sizes.max() <= sB + sB // 10 and costs.max() <= cB + cB // 10 and sizes.min() >= 1


def test_mincut_degenerate_sizes():
    rng = np.random.default_rng(9)
    cp, ri = local_graph(20, rng)
    assert oracle.partition_mincut(cp, ri, 1).tolist() == [0, 20]
    # as many sets as nodes: the CB targets of unequal costs leave some sets
    # empty, and the windows are at most one position wide
    got = oracle.partition_mincut(cp, ri, 20).tolist()
    assert got == brute_plan(cp, ri, 20)[0]
    assert got[0] == 0 and got[-1] == 20 and all(a <= b for a, b in zip(got, got[1:]))
    with pytest.raises(ValueError):
        oracle.partition_mincut(cp, ri, 21)
    cp1, ri1 = csc_from_edges(1, [(0, 0)])
    assert oracle.partition_mincut(cp1, ri1, 1).tolist() == [0, 1]
