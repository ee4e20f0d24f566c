"""Write exact_small.json: exact rational solutions X of X = P X + B (equation
affine, Section 1) for small hand-made graphs, by Gauss-Jordan elimination over
the rationals. It uses the problem definition only (p_ji = d / #out_i per
out-link entry, Section 2.2); it calls neither the oracle nor the GPU library.

Run:  python tests/golden/make_exact_golden.py
"""
import json
import os
from fractions import Fraction

D = Fraction(85, 100)

# (name, n, out-links as (source, target) in CSC order, B as fractions)
CASES = [
    # self-loop on 0, repeated link 1->2, dangling node 4, link into the dangling node
    ("mixed6", 6, [(0, 0), (0, 1), (0, 3), (1, 2), (1, 2), (1, 5), (2, 0), (3, 4), (5, 1), (5, 4)],
     [Fraction(3, 20)] * 6),
    # chain 0->1->2->3 with uneven B
    ("chain4", 4, [(0, 1), (1, 2), (2, 3)],
     [Fraction(1, 10), Fraction(0), Fraction(1, 5), Fraction(1, 20)]),
    # two hubs pointing at each other and at three leaves
    ("hubs5", 5, [(0, 1), (0, 2), (0, 3), (0, 4), (1, 0), (1, 2), (2, 0), (3, 0), (4, 1)],
     [Fraction(3, 100)] * 5),
]


def exact_solution(n, edges, b):
    outdeg = [0] * n
    for s, _ in edges:
        outdeg[s] += 1
    # A = I - P
    a = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for s, t in edges:
        a[t][s] -= D / outdeg[s]
    x = list(b)
    for c in range(n):
        piv = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[piv] = a[piv], a[c]
        x[c], x[piv] = x[piv], x[c]
        inv = 1 / a[c][c]
        a[c] = [v * inv for v in a[c]]
        x[c] *= inv
        for r in range(n):
            if r != c and a[r][c] != 0:
                f = a[r][c]
                a[r] = [vr - f * vc for vr, vc in zip(a[r], a[c])]
                x[r] -= f * x[c]
    return x


def main():
    out = {"source": "exact rational solve of X = P X + B, d = 17/20 (equation affine, Section 1;"
                     " P of Section 2.2)", "cases": []}
    for name, n, edges, b in CASES:
        x = exact_solution(n, edges, b)
        out["cases"].append({"name": name, "n": n, "edges": edges,
                             "b": [str(v) for v in b], "x": [str(v) for v in x]})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_small.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
