"""Write tests/golden/tiny_grid.json: a two-sub-grid, three-flavour grid written
out in full, query points covering every region of the method (inside,
x below the grid, Q^2 below and above it, the corners, the knots, the flavour
threshold, invalid points) and the FP64 oracle's values there.

The stored values come from oracle/ only (the plain FP64 CPU implementation of
the paper's section 2.2 interpolation and extrapolation and of section 2.3
alpha_s); the file is a regression fixture for the oracle and a fixed parity
target for the GPU path.  Run from the repository root:
    python3 tests/golden/make_golden.py
"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_grid.json")


def grid():
    xk = [1e-5, 1e-4, 1e-3, 1e-2, 0.1, 0.3, 0.6, 1.0]
    q_lo = [1.0, 1.4, 2.0, 2.89]              # Q^2 knots of sub-grid 0, threshold at 2.89
    q_hi = [2.89, 5.0, 12.0, 40.0, 150.0]     # sub-grid 1 repeats the threshold knot
    pids = [21, 2, 4]                         # gluon, up, charm (zero below the threshold)
    vals = []
    for k, qk in enumerate((q_lo, q_hi)):
        v = np.zeros((len(xk), len(qk), 3))
        for i, x in enumerate(xk):
            for j, q in enumerate(qk):
                L = math.log(q / 2.0)
                v[i, j, 0] = x ** -0.2 * (1 - x) ** 4 * (1 + 0.08 * L)
                v[i, j, 1] = x ** 0.5 * (1 - x) ** 3 * (1 + 2 * x) * (1 - 0.03 * L)
                v[i, j, 2] = 0.0 if k == 0 else 0.1 * x ** -0.1 * (1 - x) ** 5 * math.log(q / 2.89)
        vals.append(v)
    return [np.array(xk), np.array(xk)], [np.array(q_lo), np.array(q_hi)], vals, pids


def points():
    xs = [3e-6, 1e-5, 5e-5, 1e-4, 3.3e-3, 0.05, 0.3, 0.45, 0.95, 1.0]
    qs = [0.5, 1.0, 1.2, 2.0, 2.89, np.nextafter(2.89, 0.0), 3.5, 40.0, 150.0, 400.0]
    x = [a for a in xs for _ in qs] + [0.0, -1.0, 1.5, 0.5, 0.5]
    q2 = [b for _ in xs for b in qs] + [10.0, 10.0, 10.0, 0.0, -2.0]
    return np.array(x), np.array(q2)


def main():
    xk, qk, vals, pids = grid()
    g = oracle.Grid(xk, qk, vals, pids)
    x, q2 = points()
    xf, scale = oracle.xfxq2(g, pids, x, q2, with_scale=True)
    aq = np.array([1.0, 1.4, 2.0, 2.89, 2.89, 5.0, 12.0, 40.0, 150.0])
    av = np.array([0.30, 0.27, 0.25, 0.23, 0.231, 0.20, 0.175, 0.15, 0.13])
    al = oracle.alphas_q2(aq, av, q2)
    doc = {
        "about": "oracle/ values (plain FP64 CPU interpolation, paper sections 2.2-2.3) on a tiny grid; "
                 "written by tests/golden/make_golden.py",
        "pids": pids,
        "xknots": [list(map(float, a)) for a in xk],
        "q2knots": [list(map(float, a)) for a in qk],
        "values": [v.tolist() for v in vals],
        "alphas_q2knots": aq.tolist(), "alphas_values": av.tolist(),
        "x": [repr(float(a)) for a in x], "q2": [repr(float(a)) for a in q2],
        "xf": [[repr(float(v)) for v in row] for row in xf],
        "xf_scale": [[repr(float(v)) for v in row] for row in scale],
        "alphas": [repr(float(v)) for v in al],
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
