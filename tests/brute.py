"""Brute-force reference for tiny grids, written independently of the oracle.

Different route to the same readings of the paper's section 2.2 / 2.3 (log-
bicubic interpolation with finite-difference slopes, x then Q^2, sub-grids
evaluated independently, extrapolation outside the grid):
  * knot search with numpy.searchsorted (the oracle scans linearly);
  * slopes from differences of ln-knots (the oracle takes logs of ratios);
  * each cubic is solved in the power basis from its four Hermite conditions
    with numpy.linalg.solve (the oracle evaluates the Hermite basis);
  * extrapolation formulas restated from the definitions.
Pure Python loops: only for small inputs.
"""
import math

import numpy as np

TAU_X, TAU_Q, X_HIGH = 1e-3, 1e-5, 0.9


def _cell(knots, v):
    i = int(np.searchsorted(knots, v, side="right")) - 1
    return min(max(i, 0), len(knots) - 2)


def _slopes(t, f):
    """Finite-difference slope at every knot of a 1D table in ln coordinates."""
    lt = np.log(t)
    sec = np.diff(f) / np.diff(lt)
    d = np.empty(len(t))
    d[0], d[-1] = sec[0], sec[-1]
    d[1:-1] = 0.5 * (sec[:-1] + sec[1:])
    return d


def _cubic_power_basis(t0, t1, f0, f1, d0, d1, tq):
    """Cubic p with p(t0)=f0, p'(t0)=d0, p(t1)=f1, p'(t1)=d1 (t in ln units),
    solved in the power basis around t0 and evaluated at tq."""
    h = t1 - t0
    A = np.array([[1.0, 0.0, 0.0, 0.0],
                  [0.0, 1.0, 0.0, 0.0],
                  [1.0, h, h * h, h ** 3],
                  [0.0, 1.0, 2 * h, 3 * h * h]])
    c = np.linalg.solve(A, np.array([f0, d0, f1, d1]))
    s = tq - t0
    return c[0] + s * (c[1] + s * (c[2] + s * c[3]))


def interp1d(knots, f, v):
    i = _cell(knots, v)
    d = _slopes(knots, f)
    lt = np.log(knots)
    if v == knots[i]:
        return f[i]
    if v == knots[i + 1]:
        return f[i + 1]
    return _cubic_power_basis(lt[i], lt[i + 1], f[i], f[i + 1], d[i], d[i + 1], math.log(v))


def interp2d(xk, qk, V, x, q2):
    """V[ix][iq]: x step on every Q^2 row, then the Q^2 step."""
    rows = np.array([interp1d(xk, V[:, r], x) for r in range(len(qk))])
    return interp1d(qk, rows, q2)


def _subgrid(grid, q2):
    k = 0
    for j in range(grid.K):
        if grid.q2knots[j][0] <= q2:
            k = j
    return k


def xf(grid, col, x, q2):
    """Brute-force value of stored column ``col`` (extrapolation included)."""
    xk0 = grid.xknots[0]
    if not (np.isfinite(x) and np.isfinite(q2)) or x <= 0 or q2 <= 0 or x > xk0[-1]:
        return float("nan")
    K = grid.K

    def inside(k, xx, qq):
        return interp2d(grid.xknots[k], grid.q2knots[k], grid.values[k][:, :, col], xx, qq)

    def lowx(k, xx, qq):
        xk = grid.xknots[k]
        f0, f1 = inside(k, xk[0], qq), inside(k, xk[1], qq)
        s = (math.log(xx) - math.log(xk[0])) / (math.log(xk[1]) - math.log(xk[0]))
        if f0 > TAU_X and f1 > TAU_X:
            return math.exp(math.log(f0) + s * (math.log(f1) - math.log(f0)))
        return (1 - s) * f0 + s * f1

    def at(k, xx, qq):
        return lowx(k, xx, qq) if xx < grid.xknots[k][0] else inside(k, xx, qq)

    qlo, qhi = grid.q2knots[0][0], grid.q2knots[K - 1][-1]
    if q2 < qlo:
        qk = grid.q2knots[0]
        f0, f1 = at(0, x, qk[0]), at(0, x, qk[1])
        r = q2 / qk[0]
        if f0 > TAU_Q and f1 > TAU_Q and x <= X_HIGH:
            g = (math.log(f1) - math.log(f0)) / (math.log(qk[1]) - math.log(qk[0]))
        else:
            g = 1.0
        return f0 * math.exp((g * r + 1 - r) * math.log(r))
    if q2 > qhi:
        qk = grid.q2knots[K - 1]
        f0, f1 = at(K - 1, x, qk[-2]), at(K - 1, x, qk[-1])
        s = (math.log(q2) - math.log(qk[-1])) / (math.log(qk[-1]) - math.log(qk[-2]))
        if f0 > TAU_X and f1 > TAU_X:
            return math.exp(math.log(f1) + s * (math.log(f1) - math.log(f0)))
        return (1 + s) * f1 - s * f0
    k = _subgrid(grid, q2)
    return at(k, x, q2)


def alphas(q2k, a, q2):
    if not np.isfinite(q2) or q2 <= 0:
        return float("nan")
    if q2 < q2k[0]:
        return a[0]
    if q2 > q2k[-1]:
        return a[-1]
    # segments split at repeated knots; a repeated knot belongs to the upper one
    starts = [0] + [j for j in range(1, len(q2k)) if q2k[j] == q2k[j - 1]]
    ends = [s - 1 for s in starts[1:]] + [len(q2k) - 1]
    seg = max(j for j, s in enumerate(starts) if q2k[s] <= q2)
    lo, hi = starts[seg], ends[seg]
    if hi == lo:
        return a[lo]
    return interp1d(np.asarray(q2k[lo:hi + 1]), np.asarray(a[lo:hi + 1]), q2)
