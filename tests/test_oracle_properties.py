"""Property-based checks of the FP64 oracle (no GPU).  hypothesis draws small
grids (sub-grid count, knot counts, values from a seed) and query points, and
each test checks what the method fixes whatever the draw (section 2.2 for the
PDFs, section 2.3 for alpha_s):
  * the interpolant passes through every stored value (at a threshold knot the
    upper sub-grid's value);
  * data of the form a + b ln x + c ln Q^2 + d ln x ln Q^2 is reproduced at
    every point inside the grid: each row is linear in ln x and the row values
    are linear in ln Q^2, and the finite-difference slopes of a linear function
    are exact, so every cubic piece is that line;
  * the independent brute-force evaluator (tests/brute.py) agrees at arbitrary
    points, inside the grid and in every extrapolation region;
  * alpha_s agrees with the brute-force 1D evaluator, passes through its knots
    and is constant beyond its table.
"""
import math

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import brute
import oracle
from paper_2009_06635_amd import synth

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])

# (sub-grids, x knots, Q^2 knots per sub-grid, seed of knots and values)
shapes = st.tuples(st.integers(1, 3), st.integers(2, 7), st.lists(st.integers(2, 6), min_size=3, max_size=3),
                   st.integers(0, 2**31 - 1))


def make_grid(shape, npid=2):
    K, nx, nqs, seed = shape
    r = np.random.default_rng(seed)
    return synth.tiny_grid(r, K=K, nx=nx, nq=nqs[:K], npid=npid), r


def ogrid(g):
    return oracle.Grid(g.xknots, g.q2knots, g.values, g.pids)


@SETTINGS
@given(shapes, st.integers(0, 2**31 - 1))
def test_passes_through_stored_values(shape, pick):
    g, _ = make_grid(shape, npid=3)
    r = np.random.default_rng(pick)
    og = ogrid(g)
    for k in range(g.K):
        ix = r.integers(0, len(g.xknots[k]), 6)
        iq = r.integers(0, len(g.q2knots[k]), 6)
        x, q2 = g.xknots[k][ix], g.q2knots[k][iq]
        out = oracle.xfxq2(og, g.pids, x, q2)
        for j in range(len(g.pids)):
            want = g.values[k][ix, iq, j].copy()
            top = (iq == len(g.q2knots[k]) - 1) & (k + 1 < g.K)  # threshold knot: the upper sub-grid's row 0
            if top.any():
                want[top] = g.values[k + 1][ix[top], 0, j]
            assert np.array_equal(out[:, j], want), (k, j)


@SETTINGS
@given(shapes, st.tuples(*[st.floats(-3.0, 3.0) for _ in range(4)]), st.integers(0, 2**31 - 1))
def test_bilinear_log_data_reproduced_inside(shape, coef, pick):
    g, _ = make_grid(shape, npid=1)
    a, b, c, d = coef

    def f(x, q2):
        lx, lq = np.log(x), np.log(q2)
        return a + b * lx + c * lq + d * lx * lq

    vals = [f(xk[:, None], qk[None, :])[:, :, None] for xk, qk in zip(g.xknots, g.q2knots)]
    g = g.with_values(vals)
    r = np.random.default_rng(pick)
    x = np.exp(r.uniform(np.log(g.xknots[0][0]), 0.0, 25))
    q2 = np.exp(r.uniform(np.log(g.q2knots[0][0]), np.log(g.q2knots[-1][-1]), 25))
    out = oracle.xfxq2(ogrid(g), g.pids, x, q2)[:, 0]
    lx, lq = np.log(x), np.log(q2)
    scale = abs(a) + abs(b * lx) + abs(c * lq) + abs(d * lx * lq) + 1e-300
    assert np.all(np.abs(out - f(x, q2)) <= 1e-12 * scale)


@SETTINGS
@given(shapes, st.booleans(), st.lists(st.tuples(st.floats(-3.0, 0.0), st.floats(-0.4, 1.4)), min_size=1,
                                        max_size=12))
def test_agrees_with_brute_force(shape, positive, pts):
    g, _ = make_grid(shape, npid=2)
    if positive:  # positive values: the power-law extrapolation branches
        g = g.with_values([np.abs(v) + 0.01 for v in g.values])
    lx0 = math.log(g.xknots[0][0])
    lqlo, lqhi = math.log(g.q2knots[0][0]), math.log(g.q2knots[-1][-1])
    # ln x from 3 below the first knot's up to 0; ln Q^2 from 40 % of the range below it to 40 % above
    x = np.array([min(1.0, math.exp((lx0 - 3.0) * (-u / 3.0))) for u, _ in pts])
    q2 = np.array([math.exp(lqlo + v * (lqhi - lqlo)) for _, v in pts])
    out, sc = oracle.xfxq2(ogrid(g), g.pids, x, q2, with_scale=True)
    for i in range(len(x)):
        for j in range(len(g.pids)):
            b = brute.xf(g, j, x[i], q2[i])
            if math.isnan(b):
                assert math.isnan(out[i, j])
            else:
                assert abs(out[i, j] - b) <= 1e-12 * abs(b) + 1e-12 * sc[i, j], (x[i], q2[i], j)


@SETTINGS
@given(st.integers(2, 12), st.integers(0, 2**31 - 1))
def test_alphas_agrees_with_brute_force(n, seed):
    r = np.random.default_rng(seed)
    qk = np.exp(np.cumsum(r.uniform(0.2, 1.5, n)))
    a = r.uniform(0.05, 0.4, n)
    assert np.array_equal(oracle.alphas_q2(qk, a, qk), a)
    beyond = np.array([qk[0] * 0.5, qk[-1] * 2.0])
    assert np.array_equal(oracle.alphas_q2(qk, a, beyond), np.array([a[0], a[-1]]))
    q = np.exp(r.uniform(math.log(qk[0]), math.log(qk[-1]), 20))
    out = oracle.alphas_q2(qk, a, q)
    for i in range(len(q)):
        b = brute.alphas(qk, a, q[i])
        assert abs(out[i] - b) <= 1e-13 * abs(b), (q[i], out[i], b)
