"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each check is chosen so a plausible slip in the oracle (dropped term, wrong
sign or index, transposed operand, wrong slope rule, wrong branch) fails one of
them:
  * knot reproduction, bit-exact (section 2.2: the interpolant passes through
    the stored grid values);
  * exactness on data linear in (ln x, ln Q^2) everywhere, and on data
    quadratic in (ln x, ln Q^2) where the 4x4 stencil is interior on
    log-uniform knots (finite-difference slopes are exact there);
  * separable data factorises into two 1D interpolants, each equal to scipy's
    CubicHermiteSpline with the same slopes, and to the Catmull-Rom spline on
    uniform interior cells;
  * two knots reduce to linear interpolation in ln x;
  * sub-grid thresholds: Q^2 at a repeated knot is served by the upper grid;
  * extrapolation closed forms / invariants (power laws continued exactly,
    continuity at the grid edge, log-slope and vanishing limit below Q^2_min);
  * independent brute force on tiny grids (tests/brute.py);
  * alpha_s: knots, constant extrapolation, quadratic exactness, closed form.
"""
import math

import numpy as np
import pytest
import scipy.interpolate as si

import brute
import oracle
from paper_2009_06635_amd import synth


def ogrid(g):
    return oracle.Grid(g.xknots, g.q2knots, g.values, g.pids)


def rng(seed):
    return np.random.default_rng(seed)


def relerr(a, b):
    return np.abs(a - b) / (np.abs(b) + 1e-300)


# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("K,nx,nq", [(1, 2, 2), (1, 3, 4), (2, 4, 3), (3, 7, 5), (2, 5, [2, 6])])
def test_knot_reproduction_bit_exact(K, nx, nq):
    g = synth.tiny_grid(rng(11 + K), K=K, nx=nx, nq=nq, npid=3)
    og = ogrid(g)
    for k in range(K):
        xs, qs = np.meshgrid(g.xknots[k], g.q2knots[k], indexing="ij")
        x, q2 = xs.ravel(), qs.ravel()
        out = oracle.xfxq2(og, g.pids, x, q2)
        for j in range(len(g.pids)):
            want = g.values[k][:, :, j].ravel().copy()
            # a threshold knot (first knot of grid k+1 == last of grid k) is served by grid k+1
            if k + 1 < K:
                top = q2 == g.q2knots[k][-1]
                want[top] = g.values[k + 1][:, 0, j][np.searchsorted(g.xknots[k], x[top])]
            assert np.array_equal(out[:, j], want), (k, j)


def _loguniform_grid(nx, nq, fn, K=1):
    xk = np.exp(np.linspace(np.log(1e-5), 0.0, nx))
    xk[-1] = 1.0
    qk = np.exp(np.linspace(np.log(2.0), np.log(2e4), nq))
    V = fn(np.log(xk)[:, None], np.log(qk)[None, :])[:, :, None]
    return synth.SynthGrid([xk], [qk], [V], [21])


def test_linear_data_exact_everywhere_nonuniform():
    r = rng(5)
    g = synth.tiny_grid(r, K=1, nx=9, nq=8, npid=1)
    a, b, c = 0.7, -0.3, 0.45
    lx = np.log(g.xknots[0])[:, None]
    lq = np.log(g.q2knots[0])[None, :]
    g = g.with_values([(a + b * lx + c * lq)[:, :, None]])
    x = np.exp(r.uniform(np.log(g.xknots[0][0]), 0.0, 4000))
    q2 = np.exp(r.uniform(np.log(g.q2knots[0][0]), np.log(g.q2knots[0][-1]), 4000))
    out = oracle.xfxq2(ogrid(g), [21], x, q2)[:, 0]
    want = a + b * np.log(x) + c * np.log(q2)
    assert np.max(np.abs(out - want)) < 2e-14 * np.max(np.abs(want)) * 50


def test_quadratic_data_exact_on_interior_stencils():
    coef = (0.3, -0.2, 0.15, 0.04, -0.03, 0.02)

    def fn(lx, lq):
        return coef[0] + coef[1] * lx + coef[2] * lq + coef[3] * lx * lx + coef[4] * lx * lq + coef[5] * lq * lq

    g = _loguniform_grid(12, 10, fn)
    r = rng(7)
    xk, qk = g.xknots[0], g.q2knots[0]
    # cells 1..n-3 have all four stencil knots inside the grid in both directions
    x = np.exp(r.uniform(np.log(xk[1]), np.log(xk[-2]), 4000))
    q2 = np.exp(r.uniform(np.log(qk[1]), np.log(qk[-2]), 4000))
    out = oracle.xfxq2(ogrid(g), [21], x, q2)[:, 0]
    want = fn(np.log(x), np.log(q2))
    assert np.max(relerr(out, want)) < 1e-12
    # and NOT exact on an edge cell (one-sided slope): guards against a silent
    # central-difference at the boundary
    xe = np.exp(np.log(xk[0]) + 0.5 * (np.log(xk[1]) - np.log(xk[0]))) * np.ones(1)
    qe = np.exp(0.5 * (np.log(qk[4]) + np.log(qk[5]))) * np.ones(1)
    oe = oracle.xfxq2(ogrid(g), [21], xe, qe)[0, 0]
    assert abs(oe - fn(np.log(xe[0]), np.log(qe[0]))) > 1e-6


def _fd_slopes(t, f):
    lt = np.log(t)
    s = np.diff(f) / np.diff(lt)
    d = np.concatenate([[s[0]], 0.5 * (s[:-1] + s[1:]), [s[-1]]])
    return d


def test_separable_equals_scipy_hermite_product():
    r = rng(9)
    g0 = synth.tiny_grid(r, K=1, nx=9, nq=7, npid=1)
    xk, qk = g0.xknots[0], g0.q2knots[0]
    gx = r.uniform(0.5, 2.0, len(xk))
    hq = r.uniform(0.5, 2.0, len(qk))
    g = g0.with_values([(gx[:, None] * hq[None, :])[:, :, None]])
    sx = si.CubicHermiteSpline(np.log(xk), gx, _fd_slopes(xk, gx))
    sq = si.CubicHermiteSpline(np.log(qk), hq, _fd_slopes(qk, hq))
    x = np.exp(r.uniform(np.log(xk[0]), 0.0, 3000))
    q2 = np.exp(r.uniform(np.log(qk[0]), np.log(qk[-1]), 3000))
    out = oracle.xfxq2(ogrid(g), [21], x, q2)[:, 0]
    want = sx(np.log(x)) * sq(np.log(q2))
    assert np.max(relerr(out, want)) < 1e-13


def test_uniform_interior_cell_is_catmull_rom():
    r = rng(13)
    n = 10
    xk = np.exp(np.linspace(np.log(1e-3), 0.0, n))
    xk[-1] = 1.0
    qk = np.array([4.0, 9.0])
    f = r.uniform(-1, 2, n)
    V = np.stack([f, f], axis=1)[:, :, None]   # constant along Q^2
    g = synth.SynthGrid([xk], [qk], [V], [21])
    i = 4
    u = r.uniform(0, 1, 200)
    x = np.exp(np.log(xk[i]) + u * (np.log(xk[i + 1]) - np.log(xk[i])))
    out = oracle.xfxq2(ogrid(g), [21], x, np.full(200, 5.0))[:, 0]
    p0, p1, p2, p3 = f[i - 1], f[i], f[i + 1], f[i + 2]
    cr = 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u ** 2
                + (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3)
    assert np.max(np.abs(out - cr)) < 1e-13


def test_two_knots_is_linear_in_log():
    xk = np.array([1e-3, 1.0])
    qk = np.array([3.0, 50.0])
    V = np.array([[[1.5], [0.5]], [[-0.25], [2.0]]])
    g = synth.SynthGrid([xk], [qk], [V], [21])
    r = rng(17)
    ux, uq = r.uniform(0, 1, 500), r.uniform(0, 1, 500)
    x = np.exp(np.log(1e-3) * (1 - ux))
    q2 = np.exp(np.log(3.0) + uq * np.log(50.0 / 3.0))
    ux = np.log(x / 1e-3) / np.log(1e3)
    uq = np.log(q2 / 3.0) / np.log(50.0 / 3.0)
    want = ((1 - ux) * (1 - uq) * 1.5 + (1 - ux) * uq * 0.5 + ux * (1 - uq) * -0.25 + ux * uq * 2.0)
    out = oracle.xfxq2(ogrid(g), [21], x, q2)[:, 0]
    assert np.max(np.abs(out - want)) < 1e-14


def test_threshold_goes_to_upper_subgrid_and_is_continuous():
    r = rng(19)
    g = synth.tiny_grid(r, K=3, nx=6, nq=5, npid=1)

    def smooth(lx, lq):
        return 1.0 + 0.3 * np.sin(lx) + 0.2 * np.cos(0.7 * lq) + 0.05 * lx * lq

    vals = [smooth(np.log(g.xknots[k])[:, None], np.log(g.q2knots[k])[None, :])[:, :, None] for k in range(3)]
    g = g.with_values(vals)
    og = ogrid(g)
    x = np.exp(r.uniform(np.log(g.xknots[0][0]), 0.0, 50))
    for k in (1, 2):
        t = g.q2knots[k][0]
        at = oracle.xfxq2(og, [21], x, np.full(50, t))[:, 0]
        # exactly at the threshold: the upper grid's first row = its x-interpolant of row 0
        upper_row = np.array([brute.interp1d(g.xknots[k], g.values[k][:, 0, 0], xi) for xi in x])
        assert np.max(np.abs(at - upper_row)) < 1e-13
        below = oracle.xfxq2(og, [21], x, np.full(50, np.nextafter(t, 0.0)))[:, 0]
        assert np.max(np.abs(below - at)) < 1e-12
    # a grid whose flavour is zero below a threshold: each side reproduces its own grid
    vals2 = [v.copy() for v in vals]
    vals2[0][:] = 0.0
    g2 = g.with_values(vals2)
    t = g2.q2knots[1][0]
    below = oracle.xfxq2(ogrid(g2), [21], x, np.full(50, np.nextafter(t, 0.0)))[:, 0]
    assert np.all(below == 0.0)


# ---------------------------------------------------------------------------------------------
def _powerlaw_grid(p_x=0.0, p_q=0.0, C=2.0, nx=8, nq=6):
    xk = np.exp(np.linspace(np.log(1e-4), 0.0, nx))
    xk[-1] = 1.0
    qk = np.exp(np.linspace(np.log(2.0), np.log(1e3), nq))
    V = (C * xk[:, None] ** p_x * qk[None, :] ** p_q)[:, :, None]
    return synth.SynthGrid([xk], [qk], [V], [21])


def test_lowx_continues_power_law_exactly():
    g = _powerlaw_grid(p_x=-0.35)
    r = rng(23)
    x = np.exp(r.uniform(np.log(1e-9), np.log(1e-4), 500))
    x = x[x < 1e-4]
    q2 = np.exp(r.uniform(np.log(2.0), np.log(1e3), len(x)))
    out = oracle.xfxq2(ogrid(g), [21], x, q2)[:, 0]
    assert np.max(relerr(out, 2.0 * x ** -0.35)) < 1e-12


def test_highq_continues_power_law_exactly():
    g = _powerlaw_grid(p_q=0.12)
    r = rng(29)
    q2 = np.exp(r.uniform(np.log(1e3), np.log(1e7), 500))
    q2 = q2[q2 > 1e3 * (1 + 1e-12)]
    x = np.exp(r.uniform(np.log(1e-4), 0.0, len(q2)))
    out = oracle.xfxq2(ogrid(g), [21], x, q2)[:, 0]
    assert np.max(relerr(out, 2.0 * q2 ** 0.12)) < 1e-11


def test_lowx_linear_branch_below_threshold():
    # values below TAU_X -> linear continuation in ln x: second differences vanish
    g = _powerlaw_grid(p_x=0.5, C=1e-5)
    x = np.exp(np.linspace(np.log(1e-8), np.log(0.9e-4), 9))
    out = oracle.xfxq2(ogrid(g), [21], x, np.full(9, 10.0))[:, 0]
    assert np.max(np.abs(np.diff(out, 2))) < 1e-18
    # continuity at x_min
    e = oracle.xfxq2(ogrid(g), [21], np.array([np.nextafter(1e-4, 0), 1e-4]), np.full(2, 10.0))[:, 0]
    assert abs(e[0] - e[1]) < 1e-18


def test_lowq_invariants():
    g = _powerlaw_grid(p_x=-0.2, p_q=0.08)
    og = ogrid(g)
    q0, q1 = g.q2knots[0][0], g.q2knots[0][1]
    x = np.array([1e-3, 0.05, 0.3])
    f0 = oracle.xfxq2(og, [21], x, np.full(3, q0))[:, 0]
    f1 = oracle.xfxq2(og, [21], x, np.full(3, q1))[:, 0]
    gamma = np.log(f1 / f0) / np.log(q1 / q0)
    # continuity at q0
    just_below = oracle.xfxq2(og, [21], x, np.full(3, np.nextafter(q0, 0)))[:, 0]
    assert np.max(relerr(just_below, f0)) < 1e-14
    # log-slope at q0 from below equals gamma (one-sided finite difference)
    h = 1e-6
    fb = oracle.xfxq2(og, [21], x, np.full(3, q0 * math.exp(-h)))[:, 0]
    slope = (np.log(f0) - np.log(fb)) / h
    assert np.max(np.abs(slope - gamma)) < 1e-5
    # vanishes as Q^2 -> 0
    tiny = oracle.xfxq2(og, [21], x, np.full(3, 1e-12))[:, 0]
    assert np.all(np.abs(tiny) < 1e-9)
    # x above 0.9: gamma = 1, so xf = f0 * Q^2 / q0 exactly
    xh = np.array([0.95])
    fh0 = oracle.xfxq2(og, [21], xh, np.array([q0]))[0, 0]
    fh = oracle.xfxq2(og, [21], xh, np.array([0.5 * q0]))[0, 0]
    assert abs(fh - 0.5 * fh0) <= 1e-15 * abs(fh0)


# ---------------------------------------------------------------------------------------------
def _queries_everywhere(r, g, n_rand=60):
    xk0 = g.xknots[0]
    qlo, qhi = g.q2knots[0][0], g.q2knots[-1][-1]
    xs = list(np.exp(r.uniform(np.log(xk0[0]) - 2.0, 0.0, n_rand)))
    qs = list(np.exp(r.uniform(np.log(qlo) - 2.0, np.log(qhi) + 2.0, n_rand)))
    for xv in xk0:
        for qv in [qlo, qhi] + [q[0] for q in g.q2knots]:
            for dx in (xv, np.nextafter(xv, 0), np.nextafter(xv, 2)):
                for dq in (qv, np.nextafter(qv, 0), np.nextafter(qv, np.inf)):
                    xs.append(dx)
                    qs.append(dq)
    x, q = np.array(xs), np.array(qs)
    keep = x <= 1.0
    return x[keep], q[keep]


@pytest.mark.parametrize("seed", range(6))
def test_oracle_matches_brute_force_on_tiny_grids(seed):
    r = rng(100 + seed)
    K = 1 + seed % 3
    nx = [2, 3, 4, 5, 6, 7][seed]
    nq = [[2, 3, 4][(seed + k) % 3] for k in range(K)]
    g = synth.tiny_grid(r, K=K, nx=nx, nq=nq, npid=2)
    # positive values so that both extrapolation branches occur
    if seed % 2:
        g = g.with_values([np.abs(v) + 0.01 for v in g.values])
    x, q2 = _queries_everywhere(r, g)
    out, scale = oracle.xfxq2(ogrid(g), g.pids, x, q2, with_scale=True)
    for i in range(len(x)):
        for c in range(len(g.pids)):
            b = brute.xf(g, c, x[i], q2[i])
            o = out[i, c]
            if math.isnan(b):
                assert math.isnan(o)
                continue
            assert abs(o - b) <= 1e-12 * abs(b) + 1e-12 * scale[i, c], (i, c, x[i], q2[i], o, b)


def test_locate_matches_searchsorted():
    g = synth.config2_grid()
    og = ogrid(g)
    x, q2 = synth.config2_queries(n=20000, seed=77, out_fraction=0.05)
    # every knot and its float neighbours (ties: a query on an interior knot opens that knot's cell)
    xk = g.xknots[0]
    qk_all = np.concatenate(g.q2knots)
    xs = np.concatenate([xk, np.nextafter(xk, 0.0), np.nextafter(xk[:-1], 2.0)])
    qs = np.concatenate([qk_all, np.nextafter(qk_all, 0.0), np.nextafter(qk_all, np.inf)])
    r = rng(78)
    x = np.concatenate([x, xs, xs[r.integers(0, len(xs), len(qs))]])
    q2 = np.concatenate([q2, qs[r.integers(0, len(qs), len(xs))], qs])
    k, ix, iq, reg = oracle.locate(og, x, q2)
    firsts = np.array([q[0] for q in g.q2knots])
    kk = np.clip(np.searchsorted(firsts, q2, side="right") - 1, 0, 2)
    assert np.array_equal(k, kk)
    ixx = np.clip(np.searchsorted(g.xknots[0], x, side="right") - 1, 0, len(g.xknots[0]) - 2)
    assert np.array_equal(ix, ixx)
    for kv in range(3):
        m = k == kv
        qk = g.q2knots[kv]
        iqq = np.clip(np.searchsorted(qk, q2[m], side="right") - 1, 0, len(qk) - 2)
        assert np.array_equal(iq[m], iqq)
    want = ((x < g.xknots[0][0]) * 1 + (q2 < g.q2knots[0][0]) * 2 + (q2 > g.q2knots[2][-1]) * 4)
    assert np.array_equal(reg, want.astype(np.int8))


def test_invalid_points_and_pid_rules():
    g = synth.config1_grid()
    og = ogrid(g)
    x = np.array([0.1, -0.1, 0.0, 1.5, np.nan, 0.1, 0.1, np.inf])
    q2 = np.array([10.0, 10.0, 10.0, 10.0, 10.0, -1.0, np.nan, 10.0])
    out = oracle.xfxq2(og, [21, 0, 6, -6, 2], x, q2)
    assert np.all(np.isfinite(out[0, [0, 1, 4]]))
    assert out[0, 0] == out[0, 1]            # pid 0 is the gluon
    assert out[0, 2] == 0.0 and out[0, 3] == 0.0   # top absent from an 11-flavour grid
    assert np.all(np.isnan(out[1:]))
    with pytest.raises(ValueError):
        oracle.xfxq2(og, [7], x, q2)


def test_config_generators_shapes():
    g = synth.config2_grid()
    assert g.K == 3 and [len(q) for q in g.q2knots] == [17, 17, 17]
    assert len(g.xknots[0]) == 196 and g.values[2].shape == (196, 17, 13)
    assert g.q2knots[0][-1] == g.q2knots[1][0] and g.q2knots[1][-1] == g.q2knots[2][0]
    j = {p: i for i, p in enumerate(g.pids)}
    assert np.all(g.values[0][:, :, j[4]] == 0) and np.any(g.values[1][:, :, j[4]] != 0)
    assert np.all(g.values[1][:, :, j[-5]] == 0) and np.any(g.values[2][:, :, j[-5]] != 0)
    assert all(np.all(v[:, :, j[6]] == 0) for v in g.values)
    x, q2 = synth.config2_queries(n=100000)
    out = (x < 1e-9) | (q2 < 1.0) | (q2 > 1e10)
    assert abs(out.mean() - 0.01) < 0.001
    x1, q1 = synth.config2_queries(n=1000)
    x2, q2b = synth.config2_queries(n=1000)
    assert np.array_equal(x1, x2) and np.array_equal(q1, q2b)


# ---------------------------------------------------------------------------------------------
def test_alphas_pins():
    qk, a = synth.config1_alphas()
    # knot reproduction
    assert np.array_equal(oracle.alphas_q2(qk, a, qk), a)
    # constant extrapolation both sides
    out = oracle.alphas_q2(qk, a, np.array([1e-3, qk[0] * 0.999, qk[-1] * 1.001, 1e12]))
    assert np.array_equal(out, [a[0], a[0], a[-1], a[-1]])
    # closed form of the table: smoke bound only (interpolation error), not parity
    r = rng(31)
    q2 = np.exp(r.uniform(np.log(qk[0]), np.log(qk[-1]), 2000))
    assert np.max(relerr(oracle.alphas_q2(qk, a, q2), synth.alphas_closed_form(q2))) < 1e-4
    # quadratic in ln Q^2 on uniform knots: exact on interior cells
    lq = np.log(qk)
    aq = 0.1 + 0.01 * lq - 0.002 * lq * lq
    q2i = np.exp(r.uniform(lq[1], lq[-2], 2000))
    li = np.log(q2i)
    want = 0.1 + 0.01 * li - 0.002 * li * li
    # the quadratic crosses zero: compare against the data's magnitude
    assert np.max(np.abs(oracle.alphas_q2(qk, aq, q2i) - want)) < 1e-13 * np.max(np.abs(aq))
    # cubic in ln Q and in ln Q^2 are the same interpolant (affine reparametrisation)
    q = np.sqrt(qk)
    sq = si.CubicHermiteSpline(np.log(q), a, _fd_slopes(q, a))
    qq = np.sqrt(q2)
    assert np.max(relerr(oracle.alphas_q2(qk, a, q2), sq(np.log(qq)))) < 1e-13
    # invalid
    assert np.all(np.isnan(oracle.alphas_q2(qk, a, np.array([0.0, -1.0, np.nan]))))


def test_alphas_segments_at_repeated_knots():
    qk, a = synth.config2_alphas()
    a = a.copy()
    a[17:34] += 0.01      # a jump at the first threshold
    # at the threshold the upper segment's value is used
    t = qk[17]
    assert oracle.alphas_q2(qk, a, np.array([t]))[0] == a[17]
    assert oracle.alphas_q2(qk, a, np.array([np.nextafter(t, 0)]))[0] == pytest.approx(a[16], rel=1e-12)
    r = rng(37)
    q2 = np.exp(r.uniform(np.log(qk[0]) - 1, np.log(qk[-1]) + 1, 300))
    q2 = np.concatenate([q2, qk, np.nextafter(qk, 0), np.nextafter(qk, np.inf)])
    o = oracle.alphas_q2(qk, a, q2)
    b = np.array([brute.alphas(qk, a, v) for v in q2])
    assert np.max(relerr(o, b)) < 1e-13


# ---------------------------------------------------------------------------------------------
# The error scale s that the oracle returns beside each value (the floor of every
# parity criterion) against quantities computed without it: the largest stencil
# magnitude, found here by searchsorted, and the value's first-order sensitivity
# to relative changes of the grid values, found by central differences of the
# oracle's values.  Too small an s would make the parity floors too tight; too
# large an s would loosen every parity test silently.

def _data_sensitivity(g, x, q2, h=1e-6):
    W = np.zeros((len(x), len(g.pids)))
    for k in range(len(g.values)):
        for idx in np.ndindex(g.values[k].shape):
            f = g.values[k][idx]
            if f == 0.0:
                continue
            F = []
            for sgn in (1.0, -1.0):
                vals = [v.copy() for v in g.values]
                vals[k][idx] = f * (1.0 + sgn * h)
                F.append(oracle.xfxq2(oracle.Grid(g.xknots, g.q2knots, vals, g.pids), g.pids, x, q2))
            W += np.abs(F[0] - F[1]) / (2.0 * h)
    return W


def _scale_grid(r, positive):
    """Two sub-grids with log-uniform knots; smooth positive data (varying by less
    than a factor 2 across any stencil) or signed random data."""
    xk = np.exp(np.linspace(np.log(1e-4), 0.0, 6))
    q0 = np.exp(np.linspace(np.log(1.5), np.log(6.0), 5))
    q1 = np.exp(np.linspace(np.log(6.0), np.log(200.0), 6))
    q1[0] = q0[-1]
    vals = []
    for qk in (q0, q1):
        lx, lq = np.log(xk)[:, None, None], np.log(qk)[None, :, None]
        if positive:
            a = r.uniform(-0.15, 0.15, (1, 1, 2))
            b = r.uniform(-0.05, 0.05, (1, 1, 2))
            vals.append(np.exp(a * lx + b * lq + 0.05 * np.sin(lx + lq)))
        else:
            vals.append(r.uniform(-1.0, 2.0, (len(xk), len(qk), 2)))
    return synth.SynthGrid([xk, xk], [q0, q1], vals, [21, 2])


@pytest.mark.parametrize("positive", [False, True])
def test_error_scale_is_stencil_magnitude_inside(positive):
    r = rng(31 + positive)
    g = _scale_grid(r, positive)
    x, q2 = _queries_everywhere(r, g)
    out, s = oracle.xfxq2(ogrid(g), g.pids, x, q2, with_scale=True)
    inside = (x >= g.xknots[0][0]) & (q2 >= g.q2knots[0][0]) & (q2 <= g.q2knots[-1][-1])
    assert inside.sum() > 50
    for i in np.flatnonzero(inside):
        k = 1 if q2[i] >= g.q2knots[1][0] else 0
        xk, qk = g.xknots[k], g.q2knots[k]
        ix = min(max(np.searchsorted(xk, x[i], side="right") - 1, 0), len(xk) - 2)
        iq = min(max(np.searchsorted(qk, q2[i], side="right") - 1, 0), len(qk) - 2)
        win = g.values[k][max(ix - 1, 0):ix + 3, max(iq - 1, 0):iq + 3, :]
        assert np.array_equal(s[i], np.max(np.abs(win), axis=(0, 1))), (x[i], q2[i])


@pytest.mark.parametrize("positive", [False, True])
def test_error_scale_bounds_data_sensitivity(positive):
    """Every valid value, extrapolations included: its sensitivity to relative
    changes of the grid values is at most 2 s (log-uniform knots: the weights of
    a 4 x 4 stencil have sum |w| <= 1.25^2); on smooth positive data s is also at
    most 3 times that sensitivity (not inflated)."""
    r = rng(41 + positive)
    g = _scale_grid(r, positive)
    x, q2 = _queries_everywhere(r, g, n_rand=200)
    out, s = oracle.xfxq2(ogrid(g), g.pids, x, q2, with_scale=True)
    ok = np.isfinite(out) & (s > 0)
    W = _data_sensitivity(g, x, q2)
    assert np.all(W[ok] <= 2.0 * s[ok] * (1 + 1e-9)), np.max(W[ok] / s[ok])
    if positive:
        assert np.all(s[ok] <= 3.0 * W[ok]), np.max(s[ok] / W[ok])
