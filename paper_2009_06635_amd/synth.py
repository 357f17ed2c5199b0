"""Seeded synthetic grids and query sets.

These stand in for the LHAPDF grids (NNPDF3.1 NLO, MMHT2014 NLO) and the
FastKernel x-grid the paper measures on (sections 3.2-3.3, 4.3), which are not
available here.  Shapes follow the workloads the paper benchmarks: all flavours
of a set evaluated on log-distributed (x, Q) clouds inside the grid (section
3.3), heavy-flavour sub-grids split at quark-mass thresholds (section 2.2),
many replica members (section 4.3), and Monte-Carlo-integrand-style loads
(section 4.1).

This module holds no interpolation arithmetic: it only draws knots, grid
values from a smooth closed form, and query points.  Both the oracle tests and
the GPU path take their inputs from here.

Grid values use  x f = A x^a (1-x)^b (1 + c sqrt(x) + d x) (1 + e ln(Q^2/2.7))
with A = 1 and per-flavour parameters drawn uniformly: a in [-0.3, 0.8],
b in [2, 6], c, d in [-1, 2], e in [-0.1, 0.1].  Q^2 knots are Q*Q in FP64.
"""
import numpy as np

PIDS_11 = [-5, -4, -3, -2, -1, 21, 1, 2, 3, 4, 5]
PIDS_13 = [-6, -5, -4, -3, -2, -1, 21, 1, 2, 3, 4, 5, 6]


class SynthGrid:
    """One member: per sub-grid x knots, Q^2 knots and values[ix][iq][column]."""

    def __init__(self, xknots, q2knots, values, pids, params=None):
        self.xknots = [np.ascontiguousarray(x, np.float64) for x in xknots]
        self.q2knots = [np.ascontiguousarray(q, np.float64) for q in q2knots]
        self.values = [np.ascontiguousarray(v, np.float64) for v in values]
        self.pids = list(pids)
        self.params = params

    @property
    def K(self):
        return len(self.xknots)

    def with_values(self, values):
        return SynthGrid(self.xknots, self.q2knots, values, self.pids, self.params)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def draw_params(rng, npid):
    """[npid][5] = (a, b, c, d, e), drawn per flavour in column order."""
    lo = np.array([-0.3, 2.0, -1.0, -1.0, -0.1])
    hi = np.array([0.8, 6.0, 2.0, 2.0, 0.1])
    return lo + (hi - lo) * rng.random((npid, 5))


def closed_form(params, x, q2):
    """The generating function, broadcast over x[:, None] and q2[None, :]
    for one flavour: x f(x, Q^2) = x^a (1-x)^b (1 + c sqrt(x) + d x)(1 + e ln(Q^2/2.7))."""
    a, b, c, d, e = params
    x = np.asarray(x, np.float64)[:, None]
    q2 = np.asarray(q2, np.float64)[None, :]
    return x ** a * (1.0 - x) ** b * (1.0 + c * np.sqrt(x) + d * x) * (1.0 + e * np.log(q2 / 2.7))


def _fill(params, xk, qk):
    return np.stack([closed_form(params[j], xk, qk) for j in range(params.shape[0])], axis=-1)


def logspace_q2(qlo, qhi, n):
    q = np.exp(np.linspace(np.log(qlo), np.log(qhi), n))
    q[0], q[-1] = qlo, qhi
    return q * q


def alphas_closed_form(q2):
    """alpha_s table values of the synthetic sets: 0.118 / (1 + 0.02 ln(8315/Q^2))."""
    return 0.118 / (1.0 + 0.02 * np.log(8315.0 / np.asarray(q2, np.float64)))


# --------------------------------------------------------------------------------------
# config 1: one member, one sub-grid, 50 x 30 knots, 11 flavours


def config1_grid(seed=1001):
    rng = _rng(seed)
    xk = 10.0 ** (-6.0 + 6.0 * np.arange(50) / 49.0)
    xk[-1] = 1.0
    qk = logspace_q2(1.65, 1e4, 30)
    params = draw_params(rng, len(PIDS_11))
    return SynthGrid([xk], [qk], [_fill(params, xk, qk)], PIDS_11, params)


def config1_alphas():
    qk = logspace_q2(1.65, 1e4, 30)
    return qk, alphas_closed_form(qk)


def loguniform(rng, lo, hi, n, include_hi=True):
    v = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    if not include_hi:
        v = np.minimum(v, np.nextafter(hi, 0.0))
    return v


def config1_queries(n=100_000, seed=2001):
    """x log-uniform in [1e-6, 1), Q log-uniform in [1.65, 1e4]; returns (x, q2)."""
    rng = _rng(seed)
    x = loguniform(rng, 1e-6, 1.0, n, include_hi=False)
    q = loguniform(rng, 1.65, 1e4, n)
    return x, q * q


# --------------------------------------------------------------------------------------
# config 2: three sub-grids split at Q = 1.51 and 4.92 GeV, 196 x knots, 13 flavours

THRESHOLDS_Q = (1.0, 1.51, 4.92, 1e5)


def config2_grid(seed=1002):
    rng = _rng(seed)
    xk = 10.0 ** (-9.0 + 9.0 * np.arange(196) / 195.0)
    xk[-1] = 1.0
    params = draw_params(rng, len(PIDS_13))
    xks, qks, vals = [], [], []
    for k in range(3):
        qk = logspace_q2(THRESHOLDS_Q[k], THRESHOLDS_Q[k + 1], 17)
        v = _fill(params, xk, qk)
        for j, pid in enumerate(PIDS_13):
            heavy = abs(pid)
            if (heavy == 4 and k < 1) or (heavy == 5 and k < 2) or heavy == 6:
                v[:, :, j] = 0.0
        xks.append(xk.copy())
        qks.append(qk)
        vals.append(v)
    return SynthGrid(xks, qks, vals, PIDS_13, params)


def config2_alphas():
    qk = np.concatenate([logspace_q2(THRESHOLDS_Q[k], THRESHOLDS_Q[k + 1], 17) for k in range(3)])
    return qk, alphas_closed_form(qk)


def config2_queries(n=10_000_000, seed=2002, out_fraction=0.01):
    """99% inside (x in [1e-9, 1), Q in [1, 1e5]); 1% outside: a quarter each
    low-x (x in [1e-11, 1e-9)), low-Q (Q in [0.5, 1)), high-Q (Q in (1e5, 1e6]),
    and corners (low-x with low- or high-Q).  Log-uniform, interleaved."""
    rng = _rng(seed)
    x = loguniform(rng, 1e-9, 1.0, n, include_hi=False)
    q = loguniform(rng, 1.0, 1e5, n)
    n_out = int(round(out_fraction * n))
    if n_out:
        idx = rng.permutation(n)[:n_out]
        kind = np.arange(n_out) % 4
        lowx = (kind == 0) | (kind == 3)
        x[idx[lowx]] = loguniform(rng, 1e-11, 1e-9, int(lowx.sum()), include_hi=False)
        lowq = (kind == 1) | ((kind == 3) & (rng.random(n_out) < 0.5))
        highq = ((kind == 2) | (kind == 3)) & ~lowq
        q[idx[lowq]] = loguniform(rng, 0.5, 1.0, int(lowq.sum()), include_hi=False)
        q[idx[highq]] = np.maximum(loguniform(rng, 1e5, 1e6, int(highq.sum())), np.nextafter(1e5, 2e5))
    return x, q * q


# --------------------------------------------------------------------------------------
# config 3: 101 members (central + 100 log-normal replicas), 200 uneven requests


def config3_members(seed=1003, n_members=101):
    base = config1_grid()
    rng = _rng(seed)
    members = [base]
    for _ in range(1, n_members):
        z = rng.standard_normal(base.values[0].shape)
        members.append(base.with_values([base.values[0] * np.exp(0.05 * z)]))
    return members


def config3_requests(seed=2003, n_requests=200, n_members=101):
    """List of dicts {member, pids, x, q2}: log10 n ~ N(4.5, 0.75) clipped to
    [3, 6]; member uniform; pid subset of size U{1..11} in random order;
    points drawn as config 1."""
    rng = _rng(seed)
    reqs = []
    for _ in range(n_requests):
        n = int(round(10.0 ** np.clip(rng.normal(4.5, 0.75), 3.0, 6.0)))
        member = int(rng.integers(0, n_members))
        size = int(rng.integers(1, len(PIDS_11) + 1))
        pids = [int(p) for p in rng.permutation(PIDS_11)[:size]]
        x = loguniform(rng, 1e-6, 1.0, n, include_hi=False)
        q = loguniform(rng, 1.65, 1e4, n)
        reqs.append({"member": member, "pids": pids, "x": x, "q2": q * q})
    return reqs


# --------------------------------------------------------------------------------------
# config 5: Monte-Carlo-integrand-shaped load


def config5_chunk(chunk, n=1_000_000, seed=2005):
    """x1, x2 log-uniform in [1e-5, 1), shared Q log-uniform in [10, 1e3]."""
    rng = _rng([seed, chunk])
    x1 = loguniform(rng, 1e-5, 1.0, n, include_hi=False)
    x2 = loguniform(rng, 1e-5, 1.0, n, include_hi=False)
    q = loguniform(rng, 10.0, 1e3, n)
    return x1, x2, q * q


def tiny_grid(rng, K=1, nx=4, nq=4, npid=2, pids=None, loguniform_knots=False):
    """Small random grid for brute-force checks: monotone knots (random gaps
    unless ``loguniform_knots``), sub-grids sharing their threshold knot, random
    values of mixed sign."""
    nxs = [nx] * K if np.isscalar(nx) else list(nx)
    nqs = [nq] * K if np.isscalar(nq) else list(nq)
    if loguniform_knots:
        xk = np.exp(np.linspace(np.log(1e-4), 0.0, nxs[0]))
    else:
        xk = np.exp(np.cumsum(rng.uniform(0.3, 1.5, nxs[0])))
        xk = xk / xk[-1]
    xk[-1] = 1.0
    edges = [2.0]
    for k in range(K):
        edges.append(edges[-1] * np.exp(rng.uniform(1.0, 3.0)))
    xks, qks, vals = [], [], []
    for k in range(K):
        if loguniform_knots:
            qk = np.exp(np.linspace(np.log(edges[k]), np.log(edges[k + 1]), nqs[k]))
        else:
            g = np.cumsum(np.concatenate([[0.0], rng.uniform(0.3, 1.5, nqs[k] - 1)]))
            qk = np.exp(np.log(edges[k]) + g / g[-1] * (np.log(edges[k + 1]) - np.log(edges[k])))
        qk[0], qk[-1] = edges[k], edges[k + 1]
        xks.append(xk.copy() if k == 0 else xks[0].copy())
        qks.append(qk)
        vals.append(rng.uniform(-1.0, 2.0, (len(xk), nqs[k], npid)))
    if pids is None:
        pids = [21, 1, 2, -1, 3, -3, 4, -4, 5, -5, -2, 6, -6][:npid]
    return SynthGrid(xks, qks, vals, pids)
