"""Monte-Carlo-integrand load (config 5 shape): two PDF lookups per point at a
shared scale plus alpha_s, and the FP64 fixed-order chunk sum, vs the oracle."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2009_06635_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2009_06635_amd import pdfmi  # noqa: E402

DEV = "cuda:0"
PIDS = synth.PIDS_13


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(DEV)


def oracle_chunk(g, qk, a, x1, x2, q2):
    og = oracle.Grid(g.xknots, g.q2knots, g.values, g.pids)
    th = os.cpu_count() or 1
    f1 = oracle.xfxq2(og, PIDS, x1, q2, n_threads=th)
    f2 = oracle.xfxq2(og, PIDS, x2, q2, n_threads=th)
    al = oracle.alphas_q2(qk, a, q2)
    terms = al * np.sum(f1 * f2, axis=1)
    return math.fsum(terms), math.fsum(np.abs(al) * np.sum(np.abs(f1 * f2), axis=1))


@pytest.mark.parametrize("n", [1, 4095, 4097, 200_000])
def test_mc_chunk_sum_matches_oracle(n):
    g = synth.config1_grid()
    qk, a = synth.config1_alphas()
    m = pdfmi.load_synth(g)
    pdfmi.load_alphas(qk, a)
    try:
        x1, x2, q2 = synth.config5_chunk(0, n=n)
        q2d = dev(q2)
        f1 = pdfmi.xfxq2(m, PIDS, dev(x1), q2d)
        f2 = pdfmi.xfxq2(m, PIDS, dev(x2), q2d)
        al = pdfmi.alphas_q2(q2d)
        s1 = pdfmi.mc_chunk_sum(f1, f2, al).item()
        s2 = pdfmi.mc_chunk_sum(f1, f2, al).item()
        assert s1 == s2                      # fixed summation order
        so, sabs = oracle_chunk(g, qk, a, x1, x2, q2)
        assert abs(s1 - so) <= 1e-11 * sabs, (s1, so)
    finally:
        pdfmi.unload(m)


def test_mc_empty_chunk():
    e2 = torch.empty((0, 13), dtype=torch.float64, device=DEV)
    e1 = torch.empty(0, dtype=torch.float64, device=DEV)
    assert pdfmi.mc_chunk_sum(e2, e2, e1).item() == 0.0


def test_mc_full_chunk_sampled():
    """One full 1e6-point chunk as the benchmark runs it, against the oracle."""
    g = synth.config1_grid()
    qk, a = synth.config1_alphas()
    m = pdfmi.load_synth(g)
    pdfmi.load_alphas(qk, a)
    try:
        x1, x2, q2 = synth.config5_chunk(3)
        q2d = dev(q2)
        f1 = pdfmi.xfxq2(m, PIDS, dev(x1), q2d)
        f2 = pdfmi.xfxq2(m, PIDS, dev(x2), q2d)
        s = pdfmi.mc_chunk_sum(f1, f2, pdfmi.alphas_q2(q2d)).item()
        so, sabs = oracle_chunk(g, qk, a, x1, x2, q2)
        assert abs(s - so) <= 1e-11 * sabs, (s, so)
    finally:
        pdfmi.unload(m)


def _mixed_chunk(n, seed, invalid=True):
    """config-5 points with a share moved outside the grid in x and Q^2 (all
    extrapolation regions) and, with ``invalid``, a few invalid points (whose
    NaN values make the chunk sum NaN)."""
    x1, x2, q2 = synth.config5_chunk(1, n=n)
    x1, x2, q2 = x1.copy(), x2.copy(), q2.copy()
    rng = np.random.default_rng(seed)
    k = max(1, n // 20)
    idx = rng.choice(n, size=min(n, 4 * k), replace=False)
    a, b, c, d = np.array_split(idx, 4)
    x1[a] = np.exp(rng.uniform(np.log(1e-8), np.log(1e-6), len(a)))   # below x_min
    q2[b] = np.exp(rng.uniform(np.log(0.5), np.log(2.0), len(b)))     # below Q^2_min
    q2[c] = np.exp(rng.uniform(np.log(2e8), np.log(1e10), len(c)))    # above Q^2_max
    x2[d] = np.exp(rng.uniform(np.log(1e-8), np.log(1e-6), len(d)))   # corner with some of the above
    q2[d] = np.exp(rng.uniform(np.log(0.5), np.log(2.0), len(d)))
    if invalid and n > 10:
        x1[3], q2[5], x2[7] = -1.0, np.nan, 1.5
    return x1, x2, q2


@pytest.mark.parametrize("n", [1, 4095, 4097, 16385, 200_000, 1_000_000])
@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("mixed", ["none", "extrap", "invalid"])
@pytest.mark.parametrize("pids", ["p13", "all"])
def test_fused_equals_unfused(n, f32, mixed, pids):
    g = synth.config1_grid()
    qk, a = synth.config1_alphas()
    m = pdfmi.load_synth(g)
    pdfmi.load_alphas(qk, a)
    plist = PIDS if pids == "p13" else list(g.pids)
    try:
        if mixed == "none":
            x1, x2, q2 = synth.config5_chunk(2, n=n)
        else:
            x1, x2, q2 = _mixed_chunk(n, 9, invalid=mixed == "invalid")
        d1, d2, dq = dev(x1), dev(x2), dev(q2)
        ev = pdfmi.xfxq2_f32 if f32 else pdfmi.xfxq2
        pdfmi.error_count(reset=True)
        f1 = ev(m, plist, d1, dq)
        f2 = ev(m, plist, d2, dq)
        s_ref = pdfmi.mc_chunk_sum(f1, f2, pdfmi.alphas_q2(dq)).cpu().numpy()
        e_ref = pdfmi.error_count(reset=True)
        s = pdfmi.mc_fused(m, plist, d1, d2, dq, f32=f32).cpu().numpy()
        e = pdfmi.error_count(reset=True)
        assert s.view(np.uint64)[0] == s_ref.view(np.uint64)[0], (s, s_ref)
        assert e == e_ref
        assert np.isnan(s[0]) == (mixed == "invalid" and n > 10)
    finally:
        pdfmi.unload(m)


def test_fused_matches_oracle_and_empty():
    g = synth.config1_grid()
    qk, a = synth.config1_alphas()
    m = pdfmi.load_synth(g)
    pdfmi.load_alphas(qk, a)
    try:
        x1, x2, q2 = synth.config5_chunk(4, n=100_000)
        s = pdfmi.mc_fused(m, PIDS, dev(x1), dev(x2), dev(q2)).item()
        so, sabs = oracle_chunk(g, qk, a, x1, x2, q2)
        assert abs(s - so) <= 1e-11 * sabs, (s, so)
        e = torch.empty(0, dtype=torch.float64, device=DEV)
        assert pdfmi.mc_fused(m, PIDS, e, e, e).item() == 0.0
    finally:
        pdfmi.unload(m)


def test_fused_large_grid_reads_global():
    """config-2 grid: too large for LDS, the fused kernel reads it from global memory."""
    g = synth.config2_grid()
    qk, a = synth.config2_alphas()
    m = pdfmi.load_synth(g)
    pdfmi.load_alphas(qk, a)
    try:
        x, q2 = synth.config2_queries(n=60_000, seed=12)
        x2 = np.roll(x, 7)
        d1, d2, dq = dev(x), dev(x2), dev(q2)
        for f32 in (False, True):
            ev = pdfmi.xfxq2_f32 if f32 else pdfmi.xfxq2
            s_ref = pdfmi.mc_chunk_sum(ev(m, g.pids, d1, dq), ev(m, g.pids, d2, dq), pdfmi.alphas_q2(dq)).cpu().numpy()
            s = pdfmi.mc_fused(m, g.pids, d1, d2, dq, f32=f32).cpu().numpy()
            assert s.view(np.uint64)[0] == s_ref.view(np.uint64)[0], (f32, s, s_ref)
    finally:
        pdfmi.unload(m)


# Requests whose stored columns fall into the 16-byte column groups of the
# LDS-staged grid in every way: whole groups in order, groups entered at an
# odd column, reversed order, a column repeated (0 and 21 are both the gluon),
# absent flavours between stored ones, single flavours.
GROUP_REQUESTS = {
    "reversed": PIDS[::-1],
    "odd_start": [-4, -3, -2, -1, 21, 1, 2],
    "repeat": [21, 0, 21, 1, 1, -1],
    "absent_between": [-5, 6, -4, -3, -6, -2, -6, -1],
    "swapped_pairs": [-4, -5, -2, -3, 21, -1, 2, 1],
    "single": [3],
    "single_absent": [6],
    "max_request": (PIDS * 5)[:64],  # the most flavours one call takes: every step slot in use
}


@pytest.mark.parametrize("name", sorted(GROUP_REQUESTS))
@pytest.mark.parametrize("f32", [False, True])
def test_fused_column_group_requests(name, f32):
    """The fused sum reads the staged grid a column group at a time and
    applies the request's flavours in request order: bit-identical to the
    unfused calls for every way a request can fall into the groups, with
    extrapolated and invalid points mixed in."""
    g = synth.config1_grid()
    qk, a = synth.config1_alphas()
    m = pdfmi.load_synth(g)
    pdfmi.load_alphas(qk, a)
    plist = GROUP_REQUESTS[name]
    try:
        ev = pdfmi.xfxq2_f32 if f32 else pdfmi.xfxq2
        for invalid in (False, True):
            x1, x2, q2 = _mixed_chunk(20_000, 17, invalid=invalid)
            d1, d2, dq = dev(x1), dev(x2), dev(q2)
            s_ref = pdfmi.mc_chunk_sum(ev(m, plist, d1, dq), ev(m, plist, d2, dq),
                                       pdfmi.alphas_q2(dq)).cpu().numpy()
            s = pdfmi.mc_fused(m, plist, d1, d2, dq, f32=f32).cpu().numpy()
            assert s.view(np.uint64)[0] == s_ref.view(np.uint64)[0], (invalid, s, s_ref)
            # an invalid point's values are NaN, also for flavours absent from the grid
            assert np.isnan(s[0]) == invalid
            assert invalid or name == "single_absent" or s[0] != 0.0
    finally:
        pdfmi.unload(m)


def test_fused_unpadded_lds_rows():
    """A 60 x 53-knot, 11-flavour grid: in FP32 its rows padded to 12 columns
    (152.6 KB) and the other LDS contents exceed 160 KB, rows of 11 columns
    (139.9 KB) do not, so the fused kernel reads one column at a time from
    the grid staged in LDS; in FP64 the grid (280 KB) is read from global
    memory.  Both bit-identical to the unfused calls."""
    g = synth.tiny_grid(np.random.default_rng(60), K=1, nx=60, nq=53, npid=11)
    qk, a = synth.config1_alphas()
    m = pdfmi.load_synth(g)
    pdfmi.load_alphas(qk, a)
    try:
        r = np.random.default_rng(5)
        n = 30_000
        lx0 = np.log(g.xknots[0][0])
        x1 = np.exp(r.uniform(lx0 - 1.0, 0.0, n))
        x2 = np.exp(r.uniform(lx0 - 1.0, 0.0, n))
        q2 = np.exp(r.uniform(np.log(g.q2knots[0][0]) - 0.5, np.log(g.q2knots[0][-1]) + 0.5, n))
        d1, d2, dq = dev(x1), dev(x2), dev(q2)
        for f32 in (False, True):
            for plist in (list(g.pids), [int(p) for p in g.pids[::-1]] + [0]):
                ev = pdfmi.xfxq2_f32 if f32 else pdfmi.xfxq2
                s_ref = pdfmi.mc_chunk_sum(ev(m, plist, d1, dq), ev(m, plist, d2, dq),
                                           pdfmi.alphas_q2(dq)).cpu().numpy()
                s = pdfmi.mc_fused(m, plist, d1, d2, dq, f32=f32).cpu().numpy()
                assert s.view(np.uint64)[0] == s_ref.view(np.uint64)[0], (f32, plist, s, s_ref)
    finally:
        pdfmi.unload(m)


@pytest.mark.parametrize("P", [1, 13, 40, 64])
@pytest.mark.parametrize("f32", [False, True])
def test_chunk_sum_any_width(P, f32):
    """Widths that stage rows in LDS and widths that read them directly."""
    rng = np.random.default_rng(P + 100 * f32)
    n = 5000
    a = rng.normal(size=(n, P))
    b = rng.normal(size=(n, P))
    w = rng.uniform(0.1, 0.3, n)
    if f32:
        a, b = a.astype(np.float32), b.astype(np.float32)
    ta = torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    tb = torch.from_numpy(np.ascontiguousarray(b)).to(DEV)
    s1 = pdfmi.mc_chunk_sum(ta, tb, dev(w)).item()
    s2 = pdfmi.mc_chunk_sum(ta, tb, dev(w)).item()
    assert s1 == s2
    terms = w * np.sum(a.astype(np.float64) * b.astype(np.float64), axis=1)
    ref = math.fsum(terms)
    scale = math.fsum(np.abs(w) * np.sum(np.abs(a.astype(np.float64) * b.astype(np.float64)), axis=1))
    assert abs(s1 - ref) <= 1e-12 * scale


def test_full_workload_fused_equals_unfused():
    """The benchmarked load: 100 chunks of 1e6 points (1e8 points), every
    chunk sum of the fused kernel bit-identical to the unfused calls, FP64
    and FP32 (whose fused kernel reads four flavours per LDS access), and the
    FP64 total within the summation bound of the oracle on three chunks."""
    g = synth.config1_grid()
    qk, a = synth.config1_alphas()
    m = pdfmi.load_synth(g)
    pdfmi.load_alphas(qk, a)
    try:
        n = 1_000_000
        ws = pdfmi.mc_workspace(n, DEV)
        f = {dt: (torch.empty((n, len(PIDS)), dtype=dt, device=DEV), torch.empty((n, len(PIDS)), dtype=dt, device=DEV))
             for dt in (torch.float64, torch.float32)}
        al = torch.empty(n, dtype=torch.float64, device=DEV)
        unf = {k: torch.empty(100, dtype=torch.float64, device=DEV) for k in ("f64", "f32")}
        fus = {k: torch.empty(100, dtype=torch.float64, device=DEV) for k in ("f64", "f32")}
        for c in range(100):
            x1, x2, q2 = (dev(v) for v in synth.config5_chunk(c))
            pdfmi.alphas_q2(q2, out=al)
            for key, dt, ev in (("f64", torch.float64, pdfmi.xfxq2), ("f32", torch.float32, pdfmi.xfxq2_f32)):
                f1, f2 = f[dt]
                ev(m, PIDS, x1, q2, out=f1)
                ev(m, PIDS, x2, q2, out=f2)
                pdfmi.mc_chunk_sum(f1, f2, al, workspace=ws, out=unf[key][c:c + 1])
                pdfmi.mc_fused(m, PIDS, x1, x2, q2, f32=(key == "f32"), workspace=ws, out=fus[key][c:c + 1])
        for key in ("f64", "f32"):
            assert torch.equal(unf[key].view(torch.int64), fus[key].view(torch.int64)), key
        got = fus["f64"].cpu().numpy()
        for c in (0, 57, 99):
            s, absum = oracle_chunk(g, qk, a, *synth.config5_chunk(c))
            assert abs(got[c] - s) <= 1e-11 * absum, c
    finally:
        pdfmi.unload(m)
