"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Sizes: a few tiles with a ragged tail for full parity; the full 1e7-point
workload with sampled outputs checked one by one against the oracle.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2009_06635_amd import synth
from tolerance import check_f32, check_f64, describe_failures, grid_L

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2009_06635_amd import pdfmi  # noqa: E402  (fails loudly if the library is missing)

DEV = "cuda:0"


def ogrid(g):
    return oracle.Grid(g.xknots, g.q2knots, g.values, g.pids)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(DEV)


def edge_queries(g, rng, n_rand=3000):
    """Random points over and around the grid plus every knot, its float
    neighbours, thresholds, x_max, extrapolation regions and invalid inputs."""
    xk0 = g.xknots[0]
    qlo, qhi = g.q2knots[0][0], g.q2knots[-1][-1]
    x = list(np.exp(rng.uniform(np.log(xk0[0]) - 3.0, 0.0, n_rand)))
    q = list(np.exp(rng.uniform(np.log(qlo) - 2.0, np.log(qhi) + 2.0, n_rand)))
    qpts = sorted(set(np.concatenate(g.q2knots).tolist()))
    xs = xk0[:: max(1, len(xk0) // 12)].tolist() + [xk0[0], xk0[1], xk0[-2], xk0[-1]]
    for xv in xs:
        for qv in qpts[:: max(1, len(qpts) // 10)] + [qlo, qhi] + [qk[0] for qk in g.q2knots]:
            for dx in (xv, np.nextafter(xv, 0.0), np.nextafter(xv, 2.0)):
                for dq in (qv, np.nextafter(qv, 0.0), np.nextafter(qv, np.inf)):
                    x.append(dx)
                    q.append(dq)
    x += [0.0, -1.0, np.nan, 1.5, np.inf, 0.5, 0.5, 0.5, np.nextafter(1.0, 2.0)]
    q += [10.0, 10.0, 10.0, 10.0, 10.0, 0.0, -5.0, np.nan, 10.0]
    return np.array(x), np.array(q)


def run_parity(member, g, pids, x, q2, f32=False):
    og = ogrid(g)
    ora, scale = oracle.xfxq2(og, pids, x, q2, with_scale=True)
    xd, qd = dev(x), dev(q2)
    if f32:
        out = pdfmi.xfxq2_f32(member, pids, xd, qd).cpu().numpy()
        ok, lit, mx = check_f32(out, ora, scale)
    else:
        out = pdfmi.xfxq2(member, pids, xd, qd).cpu().numpy()
        ok, lit, mx = check_f64(out, ora, scale, grid_L(g))
    assert ok.all(), describe_failures(ok, out, ora, x, q2, pids)
    return out, ora, lit, mx


@pytest.fixture(scope="module")
def cfg1():
    g = synth.config1_grid()
    m = pdfmi.load_synth(g)
    yield g, m
    pdfmi.unload(m)


@pytest.fixture(scope="module")
def cfg2():
    g = synth.config2_grid()
    m = pdfmi.load_synth(g)
    yield g, m
    pdfmi.unload(m)


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["cfg1", "cfg2"])
def test_locate_bit_exact(which, request):
    g, m = request.getfixturevalue(which)
    rng = np.random.default_rng(1)
    x, q2 = edge_queries(g, rng)
    k, ix, iq, reg = pdfmi.locate(m, dev(x), dev(q2))
    ok_, oix, oiq, oreg = oracle.locate(ogrid(g), x, q2)
    assert np.array_equal(k.cpu().numpy(), ok_)
    assert np.array_equal(ix.cpu().numpy(), oix)
    assert np.array_equal(iq.cpu().numpy(), oiq)
    assert np.array_equal(reg.cpu().numpy(), oreg)


@pytest.mark.parametrize("which", ["cfg1", "cfg2"])
@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("vec", [0, 1])
def test_xfxq2_parity_edges(which, f32, vec, request):
    g, m = request.getfixturevalue(which)
    rng = np.random.default_rng(2)
    x, q2 = edge_queries(g, rng)
    pdfmi.set_lds_policy(1)
    pdfmi.set_tuning(pdfmi.TUNE_VECTOR_COLUMNS, vec)
    try:
        _, _, lit, mx = run_parity(m, g, g.pids, x, q2, f32=f32)
    finally:
        pdfmi.set_lds_policy(0)
        pdfmi.set_tuning(pdfmi.TUNE_VECTOR_COLUMNS, 1)
    print("literal pass fraction %.6f, max eq.(1) %.3g" % (lit, mx))


@pytest.mark.parametrize("f32", [False, True])
def test_xfxq2_parity_ragged_tiles(cfg2, f32):
    g, m = cfg2
    for n in (1, 255, 257, 4099):
        x, q2 = synth.config2_queries(n=n, seed=300 + n, out_fraction=0.05)
        run_parity(m, g, g.pids, x, q2, f32=f32)


@pytest.mark.parametrize("f32", [False, True])
def test_knots_bit_exact(cfg2, f32):
    g, m = cfg2
    for k in range(g.K):
        xs, qs = np.meshgrid(g.xknots[k], g.q2knots[k], indexing="ij")
        x, q2 = xs.ravel(), qs.ravel()
        if f32:
            out = pdfmi.xfxq2_f32(m, g.pids, dev(x), dev(q2)).cpu().numpy()
        else:
            out = pdfmi.xfxq2(m, g.pids, dev(x), dev(q2)).cpu().numpy()
        want = g.values[k].reshape(-1, len(g.pids)).copy()
        if k + 1 < g.K:   # threshold row served by the upper sub-grid
            top = q2 == g.q2knots[k][-1]
            want[top] = g.values[k + 1][:, 0, :]
        if f32:
            want = want.astype(np.float32)
        assert np.array_equal(out, want)


def test_lds_staged_grid_matches_global(cfg1):
    g, m = cfg1
    x, q2 = synth.config1_queries(n=70_000, seed=5)
    xd, qd = dev(x), dev(q2)
    outs = {}
    for pol in (1, 2):
        pdfmi.set_lds_policy(pol)
        outs[pol] = (pdfmi.xfxq2(m, g.pids, xd, qd).cpu().numpy(), pdfmi.xfxq2_f32(m, g.pids, xd, qd).cpu().numpy())
    pdfmi.set_lds_policy(0)
    assert np.array_equal(outs[1][0], outs[2][0])
    assert np.array_equal(outs[1][1], outs[2][1])
    ora, scale = oracle.xfxq2(ogrid(g), g.pids, x, q2, with_scale=True)
    assert check_f64(outs[2][0], ora, scale, grid_L(g))[0].all()
    assert check_f32(outs[2][1], ora, scale)[0].all()


def test_tables_in_place_below_threshold_match_staged(cfg2):
    """Calls under 32 768 points read the location tables in place, larger ones
    stage them in LDS per workgroup: the same points give bit-identical values."""
    g, m = cfg2
    n = 32_768
    x, q2 = synth.config2_queries(n=n, seed=13, out_fraction=0.05)
    xd, qd = dev(x), dev(q2)
    pdfmi.load_alphas(*synth.config2_alphas())
    big, a_big = pdfmi.xfxq2_alphas(m, g.pids, xd, qd)
    small, a_small = pdfmi.xfxq2_alphas(m, g.pids, xd[:n - 1], qd[:n - 1])
    assert torch.equal(big[:n - 1], small)
    assert torch.equal(a_big[:n - 1], a_small)
    assert torch.equal(pdfmi.xfxq2(m, g.pids, xd[:n - 1], qd[:n - 1]), small)
    sub = g.pids[::2]
    big32 = pdfmi.xfxq2_f32(m, sub, xd, qd)
    assert torch.equal(big32[:n - 1], pdfmi.xfxq2_f32(m, sub, xd[:n - 1], qd[:n - 1]))
    ora, scale = oracle.xfxq2(ogrid(g), g.pids, x[:4096], q2[:4096], with_scale=True)
    assert check_f64(small[:4096].cpu().numpy(), ora, scale, grid_L(g))[0].all()


@pytest.mark.parametrize("seed", range(8))
def test_tiny_grids_all_regions(seed):
    rng = np.random.default_rng(500 + seed)
    K = 1 + seed % 3
    nx = [2, 3, 4, 5, 6, 7, 3, 9][seed]
    nq = [[2, 3, 4, 5][(seed + k) % 4] for k in range(K)]
    g = synth.tiny_grid(rng, K=K, nx=nx, nq=nq, npid=3)
    if seed % 2:
        g = g.with_values([np.abs(v) + 0.01 for v in g.values])
    m = pdfmi.load_synth(g)
    try:
        x, q2 = edge_queries(g, rng, n_rand=800)
        for f32 in (False, True):
            for pol in (1, 2):
                for vec in (0, 1):
                    pdfmi.set_lds_policy(pol)
                    pdfmi.set_tuning(pdfmi.TUNE_VECTOR_COLUMNS, vec)
                    run_parity(m, g, g.pids, x, q2, f32=f32)
    finally:
        pdfmi.set_lds_policy(0)
        pdfmi.set_tuning(pdfmi.TUNE_VECTOR_COLUMNS, 1)
        pdfmi.unload(m)


def test_pid_subsets_and_absent_flavours(cfg1):
    g, m = cfg1
    x, q2 = synth.config1_queries(n=3000, seed=9)
    for pids in ([21], [0, 21, 2, 2], [-6, 6, 1], [5, -5, 4, -4, 3, -3, 2, -2, 1, -1, 21]):
        out, ora, _, _ = run_parity(m, g, pids, x, q2)
        for j, p in enumerate(pids):
            if abs(p) == 6:
                assert np.all(out[:, j] == 0.0)
    with pytest.raises(pdfmi.PdfError) as e:
        pdfmi.xfxq2(m, [7], dev(x), dev(q2))
    assert e.value.code == pdfmi.PDF_ERR_PID


def test_all_pids_null_request(cfg2):
    g, m = cfg2
    x, q2 = synth.config2_queries(n=2000, seed=10)
    out = pdfmi.xfxq2(m, None, dev(x), dev(q2), n_cols=len(g.pids)).cpu().numpy()
    ora, scale = oracle.xfxq2(ogrid(g), g.pids, x, q2, with_scale=True)
    assert check_f64(out, ora, scale, grid_L(g))[0].all()


def test_invalid_points_counted(cfg1):
    g, m = cfg1
    pdfmi.error_count(reset=True)
    x = np.array([0.1, 0.0, -1.0, np.nan, 2.0, 0.2])
    q2 = np.array([10.0, 10.0, 10.0, 10.0, 10.0, -1.0])
    out = pdfmi.xfxq2(m, g.pids, dev(x), dev(q2)).cpu().numpy()
    assert np.all(np.isfinite(out[0])) and np.all(np.isnan(out[1:]))
    assert pdfmi.error_count(reset=True) == 5
    pdfmi.load_alphas(*synth.config1_alphas())
    pdfmi.alphas_q2(dev(np.array([0.0, 5.0, np.nan])))
    assert pdfmi.error_count(reset=True) == 2


def test_empty_call_is_noop(cfg1):
    g, m = cfg1
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    out = pdfmi.xfxq2(m, g.pids, e, e)
    assert out.shape == (0, len(g.pids))


def test_deterministic(cfg2):
    g, m = cfg2
    x, q2 = synth.config2_queries(n=100_000, seed=11)
    xd, qd = dev(x), dev(q2)
    a = pdfmi.xfxq2(m, g.pids, xd, qd)
    b = pdfmi.xfxq2(m, g.pids, xd, qd)
    assert torch.equal(a, b)


@pytest.mark.parametrize("which", ["cfg1", "cfg2"])
def test_alphas_parity(which):
    qk, a = synth.config1_alphas() if which == "cfg1" else synth.config2_alphas()
    pdfmi.load_alphas(qk, a)
    rng = np.random.default_rng(12)
    q2 = np.concatenate([np.exp(rng.uniform(np.log(qk[0]) - 2, np.log(qk[-1]) + 2, 20000)), qk,
                         np.nextafter(qk, 0), np.nextafter(qk, np.inf), [0.0, -1.0, np.nan]])
    out = pdfmi.alphas_q2(dev(q2)).cpu().numpy()
    ora = oracle.alphas_q2(qk, a, q2)
    assert np.array_equal(np.isnan(out), np.isnan(ora))
    f = ~np.isnan(ora)
    assert np.max(np.abs(out[f] - ora[f]) / np.abs(ora[f])) < 1e-13
    # knots bit-exact
    assert np.array_equal(pdfmi.alphas_q2(dev(qk)).cpu().numpy(), ora[20000:20000 + len(qk)])


def test_full_size_sampled_config2(cfg2):
    """The 1e7-point workload in the launch configuration the benchmark times;
    outputs at sampled points checked against the oracle one by one."""
    g, m = cfg2
    x, q2 = synth.config2_queries()
    xd, qd = dev(x), dev(q2)
    out64 = pdfmi.xfxq2(m, g.pids, xd, qd)
    out32 = pdfmi.xfxq2_f32(m, g.pids, xd, qd)
    rng = np.random.default_rng(13)
    idx = np.concatenate([rng.choice(len(x), 20000, replace=False), [0, len(x) - 1]])
    idx_t = torch.from_numpy(idx).to(DEV)
    s64 = out64[idx_t].cpu().numpy()
    s32 = out32[idx_t].cpu().numpy()
    ora, scale = oracle.xfxq2(ogrid(g), g.pids, x[idx], q2[idx], with_scale=True)
    ok, lit, mx = check_f64(s64, ora, scale, grid_L(g))
    assert ok.all(), describe_failures(ok, s64, ora, x[idx], q2[idx], g.pids)
    ok32, lit32, mx32 = check_f32(s32, ora, scale)
    assert ok32.all(), describe_failures(ok32, s32, ora, x[idx], q2[idx], g.pids)
    # properties over the whole output: every valid point finite, heavy flavours zero below thresholds
    assert bool(torch.isfinite(out64).all())
    j6 = g.pids.index(6)
    assert bool((out64[:, j6] == 0).all())
    print("full-size sampled: literal FP64 pass %.6f (max %.3g), FP32 %.6f (max %.3g)" % (lit, mx, lit32, mx32))


def test_outputs_beyond_4_gib(cfg2):
    """42e6 points x 13 flavours: the FP64 output spans 4.4 GB, so rows past
    the first 4 GiB are addressed through 64-bit offsets; sampled rows there
    (and at the start) are checked against the oracle, for x*f, the fused
    alpha_s output and FP32."""
    g, m = cfg2
    n = 42_000_000
    x, q2 = synth.config2_queries(n=n, seed=14)
    xd, qd = dev(x), dev(q2)
    pdfmi.load_alphas(*synth.config2_alphas())
    out64, a = pdfmi.xfxq2_alphas(m, g.pids, xd, qd)
    assert out64.numel() * 8 > 2 ** 32
    first_far = 2 ** 32 // (8 * len(g.pids)) + 1
    rng = np.random.default_rng(15)
    idx = np.concatenate([rng.integers(first_far, n, 3000), rng.integers(0, first_far, 1000), [n - 1, first_far]])
    idx_t = torch.from_numpy(idx).to(DEV)
    s64 = out64[idx_t].cpu().numpy()
    sa = a[idx_t].cpu().numpy()
    del out64, a
    out32 = pdfmi.xfxq2_f32(m, g.pids, xd, qd)
    s32 = out32[idx_t].cpu().numpy()
    del out32
    ora, scale = oracle.xfxq2(ogrid(g), g.pids, x[idx], q2[idx], with_scale=True)
    ok = check_f64(s64, ora, scale, grid_L(g))[0]
    assert ok.all(), describe_failures(ok, s64, ora, x[idx], q2[idx], g.pids)
    ok32 = check_f32(s32, ora, scale)[0]
    assert ok32.all(), describe_failures(ok32, s32, ora, x[idx], q2[idx], g.pids)
    qk, av = synth.config2_alphas()
    oa = oracle.alphas_q2(qk, av, q2[idx])
    assert np.max(np.abs(sa - oa) / np.abs(oa)) < 1e-13


def test_extreme_but_valid_inputs(cfg2):
    """Subnormal and huge (but valid) x and Q^2: far extrapolation on both
    sides; values compared where the oracle is finite and moderate, and the
    two sides agree on which results are finite."""
    g, m = cfg2
    xs = np.array([5e-324, 1e-310, 1e-300, 1e-200, 1e-100, 1e-20, 1e-12, 0.999999, 1.0])
    qs = np.array([5e-324, 1e-300, 1e-100, 1e-10, 0.25, 10.0, 1e20, 1e100, 1e300])
    x, q2 = np.meshgrid(xs, qs, indexing="ij")
    x, q2 = x.ravel(), q2.ravel()
    out = pdfmi.xfxq2(m, g.pids, dev(x), dev(q2)).cpu().numpy()
    ora, scale = oracle.xfxq2(ogrid(g), g.pids, x, q2, with_scale=True)
    assert np.array_equal(np.isfinite(out), np.isfinite(ora))
    sel = np.isfinite(ora) & (np.abs(ora) < 1e250) & np.isfinite(scale) & (scale < 1e250)
    ok = check_f64(out, ora, scale, grid_L(g))[0] | ~sel
    assert ok.all(), describe_failures(ok, out, ora, x, q2, g.pids)
    # FP32 arithmetic: compared where the value and its scale stay well inside the FP32 range
    out32 = pdfmi.xfxq2_f32(m, g.pids, dev(x), dev(q2)).cpu().numpy()
    sel32 = sel & (np.abs(ora) < 1e30) & (scale < 1e30)
    ok32 = check_f32(out32, ora, scale)[0] | ~sel32
    assert ok32.all(), describe_failures(ok32, out32, ora, x, q2, g.pids)
    print("extreme inputs: %d of %d values compared (FP32: %d)" % (sel.sum(), sel.size, sel32.sum()))
