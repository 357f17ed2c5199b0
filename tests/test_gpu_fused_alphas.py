"""x*f and alpha_s at the same points in one launch (pdf_xfxq2_alphas /
pdf_xfxq2_alphas_f32) against the two separate calls: both outputs must be
bit-identical to pdf_xfxq2 (or _f32) and pdf_alpha_q2, in each launch shape
(grid staged in LDS, location tables staged, everything from global memory),
and invalid points counted as the two separate calls count them.  The
separate calls are themselves held to the oracle by the parity tests; the
fused outputs are also checked against the oracle here.
"""
import numpy as np
import pytest

import oracle
from paper_2009_06635_amd import synth
from tolerance import check_f32, check_f64, describe_failures, grid_L

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2009_06635_amd import pdfmi  # noqa: E402

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(DEV)


def big_table_grid():
    """Two sub-grids with their own dense x tables: the location tables exceed
    the LDS budget, so the kernel reads them from global memory."""
    rng = np.random.default_rng(77)
    xks = [np.exp(np.linspace(np.log(1e-7), 0.0, 700)), np.exp(np.linspace(np.log(1e-7), 0.0, 811))]
    qks = [synth.logspace_q2(1.65, 4.92, 12), synth.logspace_q2(4.92, 1e4, 20)]
    # smooth positive values (x^-b (1.01 - x)^c times a slow log Q^2 rise, 0.1% noise): the
    # extrapolated values stay within FP32 range
    b, c = np.linspace(0.1, 0.3, 5), np.linspace(1.0, 4.0, 5)
    vals = []
    for k in range(2):
        xs, qs = np.meshgrid(xks[k], qks[k], indexing="ij")
        base = [xs ** -b[j] * (1.01 - xs) ** c[j] * (1.0 + 0.05 * np.log(qs)) for j in range(5)]
        vals.append(np.stack(base, axis=-1) * (1.0 + 1e-3 * rng.standard_normal((len(xks[k]), len(qks[k]), 5))))
    return synth.SynthGrid(xks, qks, vals, [-1, 1, 2, 21, 5])


def queries(g, rng, n):
    xk0 = g.xknots[0]
    qlo, qhi = g.q2knots[0][0], g.q2knots[-1][-1]
    x = np.exp(rng.uniform(np.log(xk0[0]) - 2.0, 0.0, n))
    q2 = np.exp(rng.uniform(np.log(qlo) - 2.0, np.log(qhi) + 2.0, n))
    qk = np.concatenate(g.q2knots)
    q2[: len(qk)] = qk  # every Q^2 knot, thresholds included
    bad_x = [0.0, -1.0, np.nan, 1.5, 0.5, 0.5, 0.5, 0.5]
    bad_q = [10.0, 10.0, 10.0, 10.0, 0.0, -5.0, np.nan, np.inf]
    return np.concatenate([x, bad_x]), np.concatenate([q2, bad_q])


def separate(m, pids, xd, qd, f32):
    pdfmi.error_count(reset=True)
    out = (pdfmi.xfxq2_f32 if f32 else pdfmi.xfxq2)(m, pids, xd, qd)
    a = pdfmi.alphas_q2(qd)
    return out.cpu().numpy(), a.cpu().numpy(), pdfmi.error_count(reset=True)


def fused(m, pids, xd, qd, f32):
    pdfmi.error_count(reset=True)
    out, a = pdfmi.xfxq2_alphas(m, pids, xd, qd, f32=f32)
    return out.cpu().numpy(), a.cpu().numpy(), pdfmi.error_count(reset=True)


def same(a, b):
    return np.array_equal(a.view(np.uint64) if a.dtype == np.float64 else a.view(np.uint32),
                          b.view(np.uint64) if b.dtype == np.float64 else b.view(np.uint32))


@pytest.fixture(scope="module")
def grids():
    gs = {"cfg1": synth.config1_grid(), "cfg2": synth.config2_grid(), "big_tables": big_table_grid()}
    ms = {k: pdfmi.load_synth(g) for k, g in gs.items()}
    yield gs, ms
    for m in ms.values():
        pdfmi.unload(m)


@pytest.mark.parametrize("which,policy", [("cfg1", 1), ("cfg1", 2), ("cfg2", 0), ("big_tables", 0)])
@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("vec", [0, 1])
def test_fused_matches_separate_and_oracle(grids, which, policy, f32, vec):
    gs, ms = grids
    g, m = gs[which], ms[which]
    qk, av = synth.config2_alphas() if which == "cfg2" else synth.config1_alphas()
    pdfmi.load_alphas(qk, av)
    rng = np.random.default_rng(900 + len(which) + policy)
    x, q2 = queries(g, rng, 6000)
    xd, qd = dev(x), dev(q2)
    pdfmi.set_lds_policy(policy)
    pdfmi.set_tuning(pdfmi.TUNE_VECTOR_COLUMNS, vec)
    try:
        s_out, s_a, s_err = separate(m, g.pids, xd, qd, f32)
        f_out, f_a, f_err = fused(m, g.pids, xd, qd, f32)
    finally:
        pdfmi.set_lds_policy(0)
        pdfmi.set_tuning(pdfmi.TUNE_VECTOR_COLUMNS, 1)
    assert same(f_out, s_out)
    assert same(f_a, s_a)
    assert f_err == s_err and f_err == 8 + 4  # 8 invalid (x, Q^2) points for x*f, 4 invalid Q^2 for alpha_s
    ora, scale = oracle.xfxq2(oracle.Grid(g.xknots, g.q2knots, g.values, g.pids), g.pids, x, q2, with_scale=True)
    ok = check_f32(f_out, ora, scale)[0] if f32 else check_f64(f_out, ora, scale, grid_L(g))[0]
    assert ok.all(), describe_failures(ok, f_out, ora, x, q2, g.pids)
    oa = oracle.alphas_q2(qk, av, q2)
    assert np.array_equal(np.isnan(f_a), np.isnan(oa))
    fin = ~np.isnan(oa)
    assert np.max(np.abs(f_a[fin] - oa[fin]) / np.abs(oa[fin])) < 1e-13


@pytest.mark.parametrize("n", [1, 63, 65, 4099])
def test_fused_ragged_and_subsets(grids, n):
    gs, ms = grids
    g, m = gs["cfg2"], ms["cfg2"]
    pdfmi.load_alphas(*synth.config2_alphas())
    x, q2 = synth.config2_queries(n=n, seed=910 + n, out_fraction=0.05)
    xd, qd = dev(x), dev(q2)
    for pids in (g.pids, [21, 2, -2], [5]):
        for f32 in (False, True):
            s_out, s_a, _ = separate(m, pids, xd, qd, f32)
            f_out, f_a, _ = fused(m, pids, xd, qd, f32)
            assert same(f_out, s_out) and same(f_a, s_a), (pids, f32)


def test_fused_full_size(grids):
    """The 1e7-point workload in the benchmark's launch configuration: fused
    outputs bit-identical to the separate calls over every point."""
    gs, ms = grids
    g, m = gs["cfg2"], ms["cfg2"]
    pdfmi.load_alphas(*synth.config2_alphas())
    x, q2 = synth.config2_queries()
    xd, qd = dev(x), dev(q2)
    out, a = pdfmi.xfxq2_alphas(m, g.pids, xd, qd)
    assert torch.equal(out, pdfmi.xfxq2(m, g.pids, xd, qd))
    assert torch.equal(a, pdfmi.alphas_q2(qd))


def test_fused_arguments(grids):
    gs, ms = grids
    g, m = gs["cfg1"], ms["cfg1"]
    pdfmi.load_alphas(*synth.config1_alphas())
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    out, a = pdfmi.xfxq2_alphas(m, g.pids, e, e)
    assert out.shape == (0, len(g.pids)) and a.shape == (0,)
    xd = dev(np.array([0.1]))
    o = torch.empty((1, len(g.pids)), dtype=torch.float64, device=DEV)
    rc = pdfmi.library().pdf_xfxq2_alphas(int(m), None, 0, xd.data_ptr(), xd.data_ptr(), 1, o.data_ptr(), None,
                                          None)
    assert rc == pdfmi.PDF_ERR_ARG


def test_fused_call_in_a_captured_graph(grids):
    """The fused call recorded into a HIP graph (torch.cuda.graph) and replayed
    with eager work between the replays: every replay equals the eager call."""
    gs, ms = grids
    g, m = gs["cfg2"], ms["cfg2"]
    pdfmi.load_alphas(*synth.config2_alphas())
    x, q2 = synth.config2_queries(n=300_000, seed=950, out_fraction=0.05)
    xd, qd = dev(x), dev(q2)
    want_o, want_a = pdfmi.xfxq2_alphas(m, g.pids, xd, qd)
    o = torch.empty_like(want_o)
    a = torch.empty_like(want_a)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pdfmi.xfxq2_alphas(m, g.pids, xd, qd, out=o, alphas_out=a)   # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pdfmi.xfxq2_alphas(m, g.pids, xd, qd, out=o, alphas_out=a)
    for rep in range(4):
        o.fill_(float(rep))
        a.fill_(float(rep))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(torch.nan_to_num(o, nan=7.0), torch.nan_to_num(want_o, nan=7.0)), rep
        assert torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(want_a, nan=7.0)), rep
