"""Property-based parity of the HIP path with the oracle: hypothesis draws
small grids (sub-grid count, knot counts, stored flavour count, values from a
seed, values of mixed sign or positive) and a flavour request, and for every
draw, on points over and around the grid (every knot and its float
neighbours, thresholds, every extrapolation region, invalid inputs):
  * sub-grid, cell indices and region bits equal the oracle's bit for bit;
  * FP64 values meet the FP64 criterion and FP32 values the FP32 one, with the
    grid read from global memory and staged in LDS.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, example, given, settings
from hypothesis import strategies as st

import oracle
from paper_2009_06635_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2009_06635_amd import pdfmi  # noqa: E402
from test_gpu_parity import dev, edge_queries, run_parity  # noqa: E402

DEV = "cuda:0"

# (sub-grids, x knots, Q^2 knots per sub-grid, stored flavours, seed of knots and values)
shapes = st.tuples(st.integers(1, 3), st.integers(2, 9), st.lists(st.integers(2, 7), min_size=3, max_size=3),
                   st.integers(1, 13), st.integers(0, 2**31 - 1))


@settings(max_examples=25, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(shapes, st.booleans(), st.integers(0, 2**31 - 1))
@example(shape=(1, 2, [7, 2, 2], 9, 168040), positive=False, qseed=0)  # FP32 overflow below Q^2_min
def test_drawn_grids_match_oracle(shape, positive, qseed):
    K, nx, nqs, npid, seed = shape
    g = synth.tiny_grid(np.random.default_rng(seed), K=K, nx=nx, nq=nqs[:K], npid=npid)
    if positive:  # positive values: the power-law extrapolation branches
        g = g.with_values([np.abs(v) + 0.01 for v in g.values])
    r = np.random.default_rng(qseed)
    x, q2 = edge_queries(g, r, n_rand=400)
    # every stored flavour, or a drawn subset with a repeat and the gluon's alias 0
    pids = list(g.pids) if qseed % 2 else [int(p) for p in r.permutation(g.pids)[: max(1, npid // 2)]] + [0]
    m = pdfmi.load_synth(g)
    try:
        og = oracle.Grid(g.xknots, g.q2knots, g.values, g.pids)
        k, ix, iq, reg = pdfmi.locate(m, dev(x), dev(q2))
        ok_, oix, oiq, oreg = oracle.locate(og, x, q2)
        assert np.array_equal(k.cpu().numpy(), ok_)
        assert np.array_equal(ix.cpu().numpy(), oix)
        assert np.array_equal(iq.cpu().numpy(), oiq)
        assert np.array_equal(reg.cpu().numpy(), oreg)
        for policy in (1, 2):  # grid read from global memory, grid staged in LDS
            pdfmi.set_lds_policy(policy)
            for f32 in (False, True):
                run_parity(m, g, pids, x, q2, f32=f32)
    finally:
        pdfmi.set_lds_policy(0)
        pdfmi.unload(m)


@settings(max_examples=25, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(st.lists(st.integers(2, 12), min_size=1, max_size=3), st.integers(0, 2**31 - 1))
def test_drawn_alphas_tables_match_oracle(seg_sizes, seed):
    """alpha_s tables of 1-3 segments (a segment starts at a repeated knot, a
    flavour threshold): values within 1e-13 of the oracle at points over and
    around the table, knots bit-exact, NaN for invalid Q^2."""
    r = np.random.default_rng(seed)
    knots, vals = [], []
    q = float(np.exp(r.uniform(0.0, 1.0)))
    for m in seg_sizes:
        seg = [q] + list(q * np.exp(np.cumsum(r.uniform(0.1, 1.5, m - 1))))
        knots += seg
        vals += list(r.uniform(0.05, 0.4, m))
        q = seg[-1]  # the next segment starts at this knot
    qk, a = np.array(knots), np.array(vals)
    pdfmi.load_alphas(qk, a)
    q2 = np.concatenate([np.exp(r.uniform(np.log(qk[0]) - 1.0, np.log(qk[-1]) + 1.0, 2000)), qk,
                         np.nextafter(qk, 0.0), np.nextafter(qk, np.inf), [0.0, -1.0, np.nan, np.inf]])
    out = pdfmi.alphas_q2(dev(q2)).cpu().numpy()
    ora = oracle.alphas_q2(qk, a, q2)
    assert np.array_equal(np.isnan(out), np.isnan(ora))
    f = ~np.isnan(ora)
    assert np.max(np.abs(out[f] - ora[f]) / np.abs(ora[f])) < 1e-13
    assert np.array_equal(out[2000:2000 + len(qk)], ora[2000:2000 + len(qk)])


@settings(max_examples=20, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(shapes, st.booleans(), st.integers(1, 5000), st.integers(0, 2**31 - 1))
def test_drawn_mc_fused_equals_unfused(shape, f32, n, qseed):
    """The fused Monte-Carlo chunk sum on drawn grids (any sub-grid count and
    row width), point counts and flavour requests, with points in every
    region: bit-identical to the unfused calls (their own xf values, alpha_s
    and chunk sum)."""
    K, nx, nqs, npid, seed = shape
    g = synth.tiny_grid(np.random.default_rng(seed), K=K, nx=nx, nq=nqs[:K], npid=npid)
    r = np.random.default_rng(qseed)
    qlo, qhi = g.q2knots[0][0], g.q2knots[-1][-1]
    x1 = np.exp(r.uniform(np.log(g.xknots[0][0]) - 1.0, 0.0, n))
    x2 = np.exp(r.uniform(np.log(g.xknots[0][0]) - 1.0, 0.0, n))
    q2 = np.exp(r.uniform(np.log(qlo) - 0.5, np.log(qhi) + 0.5, n))
    if n > 4 and qseed % 3 == 0:
        x1[1], q2[2] = -1.0, np.nan
    pids = list(g.pids) if qseed % 2 else [int(p) for p in r.permutation(g.pids)[: max(1, npid // 2)]] + [6]
    m = pdfmi.load_synth(g)
    try:
        pdfmi.load_alphas(*synth.config1_alphas())
        d1, d2, dq = dev(x1), dev(x2), dev(q2)
        ev = pdfmi.xfxq2_f32 if f32 else pdfmi.xfxq2
        s_ref = pdfmi.mc_chunk_sum(ev(m, pids, d1, dq), ev(m, pids, d2, dq), pdfmi.alphas_q2(dq)).cpu().numpy()
        s = pdfmi.mc_fused(m, pids, d1, d2, dq, f32=f32).cpu().numpy()
        assert s.view(np.uint64)[0] == s_ref.view(np.uint64)[0], (s, s_ref)
    finally:
        pdfmi.unload(m)


@settings(max_examples=20, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(st.lists(shapes, min_size=1, max_size=4), st.lists(st.integers(0, 3000), min_size=1, max_size=8),
       st.sampled_from([64, 256, 1024, 4096]), st.booleans(), st.booleans(), st.integers(0, 2**31 - 1))
def test_drawn_batched_plans_equal_per_request(member_shapes, sizes, tile, vec, out_f64, qseed):
    """Batched plans over drawn members (tiny grids of any shape, staged in LDS
    together) and drawn requests (sizes including 0, full or partial flavour
    lists, points in every region): every output equal to its per-request
    call, for a drawn tile size and column grouping."""
    grids = [synth.tiny_grid(np.random.default_rng(s[4]), K=s[0], nx=s[1], nq=s[2][:s[0]], npid=s[3])
             for s in member_shapes]
    ids = [pdfmi.load_synth(g) for g in grids]
    r = np.random.default_rng(qseed)
    plan = None
    try:
        reqs = []
        for i, n in enumerate(sizes):
            gi = int(r.integers(0, len(grids)))
            g = grids[gi]
            pids = None if i % 2 == 0 else [int(p) for p in r.permutation(g.pids)[: int(r.integers(1, len(g.pids) + 1))]]
            P = len(g.pids) if pids is None else len(pids)
            x = np.exp(r.uniform(np.log(g.xknots[0][0]) - 1.0, 0.0, n))
            q2 = np.exp(r.uniform(np.log(g.q2knots[0][0]) - 0.5, np.log(g.q2knots[-1][-1]) + 0.5, n))
            out = torch.full((n, P), -7.0, dtype=torch.float64 if out_f64 else torch.float32, device=DEV)
            reqs.append((ids[gi], pids, dev(x), dev(q2), out, g))
        plan = pdfmi.BatchPlan([q[:5] for q in reqs], out_f64=out_f64)
        plan.configure(tile_points=tile, vector_cols=int(vec))
        plan.run()
        torch.cuda.synchronize()
        fn = pdfmi.xfxq2 if out_f64 else pdfmi.xfxq2_f32
        for m, pids, x, q2, out, g in reqs:
            if x.shape[0] == 0:
                continue
            ref = fn(m, pids, x, q2, n_cols=len(g.pids))
            assert torch.equal(torch.nan_to_num(out, nan=123.0), torch.nan_to_num(ref, nan=123.0))
    finally:
        if plan is not None:
            plan.destroy()
        for m in ids:
            pdfmi.unload(m)
