"""Batched multi-member path (persistent launch, hipGraph replay, autotuned
tiles) vs per-request calls (bit-identical) and vs the oracle."""
import numpy as np
import pytest

import oracle
from paper_2009_06635_amd import synth
from tolerance import check_f32, check_f64, grid_L

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2009_06635_amd import pdfmi  # noqa: E402

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(DEV)


@pytest.fixture(scope="module")
def members():
    grids = synth.config3_members(n_members=6)
    ids = [pdfmi.load_synth(g) for g in grids]
    yield grids, ids
    for m in ids:
        pdfmi.unload(m)


def make_requests(grids, ids, out_f64, seed=1, sizes=(1, 63, 65, 1000, 4097, 20000, 0, 777)):
    rng = np.random.default_rng(seed)
    reqs, host = [], []
    for i, n in enumerate(sizes):
        mi = int(rng.integers(0, len(ids)))
        if i % 3 == 0:
            pids = None
            P = len(grids[mi].pids)
        else:
            pids = [int(p) for p in rng.permutation(synth.PIDS_11 + [6, 0])[: int(rng.integers(1, 13))]]
            P = len(pids)
        x, q2 = synth.config1_queries(n=n, seed=100 + i)
        if n > 10:   # a few points outside the grid and invalid
            x[:3] = [1e-8, 0.5, -1.0]
            q2[:3] = [10.0, 1e9, 10.0]
        out = torch.full((n, P), -7.0, dtype=torch.float64 if out_f64 else torch.float32, device=DEV)
        reqs.append((ids[mi], pids, dev(x), dev(q2), out))
        host.append((mi, pids, x, q2))
    return reqs, host


@pytest.mark.parametrize("out_f64", [False, True])
def test_batched_equals_per_request_and_oracle(members, out_f64):
    grids, ids = members
    reqs, host = make_requests(grids, ids, out_f64)
    plan = pdfmi.BatchPlan(reqs, out_f64=out_f64)
    try:
        for tile, vec in ((64, 0), (1024, 1), (4096, 1), (8192, 0)):
            plan.configure(tile_points=tile, vector_cols=vec)
            for r in reqs:
                r[4].fill_(-7.0)
            plan.run()
            torch.cuda.synchronize()
            for (m, pids, x, q2, out), (mi, _, xh, qh) in zip(reqs, host):
                if x.shape[0] == 0:
                    continue
                fn = pdfmi.xfxq2 if out_f64 else pdfmi.xfxq2_f32
                ref = fn(m, pids, x, q2, n_cols=len(grids[mi].pids))
                assert torch.equal(torch.nan_to_num(out, nan=123.0), torch.nan_to_num(ref, nan=123.0)), (tile, vec)
        # oracle on every request
        for (m, pids, x, q2, out), (mi, p2, xh, qh) in zip(reqs, host):
            if xh.shape[0] == 0:
                continue
            g = grids[mi]
            req = g.pids if p2 is None else p2
            ora, sc = oracle.xfxq2(oracle.Grid(g.xknots, g.q2knots, g.values, g.pids), req, xh, qh, with_scale=True)
            o = out.cpu().numpy()
            ok = check_f64(o, ora, sc, grid_L(g))[0] if out_f64 else check_f32(o, ora, sc)[0]
            assert ok.all()
    finally:
        plan.destroy()


@pytest.mark.parametrize("out_f64", [False, True])
def test_lds_grids_of_other_row_widths(out_f64):
    """Grids staged in LDS with 13, 7 and 12 stored flavours (16-, 8- and
    12-float FP32 rows; the FP32 kernel has a separate code path for 12-float
    rows) beside an 11-flavour member, with full and partial flavour lists:
    every request equal to its per-request call, and within tolerance of the
    oracle."""
    rng = np.random.default_rng(5)
    grids = [synth.config3_members(n_members=1)[0],
             synth.tiny_grid(rng, K=1, nx=40, nq=25, npid=13, loguniform_knots=True),
             synth.tiny_grid(rng, K=2, nx=30, nq=[12, 14], npid=7, loguniform_knots=True),
             synth.tiny_grid(rng, K=1, nx=36, nq=20, npid=12, loguniform_knots=True)]
    ids = [pdfmi.load_synth(g) for g in grids]
    try:
        reqs, host = [], []
        for i, n in enumerate((5000, 777, 4097, 3000, 64, 20000, 1500, 999)):
            gi = i % len(grids)
            g = grids[gi]
            pids = None if i < 4 else [int(p) for p in rng.permutation(g.pids)[: max(1, len(g.pids) // 2)]]
            P = len(g.pids) if pids is None else len(pids)
            x = np.exp(rng.uniform(np.log(g.xknots[0][0]), 0.0, n))
            q2 = np.exp(rng.uniform(np.log(g.q2knots[0][0]), np.log(g.q2knots[-1][-1]), n))
            out = torch.full((n, P), -7.0, dtype=torch.float64 if out_f64 else torch.float32, device=DEV)
            reqs.append((ids[gi], pids, dev(x), dev(q2), out))
            host.append((g, pids, x, q2))
        pdfmi.set_lds_policy(2)   # stage every member grid in LDS
        try:
            plan = pdfmi.BatchPlan(reqs, out_f64=out_f64)
        finally:
            pdfmi.set_lds_policy(0)
        try:
            for tile in (64, 2048):
                plan.configure(tile_points=tile, vector_cols=0)
                for r in reqs:
                    r[4].fill_(-7.0)
                plan.run()
                torch.cuda.synchronize()
                fn = pdfmi.xfxq2 if out_f64 else pdfmi.xfxq2_f32
                for (m, pids, x, q2, out), (g, _, _, _) in zip(reqs, host):
                    ref = fn(m, pids, x, q2, n_cols=len(g.pids))
                    assert torch.equal(out, ref), (tile, len(g.pids))
            for (m, pids, x, q2, out), (g, p2, xh, qh) in zip(reqs, host):
                req = g.pids if p2 is None else p2
                ora, sc = oracle.xfxq2(oracle.Grid(g.xknots, g.q2knots, g.values, g.pids), req, xh, qh,
                                       with_scale=True)
                o = out.cpu().numpy()
                ok = check_f64(o, ora, sc, grid_L(g))[0] if out_f64 else check_f32(o, ora, sc)[0]
                assert ok.all(), len(g.pids)
        finally:
            plan.destroy()
    finally:
        for m in ids:
            pdfmi.unload(m)


@pytest.mark.parametrize("out_f64", [False, True])
def test_plan_without_lds_grid_is_identical(members, out_f64):
    """A plan created under the never-stage policy reads the member grids from
    global memory; its outputs equal those of a plan that stages them in LDS."""
    grids, ids = members
    outs = {}
    for policy in (2, 1):
        pdfmi.set_lds_policy(policy)
        try:
            reqs, _ = make_requests(grids, ids, out_f64, seed=5)
            plan = pdfmi.BatchPlan(reqs, out_f64=out_f64)
        finally:
            pdfmi.set_lds_policy(0)
        try:
            plan.configure(tile_points=1024, vector_cols=1)
            plan.run()
            torch.cuda.synchronize()
            outs[policy] = [torch.nan_to_num(r[4], nan=123.0).clone() for r in reqs]
        finally:
            plan.destroy()
    for a, b in zip(outs[2], outs[1]):
        assert torch.equal(a, b)


def test_graph_replay_matches_eager(members):
    grids, ids = members
    reqs, host = make_requests(grids, ids, False, seed=2)
    plan = pdfmi.BatchPlan(reqs)
    try:
        plan.configure(tile_points=2048, vector_cols=1, use_graph=0)
        plan.run()
        torch.cuda.synchronize()
        eager = [r[4].clone() for r in reqs]
        plan.configure(tile_points=2048, vector_cols=1, use_graph=1)
        for rep in range(4):
            for r in reqs:
                r[4].fill_(float(rep))     # eager work between replays
            torch.cuda.synchronize()
            plan.run()
            torch.cuda.synchronize()
            for r, e in zip(reqs, eager):
                assert torch.equal(torch.nan_to_num(r[4], nan=9.0), torch.nan_to_num(e, nan=9.0)), rep
    finally:
        plan.destroy()


def test_autotune_keeps_results(members):
    grids, ids = members
    reqs, host = make_requests(grids, ids, False, seed=3)
    plan = pdfmi.BatchPlan(reqs)
    try:
        plan.run()
        torch.cuda.synchronize()
        before = [r[4].clone() for r in reqs]
        tile, vec = plan.autotune(reps=1)
        assert tile in (1024, 2048, 4096, 8192, 16384) and vec in (0, 1)
        plan.run()
        torch.cuda.synchronize()
        for r, b in zip(reqs, before):
            assert torch.equal(torch.nan_to_num(r[4], nan=9.0), torch.nan_to_num(b, nan=9.0))
    finally:
        plan.destroy()


def test_autotune_cache_file(members, tmp_path):
    """A sweep appends its choice to the cache file; a choice read from the
    file (here edited by hand to a tile size the sweep never picks) is taken
    without a sweep, and the plan still gives the per-request values."""
    grids, ids = members
    reqs, host = make_requests(grids, ids, False, seed=11, sizes=(5, 6001, 333, 70))
    path = tmp_path / "tune.txt"
    pdfmi.batch_tune_cache(str(path))
    try:
        plan = pdfmi.BatchPlan(reqs)
        try:
            t1, v1 = plan.autotune(reps=1)
            lines = [ln for ln in path.read_text().splitlines() if ln.strip()]
            assert len(lines) == 1 and lines[0].split()[1:] == [str(t1), str(v1)]
            path.write_text("%s 3008 1\n" % lines[0].split()[0])
            pdfmi.batch_tune_cache(str(path))
            assert plan.autotune(reps=1) == (3008, 1)
            assert len(path.read_text().splitlines()) == 1   # no sweep, nothing appended
            for r in reqs:
                r[4].fill_(-7.0)
            plan.run()
            torch.cuda.synchronize()
            for (m, pids, x, q2, out), (mi, _, _, _) in zip(reqs, host):
                ref = pdfmi.xfxq2_f32(m, pids, x, q2, n_cols=len(grids[mi].pids))
                assert torch.equal(torch.nan_to_num(out, nan=123.0), torch.nan_to_num(ref, nan=123.0))
        finally:
            plan.destroy()
    finally:
        pdfmi.batch_tune_cache(None)


@pytest.mark.parametrize("out_f64", [False, True])
def test_one_shot_equals_per_request(members, out_f64):
    """pdf_xfxq2_batched (FP32 outputs) and pdf_xfxq2_batched_f64 against the
    per-request calls, bit for bit."""
    grids, ids = members
    reqs, host = make_requests(grids, ids, out_f64, seed=6, sizes=(100, 5, 3000, 0))
    pdfmi.xfxq2_batched(reqs, out_f64=out_f64)
    for (m, pids, x, q2, out), (mi, _, _, _) in zip(reqs, host):
        if x.shape[0] == 0:
            continue
        fn = pdfmi.xfxq2 if out_f64 else pdfmi.xfxq2_f32
        ref = fn(m, pids, x, q2, n_cols=len(grids[mi].pids))
        assert torch.equal(torch.nan_to_num(out, nan=123.0), torch.nan_to_num(ref, nan=123.0))


def test_one_shot_and_errors(members):
    grids, ids = members
    reqs, _ = make_requests(grids, ids, False, seed=4, sizes=(100, 5))
    pdfmi.xfxq2_batched(reqs)
    assert not torch.isnan(reqs[0][4][3:]).any()
    bad = [(9999, None, reqs[0][2], reqs[0][3], reqs[0][4])]
    with pytest.raises(pdfmi.PdfError) as e:
        pdfmi.BatchPlan(bad)
    assert e.value.code == pdfmi.PDF_ERR_MEMBER
    pdfmi.xfxq2_batched([])


@pytest.mark.parametrize("out_f64", [False, True])
def test_mixed_grid_shapes_read_global(members, out_f64):
    """A plan holding a three-sub-grid 13-flavour member next to the small
    ones: the largest grid does not fit LDS, so every tile reads its grid from
    global memory; outputs bit-identical to the per-request calls and within
    tolerance of the oracle."""
    grids, ids = members
    g2 = synth.config2_grid()
    m2 = pdfmi.load_synth(g2)
    try:
        rng = np.random.default_rng(9)
        reqs, host = [], []
        for i, n in enumerate((5000, 64, 1, 3000)):
            if i % 2 == 0:
                x, q2 = synth.config2_queries(n=n, seed=400 + i, out_fraction=0.05)
                m, g, pids = m2, g2, [int(p) for p in rng.permutation(g2.pids)[:7]]
            else:
                x, q2 = synth.config1_queries(n=n, seed=400 + i)
                m, g, pids = ids[i % len(ids)], grids[i % len(ids)], None
            P = len(g.pids) if pids is None else len(pids)
            out = torch.full((n, P), -7.0, dtype=torch.float64 if out_f64 else torch.float32, device=DEV)
            reqs.append((m, pids, dev(x), dev(q2), out))
            host.append((g, pids, x, q2))
        plan = pdfmi.BatchPlan(reqs, out_f64=out_f64)
        try:
            plan.configure(tile_points=1024, vector_cols=1)
            plan.run()
            torch.cuda.synchronize()
            for (m, pids, x, q2, out), (g, p2, xh, qh) in zip(reqs, host):
                fn = pdfmi.xfxq2 if out_f64 else pdfmi.xfxq2_f32
                ref = fn(m, pids, x, q2, n_cols=len(g.pids))
                assert torch.equal(torch.nan_to_num(out, nan=123.0), torch.nan_to_num(ref, nan=123.0))
                req = g.pids if p2 is None else p2
                ora, sc = oracle.xfxq2(oracle.Grid(g.xknots, g.q2knots, g.values, g.pids), req, xh, qh,
                                       with_scale=True)
                o = out.cpu().numpy()
                ok = check_f64(o, ora, sc, grid_L(g))[0] if out_f64 else check_f32(o, ora, sc)[0]
                assert ok.all()
        finally:
            plan.destroy()
    finally:
        pdfmi.unload(m2)


def test_full_size_workload_as_benchmarked():
    """The 101-member, 200-request workload in the benchmark's launch
    configuration (autotuned tiles, graph replay): every request bit-identical
    to its per-request FP32 call; a sample of each eighth request against the
    oracle."""
    grids = synth.config3_members()
    ids = [pdfmi.load_synth(g) for g in grids]
    try:
        reqs_h = synth.config3_requests()
        reqs = []
        for r in reqs_h:
            out = torch.empty((len(r["x"]), len(r["pids"])), dtype=torch.float32, device=DEV)
            reqs.append((ids[r["member"]], r["pids"], dev(r["x"]), dev(r["q2"]), out))
        plan = pdfmi.BatchPlan(reqs)
        try:
            tile, vec = plan.autotune(reps=1)
            plan.configure(tile_points=tile, vector_cols=vec, use_graph=1)
            plan.run()
            torch.cuda.synchronize()
            for i, ((m, pids, x, q2, out), r) in enumerate(zip(reqs, reqs_h)):
                ref = pdfmi.xfxq2_f32(m, pids, x, q2)
                assert torch.equal(torch.nan_to_num(out, nan=1.0), torch.nan_to_num(ref, nan=1.0)), i
                if i % 8 == 0:
                    g = grids[r["member"]]
                    k = min(500, len(r["x"]))
                    ora, sc = oracle.xfxq2(oracle.Grid(g.xknots, g.q2knots, g.values, g.pids), r["pids"],
                                           r["x"][:k], r["q2"][:k], with_scale=True)
                    assert check_f32(out[:k].cpu().numpy(), ora, sc)[0].all(), i
        finally:
            plan.destroy()
    finally:
        for m in ids:
            pdfmi.unload(m)


def test_plan_refuses_unloaded_members():
    """A plan copies its members' device pointers: after one of them is
    unloaded (and its slot reused by a new load) running or tuning the plan
    fails with PDF_ERR_MEMBER instead of reading freed memory."""
    g = synth.config1_grid()
    m = pdfmi.load_synth(g)
    x, q2 = synth.config1_queries(n=500, seed=7)
    out = torch.empty((500, len(g.pids)), dtype=torch.float32, device=DEV)
    plan = pdfmi.BatchPlan([(m, None, dev(x), dev(q2), out)])
    try:
        plan.run()
        torch.cuda.synchronize()
        pdfmi.unload(m)
        with pytest.raises(pdfmi.PdfError) as ei:
            plan.run()
        assert ei.value.code == pdfmi.PDF_ERR_MEMBER
        m2 = pdfmi.load_synth(g)   # takes the freed slot: same id, new load
        try:
            assert m2 == m
            for fn in (plan.run, lambda: plan.autotune(reps=1)):
                with pytest.raises(pdfmi.PdfError) as ei:
                    fn()
                assert ei.value.code == pdfmi.PDF_ERR_MEMBER
        finally:
            pdfmi.unload(m2)
    finally:
        plan.destroy()
