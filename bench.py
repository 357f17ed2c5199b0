"""Benchmark: PDF evaluations per second on one MI355X.

Workload of the headline line (one "step" = one pass of the hot path over one
batch): 1e7 query points of the three-sub-grid, 13-flavour synthetic set (196
x knots, 3 x 17 Q^2 knots split at the 1.51 / 4.92 GeV thresholds, 1% of the
points outside the grid), all flavours and alpha_s at every point in FP64, in
one launch (pdf_xfxq2_alphas).  Inputs are resident in device memory before
the timed region.  `value` counts PDF evaluations (points x flavours).

"variants" reports, on the same clock:
  f32        FP32 bulk arithmetic on the headline workload
             (pdf_xfxq2_alphas_f32)
  separate   the headline step as two launches (pdf_xfxq2, pdf_alphas_q2)
  small      the 1e5-point one-sub-grid workload (latency-bound), FP64
  points     evaluations per second against the number of points (1e3..1e7,
             headline grid, all flavours + alpha_s, FP64 and FP32), the
             shape of the paper's throughput-versus-points measurement
  batched    101 members, 200 requests (log-normal sizes, random flavour
             subsets), one persistent hipGraph-replayed launch with autotuned
             tiles, FP32 arithmetic; speed-up over per-request FP64 calls
  surrogate  MLP surrogate trained on 2e6 interpolator samples, inference on
             1e7 points with interpolator fallback; error vs the FP64 oracle
  mc         1e8 Monte-Carlo-style points (two lookups at a shared scale,
             alpha_s, FP64 fixed-order chunk sums), FP64 / FP32 / surrogate,
             and the fused one-kernel forms (bit-identical sums)
  members_fk 10..400 members evaluated on a 2415-point x grid at Q = 1.65
             (13 flavours, FP64, one batched launch; the paper's Table 2
             shape, its GPU seconds quoted as context), then the FP64
             matrix-core contraction with a 1024-row synthetic FK table
The dominant kernel's roofline uses its algorithmic bytes (16 B of (x, Q^2) in
+ 8 B per output value, PDF or alpha_s) over its average duration measured
with HIP events on the launch stream.  cpu_baseline times the FP64 oracle on the host cores.
"""
import argparse
import gc
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# L2 read bandwidth of the chip: 8 XCDs x 16 channels x 128 B per clock at 2.4 GHz
L2_PEAK_GBS = 8 * 16 * 128 * 2.4
# vector L1 (texture) path: 256 compute units x 64 B per clock at 2.4 GHz
L1_PEAK_GBS = 256 * 64 * 2.4


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("kernels.hip", "interp_dev.h", "pdfmi.cpp", "pdfmi_dev.h"):
        with open(os.path.join(ROOT, "paper_2009_06635_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None
    return d.get(kernel_key)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=2_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-headline", action="store_true", help="skip the variants")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--sur-steps", type=int, default=20000)
    ap.add_argument("--mc-chunks", type=int, default=100)
    ap.add_argument("--locality", action="store_true",
                    help="also measure the headline kernel on cell-sorted points, with the sort and the "
                         "scatter back to point order (what a cell-binned variant would cost)")
    ap.add_argument("--settle-ms", type=float, default=300.0,
                    help="untimed run of each timed step before its warm-up steps, so that the GPU "
                         "clocks have ramped up whatever --warmup is")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: query points shard across GPUs with no exchange, "
              "and only the single-GPU path is implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2009_06635_amd import pdfmi, synth

    dev = "cuda:0"
    torch.cuda.init()

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def timed(fn, steps, warmup):
        """(wall seconds per step, mean kernel ms between fn's own events)."""
        # The garbage collector is paused over warm-up and timed steps: a collection
        # inside the timed region stalls the launches for tens of ms, and one between
        # warm-up and timing idles the GPU long enough for its clocks to drop.
        gc.collect()
        gc.disable()
        try:
            evs = [(ev(), ev()) for _ in range(steps)]
            # clock settling: a few warm-up steps of a sub-millisecond kernel end before the
            # GPU has left its idle clocks, so the step first runs for settle_ms untimed
            t_end = time.perf_counter() + args.settle_ms * 1e-3
            while time.perf_counter() < t_end:
                for _ in range(8):
                    fn(None)
                torch.cuda.synchronize()
            for _ in range(warmup):
                fn(None)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for e in evs:
                fn(e)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / steps
        finally:
            gc.enable()
        kern = sum(e[0].elapsed_time(e[1]) for e in evs) / steps
        return wall, kern

    def dtime(fn, reps=5):
        # no collection here: the single warm-up call cannot bring the clocks back up
        # after the GPU idles through one
        gc.disable()
        try:
            e0, e1 = ev(), ev()
            fn()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
        finally:
            gc.enable()
        return e0.elapsed_time(e1) / reps

    # ---------------------------------------------------------------- headline
    log("headline workload: generating 1e7 points")
    g = synth.config2_grid()
    x, q2 = synth.config2_queries(n=args.n)
    member = pdfmi.load_synth(g)
    qk, a = synth.config2_alphas()
    pdfmi.load_alphas(qk, a)
    P = len(g.pids)
    xd = torch.from_numpy(x).to(dev)
    qd = torch.from_numpy(q2).to(dev)
    out64 = torch.empty((args.n, P), dtype=torch.float64, device=dev)
    out32 = torch.empty((args.n, P), dtype=torch.float32, device=dev)
    aout = torch.empty(args.n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def step64(e):
        if e:
            e[0].record()
        pdfmi.xfxq2_alphas(member, g.pids, xd, qd, out=out64, alphas_out=aout)
        if e:
            e[1].record()

    def step32(e):
        if e:
            e[0].record()
        pdfmi.xfxq2_alphas(member, g.pids, xd, qd, out=out32, alphas_out=aout, f32=True)
        if e:
            e[1].record()

    def step_separate(e):
        if e:
            e[0].record()
        pdfmi.xfxq2(member, g.pids, xd, qd, out=out64)
        if e:
            e[1].record()
        pdfmi.alphas_q2(qd, out=aout)

    log("timing FP64 / FP32")
    wall64, k64 = timed(step64, args.steps, args.warmup)
    wall32, k32 = timed(step32, args.steps, args.warmup)

    def copy_gbs():
        # a measured HBM figure beside the published peak: a 1 GiB device-to-device
        # copy, bytes read + written per second (context only; the roofline keeps 8 TB/s)
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        e0, e1 = ev(), ev()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        gbs = 2 * a.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del a, b
        return gbs

    hbm_copy = copy_gbs()
    evals = args.n * P
    bytes64 = args.n * (16 + 8 * P + 8)
    bytes32 = args.n * (16 + 4 * P + 8)
    ach64 = bytes64 / (k64 * 1e-3) / 1e9
    ach32 = bytes32 / (k32 * 1e-3) / 1e9
    res = {
        "metric": "PDF evals/s (points x flavours), FP64 log-bicubic interpolation",
        "value": evals / wall64,
        "unit": "PDF evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_ms": args.settle_ms,
        "ms_per_step": wall64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "xfxq2 all 13 flavours + alpha_s, 3 sub-grids (196 x 3x17 knots), "
                               "1e7 points, 1% outside the grid", "n_points": args.n, "n_flavours": P,
                   "subgrids": 3, "x_knots": 196, "q2_knots_per_subgrid": 17},
        "roofline": {"bound": "hbm", "achieved": ach64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach64 / HBM_PEAK_GBS, "traffic": measured_traffic("xfxq2_f64"),
                     "kernel": "k_xfxq2<double> with alpha_s output (pdf_xfxq2_alphas)", "kernel_ms": k64,
                     "algorithmic_bytes_per_launch": bytes64,
                     "hbm_copy_measured": {"achieved": hbm_copy, "unit": "GB/s", "frac_of_it": ach64 / hbm_copy,
                                           "what": "1 GiB device-to-device copy, bytes read + written"},
                     # the gather behind the HBM figure: every point reads its 4 x 4 stencil, 16 grid
                     # rows of 13 FP64 columns, as 16 x 128-byte lines from the L2-resident grid and as
                     # 16 rows x 7 lanes x 16 bytes through each compute unit's vector-memory (L1) path
                     "l2_gather": {"achieved": 16 * 128 * args.n / (k64 * 1e-3) / 1e9, "peak": L2_PEAK_GBS,
                                   "unit": "GB/s", "frac": 16 * 128 * args.n / (k64 * 1e-3) / 1e9 / L2_PEAK_GBS,
                                   "bytes_per_point": 16 * 128},
                     "l1_gather": {"achieved": 16 * 7 * 16 * args.n / (k64 * 1e-3) / 1e9, "peak": L1_PEAK_GBS,
                                   "unit": "GB/s", "frac": 16 * 7 * 16 * args.n / (k64 * 1e-3) / 1e9 / L1_PEAK_GBS,
                                   "bytes_per_point": 16 * 7 * 16}},
        "variants": {
            "f64_kernel_evals_per_s": evals / (k64 * 1e-3),
            "f32": {"value": evals / wall32, "ms_per_step": wall32 * 1e3, "kernel_ms": k32,
                    "kernel_evals_per_s": evals / (k32 * 1e-3), "achieved_GBs": ach32,
                    "frac": ach32 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": bytes32,
                    "speedup_vs_f64_kernel": k64 / k32,
                    # FP32 rows of 16 columns: the 4 rows of one x knot's Q^2 window span 2-3 lines;
                    # through the L1 path 16 rows x 4 lanes x 16 bytes
                    "l2_gather_frac": 4 * 2.5 * 128 * args.n / (k32 * 1e-3) / 1e9 / L2_PEAK_GBS,
                    "l1_gather_frac": 16 * 4 * 16 * args.n / (k32 * 1e-3) / 1e9 / L1_PEAK_GBS},
        },
    }
    V = res["variants"]

    # parity of the timed outputs with the FP64 oracle on a sample (outside the timed region): the
    # floored criterion the tests apply (R14: 1e-12 |o| + 4 eps64 S (1 + L); FP32: |o| <= 1e-8 or
    # 1e-5 |o| + 4 eps32 S), the literal relative criterion without the floor, and the largest eq. (1)
    # difference |g - o| / (|o| + 1e-16) where the oracle is finite (and |o| > 1e-8 for FP32)
    import oracle
    ns = min(args.n, 20000)
    sidx = np.random.default_rng(7).choice(args.n, ns, replace=False)
    sidx_t = torch.from_numpy(sidx).to(dev)
    ora, oscale = oracle.xfxq2(oracle.Grid(g.xknots, g.q2knots, g.values, g.pids), g.pids, x[sidx], q2[sidx],
                               with_scale=True, n_threads=max(1, os.cpu_count() or 1))
    Lg = float(max(np.max(1.0 / np.diff(np.log(t))) for t in g.xknots) +
               max(np.max(1.0 / np.diff(np.log(t))) for t in g.q2knots))
    eps64, eps32 = float(np.finfo(np.float64).eps), float(np.finfo(np.float32).eps)

    def parity(gv, rtol, floor_abs, c_eps, with_L, small):
        gv = gv.astype(np.float64)
        fin = np.isfinite(ora)
        both_nan = np.isnan(gv) & np.isnan(ora)
        d = np.abs(gv - ora)
        tiny = np.abs(ora) <= small if small else np.zeros_like(fin)
        floor = c_eps * oscale * ((1.0 + Lg) if with_L else 1.0)
        floored = both_nan | tiny | (d <= rtol * np.abs(ora) + floor)
        literal = both_nan | tiny | (d <= rtol * np.abs(ora))
        sel = fin & ~tiny
        r = d[sel] / (np.abs(ora[sel]) + 1e-16)
        return {"sample": int(ns), "floored_pass_frac": float(floored.mean()), "literal_pass_frac": float(literal.mean()),
                "max_eq1": float(r.max()) if r.size else 0.0, "literal_rtol": rtol}
    res["parity_vs_oracle"] = {
        "f64": parity(out64[sidx_t].cpu().numpy(), 1e-12, None, 4 * eps64, True, 0.0),
        "f32": parity(out32[sidx_t].cpu().numpy(), 1e-5, None, 4 * eps32, False, 1e-8)}
    del out32

    if args.locality:
        # What binning the points by grid cell could gain: the same kernel on the points sorted by
        # stencil cell (neighbouring lanes and waves then share grid lines, which the L1 cache
        # serves instead of L2), and what binning costs on top -- the sort of the cell keys and the
        # scatter of the output rows back to the caller's point order.
        log("locality: the headline points sorted by stencil cell")
        qall = np.concatenate(g.q2knots)
        key = np.searchsorted(qall, q2).astype(np.int64) * (len(g.xknots[0]) + 1) + np.searchsorted(g.xknots[0], x)
        perm = np.argsort(key, kind="stable")
        xs_d, qs_d = torch.from_numpy(x[perm]).to(dev), torch.from_numpy(q2[perm]).to(dev)
        perm_d, key_d = torch.from_numpy(perm).to(dev), torch.from_numpy(key).to(dev)
        outs, as_s = torch.empty_like(out64), torch.empty_like(aout)

        def step_sorted(e):
            if e:
                e[0].record()
            pdfmi.xfxq2_alphas(member, g.pids, xs_d, qs_d, out=outs, alphas_out=as_s)
            if e:
                e[1].record()
        wall_s, k_s = timed(step_sorted, args.steps, args.warmup)
        ref = out64.clone()
        t_scatter = dtime(lambda: (out64.index_copy_(0, perm_d, outs), aout.index_copy_(0, perm_d, as_s)), reps=5)
        t_sort = dtime(lambda: torch.sort(key_d, stable=True), reps=5)
        same = bool(torch.equal(out64.view(torch.int64), ref.view(torch.int64)))
        del ref, outs, as_s
        V["locality"] = {
            "sorted_kernel_ms": k_s, "unsorted_kernel_ms": k64, "scatter_to_point_order_ms": t_scatter,
            "key_sort_ms": t_sort, "binned_total_ms": k_s + t_scatter + t_sort,
            "scattered_output_equals_unsorted": same,
            "note": "sorted kernel + scatter back + key sort against the unsorted kernel; a counting sort "
                    "in a kernel of its own would replace torch's sort"}

    if not args.only_headline:
        import oracle

        log("timing the headline step as two launches")
        wall_sep, k_sep = timed(step_separate, args.steps, args.warmup)
        V["separate"] = {"ms_per_step": wall_sep * 1e3, "xfxq2_kernel_ms": k_sep,
                         "fused_speedup": wall_sep / wall64}

        def variants():
            def rel_stats(o, ora, floor=1e-8):
                ok = np.abs(ora) > floor
                r = (np.abs(o - ora) / np.abs(ora))[ok]
                return {"median_rel": float(np.median(r)), "p99_rel": float(np.percentile(r, 99)),
                        "max_rel": float(r.max()), "frac_le_1e-3": float((r <= 1e-3).mean())}

            # ---------------------------------------------------------- throughput against n
            log("throughput against the number of points")
            sweep = []
            for n_pts in (1_000, 10_000, 100_000, 1_000_000, 10_000_000):
                xs_n, qs_n = xd[:n_pts], qd[:n_pts]
                t64 = dtime(lambda: pdfmi.xfxq2_alphas(member, g.pids, xs_n, qs_n, out=out64[:n_pts],
                                                       alphas_out=aout[:n_pts]), reps=20)
                o32 = torch.empty((n_pts, P), dtype=torch.float32, device=dev)
                t32 = dtime(lambda: pdfmi.xfxq2_alphas(member, g.pids, xs_n, qs_n, out=o32, alphas_out=aout[:n_pts],
                                                       f32=True), reps=20)
                sweep.append({"n_points": n_pts, "f64_ms": t64, "f64_evals_per_s": n_pts * P / (t64 * 1e-3),
                              "f32_ms": t32, "f32_evals_per_s": n_pts * P / (t32 * 1e-3)})
                del o32
            V["points"] = sweep

            # ---------------------------------------------------------- small (1e5)
            log("small workload")
            g1 = synth.config1_grid()
            m1 = pdfmi.load_synth(g1)
            x1, q1 = synth.config1_queries()
            x1d, q1d = torch.from_numpy(x1).to(dev), torch.from_numpy(q1).to(dev)
            o1 = torch.empty((len(x1), len(g1.pids)), dtype=torch.float64, device=dev)
            ks = dtime(lambda: pdfmi.xfxq2(m1, g1.pids, x1d, q1d, out=o1), reps=20)
            sb = len(x1) * (16 + 8 * len(g1.pids))
            V["small"] = {"n_points": len(x1), "n_flavours": len(g1.pids), "kernel_ms": ks,
                          "evals_per_s": len(x1) * len(g1.pids) / (ks * 1e-3),
                          "achieved_GBs": sb / (ks * 1e-3) / 1e9, "frac_hbm": sb / (ks * 1e-3) / 1e9 / HBM_PEAK_GBS}

            # ---------------------------------------------------------- batched
            log("batched workload: 101 members, 200 requests")
            members = synth.config3_members()
            mids = [pdfmi.load_synth(mg) for mg in members]
            reqs_h = synth.config3_requests()
            reqs = []
            for r in reqs_h:
                xr = torch.from_numpy(r["x"]).to(dev)
                qr = torch.from_numpy(r["q2"]).to(dev)
                orr = torch.empty((len(r["x"]), len(r["pids"])), dtype=torch.float32, device=dev)
                reqs.append((mids[r["member"]], r["pids"], xr, qr, orr))
            plan = pdfmi.BatchPlan(reqs)
            tile, vec = plan.autotune(reps=2)
            plan.configure(tile_points=tile, vector_cols=vec, use_graph=1)
            tb = dtime(plan.run, reps=10)
            npts = sum(len(r["x"]) for r in reqs_h)
            nev = sum(len(r["x"]) * len(r["pids"]) for r in reqs_h)
            o64 = [torch.empty((t[2].shape[0], len(t[1])), dtype=torch.float64, device=dev) for t in reqs]

            def per_request_f64():
                for t, o in zip(reqs, o64):
                    pdfmi.xfxq2(t[0], t[1], t[2], t[3], out=o)
            tp = dtime(per_request_f64, reps=3)
            # error of the batched FP32 output vs the FP64 oracle on a sample of requests
            errs = []
            for i in range(0, len(reqs_h), 25):
                r = reqs_h[i]
                mg = members[r["member"]]
                k = min(2000, len(r["x"]))
                ora = oracle.xfxq2(oracle.Grid(mg.xknots, mg.q2knots, mg.values, mg.pids), r["pids"], r["x"][:k],
                                   r["q2"][:k])
                errs.append((reqs[i][4][:k].cpu().numpy().astype(np.float64), ora))
            bb = npts * 16 + nev * 4  # (x, Q^2) in, FP32 values out
            V["batched"] = {"members": len(mids), "requests": len(reqs), "points": npts, "evals": nev,
                            "tile_points": tile, "vector_cols": vec, "graph": True, "ms": tb,
                            "evals_per_s": nev / (tb * 1e-3), "achieved_GBs": bb / (tb * 1e-3) / 1e9,
                            "frac_hbm": bb / (tb * 1e-3) / 1e9 / HBM_PEAK_GBS, "per_request_f64_ms": tp,
                            "speedup_vs_per_request_f64": tp / tb,
                            "error_vs_oracle": rel_stats(np.concatenate([e[0].ravel() for e in errs]),
                                                         np.concatenate([e[1].ravel() for e in errs]))}
            plan.destroy()
            del reqs, o64
            for m_ in mids:
                pdfmi.unload(m_)

            # ---------------------------------------------------------- surrogate
            log("surrogate: training on 2e6 samples")
            xt, qt = synth.config1_queries(n=2_000_000, seed=40)
            sur = pdfmi.Surrogate(m1, seed=3)
            sur.set_data(torch.from_numpy(xt).to(dev), torch.from_numpy(qt).to(dev))
            t0 = time.perf_counter()
            sur.train(args.sur_steps, 4096, 3e-3, 3e-5, args.sur_steps)
            torch.cuda.synchronize()
            ttrain = time.perf_counter() - t0
            xs, qs = synth.config1_queries(n=10_000_000, seed=41)
            xsd, qsd = torch.from_numpy(xs).to(dev), torch.from_numpy(qs).to(dev)
            P1 = len(g1.pids)
            so = torch.empty((len(xs), P1), dtype=torch.float32, device=dev)
            ref64 = torch.empty((len(xs), P1), dtype=torch.float64, device=dev)
            ref32 = torch.empty((len(xs), P1), dtype=torch.float32, device=dev)
            t_sur = dtime(lambda: sur.xfxq2(xsd, qsd, out=so))
            t_i64 = dtime(lambda: pdfmi.xfxq2(m1, g1.pids, xsd, qsd, out=ref64))
            t_i32 = dtime(lambda: pdfmi.xfxq2_f32(m1, g1.pids, xsd, qsd, out=ref32))
            idx = np.random.default_rng(0).choice(len(xs), 20000, replace=False)
            ora = oracle.xfxq2(oracle.Grid(g1.xknots, g1.q2knots, g1.values, g1.pids), g1.pids, xs[idx], qs[idx])
            idx_t = torch.from_numpy(idx).to(dev)
            # network arithmetic per point: 2*64 + 64*64 + 64*64 + 64*16 multiply-adds (16 outputs incl.
            # padding), 3*64 tanh; layers 2-4 on the BF16 matrix cores (2.5 PFLOP/s dense peak)
            mfma_flop = 2.0 * (64 * 64 * 2 + 64 * 16) * len(xs)
            V["surrogate"] = {"n_points": len(xs), "n_flavours": P1, "train_s": ttrain, "train_steps": args.sur_steps,
                              "ms": t_sur, "evals_per_s": len(xs) * P1 / (t_sur * 1e-3),
                              "mfma_TFLOPs": mfma_flop / (t_sur * 1e-3) / 1e12,
                              "frac_bf16_mfma_peak": mfma_flop / (t_sur * 1e-3) / 2.5e15,
                              "tanh_per_s": 3 * 64 * len(xs) / (t_sur * 1e-3),
                              "interp_f64_ms": t_i64, "interp_f32_ms": t_i32,
                              "speedup_vs_f64_interp": t_i64 / t_sur, "speedup_vs_f32_interp": t_i32 / t_sur,
                              "error_vs_oracle": rel_stats(so[idx_t].cpu().numpy().astype(np.float64), ora)}
            del ref32

            # ---------------------------------------------------------- Monte-Carlo load
            nchunk = args.mc_chunks
            log("mc workload: %d chunks of 1e6 points" % nchunk)
            qk1, a1 = synth.config1_alphas()
            pdfmi.load_alphas(qk1, a1)
            ch = [synth.config5_chunk(c) for c in range(nchunk)]
            X1 = [torch.from_numpy(c[0]).to(dev) for c in ch]
            X2 = [torch.from_numpy(c[1]).to(dev) for c in ch]
            Q = [torch.from_numpy(c[2]).to(dev) for c in ch]
            PIDS = synth.PIDS_13
            n_c = len(ch[0][0])
            f1_64 = torch.empty((n_c, 13), dtype=torch.float64, device=dev)
            f2_64 = torch.empty_like(f1_64)
            f1_32 = torch.empty((n_c, 13), dtype=torch.float32, device=dev)
            f2_32 = torch.empty_like(f1_32)
            s1 = torch.empty((n_c, P1), dtype=torch.float32, device=dev)
            s2 = torch.empty_like(s1)
            al = torch.empty(n_c, dtype=torch.float64, device=dev)
            ws = pdfmi.mc_workspace(n_c, dev)
            sums = {k: torch.empty(nchunk, dtype=torch.float64, device=dev) for k in ("f64", "f32", "sur")}

            def run_mc(kind):
                for c in range(nchunk):
                    pdfmi.alphas_q2(Q[c], out=al)
                    if kind == "f64":
                        pdfmi.xfxq2(m1, PIDS, X1[c], Q[c], out=f1_64)
                        pdfmi.xfxq2(m1, PIDS, X2[c], Q[c], out=f2_64)
                        pdfmi.mc_chunk_sum(f1_64, f2_64, al, workspace=ws, out=sums[kind][c:c + 1])
                    elif kind == "f32":
                        pdfmi.xfxq2_f32(m1, PIDS, X1[c], Q[c], out=f1_32)
                        pdfmi.xfxq2_f32(m1, PIDS, X2[c], Q[c], out=f2_32)
                        pdfmi.mc_chunk_sum(f1_32, f2_32, al, workspace=ws, out=sums[kind][c:c + 1])
                    else:   # surrogate gives the stored flavours; absent ones are zero and add nothing
                        sur.xfxq2(X1[c], Q[c], out=s1)
                        sur.xfxq2(X2[c], Q[c], out=s2)
                        pdfmi.mc_chunk_sum(s1, s2, al, workspace=ws, out=sums[kind][c:c + 1])
            sums["f64_fused"] = torch.empty(nchunk, dtype=torch.float64, device=dev)
            sums["f32_fused"] = torch.empty(nchunk, dtype=torch.float64, device=dev)

            def run_fused(kind):
                for c in range(nchunk):
                    pdfmi.mc_fused(m1, PIDS, X1[c], X2[c], Q[c], f32=(kind == "f32_fused"), workspace=ws,
                                   out=sums[kind][c:c + 1])
            mc = {"points": nchunk * n_c, "chunks": nchunk, "evals_per_point": 26}
            for kind in ("f64", "f32", "sur", "f64_fused", "f32_fused"):
                fn = (lambda: run_fused(kind)) if kind.endswith("_fused") else (lambda: run_mc(kind))
                ms = dtime(fn, reps=1)
                mc[kind] = {"ms": ms, "evals_per_s": nchunk * n_c * 26 / (ms * 1e-3)}
            tot = {k: float(sums[k].sum().item()) for k in sums}
            # chunk 0 against the oracle
            og1 = oracle.Grid(g1.xknots, g1.q2knots, g1.values, g1.pids)
            th = max(1, min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1))
            oc1 = oracle.xfxq2(og1, PIDS, ch[0][0], ch[0][2], n_threads=th)
            oc2 = oracle.xfxq2(og1, PIDS, ch[0][1], ch[0][2], n_threads=th)
            oa = oracle.alphas_q2(qk1, a1, ch[0][2])
            s0 = math.fsum(oa * np.sum(oc1 * oc2, axis=1))
            for kind in ("f64", "f32", "sur", "f64_fused", "f32_fused"):
                mc[kind]["chunk0_rel_err_vs_oracle"] = abs(float(sums[kind][0].item()) - s0) / abs(s0)
                mc[kind]["total"] = tot[kind]
                mc[kind]["speedup_vs_f64"] = mc["f64"]["ms"] / mc[kind]["ms"]
            for kind in ("f64_fused", "f32_fused"):   # 24 B of (x1, x2, Q^2) per point in, one sum per chunk out
                mc[kind]["achieved_GBs"] = 24.0 * mc["points"] / (mc[kind]["ms"] * 1e-3) / 1e9
                mc[kind]["frac_hbm"] = mc[kind]["achieved_GBs"] / HBM_PEAK_GBS
                # the bound that matters: stencil gathers from the LDS-staged grid, 2 x 16 values per
                # stored flavour per point, against 128 B/clk/CU x 256 CUs x 2.4 GHz
                lds_b = 2 * 16 * len(g1.pids) * (8 if kind == "f64_fused" else 4) * mc["points"]
                mc[kind]["lds_TBs"] = lds_b / (mc[kind]["ms"] * 1e-3) / 1e12
                mc[kind]["frac_lds_peak"] = mc[kind]["lds_TBs"] / (128 * 256 * 2.4e9 / 1e12)
            mc["fused_bit_identical"] = {
                "f64": bool(torch.equal(sums["f64"].view(torch.int64), sums["f64_fused"].view(torch.int64))),
                "f32": bool(torch.equal(sums["f32"].view(torch.int64), sums["f32_fused"].view(torch.int64)))}
            V["mc"] = mc
            sur.destroy()
            del X1, X2, Q

            # ---------------------------------------------------------- multi-member x grid + FK contraction
            log("multi-member evaluation on a 2415-point x grid and FK contraction")
            nx_fk, ndat = 2415, 1024
            fk_members = synth.config3_members(n_members=400)
            fk_ids = [pdfmi.load_synth(mg) for mg in fk_members]
            xg = torch.from_numpy(np.exp(np.linspace(np.log(2e-6), np.log(0.95), nx_fk))).to(dev)
            qg = torch.full((nx_fk,), 1.65 ** 2, dtype=torch.float64, device=dev)
            table = torch.from_numpy(np.random.default_rng(11).normal(size=(ndat, nx_fk * 13))).to(dev)
            paper_gpu_s = {10: 0.07, 50: 0.35, 100: 0.69, 200: 1.46, 300: 1.29, 400: 1.69}
            fkv = {"x_points": nx_fk, "flavours": 13, "q": 1.65, "ndat": ndat, "rows": []}
            for nrep in (10, 50, 100, 200, 300, 400):
                F = torch.empty((nrep, nx_fk, 13), dtype=torch.float64, device=dev)
                plan = pdfmi.BatchPlan([(fk_ids[r], synth.PIDS_13, xg, qg, F[r]) for r in range(nrep)], out_f64=True)
                plan.configure(tile_points=2048, vector_cols=1, use_graph=1)
                t_eval = dtime(plan.run, reps=5)
                Fm = F.reshape(nrep, -1)
                T = torch.empty((nrep, ndat), dtype=torch.float64, device=dev)
                t_fk = dtime(lambda: pdfmi.fk_contract(Fm, table, out=T), reps=5)
                flops = 2.0 * nrep * ndat * nx_fk * 13
                fkv["rows"].append({"nrep": nrep, "eval_ms": t_eval, "evals_per_s": nrep * nx_fk * 13 / (t_eval * 1e-3),
                                    "contract_ms": t_fk, "contract_tflops": flops / (t_fk * 1e-3) / 1e12,
                                    "contract_frac_fp64_peak": flops / (t_fk * 1e-3) / 78.6e12,
                                    "paper_table2_gpu_s_context": paper_gpu_s[nrep]})
                plan.destroy()
                del F, T
            V["members_fk"] = fkv
            for m_ in fk_ids:
                pdfmi.unload(m_)

        try:
            variants()
        except Exception as exc:  # a failing variant must not cost the headline line
            import traceback
            traceback.print_exc()
            V["error"] = "%s: %s" % (type(exc).__name__, exc)

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(args, g, x, q2, qk, a)
    print(json.dumps(res), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, g, x, q2, qk, a):
    """The FP64 oracle timed on the host: x*f of every flavour plus alpha_s at
    each point (the GPU step's work), all cores (OpenMP over points; alpha_s in
    as many threads) and one core, wall time of the evaluation calls only,
    median of 5 after one warm-up.  Bounded samples of each workload, scaled to
    evaluations per second."""
    import statistics
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    from paper_2009_06635_amd import synth

    cores = max(1, min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1))
    pool = ThreadPoolExecutor(max_workers=cores)

    def alphas(qk_, a_, qq, threads):
        if threads == 1:
            return oracle.alphas_q2(qk_, a_, qq)
        parts = np.array_split(qq, threads)
        return np.concatenate(list(pool.map(lambda p: oracle.alphas_q2(qk_, a_, p), parts)))

    def median_time(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    def leg(name, fn_of_threads, evals, sample_desc, n1_frac):
        """fn_of_threads(threads, frac) runs the sample (frac of it on one core)."""
        t_all = median_time(lambda: fn_of_threads(cores, 1.0))
        t_one = median_time(lambda: fn_of_threads(1, n1_frac))
        return {"evals_per_s_all_cores": evals / t_all, "evals_per_s_one_core": evals * n1_frac / t_one,
                "sample": sample_desc, "all_cores_s": t_all, "one_core_s": t_one}

    out = {"unit": "PDF evals/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
           "timing": "median of 5 after one warm-up, evaluation calls only"}
    # headline: three-sub-grid grid, all 13 flavours + alpha_s
    og = oracle.Grid(g.xknots, g.q2knots, g.values, g.pids)
    nh = min(args.cpu_sample, args.n)
    xs_, qs_ = np.ascontiguousarray(x[:nh]), np.ascontiguousarray(q2[:nh])
    P = len(g.pids)

    def head(threads, frac):
        m = max(1, int(nh * frac))
        oracle.xfxq2(og, g.pids, xs_[:m], qs_[:m], n_threads=threads)
        alphas(qk, a, qs_[:m], threads)
    out["headline"] = leg("headline", head, nh * P,
                          "first %d of the %d headline points (one core: a tenth of them), all %d flavours "
                          "+ alpha_s" % (nh, args.n, P), 0.1)
    out["value"] = out["headline"]["evals_per_s_all_cores"]
    out["sample"] = out["headline"]["sample"]
    # small workload (one sub-grid, 11 flavours, 1e5 points) + alpha_s
    g1 = synth.config1_grid()
    og1 = oracle.Grid(g1.xknots, g1.q2knots, g1.values, g1.pids)
    x1, q1 = synth.config1_queries()
    qk1, a1 = synth.config1_alphas()

    def small(threads, frac):
        m = max(1, int(len(x1) * frac))
        oracle.xfxq2(og1, g1.pids, x1[:m], q1[:m], n_threads=threads)
        alphas(qk1, a1, q1[:m], threads)
    out["small"] = leg("small", small, len(x1) * len(g1.pids),
                       "all 1e5 points, 11 flavours + alpha_s (one core: a quarter)", 0.25)
    # batched workload: 101 members, 200 requests; the first 2000 points of every request
    members = synth.config3_members()
    ogm = [oracle.Grid(mg.xknots, mg.q2knots, mg.values, mg.pids) for mg in members]
    reqs = synth.config3_requests()
    sub = [(r["member"], r["pids"], np.ascontiguousarray(r["x"][:2000]), np.ascontiguousarray(r["q2"][:2000]))
           for r in reqs]
    nev = sum(len(s_[2]) * len(s_[1]) for s_ in sub)

    def batched(threads, frac):
        for mi, pids, xr, qr in sub[:max(1, int(len(sub) * frac))]:
            oracle.xfxq2(ogm[mi], pids, xr, qr, n_threads=threads)
    out["batched"] = leg("batched", batched, nev,
                         "first <= 2000 points of each of the 200 requests (one core: the first 50 requests)", 0.25)
    # Monte-Carlo load: two lookups of 13 flavours at a shared scale + alpha_s + the luminosity sum
    cx1, cx2, cq = synth.config5_chunk(0)
    nm = 200_000
    cx1, cx2, cq = cx1[:nm], cx2[:nm], cq[:nm]

    def mc(threads, frac):
        m = max(1, int(nm * frac))
        f1 = oracle.xfxq2(og1, synth.PIDS_13, cx1[:m], cq[:m], n_threads=threads)
        f2 = oracle.xfxq2(og1, synth.PIDS_13, cx2[:m], cq[:m], n_threads=threads)
        al = alphas(qk1, a1, cq[:m], threads)
        math.fsum(al * np.sum(f1 * f2, axis=1))
    out["mc"] = leg("mc", mc, nm * 26,
                    "first %d points of chunk 0 (26 evaluations + alpha_s each; one core: a tenth)" % nm, 0.1)
    pool.shutdown()
    return out


if __name__ == "__main__":
    main()
