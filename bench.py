"""Benchmark: PDF evaluations per second on one MI355X.

Workload (one "step" = one pass of the hot path over one batch): 1e7 query
points of the three-sub-grid, 13-flavour synthetic set (196 x knots, 3 x 17
Q^2 knots split at the 1.51 / 4.92 GeV thresholds, 1% of the points outside
the grid), all flavours at every point in FP64 (pdf_xfxq2) plus alpha_s at
every point (pdf_alphas_q2).  Inputs are resident in device memory before the
timed region.  `value` counts PDF evaluations (points x flavours) only.

The FP32-arithmetic variant (pdf_xfxq2_f32) is timed the same way and reported
under "variants".  The dominant kernel's roofline uses its algorithmic bytes
(16 B of (x, Q^2) in + 8 B per output value) over its average duration
measured with HIP events on the launch stream.  cpu_baseline times the FP64
oracle on the host cores over a bounded sample of the same points.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("kernels.hip", "pdfmi.cpp", "pdfmi_dev.h"):
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


def cpu_baseline(grid, x, q2, sample):
    import numpy as np

    import oracle
    og = oracle.Grid(grid.xknots, grid.q2knots, grid.values, grid.pids)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = max(1, min(cores, os.cpu_count() or 1))
    xs, qs = np.ascontiguousarray(x[:sample]), np.ascontiguousarray(q2[:sample])
    oracle.xfxq2(og, grid.pids, xs[:1000], qs[:1000], n_threads=cores)   # warm
    t0 = time.perf_counter()
    oracle.xfxq2(og, grid.pids, xs, qs, n_threads=cores)
    dt = time.perf_counter() - t0
    return {"value": sample * len(grid.pids) / dt, "unit": "PDF evals/s", "cores": cores, "kind": "oracle",
            "sample": "first %d of the %d workload points, all %d flavours, FP64 oracle (OpenMP over points), "
                      "%.1f s wall" % (sample, len(x), len(grid.pids), dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=10_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(query points shard with no exchange; see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2009_06635_amd import pdfmi, synth

    dev = "cuda:0"
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

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn(None)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in evs:
            fn(e)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern = sum(e[0].elapsed_time(e[1]) for e in evs) / steps
        return wall, kern

    def step64(e):
        if e:
            e[0].record()
        pdfmi.xfxq2(member, g.pids, xd, qd, out=out64)
        if e:
            e[1].record()
        pdfmi.alphas_q2(qd, out=aout)

    def step32(e):
        if e:
            e[0].record()
        pdfmi.xfxq2_f32(member, g.pids, xd, qd, out=out32)
        if e:
            e[1].record()
        pdfmi.alphas_q2(qd, out=aout)

    wall64, k64 = timed(step64, args.steps, args.warmup)
    wall32, k32 = timed(step32, args.steps, args.warmup)
    evals = args.n * P
    bytes64 = args.n * (16 + 8 * P)
    bytes32 = args.n * (16 + 4 * P)
    ms64 = wall64 / args.steps * 1e3
    ach64 = bytes64 / (k64 * 1e-3) / 1e9
    ach32 = bytes32 / (k32 * 1e-3) / 1e9
    t64 = measured_traffic("xfxq2_f64")
    res = {
        "metric": "PDF evals/s (points x flavours), FP64 log-bicubic interpolation",
        "value": evals / (wall64 / args.steps),
        "unit": "PDF evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "xfxq2 all 13 flavours + alpha_s, 3 sub-grids (196 x 3x17 knots), "
                               "1e7 points, 1% outside the grid", "n_points": args.n, "n_flavours": P,
                   "subgrids": 3, "x_knots": 196, "q2_knots_per_subgrid": 17},
        "roofline": {"bound": "hbm", "achieved": ach64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach64 / HBM_PEAK_GBS,
                     "traffic": t64,
                     "kernel": "k_xfxq2<double> (pdf_xfxq2)", "kernel_ms": k64,
                     "algorithmic_bytes_per_launch": bytes64},
        "variants": {
            "f32": {"value": evals / (wall32 / args.steps), "ms_per_step": wall32 / args.steps * 1e3,
                    "kernel_ms": k32, "achieved_GBs": ach32, "frac": ach32 / HBM_PEAK_GBS,
                    "algorithmic_bytes_per_launch": bytes32, "kernel_evals_per_s": evals / (k32 * 1e-3)},
            "f64_kernel_evals_per_s": evals / (k64 * 1e-3),
        },
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(g, x, q2, min(args.cpu_sample, args.n))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
