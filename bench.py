#!/usr/bin/env python3
"""Benchmark of the LAMG+ solve on one MI355X.

Metric: nnz(L) * RHS solved per second to ||b - L phi|| / ||b|| <= 1e-8, FP32 cycles inside
FP64 iterative refinement (the reported `value`) beside plain FP64 cycles, with p50/p99
solve latency. One step = one complete solve of the workload's right-hand side block
from a zero start, hierarchy resident on the device and b already in HBM.

Default workload: the 1024 x 1024 grid-aligned anisotropic 5-point Laplacian (x-weight 1,
y-weight 1e-3; n = 1,048,576, nnz(L) = 2m + n = 5,238,784), b ~ N(0,1) (mean removed by
the solver), one right-hand side. Default hierarchy: low-degree elimination levels
alternating with aggregation (--no-elimination: aggregation only).

The JSON line also carries
  roofline: the FP32 Gauss-Seidel colour pass of the finest aggregation level (the largest
            full smoothing pass, the dominant bandwidth kernel; the finest level itself is an
            elimination level on the grids):
            its algorithmic bytes per launch over its mean launch time, both summed over
            every launch in a second timed FP32+IR region of the same K solves with HIP
            events attached to every launch on the solve stream (the throughput region runs
            without events; with --graphs it replays each cycle as a HIP graph, which needs
            events off), against 8 TB/s HBM;
  coarse_tail: the same timing of the coarse-level kernel (one workgroup per column), which takes the
            largest share of the solve and is bound by dependent steps, not bytes;
  cpu_baseline: the CPU oracle (single-threaded, FP64) solving the same system once.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "aniso1024": "2D 5-point grid 1024x1024, weight 1 on x-edges and 1e-3 on y-edges",
    "lognormal128": "3D 7-point grid 128^3, lognormal(0,1) edge weights",
    "chunglu2m": "Chung-Lu n=2M, degree exponent 2.1, mean degree 16, LCC, weights U[1,2]",
    "grid64": "2D 5-point grid 64x64, unit weights",
}


def kernel_source_hash() -> str:
    """Hash of the sources the cycle kernels are built from."""
    import hashlib

    h = hashlib.sha256()
    for f in ("cycle_kernels.hip", "csr_device.h"):
        with open(os.path.join(ROOT, "paper_2606_24791_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, k: int, elimination: bool):
    """HBM bytes per launch of the timed FP32 Gauss-Seidel colour pass from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on a copy kernel), or None
    when it does not cover this workload and hierarchy or the kernel sources changed since
    it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_gs_color.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("workload") != workload or t.get("nrhs") != k or \
            bool(t.get("elimination")) != elimination or \
            t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def percentile(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs), q))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="aniso1024", choices=sorted(WORKLOADS))
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-direct", type=int, default=0,
                    help="levels up to this size are solved directly (0: library default)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed region, one device copy of this many MB (calibrates "
                         "the HBM byte counters of a profiler run)")
    ap.add_argument("--tail-rows", type=int, default=-1,
                    help="coarse-tail threshold option (-1: library default)")
    ap.add_argument("--smoother", type=int, default=0,
                    help="0: multicolour Gauss-Seidel; 1: Chebyshev on levels with > 32 colours")
    ap.add_argument("--graphs", action="store_true",
                    help="replay each cycle as a HIP graph from the second solve on")
    ap.add_argument("--no-elimination", action="store_true",
                    help="aggregation-only hierarchy (no low-degree elimination levels)")
    ap.add_argument("--profile-reps", type=int, default=0,
                    help="also time the timed level's GS colour pass in isolation (back-to-back "
                         "launches)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the solver has no multi-GPU path); got --gpus "
              f"{args.gpus}", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2606_24791_amd import inputs as I
    from paper_2606_24791_amd import lamg as B

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)

    t = time.perf_counter()
    g = I.workload(args.workload)
    log(f"graph {args.workload}: n={g.n} nnz(L)={g.nnz_laplacian} ({time.perf_counter() - t:.1f}s)")
    over = {"n_direct": args.n_direct} if args.n_direct else {}
    if args.no_elimination:
        over["elimination"] = 0
    if args.tail_rows >= 0:
        over["tail_rows"] = args.tail_rows
    if args.smoother:
        over["smoother"] = args.smoother
    if args.graphs:
        over["graphs"] = 1
    opts = B.lamg_default_options(**over)
    h = B.lamg_setup(g, opts)
    torch.cuda.synchronize()
    hi = B.lamg_hierarchy_info(h)
    lt = hi["timed_level"]
    log(f"setup {hi['setup_seconds']:.2f}s levels={hi['levels']} n={hi['n']} "
        f"elimination levels={[l for l, e in enumerate(hi['elim']) if e]} "
        f"tail from level {hi['tail_level']}, timed level {lt}")
    k = args.nrhs
    bh = I.rhs(g.n, k, seed=0)
    b = torch.tensor(bh, device=dev)
    stream = torch.cuda.current_stream()

    def run_steps(prec, phi, timed):
        """K solves between synchronisations; with `timed`, the library brackets every launch
        of the timed level's kernels and of the coarse tail with HIP events on `stream`."""
        torch.cuda.synchronize()
        if timed:
            B.lamg_timing_start(h, 65536)
        lat, stats = [], None
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            stats = B.lamg_solve(h, b, phi, tol=args.tol, precision=prec, stream=stream)
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = B.lamg_timing_stop(h) if timed else None
        return wall, lat, stats, kt

    results = {}
    for name, prec in (("fp32ir", B.FP32_IR), ("fp64", B.FP64)):
        phi = torch.empty_like(b)
        for _ in range(args.warmup):
            B.lamg_solve(h, b, phi, tol=args.tol, precision=prec, stream=stream)
        wall, lat, stats, _ = run_steps(prec, phi, False)
        wall_ev, _, _, kt = run_steps(prec, phi, True)
        ms = 1e3 * wall / args.steps
        results[name] = dict(ms=ms, value=g.nnz_laplacian * k / (wall / args.steps),
                             p50_ms=1e3 * percentile(lat, 50), p99_ms=1e3 * percentile(lat, 99),
                             cycles=stats["cycles"], relres=stats["relres_max"],
                             converged=bool(stats["converged"]), phi=phi.cpu().numpy(),
                             graph_cycles=stats["graph_cycles"],
                             kt=kt, ms_events=1e3 * wall_ev / args.steps, wall=wall_ev)
        log(f"{name}: {ms:.3f} ms/solve ({stats['graph_cycles']} of {stats['cycles']} cycles "
            f"as graphs; {results[name]['ms_events']:.3f} kernel by kernel with events), "
            f"{results[name]['value']:.3e} nnz*RHS/s, cycles={stats['cycles']} "
            f"relres={stats['relres_max']:.2e}")

    # in-situ kernel times of the FP32+IR timed region
    r32 = results["fp32ir"]
    kt = r32["kt"]

    def kstat(kern, prec):
        t = kt.get((kern, prec))
        if not t:
            return None
        return dict(launches=t["launches"], us_per_launch=round(1e6 * t["seconds"] / t["launches"], 3),
                    GBs=round(t["bytes"] / t["seconds"] / 1e9, 1) if t["bytes"] else None,
                    share=round(t["seconds"] / r32["wall"], 4))

    gs = kt[(B.KERNEL_GS_COLOR, B.FP32_IR)]
    sec = gs["seconds"] / gs["launches"]
    byt = gs["bytes"] / gs["launches"]
    achieved = byt / sec / 1e9
    log(f"gs colour pass (level {lt}, fp32, in situ): {gs['launches']} launches, {sec * 1e6:.2f} us, "
        f"{byt / 1e6:.2f} MB -> {achieved:.0f} GB/s")
    other = {"residual": kstat(B.KERNEL_RESIDUAL, B.FP32_IR),
             "restrict": kstat(B.KERNEL_RESTRICT, B.FP32_IR),
             "prolong": kstat(B.KERNEL_PROLONG, B.FP32_IR),
             "residual_fp64_outer": kstat(B.KERNEL_RESIDUAL, B.FP64),
             "gs_color": kstat(B.KERNEL_GS_COLOR, B.FP32_IR)}
    tail = kstat(B.KERNEL_TAIL, B.FP32_IR)
    log(f"coarse tail (fp32, in situ): {tail}")
    isolated = None
    if args.profile_reps > 0:
        s2, b2 = B.lamg_profile_kernel(h, lt, B.KERNEL_GS_COLOR, B.FP32_IR, k, args.profile_reps,
                                       stream=stream)
        isolated = dict(us_per_launch=s2 * 1e6, GBs=b2 / s2 / 1e9, reps=args.profile_reps)

    if args.copy_probe_mb > 0:
        nel = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nel * 4} bytes read, {nel * 4} bytes written")
        del src, dst

    # the FP64 oracle: error of every result against it, and the CPU baseline
    cpu = None
    errs = {}
    if not args.no_cpu_baseline:
        import oracle as O

        t = time.perf_counter()
        oh = O.Hierarchy(g, seed=1, n_direct=opts.n_direct, elimination=bool(opts.elimination),
                         smoother=int(opts.smoother))
        t_setup = time.perf_counter() - t
        t = time.perf_counter()
        ref, so, _ = oh.solve(bh[0], args.tol, 300)
        t_solve = time.perf_counter() - t
        for name in results:
            ph = results[name]["phi"][0]
            errs[name] = float(np.linalg.norm(ph - ref) / np.linalg.norm(ref))
        cpu = dict(value=g.nnz_laplacian / t_solve, unit="nnz*RHS/s", cores=1, kind="oracle",
                   sample=f"one FP64 solve of the same system (1 RHS, tol {args.tol:g}, "
                          f"{so['cycles']} cycles, {t_solve:.2f}s; setup {t_setup:.2f}s excluded) "
                          f"on {platform.processor() or platform.machine()}")
        log(f"oracle: setup {t_setup:.2f}s solve {t_solve:.2f}s cycles {so['cycles']}; "
            f"err fp32ir {errs.get('fp32ir'):.2e} fp64 {errs.get('fp64'):.2e}")

    traffic = measured_traffic(args.workload, k, bool(opts.elimination))
    r = results["fp32ir"]
    line = {
        "metric": "nnz*RHS solved/s to 1e-8 rel resid (FP32 cycles + FP64 refinement)",
        "value": r["value"],
        "unit": "nnz*RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {WORKLOADS[args.workload]}; b ~ N(0,1) mean-zero, "
                        f"{k} RHS, tol {args.tol:g}",
            "n": g.n, "nnz_L": g.nnz_laplacian, "nnz_2m": g.nnz, "nrhs": k,
            "levels": hi["levels"], "op_complexity": round(hi["op_complexity"], 3),
            "setup_s": round(hi["setup_seconds"], 3),
            "elimination": bool(opts.elimination), "elimination_levels": sum(hi["elim"]),
            "smoother": "chebyshev on levels with > 32 colours" if opts.smoother else "gauss-seidel",
            "chebyshev_levels": sum(hi["cheb"]),
            "tail_level": hi["tail_level"],
        },
        "latency_ms": {"p50": r["p50_ms"], "p99": r["p99_ms"]},
        "cycles": r["cycles"],
        "relres": r["relres"],
        "err_vs_oracle": errs.get("fp32ir"),
        "fp64": {"value": results["fp64"]["value"], "ms_per_step": results["fp64"]["ms"],
                 "p50_ms": results["fp64"]["p50_ms"], "p99_ms": results["fp64"]["p99_ms"],
                 "cycles": results["fp64"]["cycles"], "relres": results["fp64"]["relres"],
                 "err_vs_oracle": errs.get("fp64")},
        "roofline": {"bound": "hbm",
                     "kernel": f"k_csr<float, GS> one colour pass of level {lt} (n={hi['n'][lt]}"
                               f"{', elimination level: its eliminated rows' if hi['elim'][lt] else ''})",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": byt, "us_per_launch": sec * 1e6,
                     "launches": gs["launches"], "timing": "HIP events attached to every launch "
                     "(dispatch timestamps) in a second timed FP32+IR region of the same K solves, "
                     "launched kernel by kernel, on the solve stream"},
        "kernels_timed_level": dict(other, level=lt),
        "coarse_tail": dict(tail or {}, bound="latency (dependent steps of one workgroup)",
                            kernel="k_tail<float>"),
        "launch_modes": {"graph_cycles_per_solve": r32["graph_cycles"],
                         "fp32ir_ms_kernel_by_kernel_with_events": r32["ms_events"],
                         "fp64_ms_kernel_by_kernel_with_events": results["fp64"]["ms_events"]},
        "gs_color_isolated": isolated,
        "cpu_baseline": cpu,
        "paper_context": "0.19 us/edge median solve, 1 CPU thread Apple M5 Pro (Julia), "
                         "SuiteSparse corpus; not this workload",
    }
    print(json.dumps(line), flush=True)
    h.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
