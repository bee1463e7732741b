#!/usr/bin/env python3
"""Benchmark of the LAMG+ solve on one MI355X.

Metric: nnz(L) * RHS solved per second to ||b - L phi|| / ||b|| <= 1e-8, FP32 cycles inside
FP64 iterative refinement (the reported `value`) beside plain FP64 cycles, with p50/p99
solve latency. One step = one complete solve of the workload's right-hand-side block from
a zero start, hierarchy resident on the device and b already in HBM.

Default workload: the 128^3 7-point grid with lognormal(0,1) edge weights
(n = 2,097,152, nnz(L) = 2m + n = 14,581,760) with 32 right-hand sides b ~ N(0,1) (mean
removed by the solver) solved together: the largest nnz * RHS per solve of the measured
configurations that fits one GPU. Other workloads behind --workload / --nrhs.

The JSON line also carries
  roofline:   the dominant kernel by time (kernel kind and precision, every level) in a
              second, evented FP32+IR region of the same solves: the library attaches a pair
              of HIP events (the dispatch's own start and end timestamps) to every launch on
              the solve stream; achieved = the kind's summed algorithmic bytes / its summed
              launch durations, against 8 TB/s HBM;
  whole_solve: algorithmic bytes of every launch of one solve (the library's count) over the
              solve's wall time, with the working set beside it;
  kernels:    the same in-situ figures for every kernel kind;
  cpu_baseline: the CPU oracle (FP64, single-threaded) solving column 0 of the same block on
              one core, setup excluded, and an aggregate leg of one oracle process per
              available core (up to 15) solving one column each; the host CPU model and core
              counts; the oracle's solutions of columns 0 and k-1 give err_vs_oracle.
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
MALL_BYTES = 256 << 20
WORKLOADS = {
    "lognormal128": "3D 7-point grid 128^3, lognormal(0,1) edge weights",
    "aniso1024": "2D 5-point grid 1024x1024, weight 1 on x-edges and 1e-3 on y-edges",
    "chunglu2m": "Chung-Lu n=2M, degree exponent 2.1, mean degree 16, LCC, weights U[1,2]",
    "grid64": "2D 5-point grid 64x64, unit weights",
    "rgg1m": "random geometric graph, 1M points in the unit square, mean degree 10, LCC, unit "
             "weights, numbered in the points' random draw order",
}
KIND_SYMBOLS = {  # kernel kinds and the kernel symbols a rocprofv3 trace shows for them
    "gs_color": "k_csr / k_csr_vec / k_csr_mixed / k_csr_mixed_vec / k_csr_long with OP_GS (0)",
    "residual": "k_csr / k_csr_vec / k_csr_mixed / k_csr_mixed_vec / k_csr_long with OP_RESID (1)",
    "restrict": "k_csr / k_csr_vec / k_csr_mixed / k_csr_mixed_vec / k_csr_long with OP_SPMV (2)",
    "prolong": "k_red_partial<T, 0> + k_prolong_mu (or k_red_final<0> + k_prolong), k_inject_add",
    "tail": "k_tail",
    "reduce": "k_red_partial / k_red_final / k_rc2_fused / k_rc2_update / k_rcf_update",
    "vector": "k_copy / k_fill / k_gather_cols / k_scatter_cols / k_sub_col / k_to_f32_scaled / "
              "k_add_scaled_f32 / k_zero_cols / k_to_cols / k_from_cols / k_fill_i64 / k_coarsest",
    "cheb": "k_csr / k_csr_vec / k_csr_mixed / k_csr_mixed_vec / k_csr_long with OP_CHEB (3) + k_add_into",
    "bjgs": "k_bjgs (+ the residual launch before it, which a trace counts as residual)",
}


def kernel_kind(name: str):
    """(kind, precision) of a kernel symbol as a rocprofv3 trace shows it, in the grouping of
    the library's in-situ timer (KIND_SYMBOLS); (None, None) for setup and library kernels."""
    import re

    base = name.replace("(anonymous namespace)", "").split("(")[0]
    m = re.search(r"(k_csr_mixed_vec|k_csr_mixed|k_csr_long|k_csr_vec|k_csr)<(float|double), (\d)", base)
    if m:
        kind = {"0": "gs_color", "1": "residual", "2": "restrict", "3": "cheb"}[m.group(3)]
        return kind, "fp32" if m.group(2) == "float" else "fp64"
    prec = "fp32" if "<float" in base else ("fp64" if "<double" in base else None)
    if "k_tail" in base:
        return "tail", prec
    if "k_bjgs" in base:
        return "bjgs", prec
    for key, kind in (("k_prolong", "prolong"), ("k_inject_add", "prolong"), ("k_red_", "reduce"),
                      ("k_rc2_", "reduce"), ("k_rcf_update", "reduce"), ("k_add_into", "cheb")):
        if key in base:
            return kind, prec or "fp64"
    for key in ("k_copy", "k_fill", "k_gather_cols", "k_scatter_cols", "k_sub_col",
                "k_to_f32_scaled", "k_add_scaled_f32", "k_zero_cols", "k_to_cols", "k_from_cols",
                "k_fill_i64", "k_coarsest"):
        if key in base:
            return "vector", prec or "fp64"
    return None, None


KERNEL_SOURCES = ("cycle_kernels.hip", "csr_device.h", "tail_kernel.hip", "lamg_internal.h",
                  "solve.cpp")


def kernel_source_hash() -> str:
    """Hash of the sources that decide the solve's kernels and launches: a traffic record
    taken with other sources is not reported."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_24791_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_path(workload: str, k: int) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{workload}_k{k}.json")


def summarize_profile(d: str, workload: str, k: int, copy_bytes: int, record: bool) -> int:
    """Per kernel kind and precision: calls, total and average duration from a rocprofv3
    --stats kernel_stats.csv; from a --pmc run, the counter's KiB per dispatch, calibrated by
    the run's last device copy (the --copy-probe-mb probe, copy_bytes read and written).
    With `record`, the calibrated counters go into the workload's traffic record."""
    import csv
    import glob

    out = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        agg = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                kind, prec = kernel_kind(r["Name"])
                if kind is None:
                    continue
                a = agg.setdefault((kind, prec), [0, 0.0])
                a[0] += int(r["Calls"])
                a[1] += float(r["TotalDurationNs"])
        out.append(f"kernel statistics ({os.path.relpath(path, d)}):")
        out.append(f"  {'kind':<10} {'prec':<5} {'calls':>8} {'total ms':>10} {'avg us':>9}")
        for (kind, prec), (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
            out.append(f"  {kind:<10} {prec:<5} {c:>8} {t / 1e6:>10.2f} {t / c / 1e3:>9.3f}")
    rec = None
    if record and os.path.exists(traffic_path(workload, k)):
        with open(traffic_path(workload, k)) as fh:
            rec = json.load(fh)
        if rec.get("source_hash") != kernel_source_hash():
            rec = None
    if rec is None:
        rec = dict(workload=workload, nrhs=k, source_hash=kernel_source_hash(), kinds={},
                   probe={})
    for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        per = {}  # dispatch -> [name, {counter: value}]
        with open(path) as fh:
            for r in csv.DictReader(fh):
                e = per.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], {}])
                e[1][r["Counter_Name"]] = e[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        counters = sorted({c for _, cv in per.values() for c in cv})
        copies = [i for i, (name, _) in per.items() if "copyBuffer" in name or "k_copy" in name]
        probe_id = max(copies) if copies else None
        out.append(f"hardware counters ({os.path.relpath(path, d)}), KiB per dispatch:")
        for cn in counters:
            probe = per[probe_id][1].get(cn, 0.0) if probe_id is not None else 0.0
            factor = copy_bytes / (1024.0 * probe) if probe > 0 and copy_bytes > 0 else None
            out.append(f"  probe (last copy, {copy_bytes} bytes each way): {cn} {probe:.1f} KiB"
                       f" -> factor {factor}")
            agg = {}
            for name, cv in per.values():
                kind, prec = kernel_kind(name)
                if kind is None or cn not in cv:
                    continue
                a = agg.setdefault((kind, prec), [0, 0.0])
                a[0] += 1
                a[1] += cv[cn]
            for (kind, prec), (c, v) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
                out.append(f"  {cn:<11} {kind:<10} {prec:<5} dispatches {c:>7} "
                           f"mean {v / c:>12.2f} KiB")
                if factor is not None:
                    e = rec["kinds"].setdefault(f"{kind}_{prec}", {})
                    e["dispatches"] = c
                    e[f"{cn.lower()}_kib_per_dispatch"] = v / c
                    e[f"{cn.lower()}_bytes_per_dispatch"] = v / c * 1024.0 * factor
            rec["probe"][cn] = dict(copy_bytes=copy_bytes, counter_kib=probe, factor=factor)
            # the largest kernel symbols on their own (the timed level's passes carry
            # separate symbols)
            sym = {}
            for name, cv in per.values():
                if kernel_kind(name)[0] is None or cn not in cv:
                    continue
                short = name.replace("(anonymous namespace)::", "").replace("void ", "")
                short = short.replace("lamg::", "").split("(")[0]
                a = sym.setdefault(short, [0, 0.0])
                a[0] += 1
                a[1] += cv[cn]
            for short, (c, v) in sorted(sym.items(), key=lambda kv: -kv[1][1])[:8]:
                out.append(f"  {cn:<11} {short:<40} dispatches {c:>7} mean {v / c:>12.2f} KiB")
                if factor is not None:
                    e = rec.setdefault("symbols", {}).setdefault(short, {})
                    e["dispatches"] = c
                    e[f"{cn.lower()}_bytes_per_dispatch"] = v / c * 1024.0 * factor
    if record and rec["kinds"]:
        with open(traffic_path(workload, k), "w") as fh:
            json.dump(rec, fh, indent=1)
        out.append(f"traffic record: {os.path.relpath(traffic_path(workload, k), ROOT)}")
    print("\n".join(out))
    return 0


def traffic_of(workload: str, k: int, key: str):
    """HBM bytes per launch of a kernel kind (FETCH_SIZE + WRITE_SIZE, calibrated) from the
    workload's traffic record, if the record was taken with the current kernel sources."""
    try:
        with open(traffic_path(workload, k)) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    e = rec.get("kinds", {}).get(key, {})
    if "fetch_size_bytes_per_dispatch" not in e or "write_size_bytes_per_dispatch" not in e:
        return None
    return e["fetch_size_bytes_per_dispatch"] + e["write_size_bytes_per_dispatch"]


def host_cpu() -> dict:
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(model=model, logical_cpus=os.cpu_count(),
                usable_cpus=len(os.sched_getaffinity(0)))


# --- the CPU oracle legs (run in spawned worker processes) ------------------------------

def oracle_column(args):
    """Worker: the oracle's hierarchy of the workload and the FP64 solve of one column.
    Returns (column, phi, setup seconds, solve seconds, cycles)."""
    name, k, col, tol, opts = args
    import numpy as np  # noqa: F401

    import oracle as O
    from paper_2606_24791_amd import inputs as I

    g = I.workload(name)
    b = I.rhs(g.n, k, seed=0)[col]
    t = time.perf_counter()
    oh = O.Hierarchy(g, seed=1, **opts)
    t_setup = time.perf_counter() - t
    t = time.perf_counter()
    phi, so, _ = oh.solve(b, tol, 300)
    t_solve = time.perf_counter() - t
    return col, phi, t_setup, t_solve, so["cycles"]


def percentile(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs), q))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lognormal128", choices=sorted(WORKLOADS))
    ap.add_argument("--nrhs", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-procs", type=int, default=-1,
                    help="oracle processes of the aggregate CPU leg (-1: usable cores up to 16, "
                         "minus one; 0: no aggregate leg)")
    ap.add_argument("--n-direct", type=int, default=0,
                    help="levels up to this size are solved directly (0: library default)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed region, one device copy of this many MB (calibrates "
                         "the HBM byte counters of a profiler run)")
    ap.add_argument("--tail-rows", type=int, default=-1,
                    help="coarse-tail threshold option (-1: library default)")
    ap.add_argument("--reorder", action="store_true",
                    help="renumber the input by the self-gated reverse Cuthill-McKee order "
                         "(option reorder)")
    ap.add_argument("--no-setup-warmup", action="store_true",
                    help="skip the untimed setup and solve of a small grid that precedes the "
                         "workload's setup (profiler runs: its kernels would enter their "
                         "per-kernel averages)")
    ap.add_argument("--smoother", type=int, default=0,
                    help="0: multicolour Gauss-Seidel; 1: Chebyshev on levels with > 32 colours; "
                         "2: block-Jacobi Gauss-Seidel on those levels")
    ap.add_argument("--tail-finest", type=int, default=0,
                    help="FP32+IR cycles of a finest level up to this size run wholly in the "
                         "coarse tail (0: library default, never)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay each cycle as a HIP graph from the second solve on")
    ap.add_argument("--no-elimination", action="store_true",
                    help="aggregation-only hierarchy (no low-degree elimination levels)")
    ap.add_argument("--evented-steps", type=int, default=1,
                    help="solves per precision in the evented (per-launch timed) region "
                         "(0: none, no roofline or kernel table)")
    ap.add_argument("--fp32ir-only", action="store_true",
                    help="time only the FP32+IR solves (for hardware-counter runs)")
    ap.add_argument("--summarize-profile", metavar="DIR", default=None,
                    help="print per-kernel-kind figures of the rocprofv3 output under DIR "
                         "(kernel statistics, FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--record-traffic", action="store_true",
                    help="with --summarize-profile: store the calibrated counters in "
                         "profiles/traffic_<workload>_k<nrhs>.json")
    args = ap.parse_args()
    if args.summarize_profile:
        return summarize_profile(args.summarize_profile, args.workload, args.nrhs,
                                 args.copy_probe_mb << 20, args.record_traffic)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the solver has no multi-GPU path); got --gpus "
              f"{args.gpus}", file=sys.stderr)
        return 2
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    k = args.nrhs

    # Oracle worker processes are started before anything touches the GPU (a process that has
    # initialised the GPU must not start programs); they stay idle until the GPU part is done.
    pool, procs = None, 0
    cpu = host_cpu()
    if not args.no_cpu_baseline:
        import multiprocessing as mp

        usable = min(16, cpu["usable_cpus"])
        procs = (usable - 1) if args.cpu_procs < 0 else args.cpu_procs
        procs = max(0, min(procs, k, usable))
        pool = mp.get_context("spawn").Pool(max(1, procs))

    import numpy as np
    import torch

    from paper_2606_24791_amd import inputs as I
    from paper_2606_24791_amd import lamg as B

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

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
    if args.reorder:
        over["reorder"] = 1
    if args.graphs:
        over["graphs"] = 1
    if args.tail_finest:
        over["tail_finest"] = args.tail_finest
    opts = B.lamg_default_options(**over)
    # the first setup and solve of a process also pay the runtime's one-time start (device
    # context, first allocations, loading the library's code objects): an untimed setup and
    # solve of a small grid take them, and the workload's setup is then timed warm
    first_setup_s = None
    if not args.no_setup_warmup:
        gw = I.grid2d(48, 40)
        hw = B.lamg_setup(gw, opts)
        first_setup_s = B.lamg_hierarchy_info(hw)["setup_seconds"]
        bw = torch.tensor(I.rhs(gw.n, k, seed=0), device=dev)
        B.lamg_solve(hw, bw, torch.empty_like(bw), tol=args.tol, precision=B.FP32_IR)
        B.lamg_solve(hw, bw, torch.empty_like(bw), tol=args.tol, precision=B.FP64)
        torch.cuda.synchronize()
        hw.close()
    h = B.lamg_setup(g, opts)
    torch.cuda.synchronize()
    hi = B.lamg_hierarchy_info(h)
    log(f"setup {hi['setup_seconds']:.2f}s levels={hi['levels']} n={hi['n']} "
        f"colours={hi['ncolors']} elimination levels={[l for l, e in enumerate(hi['elim']) if e]} "
        f"tail from level {hi['tail_level']}")
    bh = I.rhs(g.n, k, seed=0)
    b = torch.tensor(bh, device=dev)
    stream = torch.cuda.current_stream()

    def run_steps(prec, phi, steps, evented):
        """`steps` solves between synchronisations; with `evented`, the library brackets every
        launch of every kernel with a pair of HIP events on `stream`."""
        torch.cuda.synchronize()
        if evented:
            B.lamg_timing_start_all(h, 1 << 18)
        lat, stats = [], None
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            stats = B.lamg_solve(h, b, phi, tol=args.tol, precision=prec, stream=stream)
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = B.lamg_timing_stop(h) if evented else None
        return wall, lat, stats, kt

    results = {}
    precs = (("fp32ir", B.FP32_IR),) if args.fp32ir_only else (("fp32ir", B.FP32_IR),
                                                                  ("fp64", B.FP64))
    for name, prec in precs:
        phi = torch.empty_like(b)
        for _ in range(args.warmup):
            B.lamg_solve(h, b, phi, tol=args.tol, precision=prec, stream=stream)
        wall, lat, stats, _ = run_steps(prec, phi, args.steps, False)
        if args.evented_steps > 0:
            wall_ev, _, _, kt = run_steps(prec, phi, args.evented_steps, True)
        else:
            wall_ev, kt = 0.0, None
        ms = 1e3 * wall / args.steps
        results[name] = dict(ms=ms, value=g.nnz_laplacian * k / (wall / args.steps),
                             p50_ms=1e3 * percentile(lat, 50), p99_ms=1e3 * percentile(lat, 99),
                             cycles=stats["cycles"], relres=stats["relres_max"],
                             converged=bool(stats["converged"]), phi=phi.cpu().numpy(),
                             graph_cycles=stats["graph_cycles"], bytes=stats["bytes"], kt=kt,
                             ev_steps=max(1, args.evented_steps), wall_ev=wall_ev)
        if kt is None:
            log(f"{name}: {ms:.3f} ms/solve, {results[name]['value']:.3e} nnz*RHS/s, "
                f"cycles={stats['cycles']}")
            continue
        log(f"{name}: {ms:.3f} ms/solve, {results[name]['value']:.3e} nnz*RHS/s, "
            f"cycles={stats['cycles']} relres={stats['relres_max']:.2e}, "
            f"{stats['bytes'] / 1e9:.2f} GB algorithmic per solve "
            f"({stats['bytes'] / (ms * 1e-3) / 1e9:.0f} GB/s); evented region "
            f"{1e3 * wall_ev / max(1, args.evented_steps):.3f} ms/solve")

    # per-kind in-situ figures of the FP32+IR evented region; the dominant kind by time
    r32 = results["fp32ir"]
    kinds = {}
    if r32["kt"] is None:  # a hardware-counter run: the timings only
        if args.copy_probe_mb > 0:
            nel = args.copy_probe_mb * (1 << 20) // 4
            src = torch.ones(nel, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            log(f"copy probe: {nel * 4} bytes read, {nel * 4} bytes written")
        print(json.dumps(dict(ms_per_step=r32["ms"], bytes_per_solve=r32["bytes"],
                              note="timings only (no evented region)")), flush=True)
        h.close()
        return 0
    for (kern, prec), t in r32["kt"].items():
        key = f"{B.KERNEL_NAMES[kern]}_{'fp32' if prec == B.FP32_IR else 'fp64'}"
        kinds[key] = dict(launches=t["launches"] // r32["ev_steps"],
                          us_per_launch=round(1e6 * t["seconds"] / t["launches"], 3),
                          GBs=round(t["bytes"] / t["seconds"] / 1e9, 1),
                          MB_per_launch=round(t["bytes"] / t["launches"] / 1e6, 4),
                          share=round(t["seconds"] / r32["wall_ev"], 4))
    (dk, dp), dt = max(r32["kt"].items(), key=lambda kv: kv[1]["seconds"])
    dname = B.KERNEL_NAMES[dk]
    achieved = dt["bytes"] / dt["seconds"] / 1e9
    log(f"dominant kernel: {dname} ({'fp32' if dp == B.FP32_IR else 'fp64'}), {dt['launches']} "
        f"launches, {1e6 * dt['seconds'] / dt['launches']:.2f} us each, "
        f"{dt['bytes'] / dt['launches'] / 1e6:.3f} MB each -> {achieved:.0f} GB/s")
    for key, v in sorted(kinds.items(), key=lambda kv: -kv[1]["share"]):
        log(f"  {key}: {v}")

    if args.copy_probe_mb > 0:
        nel = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nel * 4} bytes read, {nel * 4} bytes written")
        del src, dst

    hi2 = B.lamg_hierarchy_info(h)  # after the solves: hierarchy plus cached workspace
    h.close()

    # the CPU oracle: one core alone, then one process per core on separate columns
    cpu_line, errs = None, {}
    if pool is not None:
        oopts = dict(n_direct=opts.n_direct, elimination=bool(opts.elimination),
                     smoother=int(opts.smoother), reorder=int(opts.reorder))
        t = time.perf_counter()
        col0, phi0, ts0, tv0, cyc0 = pool.apply(oracle_column,
                                                ((args.workload, k, 0, args.tol, oopts),))
        log(f"oracle, one core: column 0 setup {ts0:.1f}s solve {tv0:.1f}s ({cyc0} cycles)")
        refs = {0: phi0}
        agg = None
        if procs > 1 or k > 1:
            cols = sorted({k - 1} | set(range(1, max(1, procs))))[:max(1, procs)]
            res = pool.map(oracle_column, [(args.workload, k, c, args.tol, oopts) for c in cols])
            for c, ph, _, _, _ in res:
                if c == k - 1:
                    refs[c] = ph
            rates = [g.nnz_laplacian / tv for _, _, _, tv, _ in res]
            if len(res) > 1:
                agg = dict(value=float(sum(rates)), unit="nnz*RHS/s", cores=len(res),
                           kind="oracle", sample=f"{len(res)} oracle processes at once, each "
                           f"solving one column of the same block (columns {cols[0]}..{cols[-1]}), "
                           f"setup excluded; value = sum of the processes' rates; solve "
                           f"{min(r[3] for r in res):.1f}-{max(r[3] for r in res):.1f}s each")
        pool.close()
        pool.join()
        for name in results:
            ph = results[name]["phi"]
            errs[name] = {f"col{c}": float(np.linalg.norm(ph[c] - ref) / np.linalg.norm(ref))
                          for c, ref in sorted(refs.items())}
        log(f"oracle errors: {errs} ({time.perf_counter() - t:.0f}s of oracle work)")
        cpu_line = dict(value=g.nnz_laplacian / tv0, unit="nnz*RHS/s", cores=1, kind="oracle",
                        sample=f"one FP64 solve of column 0 of the same block (tol {args.tol:g}, "
                               f"{cyc0} cycles, {tv0:.2f}s; setup {ts0:.2f}s excluded), one "
                               f"process alone",
                        host_cpu=cpu["model"], host_logical_cpus=cpu["logical_cpus"],
                        host_usable_cpus=cpu["usable_cpus"], nproc_leg=agg)

    r = results["fp32ir"]
    sv = lambda x: 4 if "fp32" in x else 8
    n0, e0 = hi["n"][0], hi["nnz"][0] - hi["n"][0]
    fine_ws = {p: e0 * (4 + sv(p)) + 4 * (n0 + 1) + 2 * n0 * sv(p) + 3 * k * n0 * sv(p)
               for p in ("fp32", "fp64")}
    whole = {}
    for name in results:
        rr = results[name]
        gbs = rr["bytes"] / (rr["ms"] * 1e-3) / 1e9
        whole[name] = dict(bytes_per_solve=rr["bytes"], achieved_GBs=round(gbs, 1),
                           frac=round(gbs / HBM_PEAK_GBS, 4))
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
            "workload": f"{args.workload}: {WORKLOADS[args.workload]}; {k} RHS b ~ N(0,1) "
                        f"mean-zero solved together, tol {args.tol:g}",
            "n": g.n, "nnz_L": g.nnz_laplacian, "nnz_2m": g.nnz, "nrhs": k,
            "levels": hi["levels"], "level_n": hi["n"], "op_complexity": round(hi["op_complexity"], 3),
            "setup_s": round(hi["setup_seconds"], 3),
            "first_setup_in_process_s": (None if first_setup_s is None
                                         else round(first_setup_s, 3)),
            "setup_phases_ms": {k: round(1e3 * v, 1) for k, v in hi["setup_phases"].items()},
            "elimination": bool(opts.elimination), "elimination_levels": sum(hi["elim"]),
            "smoother": {0: "gauss-seidel", 1: "chebyshev on levels with > 32 colours",
                         2: "block-jacobi gauss-seidel on levels with > 32 colours"}[opts.smoother],
            "chebyshev_levels": sum(hi["cheb"]),
            "block_jacobi_levels": sum(hi["bjgs"]),
            "reordered": hi["reordered"],
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
        "fp32ir_speedup_over_fp64": results["fp64"]["ms"] / r["ms"],
        "roofline": {"bound": "hbm",
                     "kernel": f"{dname} ({'fp32' if dp == B.FP32_IR else 'fp64'}): "
                               f"{KIND_SYMBOLS[dname]}, every level",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_of(args.workload, k,
                                           f"{dname}_{'fp32' if dp == B.FP32_IR else 'fp64'}"),
                     "traffic_source": os.path.relpath(traffic_path(args.workload, k), ROOT) +
                                       " (FETCH_SIZE + WRITE_SIZE per launch, each scaled by "
                                       "the counter's reading of a 256 MiB device copy; null "
                                       "unless taken with the current kernel sources)",
                     "bytes_per_launch": dt["bytes"] / dt["launches"],
                     "us_per_launch": 1e6 * dt["seconds"] / dt["launches"],
                     "launches_per_solve": dt["launches"] // r32["ev_steps"],
                     "share_of_solve": dt["seconds"] / r32["wall_ev"],
                     "timing": "HIP events (dispatch timestamps) on every launch of an evented "
                               "FP32+IR region of the same solves, on the solve stream"},
        "whole_solve": dict(whole, unit="GB/s", peak=HBM_PEAK_GBS,
                            bytes="algorithmic bytes of every launch of one solve "
                                  "(compulsory traffic per launch, library count)"),
        "working_set": {"device_bytes_hierarchy_and_workspace": hi2["bytes_device"],
                        "finest_level_one_sweep_bytes": fine_ws,
                        "mall_bytes": MALL_BYTES,
                        "finest_sweep_fits_mall": {p: v <= MALL_BYTES for p, v in fine_ws.items()}},
        "kernels": kinds,
        "cpu_baseline": cpu_line,
        "paper_context": "0.19 us/edge median solve, 1 CPU thread Apple M5 Pro (Julia), "
                         "SuiteSparse corpus; not this workload",
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
