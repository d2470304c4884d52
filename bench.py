"""Benchmark: SCVT P-LBFGS iterations per second at 1,048,576 generators.

Workload (one "step" = one Lloyd-preconditioned LBFGS iteration: two-loop
direction, Armijo line search with projected trial points, each trial a full
Voronoi build + cell quadrature + gradient/preconditioner/Lloyd step, and the
history update): n = 1,048,576 uniform random generators (seed 3), tanh
density with 16x spacing ratio (x_c at lat 30 lon 90, beta = pi/9,
alpha = 0.15), M = 10.  Generators start resident in HBM; the timed region is
K iterations from the seeded start, bracketed by device synchronisation.

The run ends with a serving leg at the stated accuracy: the first 16
requests of the seeded Poisson stream (20 req/s, n log-uniform in
[10,242, 655,362], each with its own tanh density) solved in mixed precision
to max |l| < 1e-8 with a 5,000-iteration cap; p50/p99 latency and throughput.

Prints one JSON line.  Options: --config C1|C2|C3|C4|C5 (default C3, the
workload above; C1 n=2,562 rho=1 to 1e-10, C2 n=163,842 8x tanh to 1e-8,
C4 the serving stream alone, 200 requests at each rate of --serving-rates,
C5 n=4,194,304 two-centre density, 100 iterations), --steps K (iteration cap,
default the workload's: 200 for C3), --warmup W, --precision fp64|mixed|both
(default both: `value` is the FP64 path, the "mixed" object the
mixed-precision path),
--no-cpu-baseline, --copy-calibration (only run a plain 256 MiB device copy,
used to scale the profiler's FETCH_SIZE / WRITE_SIZE counters), --copy-bandwidth
(only time a plain 1 GiB device copy: the practical HBM rate).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SCVT iterations/sec at 1M generators (FP64 vs mixed); p50/p99 solve latency"

# MI355X published peaks used as roofline denominators
PEAK_FP64_VECTOR_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP32_VECTOR_TFLOPS = 157.3  # published, with packed FP32 (not generated here)
PEAK_HBM_GBS = 8000.0


# Algorithmic FP64 operations of the tanh-density quadrature, counted once
# from the ISA of k_quad<tanh, fp64> as built here (FMA = 2, add/mul = 1,
# each rsqrt/reciprocal estimate = 1; clamps, rounding and exponent
# manipulation not counted):
FLOPS_PER_POINT = 89       # position, 1/|p| by its series, chord distance, table exp, logistic, moments
FLOPS_PER_LEAF = 15 + 21   # 12 midpoints per 16 leaves (20 each), det Jacobian
LEAVES_PER_EDGE = 16       # two geodesic subdivision levels
POINTS_PER_LEAF = 7


def cell_flops(mean_degree):
    leaf = POINTS_PER_LEAF * FLOPS_PER_POINT + FLOPS_PER_LEAF
    return mean_degree * LEAVES_PER_EDGE * leaf


# Sources that define the quadrature kernel: the HBM traffic recorded under
# profiles/ is reported only while these are unchanged.
QUAD_SOURCES = ["paper_1709_06924_amd/csrc/cells.hip", "paper_1709_06924_amd/csrc/cellgeom.h",
                "paper_1709_06924_amd/csrc/exp_table.h", "paper_1709_06924_amd/csrc/rules.h",
                "paper_1709_06924_amd/csrc/kernels.h"]
TRAFFIC_FILE = "profiles/hbm_traffic_k_quad_n1048576_tanh16_fp64.txt"


def quad_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in QUAD_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per k_quad dispatch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None
    when the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if kv.get("source_sha256") != quad_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


VALU_KINDS = ["f64 fma", "f64 mul", "f64 rsq", "f64 rcp", "f64 ldexp", "f64 rndne", "f64 max",
              "f32 fma", "f32 rsq", "f32 rcp", "f32 exp", "u32 add", "f64 rsq + 3 f64 fma",
              "f32 rsq + 3 f64 fma"]


def valu_rates():
    """ns per wave-instruction per SIMD of each instruction kind, and the
    FMA rates they imply (TFLOP/s over all SIMDs)."""
    import ctypes

    import torch

    from paper_1709_06924_amd import build
    torch.cuda.init()
    lib = ctypes.CDLL(build.CALIB_LIB)
    k = lib.scvt_calib_count()
    ns = (ctypes.c_double * k)()
    if lib.scvt_calib_valu(ns, 3) != 0:
        raise RuntimeError("scvt_calib_valu failed")
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    out = {"ns_per_wave_instr_per_simd": {VALU_KINDS[i]: round(ns[i], 4) for i in range(k)},
           "simds": simds}
    for name, idx in (("f64_fma_tflops", 0), ("f32_fma_tflops", 7)):
        out[name] = round(simds * 64 * 2 / (ns[idx] * 1e-9) / 1e12, 2)
    return out


def run_gpu(args, precision, Z0_dev, cfg, stream, max_iter, tol):
    import torch

    from paper_1709_06924_amd import scvt
    kw = dict(m_hist=cfg["m_hist"], precision=precision, stream=stream)
    if args.warmup > 0:
        W = scvt.Solver(Z0_dev, cfg["density"], **kw)
        for _ in range(args.warmup):
            W.step()
        W.close()
    S = scvt.Solver(Z0_dev, cfg["density"], keep_cells=False, **kw)
    F0 = S.energy()[0]
    S.set_timing(True, quad_only=True)  # two events per evaluation, around k_quad
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # max_iter iterations, or fewer when the Lloyd step falls below tol (tol 0:
    # exactly max_iter)
    info = S.solve(max_iter, tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = {"elapsed_s": t1 - t0, "info": info, "F0": F0, "iters": info["iter"]}
    ms, cnt = S.kernel_time(scvt.KERNEL_QUAD)
    out["quad"] = {"total_ms": ms, "launches": cnt}
    # the other kernels' times: every timer on, over the next iterations
    # (outside the timed region)
    S.set_timing(True)
    S.solve(info["iter"] + args.breakdown_steps, 0.0)
    for name, k in (("geom", scvt.KERNEL_CELLS), ("fallback", scvt.KERNEL_FALLBACK),
                    ("grid", scvt.KERNEL_GRID), ("lbfgs", scvt.KERNEL_LBFGS),
                    ("eval", scvt.KERNEL_EVAL), ("wide", scvt.KERNEL_CELLS_WIDE)):
        ms, cnt = S.kernel_time(k)
        out[name] = {"total_ms": ms, "launches": cnt}
    out["mean_degree"] = float(S.degrees().mean())
    S.close()
    return out


def mean_spacing(Z, nbr, deg):
    """h_i: mean chord distance from z_i to its Voronoi neighbours."""
    import numpy as np
    n = len(Z)
    rows = np.repeat(np.arange(n), deg)
    cols = nbr[np.arange(nbr.shape[1])[None, :] < deg[:, None]]
    dist = np.linalg.norm(Z[rows] - Z[cols], axis=1)
    return np.bincount(rows, dist, n) / np.maximum(deg, 1)


def mixed_errors(cfg, Z0_dev, stream, checkpoints=(0, 50, 100, 200)):
    """The mixed path's evaluation against the FP64 one at the FP64 iterates
    Z_0, Z_50, Z_100, Z_200 of the workload (both on the device): |dF|/F,
    max |dm|/m and max |d centroid| / h_i (h_i the mean distance to the
    cell's neighbours; also / R_i, the cell's circumradius)."""
    import numpy as np
    import torch

    from paper_1709_06924_amd import scvt
    kw = dict(m_hist=cfg["m_hist"], stream=stream)
    S = scvt.Solver(Z0_dev, cfg["density"], precision="fp64", keep_cells=True, **kw)
    out = []
    it = 0
    for k in checkpoints:
        while it < k:
            S.step()
            it += 1
        Z = torch.empty((S.n, 3), dtype=torch.float64, device="cuda:0")
        S.generators(Z)
        F64, m64, c64, _ = S.energy()
        R = S.vector("R")
        nbr, deg = S.neighbours()
        h = mean_spacing(S.generators(), nbr, deg)
        M = scvt.Solver(Z, cfg["density"], precision="mixed", **kw)
        Fmx, mmx, cmx, _ = M.energy()
        M.close()
        err = np.linalg.norm(cmx - c64, axis=1)
        out.append({"iteration": k, "dF_over_F": abs(Fmx - F64) / F64,
                    "max_dm_over_m": float(np.max(np.abs(mmx - m64) / m64)),
                    "max_dcentroid_over_h": float(np.max(err / h)),
                    "p99_dcentroid_over_h": float(np.percentile(err / h, 99)),
                    "max_dcentroid_over_R": float(np.max(err / R))})
    S.close()
    return out


def host_description():
    """nproc and the CPU model of the machine the oracle runs on."""
    import subprocess
    model = ""
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(cfg, Z0, iters):
    """The oracle as it stands, on the host: `iters` P-LBFGS iterations from
    the workload's start on all its threads; then the same evaluation's cell
    integrals re-timed on one thread over a sample of cells and scaled to the
    whole set (the hull and the vector algebra run on one thread anyway)."""
    import oracle
    from oracle import _clib
    L = _clib.lib()
    threads = int(L.oracle_num_threads())
    S = oracle.Solver(Z0, cfg["density"], m_hist=cfg["m_hist"])  # initial evaluation, untimed
    cells = S.cur.cells
    t0 = time.perf_counter()
    for _ in range(iters):
        S.step()
    dt = time.perf_counter() - t0
    evals = S.n_evals - 1
    n = len(Z0)
    t0 = time.perf_counter()
    oracle.cell_integrals(cells, cfg["density"])
    t_all = time.perf_counter() - t0
    sample = min(n, 131072)
    sub = type(cells).__new__(type(cells))
    sub.Z = cells.Z[:sample]
    sub.ptr = cells.ptr[:sample + 1]
    sub.verts = cells.verts
    L.oracle_set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.cell_integrals(sub, cfg["density"])
        t_one = (time.perf_counter() - t0) * n / sample
    finally:
        L.oracle_set_num_threads(threads)
    dt1 = dt + evals * (t_one - t_all)
    return {"value": iters / dt, "unit": "iterations/s", "cores": threads, "kind": "oracle",
            "sample": "%d FP64 oracle P-LBFGS iteration(s) (Qhull hull, C cell integrals on %d "
                      "threads, numpy two-loop) at n=%d from the seeded start; %d evaluation(s), "
                      "%.1f s" % (iters, threads, n, evals, dt),
            "single_thread": {"value": iters / dt1, "unit": "iterations/s", "cores": 1,
                              "sample": "the same iterations with their cell integrals re-timed "
                                        "on one thread over %d cells (%.2f s per evaluation "
                                        "against %.2f s on %d threads)"
                                        % (sample, t_one, t_all, threads)},
            "host": host_description()}


def cpu_baseline_sampled(cfg, Z0, every=16):
    """For sizes whose global hull is too slow to time within a benchmark
    run: one oracle evaluation (hull, cells, integrals on all threads) of
    every `every`-th generator of the seeded start -- a uniform random set
    of n/every points under the same density, so the same structure --
    scaled by `every` to n cells."""
    import oracle
    from oracle import _clib
    n = len(Z0)
    Zs = Z0[::every].copy()
    t0 = time.perf_counter()
    oracle.evaluate(Zs, cfg["density"])
    dt = (time.perf_counter() - t0) * n / len(Zs)
    return {"value": 1.0 / dt, "unit": "evaluations/s", "cores": int(_clib.lib().oracle_num_threads()),
            "kind": "oracle",
            "sample": "one FP64 oracle evaluation (Qhull hull, C cell integrals) of every %dth "
                      "generator of the seeded start (%d points), scaled to %d: %.1f s per "
                      "evaluation" % (every, len(Zs), n, dt),
            "host": host_description()}


WORKLOADS = {
    "C1": "n=2562 uniform start (seed 1), rho = 1, M=7, 100 iterations or max |l| < 1e-10",
    "C2": "n=163842 uniform start (seed 2), tanh density 8x (lat 30 lon 90, beta pi/6, "
          "alpha 0.2), M=7, solved to max |l| < 1e-8 (cap 20000)",
    "C3": "n=1048576 uniform start (seed 3), tanh density 16x (lat 30 lon 90, beta pi/9, "
          "alpha 0.15), M=10, 200 iterations",
    "C4": "Poisson stream (seed 4), n log-uniform in [10242, 655362], per-request tanh density "
          "(centre uniform on the sphere, beta in [pi/12, pi/4], alpha in [0.1, 0.3], ratio 4-16x), "
          "mixed precision, M=10, max |l| < 1e-8 with a 5000-iteration cap",
    "C5": "n=4194304 uniform start (seed 5), two-centre tanh density (lat +-45 lon 0, 16x and "
          "8x), M=10, 100 iterations",
}


def serve(rate, count, max_iter, slots):
    """The first `count` requests of the seeded stream at `rate` req/s,
    served to max |l| < 1e-8; per-request records and the summary."""
    import paper_1709_06924_amd.inputs as I
    from paper_1709_06924_amd import serving
    stream = I.serving_stream(seed=4, rate=rate, count=count)
    print("bench: serving %d requests at %g req/s" % (len(stream), rate), file=sys.stderr,
          flush=True)
    records, summ = serving.run_stream(
        stream, tol=1e-8, max_iter=max_iter, max_slots=slots, hbm_budget=64 << 30,
        precision="mixed", m_hist=10, log=lambda m: print(m, file=sys.stderr, flush=True))
    summ.update({"rate_rps": rate, "max_iter": max_iter, "max_slots": slots,
                 "hbm_budget_bytes": 64 << 30,
                 "n_total": sum(r["n"] for r in stream),
                 "iterations_total": sum(r["iters"] for r in records)})
    print("bench: %g req/s: %d/%d converged, p50 %.2f s, p99 %.2f s, %.3g generator-iterations/s"
          % (rate, summ["converged"], summ["requests"], summ["p50_s"], summ["p99_s"],
             summ["generator_iterations_per_s"]), file=sys.stderr, flush=True)
    return records, summ


def bench_serving(args):
    """C4: the serving stream alone at each rate; `value` is the p50 latency
    at the last rate (the stream's own 20 req/s by default)."""
    rates = [float(x) for x in args.serving_rates.split(",")]
    out = []
    for rate in rates:
        out.append(serve(rate, args.serving_requests, args.serving_max_iter, args.serving_slots)[1])
    last = out[-1]
    line = {"metric": "SCVT serving p50 solve latency at max |l| < 1e-8 (mixed)",
            "value": last["p50_s"], "unit": "s", "n_gpus": 1, "steps": last["requests"],
            "warmup": 0, "ms_per_step": 1000.0 * last["wall_s"] / max(last["requests"], 1),
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32-quadrature/f64-geometry", "data": "synthetic",
            "config": {"workload": "C4: " + WORKLOADS["C4"], "requests": args.serving_requests,
                       "rates_rps": rates, "max_iter": args.serving_max_iter,
                       "max_slots": args.serving_slots},
            "serving": out}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--config", default="C3", choices=sorted(WORKLOADS),
                    help="workload (default C3, the 1M-generator benchmark)")
    ap.add_argument("--steps", type=int, default=None,
                    help="iteration cap (default: the workload's, 200 for C3)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--copy-bandwidth", action="store_true",
                    help="only time a plain 1 GiB device copy (GB/s)")
    ap.add_argument("--valu-rates", action="store_true",
                    help="only measure vector-ALU instruction rates (libscvt_calib.so)")
    ap.add_argument("--no-mixed-errors", action="store_true",
                    help="skip the mixed-vs-FP64 evaluation errors at the FP64 iterates")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the quadrature kernel's sources and exit")
    ap.add_argument("--breakdown-steps", type=int, default=20,
                    help="iterations after the timed ones with every kernel timer on")
    ap.add_argument("--serving-requests", type=int, default=None,
                    help="requests of the serving stream (default 16 after C3, 200 for C4; "
                         "0 skips the serving leg)")
    ap.add_argument("--serving-rate", type=float, default=20.0)
    ap.add_argument("--serving-rates", default="5,10,20", help="C4: arrival rates (req/s)")
    ap.add_argument("--serving-max-iter", type=int, default=5000)
    ap.add_argument("--serving-slots", type=int, default=8)
    args = ap.parse_args()
    if args.source_hash:
        print(quad_source_hash())
        return
    if args.copy_calibration:
        import torch
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "copies": 3}))
        return
    if args.copy_bandwidth:
        # a STREAM-like copy (torch's device copy of 1 GiB, beyond the 256 MB MALL):
        # the practical HBM rate beside the 8 TB/s of the specification
        import torch
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        torch.cuda.synchronize()
        t0.record()
        for _ in range(reps):
            dst.copy_(src)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        moved = 2 * src.numel() * 8
        print(json.dumps({"copy_bytes": src.numel() * 8, "bytes_moved_per_copy": moved,
                          "ms_per_copy": round(ms, 4), "GB_per_s": round(moved / ms / 1e6, 1),
                          "fraction_of_8TBps": round(moved / ms / 1e6 / PEAK_HBM_GBS, 3)}))
        return
    if args.valu_rates:
        print(json.dumps(valu_rates()))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (its work would "
              "shard by cells, with halo exchange and one small allreduce per LBFGS pass); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.serving_requests is None:
        args.serving_requests = 200 if args.config == "C4" else 16
    if args.config == "C4":
        bench_serving(args)
        return

    import torch

    import paper_1709_06924_amd.inputs as I
    cfg = I.CONFIGS[args.config]
    n = cfg["n"]
    max_iter = args.steps if args.steps is not None else cfg["max_iter"]
    tol = cfg["tol"]
    Z0 = I.uniform_sphere(n, cfg["seed"])
    torch.cuda.set_device(0)
    Z0_dev = torch.from_numpy(Z0).to("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    print("bench: %s n=%d max_iter=%d tol=%g warmup=%d" % (args.config, n, max_iter, tol, args.warmup),
          file=sys.stderr, flush=True)

    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    if args.config in ("C1", "C2") and args.precision == "both":
        precisions = ["fp64"]  # FP64 workloads
    runs = {}
    for p in precisions:
        runs[p] = run_gpu(args, p, Z0_dev, cfg, stream, max_iter, tol)
        r = runs[p]
        print("bench: %s %.3f it/s (%d iterations, %d evals)"
              % (p, r["iters"] / r["elapsed_s"], r["iters"], r["info"]["n_evals"]),
              file=sys.stderr, flush=True)

    main_p = precisions[0]
    r = runs[main_p]
    value = r["iters"] / r["elapsed_s"]
    quad = r["quad"]
    avg_ms = quad["total_ms"] / max(quad["launches"], 1)
    flops = cell_flops(r["mean_degree"]) * n
    achieved = flops / (avg_ms * 1e-3) / 1e12
    traffic = recorded_traffic() if args.config == "C3" and main_p == "fp64" else None
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": r["iters"],
        "warmup": args.warmup,
        "ms_per_step": 1000.0 / value,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_p == "fp64" else "f32-quadrature/f64-geometry",
        "data": "synthetic",
        "config": {"workload": "%s: %s, %s" % (args.config, WORKLOADS[args.config], main_p),
                   "n": n, "m_hist": cfg["m_hist"], "quad": "7-point, 2 levels",
                   "iterations": r["iters"], "converged": bool(r["info"].get("converged")),
                   "tol": tol, "evals": r["info"]["n_evals"] - 1, "F_start": r["F0"],
                   "F_end": r["info"]["F"], "step_inf_end": r["info"]["step_inf"]},
        "kernels_ms_per_eval": {k: r[k]["total_ms"] / max(r[k]["launches"], 1)
                                for k in ("geom", "wide", "fallback", "quad", "grid", "eval")},
        "lbfgs_ms_per_iter": r["lbfgs"]["total_ms"] / max(r["lbfgs"]["launches"], 1),
        "kernels_timed": "quad: HIP events around k_quad over the timed iterations; the others: "
                         "every timer on over the %d iterations after them" % args.breakdown_steps,
        "roofline": {"kernel": "k_quad", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP64_VECTOR_TFLOPS if main_p == "fp64" else PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s",
                     "frac": achieved / (PEAK_FP64_VECTOR_TFLOPS if main_p == "fp64"
                                         else PEAK_FP32_VECTOR_TFLOPS),
                     "traffic": traffic, "flops_per_launch": flops, "avg_launch_ms": avg_ms,
                     "mean_degree": r["mean_degree"]},
    }
    for p in precisions[1:]:
        rr = runs[p]
        qms = rr["quad"]["total_ms"] / max(rr["quad"]["launches"], 1)
        qfl = cell_flops(rr["mean_degree"]) * n
        line[p] = {"value": rr["iters"] / rr["elapsed_s"], "unit": "iterations/s",
                   "ms_per_step": 1000.0 * rr["elapsed_s"] / rr["iters"],
                   "dtype": "f32 quadrature points, f64 geometry/accumulation/LBFGS",
                   "kernels_ms_per_eval": {k: rr[k]["total_ms"] / max(rr[k]["launches"], 1)
                                           for k in ("geom", "wide", "fallback", "quad", "grid", "eval")},
                   "F_end": rr["info"]["F"],
                   "roofline": {"kernel": "k_quad (mixed)", "bound": "alu",
                                "achieved": qfl / (qms * 1e-3) / 1e12,
                                "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                                "frac": qfl / (qms * 1e-3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                                "avg_launch_ms": qms}}
    if "mixed" in line and not args.no_mixed_errors:
        print("bench: mixed-vs-FP64 evaluation errors at the FP64 iterates", file=sys.stderr,
              flush=True)
        cps = tuple(k for k in (0, 50, 100, 200) if k <= max_iter)
        line["mixed"]["errors_vs_fp64"] = mixed_errors(cfg, Z0_dev, stream, cps)
    if args.serving_requests > 0 and args.config == "C3":
        line["serving"] = serve(args.serving_rate, args.serving_requests, args.serving_max_iter,
                                args.serving_slots)[1]
        line["serving"]["workload"] = ("Poisson %g req/s (seed 4), first %d requests: %s"
                                       % (args.serving_rate, args.serving_requests,
                                          WORKLOADS["C4"]))
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        if args.config == "C5":
            line["cpu_baseline"] = cpu_baseline_sampled(cfg, Z0)
        else:
            iters = {"C1": 100, "C2": 2, "C3": 1}[args.config]  # C1: the whole solve
            line["cpu_baseline"] = cpu_baseline(cfg, Z0, iters)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
