"""Benchmark of the fast random-walk Kalman filter on one MI355X.

Workload: the 256 x 256 crosswell case (N = 65536 cells, Matern nu = 3/2,
length 0.1, variance 1e-4, 24 x 20 = 480 straight rays, R = 1e-4 I, 50
assimilation steps), FP64.  Gamma (cluster tree + near-field assembly), the
ray operator, the observations and the unconditional draws are built before
the timed region and are resident in HBM.

One benchmark step is one pass of the whole hot path over the 50 observation
vectors: the generalized eigenproblem of the ray operator (cross covariance
P = Gamma H^T by H-matrix products, innovation Gram matrix, FP64 eigensolver,
basis), 50 constant-H filter steps, the variance field and 4 conditional
realizations.  The value is filter steps per second over the whole pass.
The one-column H-matrix product is benchmarked separately (HBM GB/s).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-matvec GB/s + Kalman steps/s at N=65536; mixed vs FP64 speedup @1e-6 error"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed passes")
    ap.add_argument("--warmup", type=int, default=1, help="untimed passes")
    ap.add_argument("--workload", default="crosswell-256x256")
    ap.add_argument("--realizations", type=int, default=4)
    ap.add_argument("--matvec-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(wl, H, n_panels=4, n_steps=5):
    """Time the CPU oracle on a bounded sample of one pass and extrapolate.

    One oracle pass = direct P = Gamma H^T (all row panels of 1024) + the
    exact cross-covariance filter recursion for all steps.  Sampled: n_panels
    of the direct row panels and n_steps recursion steps (on a P of the right
    shape), scaled to the full pass.
    """
    from oracle import kalman, kernels

    pts = wl.points()
    n = len(pts)
    panel = 1024
    t0 = time.perf_counter()
    for i in range(n_panels):
        rows = slice(i * panel, (i + 1) * panel)
        blk = kernels.cov_block(pts[rows], pts, wl.nu, wl.length, wl.variance)
        _ = np.asarray(H @ blk.T).T
    t_panel = (time.perf_counter() - t0) / n_panels
    n_total_panels = math.ceil(n / panel)
    # a cross covariance of the right shape with H P positive definite
    Pfake = np.asarray(H.T.todense()) * wl.variance
    ys = np.zeros((n_steps, H.shape[0]))
    R = np.full(H.shape[0], wl.noise_var)
    t0 = time.perf_counter()
    kalman.xcov_kf(Pfake, H, R, ys, wl.variance)
    t_step = (time.perf_counter() - t0) / n_steps
    t_pass = t_panel * n_total_panels + t_step * wl.steps
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = len(os.sched_getaffinity(0))
    return {"value": wl.steps / t_pass, "unit": "Kalman steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"direct Gamma H^T on {n_panels} of {n_total_panels} row panels "
                      f"({t_panel:.2f} s each) + {n_steps} of {wl.steps} cross-covariance "
                      f"filter steps ({t_step:.3f} s each), extrapolated to one pass "
                      f"({t_pass:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1405_2276_amd as fkf
    import workloads as W

    wl = W.WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    log(f"[bench] workload {wl.name} n={wl.n}")
    pts = wl.points()
    t0 = time.perf_counter()
    cov = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance, leaf_size=wl.leaf_size)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = cov.info()
    src, rcv = wl.rays()
    obs = fkf.Obs.from_rays(wl.shape, src, rcv, wl.noise_var)
    H = obs.csr()
    n_m = obs.n_m
    ys = torch.from_numpy(W.observations(wl)).to(dev)             # (steps, n_m), resident
    g = fkf.to_device(W.normals(wl, W.STREAM_DRAWS, (wl.n, args.realizations)))
    var_out = torch.empty(wl.n, dtype=torch.float64, device=dev)
    real_out = fkf.fortran_empty(wl.n, args.realizations)
    log(f"[bench] built Gamma in {t_build:.2f} s: {info}")

    def one_pass():
        f = fkf.Filter(cov)
        for k in range(wl.steps):
            f.step(obs, ys[k])
        f.variance(out=var_out)
        f.realize(g, out=real_out)
        f.close()

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    fkf.trace_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_pass()
    torch.cuda.synchronize()
    t_pass = (time.perf_counter() - t0) / args.steps
    trace = fkf.trace_report()
    fkf.trace_enable(False)
    log(f"[bench] pass {t_pass * 1e3:.2f} ms; trace {trace}")

    # ---- per-phase timing (one extra instrumented pass, events on the stream)
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    f = fkf.Filter(cov)
    ev[0].record(st)
    f.step(obs, ys[0])                   # basis (GEP) + first step
    ev[1].record(st)
    for k in range(1, wl.steps):
        f.step(obs, ys[k])
    ev[2].record(st)
    f.variance(out=var_out)
    ev[3].record(st)
    f.realize(g, out=real_out)
    ev[4].record(st)
    torch.cuda.synchronize()
    f.close()
    phases = {"gep_and_first_step": ev[0].elapsed_time(ev[1]),
              "steps_2_to_K": ev[1].elapsed_time(ev[2]),
              "variance": ev[2].elapsed_time(ev[3]),
              "realizations": ev[3].elapsed_time(ev[4])}
    step_us = phases["steps_2_to_K"] * 1e3 / max(wl.steps - 1, 1)

    # ---- one-column H-matrix product: warm and cold (Infinity Cache flushed)
    x = torch.randn(wl.n, dtype=torch.float64, device=dev)
    yv = torch.empty_like(x)
    for _ in range(3):
        cov.apply(x, out=yv)
    torch.cuda.synchronize()
    fkf.trace_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.matvec_reps):
        cov.apply(x, out=yv)
    e1.record(st)
    torch.cuda.synchronize()
    warm_us = e0.elapsed_time(e1) * 1e3 / args.matvec_reps
    tr_warm = fkf.trace_report()
    fkf.trace_enable(False)
    flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)     # 1 GiB > 256 MB MALL
    cold = []
    fkf.trace_enable(True)
    for _ in range(max(args.matvec_reps // 5, 5)):
        flush.fill_(1.0)
        e0.record(st)
        cov.apply(x, out=yv)
        e1.record(st)
        torch.cuda.synchronize()
        cold.append(e0.elapsed_time(e1) * 1e3)
    tr_cold = fkf.trace_report()
    fkf.trace_enable(False)
    del flush
    cold_us = float(np.mean(cold))
    n = wl.n
    mv_bytes = info["near_bytes"] + 8 * n + 8 * n + 8 * 2 * n   # near tiles, x, y, coordinates
    near_bytes = info["near_bytes"] + 8 * n
    c_near, ms_near = tr_cold.get("hmat_near_1rhs", (1, float("nan")))
    cold_near_us = ms_near * 1e3 / c_near
    c_nw, ms_nw = tr_warm.get("hmat_near_1rhs", (1, float("nan")))
    warm_near_us = ms_nw * 1e3 / c_nw
    hmatvec = {"cold_us": cold_us, "warm_us": warm_us,
               "alg_bytes": mv_bytes, "cold_gbs": mv_bytes / cold_us * 1e-3,
               "warm_gbs": mv_bytes / warm_us * 1e-3,
               "near_kernel_cold_us": cold_near_us, "near_kernel_warm_us": warm_near_us,
               "near_kernel_cold_gbs": near_bytes / cold_near_us * 1e-3,
               "kernel_us": {k: v[1] * 1e3 / max(v[0], 1) for k, v in tr_cold.items()}}
    log(f"[bench] hmatvec {hmatvec}")

    # ---- roofline of the dominant kernel of the pass
    per = {k: (c, ms) for k, (c, ms) in trace.items()}
    models = {
        # site: (bound, algorithmic units per launch, unit)
        "filter_gemv": ("hbm", 8.0 * n * n_m + 16.0 * n_m, "GB/s"),
        "filter_gemv_sq": ("hbm", 8.0 * n * n_m + 16.0 * n_m, "GB/s"),
        "hmat_near_multi": ("alu", 2.0 * n_m * info["n_near_pairs"] * 4096, "TFLOP/s"),
        "gep_basis_gemm": ("alu", 2.0 * n * n_m * n_m, "TFLOP/s"),
    }
    leaf_sites = [k for k in per if k not in ("gep_total", "gep_cross_cov", "filter_step")]
    dom = max(leaf_sites, key=lambda k: per[k][1])
    modelled = [k for k in leaf_sites if k in models]
    dom_m = max(modelled, key=lambda k: per[k][1]) if modelled else None
    roof = None
    if dom_m is not None:
        bound, units, unit = models[dom_m]
        c, ms = per[dom_m]
        avg_s = ms / c * 1e-3
        if unit == "GB/s":
            ach, peak = units / avg_s * 1e-9, HBM_PEAK_GBS
        else:
            ach, peak = units / avg_s * 1e-12, FP64_PEAK_TFLOPS
        roof = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                "traffic": None, "kernel": dom_m, "avg_launch_us": avg_s * 1e6,
                "launches_per_pass": c / args.steps,
                "share_of_pass": ms / args.steps / (t_pass * 1e3)}
    result = {
        "metric": METRIC,
        "value": wl.steps / t_pass,
        "unit": "Kalman steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_pass * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: N={n}, Matern nu={wl.nu} l={wl.length} "
                               f"theta={wl.variance}, {n_m} rays ({wl.n_src}x{wl.n_rcv}), "
                               f"R={wl.noise_var} I, {wl.steps} steps per pass",
                   "n": n, "n_m": n_m, "filter_steps_per_pass": wl.steps,
                   "realizations_per_pass": args.realizations, "precision": "fp64",
                   "leaf_size": wl.leaf_size, "cheb_p_per_level": info["cheb_p"],
                   "block_tol": 1e-7},
        "roofline": roof,
        "components": {
            "hmatvec_1rhs": hmatvec,
            "constant_h_step_us": step_us,
            "constant_h_steps_per_s": 1e6 / step_us,
            "phases_ms": phases,
            "dominant_site": dom,
            "sites_ms_per_pass": {k: v[1] / args.steps for k, v in per.items()},
            "gamma_build_s": t_build,
            "mixed_vs_fp64_speedup": None,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle sample")
        result["cpu_baseline"] = cpu_baseline(wl, H)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
