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
realizations.  The value is filter steps per second over the whole pass in
FP64.  Beside it: steps with a new operator every step (Section 2.4) and
steps of the extended filter for the Box-Cox observation model, both with
the relative rank truncation 1e-5, and the cost of the log-likelihood
gradient (theta, length, noise) relative to the filter run alone.  The same pass is then timed in the mixed-precision form (FP32 storage
and kernel evaluation, FP64 accumulation) and its speedup and per-result
error (against stored oracle values at sampled cells and against the FP64
form) are reported beside it.  The one-column H-matrix product is benchmarked
separately (HBM GB/s), cold and warm, in both forms.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
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
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision form")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two counter runs and exit")
    ap.add_argument("--matvec-only", choices=["fp64", "mixed"],
                    help="20 one-column products only (for profiler runs)")
    ap.add_argument("--profile", action="store_true",
                    help="one FP64 pass and a calibration copy only (for counter runs)")
    ap.add_argument("--batched-filters", type=int, default=64,
                    help="independent filters of uneven size stepped together (0: skip)")
    ap.add_argument("--varying-steps", type=int, default=4,
                    help="steps with a new measurement operator each (0: skip)")
    ap.add_argument("--no-gradient", action="store_true",
                    help="skip the log-likelihood gradient component")
    ap.add_argument("--boxcox-steps", type=int, default=4,
                    help="extended-filter steps of the Box-Cox observation model (0: skip)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_pass_time(wl, H, n_panels, n_steps):
    """Seconds of one oracle pass, extrapolated from n_panels row panels of
    the direct Gamma H^T and n_steps cross-covariance filter steps; returns
    (pass s, panel s, step s, total panels)."""
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
    return t_panel * n_total_panels + t_step * wl.steps, t_panel, t_step, n_total_panels


def cpu_baseline(wl, H, n_panels=4, n_steps=5):
    """Time the CPU oracle on a bounded sample of one pass and extrapolate,
    with the BLAS threads of the host and again on one thread.

    One oracle pass = direct P = Gamma H^T (all row panels of 1024) + the
    exact cross-covariance filter recursion for all steps.  Sampled: n_panels
    of the direct row panels and n_steps recursion steps (on a P of the right
    shape), scaled to the full pass; the one-thread figure samples half as
    many of each.
    """
    t_pass, t_panel, t_step, n_total_panels = _oracle_pass_time(wl, H, n_panels, n_steps)
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        with threadpool_limits(limits=1):
            t1 = _oracle_pass_time(wl, H, max(n_panels // 2, 1), max(n_steps // 2, 1))
    except Exception:  # pragma: no cover
        threads = len(os.sched_getaffinity(0))
        t1 = None
    out = {"value": wl.steps / t_pass, "unit": "Kalman steps/s", "cores": int(threads),
           "kind": "oracle",
           "sample": f"direct Gamma H^T on {n_panels} of {n_total_panels} row panels "
                     f"({t_panel:.2f} s each) + {n_steps} of {wl.steps} cross-covariance "
                     f"filter steps ({t_step:.3f} s each), extrapolated to one pass "
                     f"({t_pass:.1f} s)"}
    if t1 is not None:
        out["one_core"] = {"value": wl.steps / t1[0], "cores": 1,
                           "sample": f"{max(n_panels // 2, 1)} row panels ({t1[1]:.2f} s each) "
                                     f"+ {max(n_steps // 2, 1)} filter steps ({t1[2]:.3f} s "
                                     f"each), extrapolated to one pass ({t1[0]:.1f} s)"}
    return out


def time_passes(fkf, torch, cov, obs, ys, g, steps_per_pass, warmup, reps):
    """Mean wall time of one hot-path pass over `reps` timed passes, and the
    per-site trace (HIP events on the launching streams) of one further
    instrumented pass."""
    var_out = torch.empty(cov.n, dtype=torch.float64, device="cuda")
    real_out = fkf.fortran_empty(cov.n, g.shape[1])
    # one filter for all passes, returned to its initial state before each
    # (fkf_filter_reset keeps its device buffers: no allocation in the timed
    # passes once the warm-up pass has sized them)
    f = fkf.Filter(cov)

    def one_pass():
        f.reset()
        for k in range(steps_per_pass):
            f.step(obs, ys[k])
        f.variance(out=var_out)
        f.realize(g, out=real_out)

    for _ in range(warmup):
        one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one_pass()
    torch.cuda.synchronize()
    t_pass = (time.perf_counter() - t0) / reps
    # one more pass with per-site event timing (not part of the timed region)
    fkf.trace_enable(True)
    one_pass()
    torch.cuda.synchronize()
    trace = fkf.trace_report()
    fkf.trace_enable(False)
    f.close()
    return t_pass, trace


def final_results(fkf, torch, cov, obs, ys, g, steps_per_pass):
    """One instrumented pass: per-phase times and the final state, variance and
    realizations (host copies)."""
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    f = fkf.Filter(cov)
    ev[0].record(st)
    f.step(obs, ys[0])                   # basis (GEP) + first step
    ev[1].record(st)
    for k in range(1, steps_per_pass):
        f.step(obs, ys[k])
    ev[2].record(st)
    var = f.variance()
    ev[3].record(st)
    real = f.realize(g)
    ev[4].record(st)
    torch.cuda.synchronize()
    f.status()
    out = {"s": f.mean().cpu().numpy(), "var": var.cpu().numpy(), "real": real.cpu().numpy()}
    f.close()
    phases = {"gep_and_first_step": ev[0].elapsed_time(ev[1]),
              "steps_2_to_K": ev[1].elapsed_time(ev[2]),
              "variance": ev[2].elapsed_time(ev[3]),
              "realizations": ev[3].elapsed_time(ev[4])}
    return phases, out


def hmatvec_bench(fkf, torch, cov, info, reps):
    """One-column H-matrix product: warm (repeated) and cold (Infinity Cache
    flushed by a 1 GiB write before each product), both timed with the
    library's tracing off; the per-kernel breakdown comes from separate
    traced warm and cold runs."""
    n = cov.n
    st = torch.cuda.current_stream()
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    yv = torch.empty_like(x)
    for _ in range(3):
        cov.apply(x, out=yv)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")     # 1 GiB > 256 MB MALL

    def warm_loop():
        e0.record(st)
        for _ in range(reps):
            cov.apply(x, out=yv)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    def cold_loop():
        cold = []
        for _ in range(max(reps // 5, 5)):
            flush.fill_(1.0)
            e0.record(st)
            cov.apply(x, out=yv)
            e1.record(st)
            torch.cuda.synchronize()
            cold.append(e0.elapsed_time(e1) * 1e3)
        return float(np.mean(cold))

    warm_us = warm_loop()
    cold_us = cold_loop()
    fkf.trace_enable(True)
    warm_loop()
    tr_warm = fkf.trace_report()
    fkf.trace_enable(False)
    fkf.trace_enable(True)
    cold_loop()
    tr_cold = fkf.trace_report()
    fkf.trace_enable(False)
    del flush
    # algorithmic bytes of one product: stored near-field tiles, stored
    # far-field couplings, x, y and the point coordinates
    mv_bytes = info["near_bytes"] + info["far_bytes"] + 8 * n + 8 * n + 8 * 2 * n
    near_bytes = info["near_bytes"] + 8 * n
    c_near, ms_near = tr_cold.get("hmat_near_1rhs", (1, float("nan")))
    c_nw, ms_nw = tr_warm.get("hmat_near_1rhs", (1, float("nan")))
    cold_near_us, warm_near_us = ms_near * 1e3 / c_near, ms_nw * 1e3 / c_nw
    return {"cold_us": cold_us, "warm_us": warm_us,
            "alg_bytes": mv_bytes, "near_bytes": info["near_bytes"], "far_bytes": info["far_bytes"],
            "cold_gbs": mv_bytes / cold_us * 1e-3,
            "warm_gbs": mv_bytes / warm_us * 1e-3,
            "near_kernel_cold_us": cold_near_us, "near_kernel_warm_us": warm_near_us,
            "near_kernel_cold_gbs": near_bytes / cold_near_us * 1e-3,
            "kernel_us": {k: v[1] * 1e3 / max(v[0], 1) for k, v in tr_cold.items()}}


def varying_h(fkf, torch, cov, wl, ys, n_steps=4, rank_rtol=1e-5):
    """Steps with a new measurement operator every step: the crosswell rays
    and the same rays with x and y swapped (bottom-to-top), alternating.  Each
    step runs the cross covariance Gamma H_k^T, the rank update of the
    low-rank term and the innovation solve.  Returns per-step times (ms) and
    ranks; the observation vectors are the workload's own (timing only)."""
    src, rcv = wl.rays()
    obs = [fkf.Obs.from_rays(wl.shape, src, rcv, wl.noise_var),
           fkf.Obs.from_rays(wl.shape, np.ascontiguousarray(src[:, ::-1]),
                             np.ascontiguousarray(rcv[:, ::-1]), wl.noise_var)]
    st = torch.cuda.current_stream()
    f = fkf.Filter(cov, rank_rtol=rank_rtol)
    times, ranks = [], []
    for k in range(n_steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        f.step(obs[k % 2], ys[k])
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        ranks.append(f.info()["rank"])
    f.status()
    f.close()
    for o in obs:
        o.close()
    return {"step_ms": times, "rank": ranks, "rank_rtol": rank_rtol,
            "steady_steps_per_s": 1e3 / float(np.mean(times[1:])) if n_steps > 1 else None}


def extended_filter(fkf, torch, cov, wl, n_steps=4, a=4.0, rank_rtol=1e-5):
    """Steps of the extended filter for the Box-Cox observation model
    (fkf_filter_step_boxcox) with the workload's rays through the positive
    field exp(truth), transform parameter a and the paper's relative rank
    truncation 1e-5: every step linearises H_k = H diag(g'(x)) about the
    estimate, so each runs a fresh cross covariance Gamma H_k^T and the rank
    update of the low-rank term.  Returns per-step times (ms) and ranks."""
    src, rcv = wl.rays()
    obs = fkf.Obs.from_rays(wl.shape, src, rcv, wl.noise_var)
    wl_k = dataclasses.replace(wl, steps=n_steps)
    import workloads as W
    ys = torch.from_numpy(W.observations(wl_k, positive=True)).cuda()
    st = torch.cuda.current_stream()
    f = fkf.Filter(cov, rank_rtol=rank_rtol)
    times, ranks = [], []
    for k in range(n_steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        f.step_boxcox(obs, ys[k], a)
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        ranks.append(f.info()["rank"])
    f.status()
    f.close()
    obs.close()
    return {"step_ms": times, "rank": ranks, "rank_rtol": rank_rtol, "bc_alpha": a,
            "steady_steps_per_s": 1e3 / float(np.mean(times[1:])) if n_steps > 1 else None}


def loglik_gradient(fkf, torch, cov, wl, ys, reps=3):
    """The innovation log-likelihood and its derivatives in log theta, log
    length and log sigma^2 over the workload's steps: the filter run alone
    (GEP + steps, log-likelihood carried) against the same run with the length
    derivative tracked (one more n_m-column product with dGamma/d length at
    the basis build and an O(n_m^2) tangent update per step).  dGamma/d length
    is built once beforehand (its build time is reported).  Returns the
    times (best of reps), the ratio and the values."""
    pts = wl.points()
    src, rcv = wl.rays()
    obs = fkf.Obs.from_rays(wl.shape, src, rcv, wl.noise_var)
    t0 = time.perf_counter()
    dcov = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance,
                   leaf_size=wl.leaf_size, dlength=True)
    torch.cuda.synchronize()
    t_dbuild = time.perf_counter() - t0

    def run(track):
        f = fkf.Filter(cov)
        if track:
            f.track_length(dcov)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(wl.steps):
            f.step(obs, ys[k])
        out = f.loglik()
        dt = time.perf_counter() - t
        f.close()
        return dt, out

    run(True)                                   # warm-up (workspaces)
    tf = min(run(False)[0] for _ in range(reps))
    tg, vals = min((run(True) for _ in range(reps)), key=lambda r: r[0])
    dcov.close()
    obs.close()
    ll, d_th, d_nv, d_ln = vals
    return {"forward_ms": tf * 1e3, "with_gradient_ms": tg * 1e3, "gradient_over_forward": tg / tf,
            "dgamma_build_s": t_dbuild, "steps": wl.steps, "ll": ll, "dll_dlog_theta": d_th,
            "dll_dlog_length": d_ln, "dll_dlog_noise": d_nv}


# kernel (name prefix in the counter output) -> launch site of the trace
TRAFFIC_KERNELS = {
    "void fkf::(anonymous namespace)::k_tridiag<8, 1>": "eig_tridiag",
    "void fkf::k_couple_mfma2<2, false, true>": "hmat_far_couple_multi",
    "void (anonymous namespace)::k_near_sparse<double>": "hmat_near_sparse",
    "void fkf::k_down_mfma2<2>": "hmat_down_multi",
    "void (anonymous namespace)::k_up_sparse<2>": "hmat_far_up_sparse",
    "void fkf::k_gemv_panel<double, 0, false>": "filter_gemv",
    "fkf::k_gemm_tall": "gep_basis_gemm",
}
TRAFFIC_SOURCES = ["paper_1405_2276_amd/csrc/common.h", "paper_1405_2276_amd/csrc/kernels.h",
                   "paper_1405_2276_amd/csrc/hmat.hip", "paper_1405_2276_amd/csrc/linalg.hip",
                   "paper_1405_2276_amd/csrc/eig_dc.hip", "paper_1405_2276_amd/csrc/filter.hip"]


def _sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in sorted(files):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def write_traffic(fetch_csv, write_csv, out=None):
    """profiles/traffic.json from two counter runs of `bench.py --profile`
    (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, --output-format csv): the
    mean KiB per dispatch of each traced kernel, and the factors that map the
    counters of the calibration copy (2^25 doubles read after a cache flush,
    2^25 written) onto its true bytes."""
    import csv
    sites, calib = {}, {}
    for path, ctr in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != ctr:
                continue
            name = r["Kernel_Name"]
            if "AUnaryFunctor" in name and int(r["Grid_Size"]) == (1 << 23):
                calib[ctr] = float(r["Counter_Value"])
            for pref, site in TRAFFIC_KERNELS.items():
                if name.startswith(pref):
                    vals.setdefault(site, []).append(float(r["Counter_Value"]))
        for site, v in vals.items():
            sites.setdefault(site, {})["fetch_kib" if ctr == "FETCH_SIZE" else "write_kib"] = \
                float(np.mean(v))
    true_kib = (8 << 25) / 1024.0
    rec = {"fetch_factor": true_kib / calib["FETCH_SIZE"],
           "write_factor": true_kib / calib["WRITE_SIZE"],
           "calibration_kib": {"fetch": calib["FETCH_SIZE"], "write": calib["WRITE_SIZE"],
                               "true_each_way": true_kib},
           "sites": sites, "sources": TRAFFIC_SOURCES,
           "sources_sha256": _sources_sha256(TRAFFIC_SOURCES)}
    out = out or os.path.join(ROOT, "profiles", "traffic.json")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(out)


def traffic_for(site, path=None):
    """HBM bytes per launch of a kernel site from the committed counter runs
    (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE per dispatch, scaled by
    what the counters read for a copy kernel of known size), or None when
    absent or taken on different kernel sources."""
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if _sources_sha256(rec.get("sources", [])) != rec.get("sources_sha256"):
        return None
    k = rec.get("sites", {}).get(site)
    if k is None:
        return None
    return (k["fetch_kib"] * rec["fetch_factor"] + k["write_kib"] * rec["write_factor"]) * 1024.0


def many_filters(fkf, torch, count, reps=2):
    """Independent filters of uneven size (workloads.batch): every filter
    built and resident, then timed passes of `steps` steps of all filters,
    (a) together through fkf_filter_step_many (the bases' projected
    eigenproblems solved as one batch) and (b) one filter at a time.  Returns
    filter steps per second for both."""
    import workloads as W
    wls = W.batch(count)
    t0 = time.perf_counter()
    covs, obss, yss = [], [], []
    for wl in wls:
        covs.append(fkf.Cov(wl.points(), nu=wl.nu, length=wl.length, variance=wl.variance,
                            leaf_size=wl.leaf_size))
        src, rcv = wl.rays()
        obss.append(fkf.Obs.from_rays(wl.shape, src, rcv, wl.noise_var))
        yss.append(torch.from_numpy(W.observations(wl)).cuda())
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    steps = wls[0].steps

    def run(together):
        fs = [fkf.Filter(c) for c in covs]
        for k in range(steps):
            if together:
                fkf.step_many(fs, obss, [y[k] for y in yss])
            else:
                for f, o, y in zip(fs, obss, yss):
                    f.step(o, y[k])
        torch.cuda.synchronize()
        for f in fs:
            f.status()
            f.close()

    out = {"filters": count, "steps_each": steps, "n_total": int(sum(w.n for w in wls)),
           "n_m_range": [min(w.n_src * w.n_rcv for w in wls), max(w.n_src * w.n_rcv for w in wls)],
           "setup_s": t_setup}
    for name, together in (("together", True), ("one_by_one", False)):
        run(together)                               # warm-up
        t0 = time.perf_counter()
        for _ in range(reps):
            run(together)
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"pass_s": dt, "filter_steps_per_s": count * steps / dt}
    out["speedup_together"] = out["one_by_one"]["pass_s"] / out["together"]["pass_s"]
    for o in obss:
        o.close()
    for c in covs:
        c.close()
    return out


def accuracy(wl, res, ref64):
    """Per-result error of a pass: against the oracle's stored fields (when
    the workload has them; every cell) and against the FP64 GPU form over the
    whole field."""
    out = {}
    refp = os.path.join(ROOT, "tests", "golden", "headline_reference.npz")
    k = wl.steps
    if wl.name == "crosswell-256x256" and os.path.exists(refp):
        ref = np.load(refp)
        if f"s{k}" in ref and ref[f"s{k}"].shape == res["s"].shape:
            rs, rv = ref[f"s{k}"], ref[f"v{k}"]
            out["oracle_state_maxabs"] = float(np.abs(res["s"] - rs).max() / np.abs(rs).max())
            out["oracle_state_2norm"] = float(np.linalg.norm(res["s"] - rs) / np.linalg.norm(rs))
            out["oracle_var_maxabs"] = float(np.abs(res["var"] - rv).max() / np.abs(rv).max())
            out["oracle_var_cellrel"] = float((np.abs(res["var"] - rv) / np.abs(rv)).max())
    if ref64 is not None:
        out["fp64gpu_state"] = float(np.linalg.norm(res["s"] - ref64["s"])
                                     / np.linalg.norm(ref64["s"]))
        out["fp64gpu_var"] = float(np.abs(res["var"] - ref64["var"]).max()
                                   / np.abs(ref64["var"]).max())
        out["fp64gpu_realizations"] = float(np.linalg.norm(res["real"] - ref64["real"])
                                            / np.linalg.norm(ref64["real"]))
    return out


def main():
    args = parse()
    if args.traffic_from:
        write_traffic(*args.traffic_from)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
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
    n = wl.n
    ys = torch.from_numpy(W.observations(wl)).to(dev)             # (steps, n_m), resident
    g = fkf.to_device(W.normals(wl, W.STREAM_DRAWS, (wl.n, args.realizations)))
    log(f"[bench] built Gamma in {t_build:.2f} s: {info}")
    if args.matvec_only:
        # profiler runs of the one-column product alone: 20 products in the
        # given precision
        c = cov if args.matvec_only == "fp64" else fkf.Cov(
            pts, nu=wl.nu, length=wl.length, variance=wl.variance, leaf_size=wl.leaf_size,
            precision="mixed")
        x = torch.randn(wl.n, dtype=torch.float64, device=dev)
        yv = torch.empty_like(x)
        for _ in range(20):
            c.apply(x, out=yv)
        torch.cuda.synchronize()
        print(json.dumps({"matvec_only": args.matvec_only, "products": 20}), flush=True)
        return
    if args.profile:
        # counter runs: one FP64 pass and a plain copy of known size whose
        # FETCH_SIZE / WRITE_SIZE calibrate the counters (2^25 doubles read
        # from HBM after a cache flush, 2^25 written, by one elementwise kernel)
        a = torch.ones(1 << 25, dtype=torch.float64, device=dev)
        flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB > Infinity Cache
        flush.fill_(0.0)
        b = a * 2.0
        torch.cuda.synchronize()
        del flush
        t_pass, _ = time_passes(fkf, torch, cov, obs, ys, g, wl.steps, 0, 1)
        print(json.dumps({"profile_pass_ms": t_pass * 1e3, "copy_bytes_each_way": 8 << 25,
                          "check": float(b[0].item())}), flush=True)
        return

    # ---- FP64 form: the timed passes (the headline value)
    t_pass, trace = time_passes(fkf, torch, cov, obs, ys, g, wl.steps, args.warmup, args.steps)
    log(f"[bench] fp64 pass {t_pass * 1e3:.2f} ms; trace {trace}")
    phases, res64 = final_results(fkf, torch, cov, obs, ys, g, wl.steps)
    step_us = phases["steps_2_to_K"] * 1e3 / max(wl.steps - 1, 1)
    acc64 = accuracy(wl, res64, None)
    log(f"[bench] fp64 phases {phases} accuracy {acc64}")
    hmatvec = hmatvec_bench(fkf, torch, cov, info, args.matvec_reps)
    log(f"[bench] hmatvec fp64 {hmatvec}")
    many = None
    if args.batched_filters > 0:
        many = many_filters(fkf, torch, args.batched_filters)
        log(f"[bench] many filters {many}")
    vary = None
    if args.varying_steps > 0:
        vary = varying_h(fkf, torch, cov, wl, ys, args.varying_steps)
        log(f"[bench] varying-H steps {vary}")
    grad = None
    if not args.no_gradient:
        grad = loglik_gradient(fkf, torch, cov, wl, ys)
        log(f"[bench] log-likelihood gradient {grad}")
    ext = None
    if args.boxcox_steps > 0:
        ext = extended_filter(fkf, torch, cov, wl, args.boxcox_steps)
        log(f"[bench] extended (Box-Cox) steps {ext}")

    # ---- mixed form (FP32 storage / kernel evaluation, FP64 accumulation)
    mixed = None
    if not args.no_mixed:
        t0 = time.perf_counter()
        cov_m = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance,
                        leaf_size=wl.leaf_size, precision="mixed")
        torch.cuda.synchronize()
        t_build_m = time.perf_counter() - t0
        info_m = cov_m.info()
        t_pass_m, trace_m = time_passes(fkf, torch, cov_m, obs, ys, g, wl.steps, args.warmup,
                                        args.steps)
        log(f"[bench] mixed pass {t_pass_m * 1e3:.2f} ms; trace {trace_m}")
        phases_m, res_m = final_results(fkf, torch, cov_m, obs, ys, g, wl.steps)
        acc_m = accuracy(wl, res_m, res64)
        log(f"[bench] mixed phases {phases_m} accuracy {acc_m}")
        hmv_m = hmatvec_bench(fkf, torch, cov_m, info_m, args.matvec_reps)
        log(f"[bench] hmatvec mixed {hmv_m}")
        step_us_m = phases_m["steps_2_to_K"] * 1e3 / max(wl.steps - 1, 1)
        mixed = {"pass_ms": t_pass_m * 1e3, "steps_per_s": wl.steps / t_pass_m,
                 "constant_h_step_us": step_us_m, "phases_ms": phases_m,
                 "hmatvec_1rhs": hmv_m, "gamma_build_s": t_build_m,
                 "near_bytes": info_m["near_bytes"], "errors": acc_m,
                 "sites_ms_per_pass": {k: v[1] for k, v in trace_m.items()}}
        cov_m.close()

    # ---- roofline of the dominant kernel of the FP64 pass
    per = {k: (c, ms) for k, (c, ms) in trace.items()}
    # entries of the coupling matrices over all ordered admissible pairs
    k_entries = 2.0 * info["far_pair_entries"]
    models = {
        # site: (bound, algorithmic units per launch, unit)
        # basis U0 (N x n_m) read once; the state read and written (or the
        # variance written) and the n_m coefficients read
        "filter_gemv": ("hbm", 8.0 * n * n_m + 16.0 * n + 8.0 * n_m, "GB/s"),
        "filter_gemv_sq": ("hbm", 8.0 * n * n_m + 8.0 * n + 8.0 * n_m, "GB/s"),
        # n_m-column H-matrix product on the FP64 matrix cores, one FMA per
        # entry and column: couplings of the ordered admissible pairs; the
        # near-field tiles plus the downward interpolation; the upward one
        "hmat_far_couple_multi": ("mfma", 2.0 * n_m * k_entries, "TFLOP/s"),
        "hmat_near_multi": ("mfma", 2.0 * n_m * info["n_near_pairs"] * 4096.0, "TFLOP/s"),
        "hmat_down_multi": ("mfma", 2.0 * n_m * info["far_interp_entries"], "TFLOP/s"),
        "hmat_far_up_multi": ("mfma", 2.0 * n_m * info["far_interp_entries"], "TFLOP/s"),
        "gep_basis_gemm": ("mfma", 2.0 * n * n_m * n_m, "TFLOP/s"),
        # Householder reduction to tridiagonal form (one launch): 4 n^3 / 3
        # flops (a symmetric rank-2 update and a matrix-vector product per
        # reflector), on the FP64 vector units
        "eig_tridiag": ("alu", 4.0 * n_m ** 3 / 3.0, "TFLOP/s"),
    }
    # single-kernel sites (composite sites excluded)
    leaf_sites = [k for k in per if k not in ("gep_total", "gep_cross_cov", "gep_eig",
                                               "filter_step")]
    dom = max(leaf_sites, key=lambda k: per[k][1])
    roof = None
    if dom in models:
        bound, units, unit = models[dom]
        c, ms = per[dom]
        avg_s = ms / c * 1e-3
        if unit == "GB/s":
            ach, peak = units / avg_s * 1e-9, HBM_PEAK_GBS
        else:
            ach, peak = units / avg_s * 1e-12, FP64_PEAK_TFLOPS
        roof = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                "traffic": traffic_for(dom), "kernel": dom, "avg_launch_us": avg_s * 1e6,
                "launches_per_pass": c, "share_of_pass": ms / (t_pass * 1e3)}
    # the eigensolver phase against the flops of a minimal dense symmetric
    # eigen-decomposition with vectors (~9 n^3: tridiagonal reduction,
    # tridiagonal solve and back-transformation)
    eig_ms = per.get("gep_eig", (1, float("nan")))[1]
    eig_phase = {"ms_per_pass": eig_ms, "minimal_flops": 9.0 * n_m ** 3,
                 "tflops_vs_minimal": 9.0 * n_m ** 3 / (eig_ms * 1e-3) * 1e-12,
                 "frac_of_fp64_peak": 9.0 * n_m ** 3 / (eig_ms * 1e-3) * 1e-12 / FP64_PEAK_TFLOPS}
    result = {
        "metric": METRIC,
        "value": wl.steps / t_pass,
        "unit": "Kalman steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_pass * 1e3,         # one benchmark step = one pass of the hot path
        "ms_per_pass": t_pass * 1e3,
        "ms_per_filter_step": t_pass * 1e3 / wl.steps,
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
            "varying_h": vary,
            "extended_boxcox": ext,
            "loglik_gradient": grad,
            "many_filters": many,
            "phases_ms": phases,
            "errors": acc64,
            "dominant_site": dom,
            "eig_phase": eig_phase,
            "sites_ms_per_pass": {k: v[1] for k, v in per.items()},
            "gamma_build_s": t_build,
            "mixed": mixed,
            "mixed_vs_fp64_speedup": (t_pass * 1e3 / mixed["pass_ms"]) if mixed else None,
            "mixed_vs_fp64_step_speedup": (step_us / mixed["constant_h_step_us"]) if mixed
            else None,
            "mixed_vs_fp64_hmatvec_cold_speedup": (hmatvec["cold_us"]
                                                   / mixed["hmatvec_1rhs"]["cold_us"]) if mixed
            else None,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle sample")
        result["cpu_baseline"] = cpu_baseline(wl, H)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
