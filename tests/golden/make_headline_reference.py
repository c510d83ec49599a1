"""Write the oracle's reference values for the 256 x 256 crosswell workload.

Runs only the CPU oracle (direct P = Gamma H^T and the exact cross-covariance
Kalman recursion of oracle.kalman.xcov_kf) on the seeded inputs of
workloads.LARGE and stores the whole state estimate and variance field
(every one of the 65536 cells) after steps 1, 10 and 50; and the
innovation log-likelihood of the 50 steps with its central differences in
log theta (P and theta scaled), log sigma^2 (R scaled) and log length (P
recomputed directly at length e^(+-h)), h = 1e-4.

    python tests/golden/make_headline_reference.py

Output: tests/golden/headline_reference.npz (about 3 MB).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import direct, kalman, rays  # noqa: E402

STEPS_KEPT = (1, 10, 50)


def main():
    wl = W.LARGE
    pts = wl.points()
    src, rcv = wl.rays()
    H = rays.ray_operator(wl.shape, src, rcv)
    R = np.full(H.shape[0], wl.noise_var)
    ys = W.observations(wl)
    t0 = time.time()
    P = direct.cross_cov(pts, H, wl.nu, wl.length, wl.variance)
    print(f"P in {time.time() - t0:.1f} s", flush=True)
    out = kalman.xcov_kf(P, H, R, ys, wl.variance)
    print(f"filter in {time.time() - t0:.1f} s", flush=True)
    rec = {"steps": np.array(STEPS_KEPT)}
    for k in STEPS_KEPT:
        rec[f"s{k}"] = out[k - 1]["s"]
        rec[f"v{k}"] = out[k - 1]["var"]
    # log-likelihood and its derivatives (central differences, h = 1e-4)
    h = 1e-4
    rec["ll"] = out[-1]["ll"]

    def ll_of(Pm, Rm, theta):
        return kalman.xcov_kf(Pm, H, Rm, ys, theta)[-1]["ll"]
    e = np.exp(h)
    rec["dll_dlog_theta"] = (ll_of(P * e, R, wl.variance * e)
                             - ll_of(P / e, R, wl.variance / e)) / (2 * h)
    rec["dll_dlog_noise"] = (ll_of(P, R * e, wl.variance) - ll_of(P, R / e, wl.variance)) / (2 * h)
    Pp = direct.cross_cov(pts, H, wl.nu, wl.length * e, wl.variance)
    Pm = direct.cross_cov(pts, H, wl.nu, wl.length / e, wl.variance)
    rec["dll_dlog_length"] = (ll_of(Pp, R, wl.variance) - ll_of(Pm, R, wl.variance)) / (2 * h)
    print(f"log-likelihood and derivatives in {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "headline_reference.npz"), **rec)
    print("written", flush=True)


if __name__ == "__main__":
    main()
