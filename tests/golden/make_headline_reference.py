"""Write the oracle's reference values for the 256 x 256 crosswell workload.

Runs only the CPU oracle (direct P = Gamma H^T and the exact cross-covariance
Kalman recursion of oracle.kalman.xcov_kf) on the seeded inputs of
workloads.LARGE and stores the state estimate and variance at 4096 sampled
cells after steps 1, 10 and 50, plus their full-vector 2-norms.

    python tests/golden/make_headline_reference.py

Output: tests/golden/headline_reference.npz (a few hundred KB).
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
    idx = np.sort(W.rng(wl.cfg_id, 7).choice(wl.n, 4096, replace=False))
    rec = {"idx": idx, "steps": np.array(STEPS_KEPT)}
    for k in STEPS_KEPT:
        rec[f"s{k}"] = out[k - 1]["s"][idx]
        rec[f"v{k}"] = out[k - 1]["var"][idx]
        rec[f"s{k}_norm"] = np.linalg.norm(out[k - 1]["s"])
        rec[f"v{k}_max"] = np.abs(out[k - 1]["var"]).max()
    np.savez_compressed(os.path.join(HERE, "headline_reference.npz"), **rec)
    print("written", flush=True)


if __name__ == "__main__":
    main()
