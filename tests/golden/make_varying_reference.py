"""Write the oracle's reference values for steps with a new measurement
operator every step at n_m = 480 on the 128 x 128 grid.

Workload: the 128 x 128 grid of workloads.MEDIUM (N = 16384, Matern 3/2,
length 0.2, variance 1e-4), two 480-ray geometries taken in turn, A, B, A, B,
A, B: crosswell left edge -> right edge (24 sources x 20 receivers) and the
same turned by a right angle (bottom edge -> top edge).  Data: travel times of
the synthetic truth of workloads.Truth along each step's rays plus N(0, R)
noise, R = 1e-4 I.  Runs only the oracle's dense Kalman filter
(oracle.kalman.dense_kf: Algorithm 1 with F = I, s_0 = Sigma_0 = 0; Gamma is
2 GiB on the host) and stores, for every step, the data, the whole state
estimate and the whole variance field.

    python tests/golden/make_varying_reference.py

Output: tests/golden/varying_reference.npz (about 1.6 MB).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import direct, kalman, rays  # noqa: E402

SEQUENCE = (0, 1, 0, 1, 0, 1)   # geometry of each step
CFG_ID = 6                      # random streams of this reference


def geometries():
    return [W.crosswell_2d(24, 20), W.crosswell_vertical(24, 20)]


def main():
    wl = W.MEDIUM
    pts = wl.points()
    geo = geometries()
    Hs = [rays.ray_operator(wl.shape, s, r) for s, r in geo]
    truth = W.Truth(W.tiny(shape=wl.shape, nu=wl.nu, length=wl.length, variance=wl.variance,
                           steps=len(SEQUENCE), drift_sigma=wl.drift_sigma, cfg_id=CFG_ID))
    noise = W.rng(CFG_ID, W.STREAM_NOISE)
    ys = []
    for k, g in enumerate(SEQUENCE, start=1):
        src, rcv = geo[g]
        y = truth.travel_times(k, src, rcv)
        ys.append(y + np.sqrt(wl.noise_var) * noise.standard_normal(len(y)))
    t0 = time.time()
    Gamma = direct.dense_cov(pts, wl.nu, wl.length, wl.variance)
    print(f"Gamma in {time.time() - t0:.1f} s", flush=True)
    R = np.full(480, wl.noise_var)
    out = kalman.dense_kf(Gamma, [Hs[g] for g in SEQUENCE], [R] * len(SEQUENCE), ys,
                          keep_cov=False)
    print(f"filter in {time.time() - t0:.1f} s", flush=True)
    rec = {"sequence": np.array(SEQUENCE), "ys": np.array(ys)}
    for k, o in enumerate(out, start=1):
        rec[f"s{k}"] = o["s"]
        rec[f"v{k}"] = o["var"]
    np.savez_compressed(os.path.join(HERE, "varying_reference.npz"), **rec)
    print("written", flush=True)


if __name__ == "__main__":
    main()
