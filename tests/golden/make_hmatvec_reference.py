"""Write the oracle's direct products y = Gamma x on the 256 x 256 grid.

Runs only oracle.direct.cov_matvec (every entry of Gamma evaluated, summed in
row panels; never an H-matrix) for the covariance of workloads.LARGE (Matern
3/2, length 0.1, variance 1e-4, N = 65536) and two seeded standard normal
vectors (stream STREAM_VECTORS of that workload), and stores x and y whole.

    python tests/golden/make_hmatvec_reference.py

Output: tests/golden/hmatvec_reference.npz (about 2 MB).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import direct  # noqa: E402


def main():
    wl = W.LARGE
    pts = wl.points()
    x = W.normals(wl, W.STREAM_VECTORS, (wl.n, 2))
    t0 = time.time()
    y = direct.cov_matvec(pts, x, wl.nu, wl.length, wl.variance)
    print(f"direct product in {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "hmatvec_reference.npz"), x=x, y=y)
    print("written", flush=True)


if __name__ == "__main__":
    main()
