"""Direct covariance products: never an H-matrix (Section 2.2.1).

y = Gamma x with Gamma[i, j] = theta C(|x_i - x_j|) summed exactly, in row
panels so that memory stays bounded.  Cost O(N^2) kernel evaluations.
"""
from __future__ import annotations

import numpy as np

from .kernels import cov_block


def cov_matvec(pts: np.ndarray, X: np.ndarray, nu, ell, theta, panel: int = 1024,
               dlength: bool = False):
    """Y = Gamma X for X of shape (N,) or (N, k) (dlength: Y = dGamma/d ell X)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.empty_like(X)
    N = pts.shape[0]
    for i0 in range(0, N, panel):
        i1 = min(N, i0 + panel)
        Y[i0:i1] = cov_block(pts[i0:i1], pts, nu, ell, theta, dlength) @ X
    return Y


def cov_rows(pts: np.ndarray, rows: np.ndarray, X: np.ndarray, nu, ell, theta):
    """Selected rows of Gamma X (for spot checks at large N)."""
    return cov_block(pts[rows], pts, nu, ell, theta) @ X


def cross_cov(pts: np.ndarray, H, nu, ell, theta, panel: int = 1024):
    """P = Gamma H^T (the cross covariance of Algorithm 2), shape (N, n_m)."""
    N = pts.shape[0]
    P = np.empty((N, H.shape[0]))
    for i0 in range(0, N, panel):
        i1 = min(N, i0 + panel)
        blk = cov_block(pts[i0:i1], pts, nu, ell, theta)
        P[i0:i1] = np.asarray(H @ blk.T).T
    return P


def dense_cov(pts: np.ndarray, nu, ell, theta, dlength: bool = False):
    """The full Gamma, or dGamma/d ell (small N only)."""
    return cov_block(pts, pts, nu, ell, theta, dlength)
