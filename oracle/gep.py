"""Generalized eigenproblem and the constant-H per-mode recursion.

Section 2.2.2: H^T R^-1 H x = lambda Gamma^-1 x, with the decomposition
H^T R^-1 H = Gamma^-1 U Lambda U^T Gamma^-1, U^T Gamma^-1 U = I
(eqs. ghep, geneigendecomposition).  ``gep_dense`` solves it as a library
generalized symmetric eigenproblem (scipy ``eigh(A, B)``), which is the plain
definition.

Section 2.3 (Algorithms 2 and 3): with constant H and Sigma_{k|k} =
alpha_k Gamma - U D_k U^T, each mode evolves on its own.  Writing
c = alpha - D (the weight of mode i in Sigma, in the basis Gamma^-1 U), the
printed update D_{k+1} = D_k + ((alpha_{k+1} - D_k)^-1 Lambda^-1 + 1)^-1
(alpha_{k+1} - D_k) becomes, with a = c_k + 1 (alpha grows by one per step),
c_{k+1} = a / (1 + a lambda).  ``mode_weights`` iterates that scalar map.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def gep_dense(H, R, Gamma: np.ndarray):
    """All N generalized eigenpairs, eigenvalues descending.

    Returns (lam, U) with U^T Gamma^-1 U = I.  B = Gamma^-1 is formed densely
    (small N only).
    """
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    A = Hd.T @ (Hd / np.asarray(R)[:, None])
    B = np.linalg.inv(Gamma)
    B = 0.5 * (B + B.T)
    lam, X = sla.eigh(A, B)          # X^T B X = I
    order = np.argsort(lam)[::-1]
    return lam[order], X[:, order]


def mode_weights(lam: np.ndarray, alpha0: float, k: int) -> np.ndarray:
    """c_k = alpha_k - D_k per mode after k constant-H steps from Sigma_0 = alpha0 Gamma."""
    c = np.full_like(np.asarray(lam, dtype=np.float64), alpha0)
    for _ in range(k):
        a = c + 1.0
        c = a / (1.0 + a * lam)
    return c
