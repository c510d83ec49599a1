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

Appendix B (randomized algorithm for the GHEP A x = lambda B x with
A = H^T R^-1 H, B = Gamma^-1): ``randomized_ghep`` follows its steps with a
given Gaussian Omega: Ybar = A Omega; Qhat with Qhat^T B^-1 Qhat = I by
modified Gram-Schmidt in the B^-1 = Gamma inner product (as the appendix
suggests; columns that are dependent to rounding are dropped); Q = B^-1 Qhat;
T = Q^T A Q = S Lambda S^T; U = Q S for the k largest.  With a truncated
decomposition (k below the rank of H) the filter of Section 2.3 runs on the
information the decomposition keeps, H^T R^-1 H ~ B U Lambda U^T B; in
observation form that is the whitened k-dimensional data
y' = Lambda^-1/2 U^T H^T R^-1 y with operator H' = Lambda^1/2 (B U)^T and
unit noise (``projected_observation``).
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


def randomized_ghep(H, R, Gamma: np.ndarray, Omega: np.ndarray, k: int, drop: float = 1e-10):
    """Appendix B's randomized eigenpairs: (lam (k, descending), U (N x k),
    Q (N x m), Qhat (N x m)) with U^T Gamma^-1 U = I, Qhat^T Gamma Qhat = I and
    Q = Gamma Qhat."""
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    Rinv = 1.0 / np.asarray(R, dtype=np.float64)
    A = Hd.T @ (Hd * Rinv[:, None])
    Ybar = A @ Omega
    # modified Gram-Schmidt in the Gamma inner product, twice per column
    cols = []
    norm0 = max(np.sqrt(abs(y @ Gamma @ y)) for y in Ybar.T)
    for y in Ybar.T:
        v = y.copy()
        for _ in range(2):
            for q in cols:
                v = v - (q @ Gamma @ v) * q
        nv = np.sqrt(max(v @ Gamma @ v, 0.0))
        if nv > drop * norm0:
            cols.append(v / nv)
    Qhat = np.array(cols).T
    Q = Gamma @ Qhat
    T = Q.T @ A @ Q
    T = 0.5 * (T + T.T)
    lam, S = np.linalg.eigh(T)
    order = np.argsort(lam)[::-1][:k]
    return lam[order], Q @ S[:, order], Q, Qhat


def projected_observation(U, lam, Gamma, H, R, y):
    """The k-dimensional whitened data y' and operator H' (unit noise) that
    carry what the decomposition H^T R^-1 H ~ Gamma^-1 U Lambda U^T Gamma^-1
    keeps of the observation (H, R, y)."""
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    BU = np.linalg.solve(Gamma, U)
    Hp = np.sqrt(lam)[:, None] * BU.T
    yp = (U.T @ (Hd.T @ (np.asarray(y) / np.asarray(R)))) / np.sqrt(lam)
    return Hp, yp
