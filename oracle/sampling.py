"""Conditional realizations (Section 3.3).

With Sigma = alpha Gamma - U D U^T and U^T Gamma^-1 U = I, the paper factors
Sigma = L L^T with L = alpha^{1/2} Gamma^{1/2} (I - W Sigma_pm W^T),
W = Gamma^{-1/2} U, where Sigma_pm solves Sigma^2 - 2 Sigma + alpha^-1 D = 0.
Reading: take the root Sigma_- = I - (I - D/alpha)^{1/2}; then
I - W Sigma_- W^T is the principal square root of M = Gamma^{-1/2} Sigma
Gamma^{-1/2} / alpha, a basis-free matrix.  Given an unconditional draw
g = Gamma^{1/2} s_u the realization is

    s = s_hat + alpha^{1/2} Gamma^{1/2} M^{1/2} Gamma^{-1/2} g,

which this module evaluates densely with symmetric eigendecompositions.
"""
from __future__ import annotations

import numpy as np


def _sym_fn(A, fn):
    w, Q = np.linalg.eigh(0.5 * (A + A.T))
    return (Q * fn(w)) @ Q.T


def realize(s_hat, Sigma, alpha: float, Gamma, g):
    """Conditional realization(s) for draws g (N,) or (N, ns)."""
    if alpha == 0.0:
        return np.broadcast_to(s_hat[:, None] if np.ndim(g) == 2 else s_hat,
                               np.shape(g)).copy()
    G_half = _sym_fn(Gamma, lambda w: np.sqrt(np.maximum(w, 0.0)))
    G_ihalf = _sym_fn(Gamma, lambda w: 1.0 / np.sqrt(w))
    M = G_ihalf @ Sigma @ G_ihalf / alpha
    M_half = _sym_fn(M, lambda w: np.sqrt(np.maximum(w, 0.0)))
    T = G_half @ M_half @ G_ihalf
    out = np.sqrt(alpha) * (T @ g)
    return (out + (s_hat[:, None] if np.ndim(g) == 2 else s_hat))


def realization_factor(Sigma, alpha, Gamma):
    """L with L L^T = Sigma (the operator applied to s_u)."""
    G_half = _sym_fn(Gamma, lambda w: np.sqrt(np.maximum(w, 0.0)))
    G_ihalf = _sym_fn(Gamma, lambda w: 1.0 / np.sqrt(w))
    M = G_ihalf @ Sigma @ G_ihalf / alpha
    M_half = _sym_fn(M, lambda w: np.sqrt(np.maximum(w, 0.0)))
    return np.sqrt(alpha) * G_half @ M_half
