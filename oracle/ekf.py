"""Extended Kalman filter for the Box-Cox observation model.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Extended Kalman Filter" of the numerical experiments, Algorithm 4.
The filtered state is the transformed field x (the paper's s-hat); the
physical field is the inverse of the Box-Cox transform (eq. nonlinear),

    s = g(x) = ((x + a) / a)^a,        x = a (s^(1/a) - 1),

with a > 0 the transform's own parameter (printed as alpha in the paper, a
different alpha from the weight alpha_k of Gamma).  Measurements are
y_k = H g(x_k) + v_k with the linear travel-time operator H, and the
random-walk forecast (F = I) acts on x.  Each step linearizes h(x) = H g(x)
about the predicted estimate,

    H_k = H diag(g'(x)),   g'(x) = ((x + a) / a)^(a - 1),

and takes the Kalman update with that H_k and the innovation y_k - h(x):
the gain form of the update in Algorithm 4, with the predicted covariance
Sigma_{k|k-1} = Sigma_{k-1|k-1} + Gamma.

Readings (the paper does not state them):
* outside the transform's domain, x < -a, the base (x + a)/a is taken as 0:
  g = 0 there and g' is its one-sided limit at the boundary (1 for a = 1,
  0 for a > 1; 0 also for a < 1, where no finite limit exists);
* the initial estimate is x_0 = 0 (the paper's initial field of zero, read in
  the filtered variable: s = g(0) = 1), with Sigma_{0|0} = alpha0 Gamma;
* one linearization per step (the optional extra linearizations of
  Algorithm 4 are not taken).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def boxcox_forward(s, a: float):
    """The Box-Cox transform x = a (s^(1/a) - 1) of eq. nonlinear (s >= 0)."""
    s = np.asarray(s, dtype=np.float64)
    return a * (np.power(s, 1.0 / a) - 1.0)


def boxcox_inverse(x, a: float):
    """s = g(x) = ((x + a)/a)^a, with the base clamped at 0 below the domain."""
    t = np.maximum((np.asarray(x, dtype=np.float64) + a) / a, 0.0)
    return np.power(t, a)


def boxcox_inverse_deriv(x, a: float):
    """g'(x) = ((x + a)/a)^(a - 1); at and below the domain's edge, the
    one-sided limit (1 for a = 1, else 0)."""
    t = np.maximum((np.asarray(x, dtype=np.float64) + a) / a, 0.0)
    out = np.zeros_like(t)
    pos = t > 0
    out[pos] = np.power(t[pos], a - 1.0)
    if a == 1.0:
        out[~pos] = 1.0
    return out


def _dense(H):
    return H.toarray() if hasattr(H, "toarray") else np.asarray(H, dtype=np.float64)


def dense_ekf(Gamma: np.ndarray, H, R, ys, a: float, alpha0: float = 0.0, x0=None):
    """Run the extended filter for ys (steps x n_m) with one operator H.

    R is the diagonal of the measurement-noise covariance.  Returns per step
    a dict with the estimate ``x`` of the filtered field, its covariance
    ``Sigma`` and variances ``var``, the linearization used (``Hk``,
    innovation ``nu``) and the innovation log-likelihood of the steps so far
    (``ll``: the sum of -(nu^T S^-1 nu + log det S + n_m log 2 pi)/2).
    """
    H = _dense(H)
    R = np.asarray(R, dtype=np.float64)
    N = Gamma.shape[0]
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    Sigma = alpha0 * Gamma.copy()
    out = []
    ll = 0.0
    for k, y in enumerate(ys, start=1):
        Sp = Sigma + Gamma                           # prediction (F = I)
        Hk = H * boxcox_inverse_deriv(x, a)[None, :]  # H diag(g'(x))
        nu = np.asarray(y, dtype=np.float64) - H @ boxcox_inverse(x, a)
        C = Sp @ Hk.T                                # Sigma_{k|k-1} H_k^T
        S = Hk @ C + np.diag(R)
        cf = sla.cho_factor(S)
        ll -= 0.5 * (nu @ sla.cho_solve(cf, nu) + 2 * np.sum(np.log(np.diag(cf[0])))
                     + len(nu) * np.log(2 * np.pi))
        x = x + C @ sla.cho_solve(cf, nu)
        Sigma = Sp - C @ sla.cho_solve(cf, C.T)
        Sigma = 0.5 * (Sigma + Sigma.T)
        out.append({"x": x.copy(), "Sigma": Sigma.copy(), "var": np.diag(Sigma).copy(),
                    "alpha": alpha0 + k, "Hk": Hk, "nu": nu, "ll": ll})
    return out
