"""The standard Kalman filter with the random-walk forecast model.

Algorithm 1 with F_k = I (Section 2.1, "Assumptions"): prediction
s_{k|k-1} = s_{k-1|k-1}, Sigma_{k|k-1} = Sigma_{k-1|k-1} + Gamma; update with
innovation covariance S = H Sigma_{k|k-1} H^T + R, gain K = Sigma_{k|k-1} H^T S^-1,
s_{k|k} = s_{k|k-1} + K (y_k - H s_{k|k-1}) and the posterior covariance.  The
paper prints the covariance update in information form,
Sigma_{k|k} = (Sigma_{k|k-1}^-1 + H^T R^-1 H)^-1; ``dense_kf`` evaluates the
algebraically identical gain form Sigma_{k|k-1} - K H Sigma_{k|k-1}
(no N x N inverse), and a test pins the two against each other.

Reading of the time index (the model writes y_{k+1}, the algorithms y_k):
step k = 1..N_t predicts from step k-1 and assimilates y_k.  The initial
condition is s_0 (default 0) and Sigma_{0|0} = alpha_0 Gamma (alpha_0 = 0 gives
the paper's s_0 = Sigma_0 = 0 of Section 4.1).

``xcov_kf`` is the same filter for a constant H evaluated without ever forming
an N x N matrix: it carries C = Sigma H^T, A = H Sigma H^T and diag Sigma only
(the cross-covariance idea the paper attributes to earlier work in Section 1);
every line is Algorithm 1 multiplied by H^T on the right.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _dense(H):
    return H.toarray() if hasattr(H, "toarray") else np.asarray(H, dtype=np.float64)


def dense_kf(Gamma: np.ndarray, Hs, Rs, ys, alpha0: float = 0.0, s0=None,
             keep_cov: bool = True):
    """Run Algorithm 1 (F = I).  Hs, Rs, ys are per-step sequences.

    Rs[k] is the diagonal of the measurement-noise covariance.  Returns a list
    of dicts with the estimate ``s``, covariance ``Sigma`` (or only ``var``
    when keep_cov is False) and ``alpha`` (alpha_0 + k, the weight of Gamma in
    the paper's representation).
    """
    N = Gamma.shape[0]
    s = np.zeros(N) if s0 is None else np.array(s0, dtype=np.float64)
    Sigma = alpha0 * Gamma.copy()
    out = []
    for k, (H, R, y) in enumerate(zip(Hs, Rs, ys), start=1):
        H = _dense(H)
        Sp = Sigma + Gamma                      # predict (F = I)
        C = Sp @ H.T                            # Sigma_{k|k-1} H^T
        S = H @ C + np.diag(np.asarray(R, dtype=np.float64))
        cf = sla.cho_factor(S)
        nu = np.asarray(y, dtype=np.float64) - H @ s
        s = s + C @ sla.cho_solve(cf, nu)
        Sigma = Sp - C @ sla.cho_solve(cf, C.T)
        Sigma = 0.5 * (Sigma + Sigma.T)
        rec = {"s": s.copy(), "alpha": alpha0 + k, "var": np.diag(Sigma).copy()}
        if keep_cov:
            rec["Sigma"] = Sigma.copy()
        out.append(rec)
    return out


def information_update(Sigma_pred: np.ndarray, H, R):
    """Posterior covariance in the information form printed in Algorithm 1."""
    H = _dense(H)
    Hred = H.T @ (H / np.asarray(R, dtype=np.float64)[:, None])
    return np.linalg.inv(np.linalg.inv(Sigma_pred) + Hred)


def xcov_kf(P: np.ndarray, H, R, ys, theta: float, alpha0: float = 0.0, s0=None):
    """Exact filter for constant H carrying only N x n_m quantities.

    P = Gamma H^T (from ``direct.cross_cov``), theta = diag(Gamma).  With
    Sigma_{0|0} = alpha0 Gamma: C = Sigma H^T = alpha0 P, A = H C, v = diag Sigma.
    Per step: C^- = C + P, A^- = A + H P, v^- = v + theta; S = A^- + R;
    K = C^- S^-1; s += K (y - H s); C = C^- - K A^-; A = A^- - A^- S^-1 A^-;
    v = v^- - rowsum(K o C^-).  Each record also carries the innovation
    log-likelihood of the steps so far (``ll``), as ``innovation_loglik``.
    """
    Hd = H
    G = np.asarray(Hd @ P)
    G = 0.5 * (G + G.T)
    N = P.shape[0]
    s = np.zeros(N) if s0 is None else np.array(s0, dtype=np.float64)
    C = alpha0 * P
    A = alpha0 * G
    v = np.full(N, alpha0 * theta)
    Rd = np.diag(np.asarray(R, dtype=np.float64))
    out = []
    ll = 0.0
    for k, y in enumerate(ys, start=1):
        Cm = C + P
        Am = A + G
        vm = v + theta
        cf = sla.cho_factor(Am + Rd)
        nu = np.asarray(y, dtype=np.float64) - np.asarray(Hd @ s).ravel()
        ll -= 0.5 * (nu @ sla.cho_solve(cf, nu) + 2 * np.sum(np.log(np.diag(cf[0])))
                     + len(nu) * np.log(2 * np.pi))
        s = s + Cm @ sla.cho_solve(cf, nu)
        K = sla.cho_solve(cf, Cm.T).T
        C = Cm - K @ Am
        A = Am - Am @ sla.cho_solve(cf, Am)
        A = 0.5 * (A + A.T)
        v = vm - np.sum(K * Cm, axis=1)
        out.append({"s": s.copy(), "alpha": alpha0 + k, "var": v.copy(), "ll": ll})
    return out


def innovation_loglik(Gamma, Hs, Rs, ys, alpha0=0.0):
    """Innovation log-likelihood sum_k -1/2 (nu^T S^-1 nu + logdet S + n log 2 pi)."""
    N = Gamma.shape[0]
    s = np.zeros(N)
    Sigma = alpha0 * Gamma.copy()
    ll = 0.0
    for H, R, y in zip(Hs, Rs, ys):
        H = _dense(H)
        Sp = Sigma + Gamma
        C = Sp @ H.T
        S = H @ C + np.diag(R)
        cf = sla.cho_factor(S)
        nu = y - H @ s
        ll -= 0.5 * (nu @ sla.cho_solve(cf, nu) + 2 * np.sum(np.log(np.diag(cf[0])))
                     + len(y) * np.log(2 * np.pi))
        s = s + C @ sla.cho_solve(cf, nu)
        Sigma = Sp - C @ sla.cho_solve(cf, C.T)
        Sigma = 0.5 * (Sigma + Sigma.T)
    return ll


def loglik_log_derivatives_fd(Gamma, Hs, Rs, ys, alpha0=0.0, h=1e-4):
    """Central differences of ``innovation_loglik`` in log theta (Gamma scaled
    by e^t) and in log sigma^2 (every R_k scaled by e^t), step h."""
    def ll(a, s):
        return innovation_loglik(a * Gamma, Hs, [s * np.asarray(R, dtype=np.float64) for R in Rs],
                                 ys, alpha0)
    e, ie = np.exp(h), np.exp(-h)
    d_theta = (ll(e, 1.0) - ll(ie, 1.0)) / (2 * h)
    d_noise = (ll(1.0, e) - ll(1.0, ie)) / (2 * h)
    return d_theta, d_noise
