"""Matern covariance kernel (Section 2.2.1, eq. maternfamily).

The paper writes C_{alpha,nu}(r) = 2^{1-nu}/Gamma(nu) (sqrt(2 nu) alpha r)^nu
K_nu(sqrt(2 nu) alpha r) with a scaling factor alpha and no variance.  Reading
used throughout: alpha = 1/ell (ell the length scale) and the entries are
multiplied by a variance theta, so C(0) = theta.  For nu = 1/2 + n the Bessel
form reduces to an exponential times a polynomial of order n (stated in the
same section); the closed forms below are those reductions.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def matern(r, nu: float, ell: float, theta: float = 1.0):
    """Closed-form Matern entries theta * C(r) for nu in {1/2, 3/2, 5/2}."""
    r = np.asarray(r, dtype=np.float64)
    if nu == 0.5:
        return theta * np.exp(-r / ell)
    if nu == 1.5:
        t = np.sqrt(3.0) * r / ell
        return theta * (1.0 + t) * np.exp(-t)
    if nu == 2.5:
        t = np.sqrt(5.0) * r / ell
        return theta * (1.0 + t + t * t / 3.0) * np.exp(-t)
    raise ValueError(f"unsupported smoothness nu={nu}")


def matern_bessel(r, nu: float, ell: float, theta: float = 1.0):
    """The Bessel-function form of eq. maternfamily, for any nu > 0.

    Used only to pin the closed forms.  At r = 0 the limit value theta is
    returned.
    """
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    x = np.sqrt(2.0 * nu) * r / ell
    out = np.empty_like(x)
    z = x == 0
    out[z] = 1.0
    xz = x[~z]
    out[~z] = (2.0 ** (1.0 - nu) / special.gamma(nu)) * xz ** nu * special.kv(nu, xz)
    return theta * out


def matern_dlength(r, nu: float, ell: float, theta: float = 1.0):
    """d/d ell of ``matern``: with t = c r / ell (c = 1, sqrt 3, sqrt 5),
    d/d ell theta C(t) = theta C'(t) (-t / ell), written out per closed form
    (the operator whose products give the length derivative of the
    likelihood; the paper has no parameter estimation)."""
    r = np.asarray(r, dtype=np.float64)
    if nu == 0.5:
        t = r / ell
        return theta / ell * t * np.exp(-t)              # C' = -e^-t
    if nu == 1.5:
        t = np.sqrt(3.0) * r / ell
        return theta / ell * t * t * np.exp(-t)          # C' = -t e^-t
    if nu == 2.5:
        t = np.sqrt(5.0) * r / ell
        return theta / ell * t * t * (1.0 + t) / 3.0 * np.exp(-t)   # C' = -t (1 + t) e^-t / 3
    raise ValueError(f"unsupported smoothness nu={nu}")


def cov_block(pts_a: np.ndarray, pts_b: np.ndarray, nu, ell, theta, dlength: bool = False):
    """Dense block Gamma[a, b] = theta C(|x_a - x_b|) (or its length
    derivative)."""
    d = pts_a[:, None, :] - pts_b[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=-1))
    return (matern_dlength if dlength else matern)(r, nu, ell, theta)
