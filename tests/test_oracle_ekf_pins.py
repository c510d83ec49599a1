"""Pins of the oracle's extended Kalman filter for the Box-Cox observation
model (Algorithm 4) against facts fixed by the paper and by mathematics.

Each pin takes an independent route: the transform's printed forward form and
its logarithmic limit, central differences of h(x) = H g(x), the linear
filter in the case a = 1 where the model is affine, and, for every step, the
minimiser of the linearised least-squares problem solved by a library
least-squares routine together with the information form of the covariance.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import ekf, kalman, kernels

A_VALUES = [0.5, 1.0, 2.0, 4.0, 6.0]


@pytest.mark.parametrize("a", A_VALUES)
def test_inverse_transform_inverts_the_printed_forward_transform(a):
    # eq. nonlinear: x = a (s^(1/a) - 1) and s = ((x + a)/a)^a are inverse maps
    # (x + a cancels for small s: the bound is absolute there)
    s = np.concatenate([[0.0], np.geomspace(1e-6, 50.0, 400)])
    np.testing.assert_allclose(ekf.boxcox_inverse(ekf.boxcox_forward(s, a), a), s,
                               rtol=1e-12, atol=1e-10)
    x = np.linspace(-a + 1e-9, 5.0, 300)
    np.testing.assert_allclose(ekf.boxcox_forward(ekf.boxcox_inverse(x, a), a), x,
                               rtol=1e-10, atol=1e-10)
    assert ekf.boxcox_forward(0.0, a) == -a and ekf.boxcox_inverse(0.0, a) == 1.0


def test_forward_transform_tends_to_log():
    # the paper's remark: a (s^(1/a) - 1) -> log s as a grows
    s = np.geomspace(1e-3, 1e3, 50)
    np.testing.assert_allclose(ekf.boxcox_forward(s, 1e7), np.log(s), rtol=0, atol=1e-5)


@pytest.mark.parametrize("a", A_VALUES)
def test_derivative_matches_central_differences(a):
    x = np.linspace(-0.9 * a, 3.0, 101)
    h = 1e-6
    fd = (ekf.boxcox_inverse(x + h, a) - ekf.boxcox_inverse(x - h, a)) / (2 * h)
    np.testing.assert_allclose(ekf.boxcox_inverse_deriv(x, a), fd, rtol=1e-7, atol=1e-9)


def test_reading_below_the_domain():
    for a in A_VALUES:
        x = np.array([-a - 1.0, -a])
        assert np.all(ekf.boxcox_inverse(x, a) == 0.0)
        want = 1.0 if a == 1.0 else 0.0
        assert np.all(ekf.boxcox_inverse_deriv(x, a) == want)


def _problem(N=24, nm=5, steps=4, seed=7, theta=0.05):
    g = np.random.default_rng(seed)
    pts = g.uniform(0, 1, (N, 2))
    Gamma = kernels.cov_block(pts, pts, 0.5, 0.3, theta)
    H = np.abs(g.standard_normal((nm, N))) / N
    R = g.uniform(1e-3, 3e-3, nm)
    ys = [H @ np.exp(0.3 * g.standard_normal(N)) + np.sqrt(R) * g.standard_normal(nm)
          for _ in range(steps)]
    return Gamma, H, R, np.array(ys)


@pytest.mark.parametrize("a", [2.0, 4.0])
def test_linearisation_is_the_jacobian_of_h(a):
    Gamma, H, R, ys = _problem()
    out = ekf.dense_ekf(Gamma, H, R, ys, a)
    x = out[1]["x"]                              # estimate the third step linearises about
    Hk = out[2]["Hk"]
    d = np.random.default_rng(1).standard_normal(x.size)
    e = 1e-6
    fd = (H @ ekf.boxcox_inverse(x + e * d, a) - H @ ekf.boxcox_inverse(x - e * d, a)) / (2 * e)
    np.testing.assert_allclose(Hk @ d, fd, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(out[2]["nu"], ys[2] - H @ ekf.boxcox_inverse(x, a), rtol=1e-14)


def test_affine_case_is_the_linear_filter():
    # a = 1: g(x) = x + 1, so the model is y = H x + H 1 + v, the linear filter
    # on data y - H 1 (valid while the estimate stays in the domain x > -1)
    Gamma, H, R, ys = _problem(steps=5)
    out = ekf.dense_ekf(Gamma, H, R, ys, 1.0, alpha0=0.4)
    ref = kalman.dense_kf(Gamma, [H] * len(ys), [R] * len(ys), ys - H @ np.ones(H.shape[1]),
                          alpha0=0.4)
    Hs, Rs = [H] * len(ys), [R] * len(ys)
    for k, (o, r) in enumerate(zip(out, ref), start=1):
        ll = kalman.innovation_loglik(Gamma, Hs[:k], Rs[:k], (ys - H @ np.ones(H.shape[1]))[:k],
                                      alpha0=0.4)
        assert abs(o["ll"] - ll) <= 1e-10 * abs(ll)
        assert o["x"].min() > -1.0
        np.testing.assert_allclose(o["x"], r["s"], rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(o["Sigma"], r["Sigma"], rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("a", [2.0, 6.0])
def test_each_step_minimises_the_linearised_least_squares(a):
    # the update is the minimiser of
    #   |R^-1/2 (y - h(x-) - H_k (z - x-))|^2 + |L^-1 (z - x-)|^2,  Sigma_{k|k-1} = L L^T,
    # and the covariance its information form (Sigma^-1 + H_k^T R^-1 H_k)^-1
    Gamma, H, R, ys = _problem(steps=4)
    out = ekf.dense_ekf(Gamma, H, R, ys, a, alpha0=0.2)
    x_prev, S_prev = np.zeros(H.shape[1]), 0.2 * Gamma
    for k, o in enumerate(out):
        Sp = S_prev + Gamma
        L = np.linalg.cholesky(Sp)
        Hk = H * ekf.boxcox_inverse_deriv(x_prev, a)[None, :]
        r = ys[k] - H @ ekf.boxcox_inverse(x_prev, a)
        M = np.vstack([Hk / np.sqrt(R)[:, None], sla.solve_triangular(L, np.eye(L.shape[0]),
                                                                      lower=True)])
        rhs = np.concatenate([r / np.sqrt(R), np.zeros(L.shape[0])])
        dz = np.linalg.lstsq(M, rhs, rcond=None)[0]
        np.testing.assert_allclose(o["x"], x_prev + dz, rtol=1e-8, atol=1e-10)
        Si = kalman.information_update(Sp, Hk, R)
        np.testing.assert_allclose(o["Sigma"], Si, rtol=1e-8, atol=1e-12)
        np.testing.assert_allclose(o["var"], np.diag(o["Sigma"]), rtol=0, atol=0)
        x_prev, S_prev = o["x"], o["Sigma"]


def test_first_step_from_zero_does_not_depend_on_a():
    # at x_0 = 0, g = 1 and g' = 1 for every a: the first update is the same
    Gamma, H, R, ys = _problem(steps=2)
    o2 = ekf.dense_ekf(Gamma, H, R, ys, 2.0)
    o6 = ekf.dense_ekf(Gamma, H, R, ys, 6.0)
    np.testing.assert_allclose(o2[0]["x"], o6[0]["x"], rtol=1e-13, atol=1e-15)
    assert np.linalg.norm(o2[1]["x"] - o6[1]["x"]) > 1e-6 * np.linalg.norm(o2[1]["x"])
