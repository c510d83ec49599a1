"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-type the oracle's own formulas: each compares it with an
independent route (a library special function, an analytic inverse, a
brute-force joint Gaussian, hand-computed geometry, sampling).
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from oracle import direct, gep, kalman, kernels, rays, sampling

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- kernels ---
@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
@pytest.mark.parametrize("ell", [0.1, 0.3, 2.0])
def test_matern_closed_forms_match_bessel_definition(nu, ell):
    # eq. maternfamily: nu = 1/2 + n reduces to exponential x polynomial
    r = np.concatenate([[0.0], np.geomspace(1e-6, 5.0, 200)])
    a = kernels.matern(r, nu, ell, 2.5)
    b = kernels.matern_bessel(r, nu, ell, 2.5)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-300)
    assert a[0] == 2.5


def test_matern_exponential_value():
    # nu = 1/2 is the exponential covariance: C(ell) = theta / e
    assert kernels.matern(0.3, 0.5, 0.3, 7.0) == pytest.approx(7.0 / math.e, rel=1e-15)


# ------------------------------------------------------------------- rays ---
def _golden_rays():
    cases = []
    with open(os.path.join(GOLDEN, "rays_hand.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, tail = line.split("|")
            v = head.split()
            nx, ny = int(v[0]), int(v[1])
            a = (float(v[2]), float(v[3]))
            b = (float(v[4]), float(v[5]))
            exp = {int(t.split(":")[0]): float(t.split(":")[1]) for t in tail.split()}
            cases.append(((nx, ny), a, b, exp))
    return cases


@pytest.mark.parametrize("case", _golden_rays())
def test_rays_hand_computed(case):
    shape, a, b, exp = case
    H = rays.ray_operator(shape, np.array([a]), np.array([b])).toarray()[0]
    got = {int(c): H[c] for c in np.nonzero(H)[0]}
    assert set(got) == set(exp)
    for c in exp:
        assert got[c] == pytest.approx(exp[c], rel=1e-13)


def test_rays_row_sums_are_ray_lengths_and_match_sampling():
    src, rcv = W.crosswell_2d(8, 8)
    shape = (32, 32)
    H = rays.ray_operator(shape, src, rcv)
    L = np.linalg.norm(rcv - src, axis=1)
    np.testing.assert_allclose(np.asarray(H.sum(axis=1)).ravel(), L, rtol=1e-13)
    assert H.min() >= 0
    # independent route: dense midpoint sampling of one oblique ray
    m = 13
    n_s = 400000
    t = (np.arange(n_s) + 0.5) / n_s
    p = src[m] + t[:, None] * (rcv[m] - src[m])
    cells = np.minimum((p * 32).astype(int), 31)
    flat = cells[:, 0] + 32 * cells[:, 1]
    approx = np.bincount(flat, minlength=1024) * (L[m] / n_s)
    np.testing.assert_allclose(H.toarray()[m], approx, atol=5e-5)


def test_rays_3d_row_sums():
    src, rcv = W.crosswell_3d((2, 3), (3, 2))
    H = rays.ray_operator((6, 5, 4), src, rcv)
    L = np.linalg.norm(rcv - src, axis=1)
    np.testing.assert_allclose(np.asarray(H.sum(axis=1)).ravel(), L, rtol=1e-13)


# ----------------------------------------------------------------- direct ---
def test_direct_matvec_against_analytic_inverse_of_exponential_kernel():
    # Points on a line with the exponential kernel form a Markov chain: Gamma^-1
    # is tridiagonal with rho = exp(-h/ell):
    #   Gamma^-1 = 1/(theta (1 - rho^2)) * tridiag(-rho, 1 + rho^2, -rho), corners 1.
    n, h, ell, theta = 40, 0.025, 0.3, 1.7
    pts = np.stack([np.arange(n) * h + 0.1, np.full(n, 0.5)], axis=1)
    rho = math.exp(-h / ell)
    Ti = np.diag(np.full(n, 1 + rho * rho)) - rho * (np.eye(n, k=1) + np.eye(n, k=-1))
    Ti[0, 0] = Ti[-1, -1] = 1.0
    Ti /= theta * (1 - rho * rho)
    x = np.random.default_rng(0).standard_normal(n)
    y = direct.cov_matvec(pts, Ti @ x, 0.5, ell, theta, panel=7)
    np.testing.assert_allclose(y, x, rtol=0, atol=1e-11)


def test_cross_cov_equals_matvec_of_dense_transpose():
    wl = W.tiny(shape=(10, 9))
    pts = wl.points()
    src, rcv = wl.rays()
    H = rays.ray_operator(wl.shape, src, rcv)
    P = direct.cross_cov(pts, H, wl.nu, wl.length, wl.variance, panel=13)
    P2 = direct.cov_matvec(pts, H.T.toarray(), wl.nu, wl.length, wl.variance, panel=29)
    np.testing.assert_allclose(P, P2, rtol=1e-13, atol=1e-14)


# ------------------------------------------------------------------ kalman ---
def _tiny_problem(N=6, steps=3, seed=3, varying=True):
    g = np.random.default_rng(seed)
    pts = g.uniform(0, 1, (N, 2))
    Gamma = kernels.cov_block(pts, pts, 1.5, 0.4, 0.8)
    Hs, Rs, ys = [], [], []
    for k in range(steps):
        nm = 2 + (k % 2) if varying else 2
        gk = np.random.default_rng(seed + (k if varying else 0) + 100)
        Hs.append(gk.standard_normal((nm, N)))
        Rs.append(gk.uniform(0.1, 0.5, nm))
        ys.append(g.standard_normal(nm))
    return Gamma, Hs, Rs, ys


def _joint_gaussian_posterior(Gamma, Hs, Rs, ys, alpha0, s0):
    """E[s_K | y_1..y_K] and Cov by conditioning the stacked Gaussian directly.

    s_j = s_0 + w_0 + ... with Cov(s_i, s_j) = (alpha0 + min(i, j)) Gamma and
    y_j = H_j s_j + v_j (the model of Section 2.1 with F = I).
    """
    K = len(Hs)
    blocks_sy = []
    rows = []
    for i in range(K):
        row = []
        for j in range(K):
            row.append((alpha0 + min(i, j) + 1) * Hs[i] @ Gamma @ Hs[j].T)
        rows.append(row)
    Syy = np.block(rows) + np.diag(np.concatenate(Rs))
    Ssy = np.hstack([(alpha0 + min(K - 1, j) + 1) * Gamma @ Hs[j].T for j in range(K)])
    ymean = np.concatenate([H @ s0 for H in Hs])
    yv = np.concatenate(ys)
    mean = s0 + Ssy @ np.linalg.solve(Syy, yv - ymean)
    cov = (alpha0 + K) * Gamma - Ssy @ np.linalg.solve(Syy, Ssy.T)
    return mean, cov


@pytest.mark.parametrize("alpha0", [0.0, 0.7])
def test_dense_kf_equals_brute_force_joint_gaussian(alpha0):
    Gamma, Hs, Rs, ys = _tiny_problem()
    s0 = np.linspace(-0.3, 0.4, Gamma.shape[0])
    out = kalman.dense_kf(Gamma, Hs, Rs, ys, alpha0=alpha0, s0=s0)
    for k in range(1, len(Hs) + 1):
        m, c = _joint_gaussian_posterior(Gamma, Hs[:k], Rs[:k], ys[:k], alpha0, s0)
        np.testing.assert_allclose(out[k - 1]["s"], m, rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(out[k - 1]["Sigma"], c, rtol=1e-10, atol=1e-12)
        assert out[k - 1]["alpha"] == alpha0 + k


def test_gain_form_equals_information_form():
    Gamma, Hs, Rs, ys = _tiny_problem(N=8, steps=1)
    Sp = 1.3 * Gamma
    Si = kalman.information_update(Sp, Hs[0], Rs[0])
    out = kalman.dense_kf(Gamma, Hs, Rs, ys, alpha0=0.3)
    np.testing.assert_allclose(out[0]["Sigma"], Si, rtol=1e-10, atol=1e-13)


def test_xcov_kf_equals_dense_kf():
    wl = W.tiny(shape=(12, 10), nu=1.5, length=0.3, variance=1e-2, noise_var=1e-3, steps=5)
    pts = wl.points()
    src, rcv = wl.rays()
    H = rays.ray_operator(wl.shape, src, rcv)
    Gamma = direct.dense_cov(pts, wl.nu, wl.length, wl.variance)
    ys = W.observations(wl)
    R = np.full(H.shape[0], wl.noise_var)
    d = kalman.dense_kf(Gamma, [H] * wl.steps, [R] * wl.steps, ys, alpha0=0.5)
    P = direct.cross_cov(pts, H, wl.nu, wl.length, wl.variance)
    x = kalman.xcov_kf(P, H, R, ys, wl.variance, alpha0=0.5)
    for k, (a, b) in enumerate(zip(d, x), start=1):
        np.testing.assert_allclose(b["s"], a["s"], rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(b["var"], a["var"], rtol=1e-10, atol=1e-14)
        ll = kalman.innovation_loglik(Gamma, [H] * k, [R] * k, ys[:k], alpha0=0.5)
        assert b["ll"] == pytest.approx(ll, rel=1e-11)


# --------------------------------------------------------------------- gep ---
def test_gep_identities_and_data_space_eigenvalues():
    wl = W.tiny(shape=(9, 8), nu=0.5, length=0.3, variance=1.0, noise_var=1e-2)
    pts = wl.points()
    src, rcv = wl.rays()
    H = rays.ray_operator(wl.shape, src, rcv)
    R = np.full(H.shape[0], wl.noise_var)
    Gamma = direct.dense_cov(pts, wl.nu, wl.length, wl.variance)
    lam, U = gep.gep_dense(H, R, Gamma)
    nm = H.shape[0]
    Gi = np.linalg.inv(Gamma)
    # eq. geneigendecomposition: U^T Gamma^-1 U = I and the reconstruction
    np.testing.assert_allclose(U.T @ Gi @ U, np.eye(len(lam)), atol=1e-8)
    Hd = H.toarray()
    np.testing.assert_allclose(Gi @ U @ np.diag(lam) @ U.T @ Gi, Hd.T @ (Hd / R[:, None]),
                               atol=1e-7 * np.abs(lam).max())
    # rank <= n_m; nonzero part = eig of R^-1/2 H Gamma H^T R^-1/2 (data space)
    A = (Hd / np.sqrt(R)[:, None]) @ Gamma @ (Hd / np.sqrt(R)[:, None]).T
    ev = np.sort(np.linalg.eigvalsh(A))[::-1]
    np.testing.assert_allclose(lam[:nm], ev, rtol=1e-8, atol=1e-8 * ev[0])
    assert np.all(np.abs(lam[nm:]) <= 1e-8 * ev[0])


@pytest.mark.parametrize("alpha0", [0.0, 2.0])
def test_mode_weights_match_dense_kf_in_gep_basis(alpha0):
    # Sigma_k = alpha_k Gamma - U D_k U^T: in the basis Gamma^-1 U the dense
    # filter's covariance must be diag(alpha_k - D_k) = diag(c_k).
    wl = W.tiny(shape=(7, 6), nu=1.5, length=0.4, variance=0.5, noise_var=1e-2, steps=4)
    pts = wl.points()
    src, rcv = wl.rays()
    H = rays.ray_operator(wl.shape, src, rcv)
    R = np.full(H.shape[0], wl.noise_var)
    Gamma = direct.dense_cov(pts, wl.nu, wl.length, wl.variance)
    lam, U = gep.gep_dense(H, R, Gamma)
    Ut = np.linalg.solve(Gamma, U)
    ys = W.observations(wl)
    out = kalman.dense_kf(Gamma, [H] * wl.steps, [R] * wl.steps, ys, alpha0=alpha0)
    for k, rec in enumerate(out, start=1):
        M = Ut.T @ rec["Sigma"] @ Ut
        c = gep.mode_weights(lam, alpha0, k)
        np.testing.assert_allclose(M, np.diag(c), atol=1e-8 * max(1.0, c.max()))


# ---------------------------------------------------------------- sampling ---
def test_realization_factor_reproduces_covariance_and_paper_formula():
    wl = W.tiny(shape=(6, 6), nu=1.5, length=0.4, variance=0.5, noise_var=1e-2, steps=3)
    pts = wl.points()
    src, rcv = wl.rays()
    H = rays.ray_operator(wl.shape, src, rcv)
    R = np.full(H.shape[0], wl.noise_var)
    Gamma = direct.dense_cov(pts, wl.nu, wl.length, wl.variance)
    ys = W.observations(wl)
    out = kalman.dense_kf(Gamma, [H] * 3, [R] * 3, ys)
    rec = out[-1]
    L = sampling.realization_factor(rec["Sigma"], rec["alpha"], Gamma)
    np.testing.assert_allclose(L @ L.T, rec["Sigma"], atol=1e-12)
    # the paper's form: g - U Sigma_- U^T Gamma^-1 g with Sigma_- = 1 - (1 - D/alpha)^1/2
    lam, U = gep.gep_dense(H, R, Gamma)
    a = rec["alpha"]
    D = a - gep.mode_weights(lam, 0.0, 3)
    Sm = 1.0 - np.sqrt(np.maximum(1.0 - D / a, 0.0))
    g = np.random.default_rng(5).standard_normal((Gamma.shape[0], 2))
    want = rec["s"][:, None] + math.sqrt(a) * (g - U @ (Sm[:, None] * (U.T @ np.linalg.solve(Gamma, g))))
    got = sampling.realize(rec["s"], rec["Sigma"], a, Gamma, g)
    np.testing.assert_allclose(got, want, atol=1e-9)


def test_innovation_loglik_equals_joint_gaussian_log_density():
    # the innovation decomposition of the log-likelihood equals the log density
    # of the stacked observations under the joint Gaussian model
    Gamma, Hs, Rs, ys = _tiny_problem(N=5, steps=3)
    ll = kalman.innovation_loglik(Gamma, Hs, Rs, ys, alpha0=0.4)
    K = len(Hs)
    rows = [[(0.4 + min(i, j) + 1) * Hs[i] @ Gamma @ Hs[j].T for j in range(K)] for i in range(K)]
    Syy = np.block(rows) + np.diag(np.concatenate(Rs))
    y = np.concatenate(ys)
    sign, logdet = np.linalg.slogdet(Syy)
    want = -0.5 * (y @ np.linalg.solve(Syy, y) + logdet + len(y) * np.log(2 * np.pi))
    assert sign > 0
    assert ll == pytest.approx(want, rel=1e-11)


@pytest.mark.parametrize("alpha0", [0.0, 0.4])
def test_loglik_derivatives_match_joint_gaussian_closed_form(alpha0):
    # y (stacked) ~ N(0, C) with C = a C_G + s C_R (Gamma scaled by a, every R
    # by s): d ll / d log a = -a (tr(C^-1 C_G) - y^T C^-1 C_G C^-1 y) / 2 at
    # a = 1, and likewise for s; the oracle's central differences must agree
    Gamma, Hs, Rs, ys = _tiny_problem(N=6, steps=3)
    K = len(Hs)
    CG = np.block([[(alpha0 + min(i, j) + 1) * Hs[i] @ Gamma @ Hs[j].T for j in range(K)]
                   for i in range(K)])
    CR = np.diag(np.concatenate(Rs))
    C = CG + CR
    y = np.concatenate(ys)
    Ci_y = np.linalg.solve(C, y)
    want = [-0.5 * (np.trace(np.linalg.solve(C, M)) - Ci_y @ M @ Ci_y) for M in (CG, CR)]
    got = kalman.loglik_log_derivatives_fd(Gamma, Hs, Rs, ys, alpha0=alpha0)
    np.testing.assert_allclose(got, want, rtol=1e-7, atol=1e-10)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
@pytest.mark.parametrize("ell", [0.1, 0.3])
def test_matern_length_derivative_matches_central_differences_of_bessel_form(nu, ell):
    # differentiate the Bessel form itself (an independent route to C)
    r = np.geomspace(1e-4, 3.0, 120)
    h = 1e-4 * ell
    fd = (kernels.matern_bessel(r, nu, ell + h, 2.5) - kernels.matern_bessel(r, nu, ell - h, 2.5)) / (2 * h)
    np.testing.assert_allclose(kernels.matern_dlength(r, nu, ell, 2.5), fd, rtol=1e-6, atol=1e-9)
    assert kernels.matern_dlength(0.0, nu, ell, 2.5) == 0.0


@pytest.mark.parametrize("alpha0", [0.0, 0.4])
def test_loglik_length_derivative_matches_joint_gaussian_closed_form(alpha0):
    # d ll / d log ell = ell * -(tr(C^-1 C') - y^T C^-1 C' C^-1 y)/2 with
    # C' built from dGamma/d ell; against central differences of the oracle's
    # prediction-error log-likelihood over log ell
    g = np.random.default_rng(4)
    pts = g.uniform(0, 1, (7, 2))
    nu, ell, theta = 1.5, 0.4, 0.8
    Hs = [g.standard_normal((2 + k % 2, 7)) for k in range(3)]
    Rs = [g.uniform(0.1, 0.5, H.shape[0]) for H in Hs]
    ys = [g.standard_normal(H.shape[0]) for H in Hs]
    Gamma = kernels.cov_block(pts, pts, nu, ell, theta)
    dG = kernels.cov_block(pts, pts, nu, ell, theta, dlength=True)
    K = len(Hs)
    C = np.block([[(alpha0 + min(i, j) + 1) * Hs[i] @ Gamma @ Hs[j].T for j in range(K)]
                  for i in range(K)]) + np.diag(np.concatenate(Rs))
    Cp = np.block([[(alpha0 + min(i, j) + 1) * Hs[i] @ dG @ Hs[j].T for j in range(K)]
                   for i in range(K)])
    y = np.concatenate(ys)
    Ci_y = np.linalg.solve(C, y)
    want = -0.5 * ell * (np.trace(np.linalg.solve(C, Cp)) - Ci_y @ Cp @ Ci_y)
    hh = 1e-4

    def ll(e):
        return kalman.innovation_loglik(kernels.cov_block(pts, pts, nu, e, theta), Hs, Rs, ys,
                                        alpha0=alpha0)
    fd = (ll(ell * np.exp(hh)) - ll(ell * np.exp(-hh))) / (2 * hh)
    assert fd == pytest.approx(want, rel=1e-7, abs=1e-10)
