"""CPU pins of the oracle's randomized generalized eigensolver (Appendix B)
and of its Gaussian sketch generator.

* Philox4x32-10 against the generator's published known-answer vectors.
* The Box-Muller normals: mean, variance and a Kolmogorov-Smirnov test
  against the normal law; distinct seeds and columns uncorrelated.
* With a sketch of at least n_m columns the sketch spans range(H^T), and the
  randomized eigenpairs are the exact ones: eigenvalues equal the library
  generalized eigensolver's, U^T Gamma^-1 U = I and
  H^T R^-1 H = Gamma^-1 U Lambda U^T Gamma^-1.
* With a smaller sketch the Ritz values lie below the exact eigenvalues
  (Rayleigh-Ritz on a subspace) and within the appendix's bound
  |lambda - lambda~| <= 2 eps, eps = ||(I - Q Q^T B) B^-1 A||_B.
* The projected observation of an untruncated decomposition reproduces the
  plain filter (state and covariance).
"""
import numpy as np
import pytest
import scipy.stats

import workloads as W
from oracle import direct, gep, kalman, rays, sketch

KAT = [  # (counter, key, output), Philox4x32-10 known-answer vectors
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    got = sketch.philox4x32_10([np.array([c], dtype=np.uint64) for c in ctr], key)
    assert tuple(int(x[0]) for x in got) == want


def test_sketch_normals_are_standard_normal():
    z = sketch.normals(2024, 200_000)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # even and odd numbers (cosine and sine of one pair) and two seeds are
    # uncorrelated
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 0.01
    z2 = sketch.normals(2025, 200_000)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.01
    om = sketch.sketch(2024, 1000, 3)
    assert np.array_equal(om[:, 1], z[1000:2000])


def _problem(shape=(10, 9), n_src=4, n_rcv=5, noise=1e-2):
    pts = W.grid_points(shape)
    Gamma = direct.dense_cov(pts, 1.5, 0.35, 0.7)
    src, rcv = W.crosswell_2d(n_src, n_rcv)
    H = rays.ray_operator(shape, src, rcv)
    R = np.full(H.shape[0], noise)
    return pts, Gamma, H, R


@pytest.mark.parametrize("oversample", [0, 20])
def test_randomized_ghep_is_exact_with_a_full_sketch(oversample):
    pts, Gamma, H, R = _problem()
    nm, n = H.shape
    Om = sketch.sketch(11, n, nm + oversample)
    lam, U, Q, Qh = gep.randomized_ghep(H, R, Gamma, Om, nm)
    lam_ref, _ = gep.gep_dense(H, R, Gamma)
    assert np.allclose(lam, lam_ref[:nm], rtol=1e-9, atol=1e-9 * lam_ref[0])
    B = np.linalg.inv(Gamma)
    assert np.abs(U.T @ B @ U - np.eye(nm)).max() < 1e-9
    Hd = H.toarray()
    A = Hd.T @ (Hd / R[:, None])
    BU = B @ U
    assert np.abs(A - (BU * lam) @ BU.T).max() < 1e-8 * np.abs(A).max()
    assert np.abs(Q - Gamma @ Qh).max() < 1e-12 * np.abs(Q).max()


@pytest.mark.parametrize("k,p", [(6, 4), (10, 2)])
def test_randomized_ghep_ritz_values_within_the_appendix_bound(k, p):
    pts, Gamma, H, R = _problem()
    nm, n = H.shape
    lam, U, Q, Qh = gep.randomized_ghep(H, R, Gamma, sketch.sketch(5, n, k + p), k)
    lam_ref, _ = gep.gep_dense(H, R, Gamma)
    B = np.linalg.inv(Gamma)
    Hd = H.toarray()
    A = Hd.T @ (Hd / R[:, None])
    # eps = ||(I - Q Q^T B) B^-1 A||_B, ||X||_B = ||B^1/2 X B^-1/2||_2
    wB, VB = np.linalg.eigh(0.5 * (B + B.T))
    Bh = (VB * np.sqrt(wB)) @ VB.T
    Bih = (VB / np.sqrt(wB)) @ VB.T
    E = (np.eye(n) - Q @ Q.T @ B) @ (Gamma @ A)
    eps = np.linalg.norm(Bh @ E @ Bih, 2)
    err = lam_ref[:k] - lam
    assert np.all(err >= -1e-10 * lam_ref[0])        # Ritz values below the exact ones
    assert np.all(err <= 2 * eps + 1e-10 * lam_ref[0])
    assert eps > 0 and err[0] < 1e-3 * lam_ref[0]     # the dominant mode is resolved


def test_projected_observation_of_full_decomposition_reproduces_the_filter():
    pts, Gamma, H, R = _problem()
    nm, n = H.shape
    lam, U, _, _ = gep.randomized_ghep(H, R, Gamma, sketch.sketch(3, n, nm + 5), nm)
    g = np.random.default_rng(1)
    ys = [g.standard_normal(nm) for _ in range(3)]
    ref = kalman.dense_kf(Gamma, [H] * 3, [R] * 3, ys, alpha0=0.2)
    proj = [gep.projected_observation(U, lam, Gamma, H, R, y) for y in ys]
    got = kalman.dense_kf(Gamma, [p[0] for p in proj], [np.ones(nm)] * 3, [p[1] for p in proj],
                          alpha0=0.2)
    for a, b in zip(got, ref):
        assert np.linalg.norm(a["s"] - b["s"]) <= 1e-9 * np.linalg.norm(b["s"])
        assert np.abs(a["Sigma"] - b["Sigma"]).max() <= 1e-9 * np.abs(b["Sigma"]).max()
