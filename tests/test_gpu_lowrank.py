"""GPU pins of the low-rank representation Sigma_{k|k} = alpha_k Gamma - W D W^T
(Section 2.3, eq. sigmakk) and of the method's degenerate case lambda -> 0
(duplicate and near-duplicate rays), through the C ABI.

* W^T Gamma^-1 W = I and Wd = Gamma^-1 W (Section 2.4: the basis is
  Gamma^-1-orthonormal; the library carries the dual Wd instead of solving with
  Gamma): Wd^T W = I and Gamma Wd = W to 1e-10, on grids small enough that the
  H-matrix is exactly the dense Gamma (every leaf pair in the near field).
* The reconstruction alpha Gamma - W D W^T equals the oracle's dense
  covariance to 1e-9 of its largest entry (constant H and every varying-H
  step, untruncated: the AddLowRank update of Algorithm 5 without loss), and
  it is symmetric positive semi-definite.
* Duplicate rays make H H^T singular and give generalized eigenvalues 0
  (near-duplicates: eigenvalues far below the largest).  That is not an error:
  the filter steps with status FKF_OK and matches the oracle's dense filter
  (state and variance within 1e-6), in the constant-H and the varying-H form.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import direct, kalman, rays

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


SHAPE = (12, 10)   # 120 points, two leaves of 60: the H-matrix is the dense Gamma


def _geometries():
    return [W.crosswell_2d(3, 4), W.crosswell_vertical(3, 3), W.crosswell_2d(2, 5)]


def _check_lowrank(tag, f, alpha, Gamma, Sigma_ref):
    Wt, Wdt, Dt = f.lowrank()
    Wm, Wd, D = _host(Wt), _host(Wdt), _host(Dt)
    r = Wm.shape[1]
    e_orth = np.abs(Wd.T @ Wm - np.eye(r)).max()
    e_dual = np.linalg.norm(Gamma @ Wd - Wm) / np.linalg.norm(Wm)
    Sig = alpha * Gamma - (Wm * D) @ Wm.T
    e_sig = np.abs(Sig - Sigma_ref).max() / np.abs(Sigma_ref).max()
    e_sym = np.abs(Sig - Sig.T).max() / np.abs(Sig).max()
    ev_min = np.linalg.eigvalsh(0.5 * (Sig + Sig.T)).min() / np.abs(Sig).max()
    _say(f"[lowrank] {tag} rank={r} WdtW-I={e_orth:.2e} GammaWd-W={e_dual:.2e} "
         f"Sigma={e_sig:.2e} sym={e_sym:.2e} min eig/max={ev_min:.2e}")
    assert e_orth <= 1e-10 and e_dual <= 1e-10
    assert e_sig <= 1e-9 and e_sym <= 1e-12 and ev_min >= -1e-12
    assert np.all(D >= 0) and np.all(D <= alpha + 1e-12)


def test_lowrank_basis_constant_and_varying_h():
    import paper_1405_2276_amd as fkf
    pts = W.grid_points(SHAPE)
    nu, ell, theta, noise = 1.5, 0.3, 0.5, 1e-2
    cov = fkf.Cov(pts, nu=nu, length=ell, variance=theta, leaf_size=64)
    assert cov.info()["n_far_pairs"] == 0
    Gamma = direct.dense_cov(pts, nu, ell, theta)
    geo = _geometries()
    obs = [fkf.Obs.from_rays(SHAPE, s, r, noise) for s, r in geo]
    Hs = [rays.ray_operator(SHAPE, s, r) for s, r in geo]
    seq = [0, 0, 0, 1, 2, 1, 0]   # three constant-H steps, then a new operator every step
    g = np.random.default_rng(77)
    ys = [g.standard_normal(Hs[i].shape[0]) * 0.3 for i in seq]
    ref = kalman.dense_kf(Gamma, [Hs[i] for i in seq], [np.full(Hs[i].shape[0], noise) for i in seq],
                          ys, alpha0=0.25)
    f = fkf.Filter(cov, alpha0=0.25)
    for k, i in enumerate(seq):
        f.step(obs[i], ys[k])
        _check_lowrank(f"step={k + 1} obs={i}", f, ref[k]["alpha"], Gamma, ref[k]["Sigma"])
    f.status()


def _duplicate_rays(shift):
    # crosswell 4 x 5 rays; rays 0..4 repeated exactly, ray 7 repeated with its
    # receiver moved by `shift` along the right edge
    src, rcv = W.crosswell_2d(4, 5)
    s2 = np.vstack([src, src[:5], src[7:8]])
    r2 = np.vstack([rcv, rcv[:5], rcv[7:8] + np.array([[0.0, shift]])])
    return s2, r2


@pytest.mark.parametrize("shift", [1e-9, 1e-4])
def test_duplicate_rays_constant_and_varying_h(shift):
    import paper_1405_2276_amd as fkf
    shape = (24, 20)
    pts = W.grid_points(shape)
    nu, ell, theta, noise = 1.5, 0.25, 1.0, 1e-4
    cov = fkf.Cov(pts, nu=nu, length=ell, variance=theta, leaf_size=64)
    Gamma = direct.dense_cov(pts, nu, ell, theta)
    src, rcv = _duplicate_rays(shift)
    geo = [(src, rcv), W.crosswell_vertical(4, 4)]
    obs = [fkf.Obs.from_rays(shape, s, r, noise) for s, r in geo]
    Hs = [rays.ray_operator(shape, s, r) for s, r in geo]
    seq = [0, 0, 0, 1, 0, 1]
    g = np.random.default_rng(5)
    ys = [g.standard_normal(Hs[i].shape[0]) for i in seq]
    ref = kalman.dense_kf(Gamma, [Hs[i] for i in seq], [np.full(Hs[i].shape[0], noise) for i in seq],
                          ys, keep_cov=False)
    f = fkf.Filter(cov)
    for k, i in enumerate(seq):
        f.step(obs[i], ys[k])
        f.status()    # FKF_OK: zero eigenvalues are not an error
        if k == 0:
            lam, w = f.modes()
            _say(f"[duplicate] shift={shift} smallest lambda/largest={lam[-1] / lam[0]:.2e} "
                 f"weights finite={np.all(np.isfinite(w))}")
            assert lam[-1] / lam[0] < 1e-6 and np.all(np.isfinite(w)) and np.all(w > 0)
        s, v = _host(f.mean()), _host(f.variance())
        es = np.abs(s - ref[k]["s"]).max() / np.abs(ref[k]["s"]).max()
        ev = np.abs(v - ref[k]["var"]).max() / np.abs(ref[k]["var"]).max()
        _say(f"[duplicate] shift={shift} step={k + 1} obs={i} rank={f.info()['rank']} "
             f"state={es:.2e} var={ev:.2e}")
        assert es <= 1e-6 and ev <= 1e-6
