"""GPU parity of the fast filter (constant H) against the oracle's plain
Kalman filter (dense for small N, cross-covariance form for larger N).

Bars: state estimate and variances within 1e-6 relative (state as relative
2-norm per step, variance as max-abs error over max variance), eigenvalues and
per-mode weights within 1e-6 of the oracle's generalized eigenproblem.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import direct, gep, kalman, rays, sampling

pytestmark = pytest.mark.gpu
TOL = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _setup(wl, block_tol=1e-7):
    import paper_1405_2276_amd as fkf
    pts = wl.points()
    cov = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance,
                  leaf_size=wl.leaf_size, block_tol=block_tol)
    src, rcv = wl.rays()
    obs = fkf.Obs.from_rays(wl.shape, src, rcv, wl.noise_var)
    H = rays.ray_operator(wl.shape, src, rcv)
    R = np.full(H.shape[0], wl.noise_var)
    return fkf, pts, cov, obs, H, R


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _var_err(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


SMALL_CASES = {
    "tiny-12x10": dict(wl=W.tiny(shape=(12, 10), nu=1.5, length=0.3, variance=0.5, n_src=3, n_rcv=4,
                                 noise_var=1e-2, steps=6, leaf_size=16), alpha0=0.0, s0=False),
    "tiny-s0-alpha0": dict(wl=W.tiny(shape=(14, 9), nu=0.5, length=0.4, variance=2.0, n_src=4,
                                     n_rcv=3, noise_var=5e-2, steps=4, leaf_size=16),
                           alpha0=0.75, s0=True),
    "small-32x32": dict(wl=W.SMALL, alpha0=0.0, s0=False),
}


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_constant_h_filter_matches_dense_kf(name):
    case = SMALL_CASES[name]
    wl = case["wl"]
    _say(f"[filter] case={name} n={wl.n}")
    fkf, pts, cov, obs, H, R = _setup(wl)
    Gamma = direct.dense_cov(pts, wl.nu, wl.length, wl.variance)
    ys = W.observations(wl)
    s0 = W.normals(wl, W.STREAM_VECTORS, wl.n) * 0.1 if case["s0"] else None
    ref = kalman.dense_kf(Gamma, [H] * wl.steps, [R] * wl.steps, ys, alpha0=case["alpha0"], s0=s0)
    f = fkf.Filter(cov, s0=s0, alpha0=case["alpha0"])
    # before any step: variance alpha0 * theta, mean s0
    v0 = _host(f.variance())
    np.testing.assert_allclose(v0, case["alpha0"] * wl.variance)
    lam_ref, _ = gep.gep_dense(H, R, Gamma)
    for k in range(wl.steps):
        f.step(obs, ys[k])
        s = _host(f.mean())
        v = _host(f.variance())
        es, ev = _rel(s, ref[k]["s"]), _var_err(v, ref[k]["var"])
        _say(f"[filter] case={name} step={k + 1} state_err={es:.2e} var_err={ev:.2e}")
        assert es <= TOL and ev <= TOL
    f.status()
    info = f.info()
    assert info["k"] == wl.steps and info["alpha"] == case["alpha0"] + wl.steps
    lam, w = f.modes()
    nm = H.shape[0]
    np.testing.assert_allclose(lam, np.maximum(lam_ref[:nm], 0), rtol=0, atol=TOL * lam_ref[0])
    c_ref = gep.mode_weights(lam_ref[:nm], case["alpha0"], wl.steps)
    np.testing.assert_allclose(w, c_ref, rtol=TOL, atol=TOL)


def test_realization_matches_oracle():
    wl = W.tiny(shape=(10, 10), nu=1.5, length=0.35, variance=0.7, n_src=3, n_rcv=3,
                noise_var=1e-2, steps=3, leaf_size=16)
    fkf, pts, cov, obs, H, R = _setup(wl)
    Gamma = direct.dense_cov(pts, wl.nu, wl.length, wl.variance)
    ys = W.observations(wl)
    ref = kalman.dense_kf(Gamma, [H] * 3, [R] * 3, ys)
    f = fkf.Filter(cov)
    g = W.normals(wl, W.STREAM_DRAWS, (wl.n, 3))
    # before any step (alpha = 0): the realization is the mean
    np.testing.assert_allclose(_host(f.realize(g)), 0.0)
    for k in range(3):
        f.step(obs, ys[k])
    got = _host(f.realize(g))
    want = sampling.realize(ref[-1]["s"], ref[-1]["Sigma"], ref[-1]["alpha"], Gamma, g)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    _say(f"[filter] realization err={err:.2e}")
    assert err <= TOL
    one = _host(f.realize(g[:, 1]))
    np.testing.assert_allclose(one, got[:, 1], rtol=1e-13, atol=1e-13)


def test_medium_filter_matches_cross_covariance_kf():
    wl = W.MEDIUM
    _say(f"[filter] medium n={wl.n}")
    fkf, pts, cov, obs, H, R = _setup(wl)
    ys = W.observations(wl)
    P = direct.cross_cov(pts, H, wl.nu, wl.length, wl.variance)
    ref = kalman.xcov_kf(P, H, R, ys, wl.variance)
    f = fkf.Filter(cov)
    worst_s = worst_v = 0.0
    for k in range(wl.steps):
        f.step(obs, ys[k])
        if k in (0, 4, wl.steps - 1):
            s = _host(f.mean())
            v = _host(f.variance())
            es, ev = _rel(s, ref[k]["s"]), _var_err(v, ref[k]["var"])
            worst_s, worst_v = max(worst_s, es), max(worst_v, ev)
            _say(f"[filter] medium step={k + 1} state_err={es:.2e} var_err={ev:.2e}")
    assert worst_s <= TOL and worst_v <= TOL


def test_error_paths():
    import torch
    wl = W.tiny(shape=(8, 8), steps=2, leaf_size=16)
    fkf, pts, cov, obs, H, R = _setup(wl)
    f = fkf.Filter(cov)
    y = np.full(H.shape[0], np.nan)
    f.step(obs, y)
    with pytest.raises(fkf.FkfError) as e:
        f.status()
    assert e.value.name == "FKF_E_NONFINITE"
    with pytest.raises(fkf.FkfError) as e:
        f.step(obs, np.zeros(H.shape[0]))
    assert e.value.name in ("FKF_E_ORDER", "FKF_E_NONFINITE")
    with pytest.raises(fkf.FkfError) as e:
        f.step(obs, np.zeros(H.shape[0]))
    assert e.value.name == "FKF_E_ORDER"
    with pytest.raises(fkf.FkfError) as e:
        fkf.Obs.from_rays(wl.shape, np.array([[0, 0.5]]), np.array([[1, 0.5]]), -1.0)
    assert e.value.name == "FKF_E_ARG"
    with pytest.raises(fkf.FkfError):
        fkf.Filter(cov, alpha0=-1.0)


def test_trace_counts_launches():
    # the tracing subsystem: one basis GEMV per constant-H step; the
    # projected eigenproblem (one per basis) records its three stages:
    # tridiagonal reduction, divide and conquer, back-transformation
    wl = W.tiny(shape=(24, 20), n_src=5, n_rcv=6, steps=3, leaf_size=16, cfg_id=120)
    fkf, pts, cov, obs, H, R = _setup(wl)
    ys = W.observations(wl)
    fkf.trace_enable(True)
    try:
        f = fkf.Filter(cov)
        for k in range(wl.steps):
            f.step(obs, ys[k])
        f.status()
        rep = fkf.trace_report()
    finally:
        fkf.trace_enable(False)
    c_gemv, ms_gemv = rep["filter_gemv"]
    eig = {k: rep[k] for k in ("eig_tridiag", "eig_dc", "eig_back")}
    print(f"[filter] trace gemv {c_gemv} launches {ms_gemv:.3f} ms; eigensolver {eig}", flush=True)
    assert c_gemv == wl.steps and ms_gemv > 0
    assert all(c == 1 and ms > 0 for c, ms in eig.values())
    assert "eig_jacobi_round" not in rep
    assert fkf.trace_report() == {}


def test_reset_reruns_bitwise_like_a_fresh_filter():
    # fkf_filter_reset returns a used filter (constant-H basis, then a step of
    # Section 2.4 with another operator) to its initial state: running it
    # again gives bitwise the results of a fresh filter
    wl = W.tiny(shape=(20, 18), nu=1.5, length=0.3, variance=0.5, n_src=4, n_rcv=3,
                noise_var=1e-2, steps=4, leaf_size=32)
    fkf, pts, cov, obs, H, R = _setup(wl)
    src2, rcv2 = W.crosswell_vertical(3, 3)
    obs2 = fkf.Obs.from_rays(wl.shape, src2, rcv2, wl.noise_var)
    ys = W.observations(wl)
    y2 = np.random.default_rng(4).standard_normal(9)

    def run(f):
        for k in range(wl.steps):
            f.step(obs, ys[k])
        f.step(obs2, y2)
        return _host(f.mean()), _host(f.variance()), f.info(), f.loglik(grad=False)

    fresh = run(fkf.Filter(cov, alpha0=0.3))
    f = fkf.Filter(cov)
    run(f)
    f.reset(alpha0=0.3)
    assert f.info() == {"k": 0, "alpha": 0.3, "rank": 0}
    again = run(f)
    _say(f"[reset] rank={again[2]['rank']} ll={again[3]:.6e}")
    assert np.array_equal(again[0], fresh[0]) and np.array_equal(again[1], fresh[1])
    assert again[2] == fresh[2] and again[3] == fresh[3]
