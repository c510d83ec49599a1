"""GPU parity of the innovation log-likelihood the filter accumulates
(fkf_filter_loglik) and of its derivatives with respect to log theta, log
length and log sigma^2, against the oracle: the dense prediction-error
log-likelihood and its central differences (themselves pinned to the
closed-form gradients of the joint Gaussian density); and of the
length-derivative operator dGamma/d length against direct products.  Bars:
1e-6 relative for the log-likelihood and the derivative operator, 1e-5
relative for the derivatives.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import direct, ekf, kalman, rays

pytestmark = pytest.mark.gpu
LL_TOL = 1e-6
GRAD_TOL = 1e-5

CASES = {
    "exp-32x32": W.tiny(shape=(32, 32), nu=0.5, length=0.3, variance=1.0, n_src=8, n_rcv=8,
                        noise_var=1e-4, steps=5, drift_sigma=1.0, leaf_size=64, cfg_id=1),
    "m32-40x24": W.tiny(shape=(40, 24), nu=1.5, length=0.2, variance=0.01, n_src=6, n_rcv=5,
                        noise_var=1e-3, steps=6, drift_sigma=0.1, leaf_size=48, cfg_id=120),
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle(wl):
    pts = wl.points()
    src, rcv = wl.rays()
    H = rays.ray_operator(wl.shape, src, rcv)
    Gamma = direct.dense_cov(pts, wl.nu, wl.length, wl.variance)
    R = np.full(H.shape[0], wl.noise_var)
    return pts, H, Gamma, R


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _fd_log_length(wl, H, R, ys, K, alpha0, h=1e-4):
    """Central difference of the oracle's log-likelihood over log length."""
    pts = wl.points()

    def ll(e):
        G = direct.dense_cov(pts, wl.nu, e, wl.variance)
        return kalman.innovation_loglik(G, [H] * K, [R] * K, ys[:K], alpha0=alpha0)
    return (ll(wl.length * np.exp(h)) - ll(wl.length * np.exp(-h))) / (2 * h)


DPTS = {
    "grid-48x40": lambda: W.grid_points((48, 40)),
    "jitter-40x31": lambda: W.grid_points((40, 31)) + np.random.default_rng(8).uniform(
        -0.004, 0.004, (1240, 2)),
    "cube-14": lambda: W.grid_points((14, 14, 14)),
}


@pytest.mark.parametrize("pname", list(DPTS))
@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_length_derivative_operator_matches_direct(pname, nu):
    import torch
    import paper_1405_2276_amd as fkf
    pts = DPTS[pname]()
    ell, theta = 0.2, 0.7
    _say(f"[loglik] dGamma/dl case={pname} nu={nu} n={len(pts)}")
    cov = fkf.Cov(pts, nu=nu, length=ell, variance=theta, leaf_size=48, dlength=True)
    X = np.random.default_rng(3).standard_normal((len(pts), 5))
    want = direct.cov_matvec(pts, X, nu, ell, theta, dlength=True)
    Xd = torch.from_numpy(np.asfortranarray(X).T.copy()).cuda().t()
    got = cov.apply(Xd)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    _say(f"[loglik] dGamma/dl case={pname} nu={nu} relerr={err:.2e}")
    assert err <= 1e-6
    with pytest.raises(fkf.FkfError):
        fkf.Filter(cov)                      # not a covariance


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("alpha0", [0.0, 0.5])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loglik_and_derivatives_constant_h(name, alpha0, precision):
    import paper_1405_2276_amd as fkf
    wl = CASES[name]
    _say(f"[loglik] case={name} alpha0={alpha0} precision={precision}")
    pts, H, Gamma, R = _oracle(wl)
    ys = W.observations(wl)
    cov = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance,
                  leaf_size=wl.leaf_size, precision=precision)
    src, rcv = wl.rays()
    obs = fkf.Obs.from_rays(wl.shape, src, rcv, wl.noise_var)
    dcov = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance,
                   leaf_size=wl.leaf_size, precision=precision, dlength=True)
    f = fkf.Filter(cov, alpha0=alpha0)
    f.track_length(dcov)
    assert f.loglik() == (0.0, 0.0, 0.0, 0.0)
    for k in range(wl.steps):
        f.step(obs, ys[k])
        ll, d_th, d_nv, d_ln = f.loglik()
        K = k + 1
        want = kalman.innovation_loglik(Gamma, [H] * K, [R] * K, ys[:K], alpha0=alpha0)
        w_th, w_nv = kalman.loglik_log_derivatives_fd(Gamma, [H] * K, [R] * K, ys[:K],
                                                      alpha0=alpha0)
        w_ln = _fd_log_length(wl, H, R, ys, K, alpha0)
        e, et, en, el = _rel(ll, want), _rel(d_th, w_th), _rel(d_nv, w_nv), _rel(d_ln, w_ln)
        _say(f"[loglik] {name} {precision} step={K} ll={ll:.6e} err={e:.1e} "
             f"dlogtheta={d_th:.4e} err={et:.1e} dlognoise={d_nv:.4e} err={en:.1e} "
             f"dloglength={d_ln:.4e} err={el:.1e}")
        assert e <= LL_TOL and et <= GRAD_TOL and en <= GRAD_TOL and el <= GRAD_TOL
    f.status()
    with pytest.raises(fkf.FkfError) as e:
        f.track_length(dcov)                 # only before the first step
    assert e.value.name == "FKF_E_ORDER"
    g = fkf.Filter(cov)
    with pytest.raises(fkf.FkfError) as e:
        g.track_length(cov)                  # not a length derivative
    assert e.value.name == "FKF_E_ARG"


def test_loglik_varying_h_and_extended_filter():
    import paper_1405_2276_amd as fkf
    wl = CASES["m32-40x24"]
    pts, H, Gamma, R = _oracle(wl)
    cov = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance, leaf_size=wl.leaf_size)
    src, rcv = wl.rays()
    geoms = [(src, rcv), (np.ascontiguousarray(src[:, ::-1]), np.ascontiguousarray(rcv[:, ::-1]))]
    obs = [fkf.Obs.from_rays(wl.shape, s, r, wl.noise_var) for s, r in geoms]
    Hs = [rays.ray_operator(wl.shape, s, r) for s, r in geoms]
    ys = W.observations(wl)
    seq = [0, 1, 0, 1]
    f = fkf.Filter(cov)
    for k, i in enumerate(seq):
        f.step(obs[i], ys[k])
        K = k + 1
        want = kalman.innovation_loglik(Gamma, [Hs[j] for j in seq[:K]], [R] * K, ys[:K])
        ll = f.loglik(grad=False)
        _say(f"[loglik] varying step={K} ll={ll:.6e} err={_rel(ll, want):.1e}")
        assert _rel(ll, want) <= LL_TOL
    with pytest.raises(fkf.FkfError) as e:
        f.loglik()
    assert e.value.name == "FKF_E_UNSUPPORTED"
    # extended filter: the log-likelihood of the linearised innovations
    a = 2.0
    yp = W.observations(wl, positive=True)
    ref = ekf.dense_ekf(Gamma, H, R, yp, a)
    fe = fkf.Filter(cov)
    for k in range(3):
        fe.step_boxcox(obs[0], yp[k], a)
        ll = fe.loglik(grad=False)
        _say(f"[loglik] extended step={k + 1} ll={ll:.6e} err={_rel(ll, ref[k]['ll']):.1e}")
        assert _rel(ll, ref[k]["ll"]) <= LL_TOL


def test_autograd_function_matches_oracle_gradient():
    import torch
    import paper_1405_2276_amd as fkf
    wl = CASES["m32-40x24"]
    pts, H, Gamma, R = _oracle(wl)
    ys = W.observations(wl)
    src, rcv = wl.rays()
    theta = torch.tensor(wl.variance, dtype=torch.float64, requires_grad=True)
    length = torch.tensor(wl.length, dtype=torch.float64, requires_grad=True)
    noise = torch.tensor(wl.noise_var, dtype=torch.float64, requires_grad=True)
    ll = fkf.innovation_loglik(theta, length, noise, pts,
                               lambda nv: fkf.Obs.from_rays(wl.shape, src, rcv, nv),
                               [y for y in ys], nu=wl.nu, leaf_size=wl.leaf_size)
    ll.backward()
    K = len(ys)
    want = kalman.innovation_loglik(Gamma, [H] * K, [R] * K, ys)
    w_th, w_nv = kalman.loglik_log_derivatives_fd(Gamma, [H] * K, [R] * K, ys)
    w_ln = _fd_log_length(wl, H, R, ys, K, 0.0)
    g_th, g_ln, g_nv = theta.grad.item(), length.grad.item(), noise.grad.item()
    _say(f"[loglik] autograd ll err={_rel(ll.item(), want):.1e} "
         f"dtheta={g_th:.5e} err={_rel(g_th, w_th / wl.variance):.1e} "
         f"dlength={g_ln:.5e} err={_rel(g_ln, w_ln / wl.length):.1e} "
         f"dnoise={g_nv:.5e} err={_rel(g_nv, w_nv / wl.noise_var):.1e}")
    assert _rel(ll.item(), want) <= LL_TOL
    assert _rel(g_th, w_th / wl.variance) <= GRAD_TOL
    assert _rel(g_ln, w_ln / wl.length) <= GRAD_TOL
    assert _rel(g_nv, w_nv / wl.noise_var) <= GRAD_TOL
