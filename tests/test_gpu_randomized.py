"""GPU parity of the randomized generalized eigensolver (Appendix B;
fkf_filter_params.gep_mode = FKF_GEP_RANDOMIZED) and of its Gaussian sketch,
through the C ABI.

* The device sketch equals the oracle's implementation of the same
  counter-based generator (Philox4x32-10 + Box-Muller), number by number.
* With k + p >= n_m the randomized modes are the exact ones: eigenvalues,
  state and variance equal the exact eigensolver's filter to 1e-10 (relative)
  and the oracle's dense filter to 1e-6.
* With k + p < n_m (truncated): the eigenvalues equal the oracle's
  Appendix B eigenvalues for the same sketch, and the state and variance equal
  the oracle's dense filter fed the data the k modes keep (the projected
  observation), on a grid where the H-matrix is the dense Gamma.
"""
import numpy as np
import pytest

import workloads as W
from oracle import direct, gep, kalman, rays, sketch

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_device_sketch_matches_oracle_generator():
    import paper_1405_2276_amd as fkf
    for seed, count in ((0, 7), (14052276, 100_001), (2 ** 63 + 12345, 4096)):
        got = _host(fkf.gaussian_sketch(seed, count))
        want = sketch.normals(seed, count)
        err = np.abs(got - want).max()
        _say(f"[sketch] seed={seed} count={count} maxdiff={err:.2e}")
        assert err <= 1e-12


def _case(shape, nu=1.5, ell=0.3, theta=0.5, n_src=4, n_rcv=5, noise=1e-2, leaf=64):
    import paper_1405_2276_amd as fkf
    pts = W.grid_points(shape)
    cov = fkf.Cov(pts, nu=nu, length=ell, variance=theta, leaf_size=leaf)
    src, rcv = W.crosswell_2d(n_src, n_rcv)
    obs = fkf.Obs.from_rays(shape, src, rcv, noise)
    H = rays.ray_operator(shape, src, rcv)
    R = np.full(H.shape[0], noise)
    Gamma = direct.dense_cov(pts, nu, ell, theta)
    return fkf, pts, cov, obs, H, R, Gamma


@pytest.mark.parametrize("shape,leaf,oversample", [((12, 10), 64, 20), ((32, 24), 64, 0)])
def test_full_sketch_equals_exact_eigensolver(shape, leaf, oversample):
    fkf, pts, cov, obs, H, R, Gamma = _case(shape, leaf=leaf)
    nm = H.shape[0]
    g = np.random.default_rng(3)
    ys = [g.standard_normal(nm) * 0.3 for _ in range(4)]
    fe = fkf.Filter(cov, alpha0=0.2)
    fr = fkf.Filter(cov, alpha0=0.2, gep="randomized", gep_rank=0, oversample=oversample,
                    seed=99)
    ref = kalman.dense_kf(Gamma, [H] * 4, [R] * 4, ys, alpha0=0.2)
    for k, y in enumerate(ys):
        fe.step(obs, y)
        fr.step(obs, y)
        se, ve = _host(fe.mean()), _host(fe.variance())
        sr, vr = _host(fr.mean()), _host(fr.variance())
        es = np.abs(sr - se).max() / np.abs(se).max()
        ev = np.abs(vr - ve).max() / np.abs(ve).max()
        # against the oracle: the method's state bar (relative 2-norm) with
        # the H-matrix approximation of Gamma (block tolerance 1e-7)
        eo = np.linalg.norm(sr - ref[k]["s"]) / np.linalg.norm(ref[k]["s"])
        _say(f"[randomized] {shape} p={oversample} step={k + 1} vs exact state={es:.2e} "
             f"var={ev:.2e} vs oracle state={eo:.2e}")
        assert es <= 1e-10 and ev <= 1e-10 and eo <= 1e-6
    le, _ = fe.modes()
    lr, _ = fr.modes()
    assert len(lr) == len(le) == nm
    assert np.abs(lr - le).max() <= 1e-10 * le[0]
    fe.status()
    fr.status()


@pytest.mark.parametrize("k,p", [(8, 4), (12, 0)])
def test_truncated_sketch_matches_oracle_appendix_b(k, p):
    shape = (12, 10)    # two leaves, both in the near field: the H-matrix is the dense Gamma
    fkf, pts, cov, obs, H, R, Gamma = _case(shape)
    assert cov.info()["n_far_pairs"] == 0
    nm, n = H.shape
    seed = 1405
    lam, U, _, _ = gep.randomized_ghep(H, R, Gamma, sketch.sketch(seed, n, k + p), k)
    g = np.random.default_rng(9)
    ys = [g.standard_normal(nm) * 0.3 for _ in range(3)]
    proj = [gep.projected_observation(U, lam, Gamma, H, R, y) for y in ys]
    ref = kalman.dense_kf(Gamma, [q[0] for q in proj], [np.ones(k)] * 3, [q[1] for q in proj])
    f = fkf.Filter(cov, gep="randomized", gep_rank=k, oversample=p, seed=seed)
    for i, y in enumerate(ys):
        f.step(obs, y)
        s, v = _host(f.mean()), _host(f.variance())
        es = np.abs(s - ref[i]["s"]).max() / np.abs(ref[i]["s"]).max()
        ev = np.abs(v - ref[i]["var"]).max() / np.abs(ref[i]["var"]).max()
        _say(f"[randomized] truncated k={k} p={p} step={i + 1} state={es:.2e} var={ev:.2e}")
        assert es <= 1e-8 and ev <= 1e-8
    lr, w = f.modes()
    _say(f"[randomized] truncated k={k} eigenvalue err={np.abs(lr - lam).max() / lam[0]:.2e}")
    assert len(lr) == k and np.abs(lr - lam).max() <= 1e-9 * lam[0]
    assert f.info()["rank"] == k
    with pytest.raises(fkf.FkfError) as e:
        f.loglik()
    assert e.value.name == "FKF_E_UNSUPPORTED"
    f.status()


def test_randomized_parameter_errors():
    import ctypes
    fkf, pts, cov, obs, H, R, Gamma = _case((12, 10))
    fp = fkf.FilterParams(ctypes.sizeof(fkf.FilterParams), 100, 0.0, 7, 0, 20, 0, 1)
    h = ctypes.c_void_p()
    rc = fkf._lib.fkf_filter_create(cov.handle, None, 0.0, ctypes.byref(fp), fkf._stream(),
                                    ctypes.byref(h))
    assert fkf.STATUS[rc] == "FKF_E_ARG"
    f = fkf.Filter(cov, gep="randomized")
    dcov = fkf.Cov(pts, nu=1.5, length=0.3, variance=0.5, dlength=True)
    with pytest.raises(fkf.FkfError) as e:
        f.track_length(dcov)
    assert e.value.name == "FKF_E_UNSUPPORTED"
