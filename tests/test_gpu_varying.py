"""GPU parity of the varying-H update (Section 2.4, Algorithm 5 with the
Gamma^-1 inner product realised by dual vectors) against the oracle's plain
Kalman filter with the same sequence of measurement operators."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import direct, kalman, rays, sampling

pytestmark = pytest.mark.gpu
TOL = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _vertical_rays(n_src, n_rcv):
    xs = (np.arange(n_src) + 0.5) / n_src
    xr = (np.arange(n_rcv) + 0.5) / n_rcv
    src = np.array([[a, 0.0] for a in xs for _ in xr])
    rcv = np.array([[b, 1.0] for _ in xs for b in xr])
    return src, rcv


def _setup(shape=(20, 24), nu=1.5, ell=0.3, theta=0.5, noise=1e-2, leaf=64):
    import paper_1405_2276_amd as fkf
    pts = W.grid_points(shape)
    cov = fkf.Cov(pts, nu=nu, length=ell, variance=theta, leaf_size=leaf)
    geoms = [W.crosswell_2d(4, 5), _vertical_rays(3, 4), W.crosswell_2d(3, 3)]
    obs, Hs = [], []
    for src, rcv in geoms:
        obs.append(fkf.Obs.from_rays(shape, src, rcv, noise))
        Hs.append(rays.ray_operator(shape, src, rcv))
    Gamma = direct.dense_cov(pts, nu, ell, theta)
    return fkf, pts, cov, obs, Hs, Gamma


@pytest.mark.parametrize("seq,alpha0", [([0, 0, 1, 0, 1, 1, 2], 0.0), ([1, 0, 2, 1], 0.6)])
def test_varying_h_matches_dense_kf(seq, alpha0):
    fkf, pts, cov, obs, Hs, Gamma = _setup()
    noise = 1e-2
    g = np.random.default_rng(21)
    ys = [g.standard_normal(Hs[i].shape[0]) * 0.3 for i in seq]
    Rs = [np.full(Hs[i].shape[0], noise) for i in seq]
    ref = kalman.dense_kf(Gamma, [Hs[i] for i in seq], Rs, ys, alpha0=alpha0)
    f = fkf.Filter(cov, alpha0=alpha0)
    for k, i in enumerate(seq):
        _say(f"[varying] seq={seq} step={k + 1} obs={i}")
        f.step(obs[i], ys[k])
        s = _host(f.mean())
        v = _host(f.variance())
        es = np.linalg.norm(s - ref[k]["s"]) / np.linalg.norm(ref[k]["s"])
        ev = np.abs(v - ref[k]["var"]).max() / np.abs(ref[k]["var"]).max()
        _say(f"[varying] step={k + 1} rank={f.info()['rank']} state_err={es:.2e} var_err={ev:.2e}")
        assert es <= TOL and ev <= TOL
    f.status()
    assert f.info()["alpha"] == alpha0 + len(seq)
    # realizations in the general form
    gd = W.normals(W.tiny(), W.STREAM_DRAWS, (len(pts), 2))
    got = _host(f.realize(gd))
    want = sampling.realize(ref[-1]["s"], ref[-1]["Sigma"], ref[-1]["alpha"], Gamma, gd)
    er = np.abs(got - want).max() / np.abs(want).max()
    _say(f"[varying] realization err={er:.2e}")
    assert er <= TOL


def test_varying_h_rank_growth_and_truncation():
    fkf, pts, cov, obs, Hs, Gamma = _setup()
    g = np.random.default_rng(3)
    f = fkf.Filter(cov)
    ranks = []
    for k, i in enumerate([0, 1, 2, 0]):
        f.step(obs[i], g.standard_normal(Hs[i].shape[0]) * 0.1)
        ranks.append(f.info()["rank"])
    # rank is at most the number of measurements so far and never decreases here
    assert ranks[0] <= 20 and ranks[1] <= 32 and ranks[-1] <= len(pts)
    assert all(b >= a for a, b in zip(ranks, ranks[1:]))
    # the constant-H mode query is refused in the general form
    with pytest.raises(fkf.FkfError):
        f.modes()
    # a small max_rank is reported as FKF_E_RANK
    f2 = fkf.Filter(cov, max_rank=10)
    f2.step(obs[0], g.standard_normal(20))
    with pytest.raises(fkf.FkfError) as e:
        f2.step(obs[1], g.standard_normal(12))
    assert e.value.name == "FKF_E_RANK"
