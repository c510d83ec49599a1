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


def test_varying_h_480_rays_full_field():
    # steps with a new operator every step at n_m = 480 on the 128 x 128 grid
    # (N = 16384, two 480-ray crosswell geometries taken in turn), untruncated
    # (rank_rtol = 0), against the oracle's dense Kalman filter
    # (tests/golden/varying_reference.npz, make_varying_reference.py): every
    # cell of the state and variance after every step
    import os
    import paper_1405_2276_amd as fkf
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_varying_reference as mv
    ref_path = os.path.join(os.path.dirname(__file__), "golden", "varying_reference.npz")
    if not os.path.exists(ref_path):
        pytest.skip("reference file not generated")
    ref = np.load(ref_path)
    wl = W.MEDIUM
    cov = fkf.Cov(wl.points(), nu=wl.nu, length=wl.length, variance=wl.variance,
                  leaf_size=wl.leaf_size)
    obs = [fkf.Obs.from_rays(wl.shape, s, r, wl.noise_var) for s, r in mv.geometries()]
    f = fkf.Filter(cov, rank_rtol=0.0)
    for k, g in enumerate(ref["sequence"].tolist(), start=1):
        f.step(obs[g], ref["ys"][k - 1])
        s, v = _host(f.mean()), _host(f.variance())
        rs, rv = ref[f"s{k}"], ref[f"v{k}"]
        es = np.abs(s - rs).max() / np.abs(rs).max()
        e2 = np.linalg.norm(s - rs) / np.linalg.norm(rs)
        ev = np.abs(v - rv).max() / np.abs(rv).max()
        _say(f"[varying480] step={k} geometry={g} rank={f.info()['rank']} state maxabs={es:.2e} "
             f"2norm={e2:.2e} var maxabs={ev:.2e}")
        assert es <= TOL and e2 <= TOL and ev <= TOL
    f.status()


def test_failed_step_leaves_the_filter_unchanged():
    # a step that fails (here: the low-rank term would exceed max_rank) leaves
    # the estimate (bitwise), the variance, alpha and the step count as they
    # were, and the filter then refuses further steps (FKF_E_ORDER)
    fkf, pts, cov, obs, Hs, Gamma = _setup()
    g = np.random.default_rng(8)
    f = fkf.Filter(cov, max_rank=24)
    f.step(obs[0], g.standard_normal(20))      # constant-H basis: rank 20
    s0, v0, i0 = _host(f.mean()), _host(f.variance()), f.info()
    with pytest.raises(fkf.FkfError) as e:
        f.step(obs[1], g.standard_normal(12))  # rank 20 + 12 > 24
    assert e.value.name == "FKF_E_RANK"
    s1, v1, i1 = _host(f.mean()), _host(f.variance()), f.info()
    assert np.array_equal(s1, s0)
    assert np.abs(v1 - v0).max() <= 1e-12 * np.abs(v0).max()
    assert (i1["k"], i1["alpha"]) == (i0["k"], i0["alpha"])
    with pytest.raises(fkf.FkfError) as e2:
        f.step(obs[0], g.standard_normal(20))
    assert e2.value.name == "FKF_E_ORDER"
