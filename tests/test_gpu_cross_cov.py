"""GPU parity of the cross covariance Gamma H^T (fkf_obs_cross_cov), which
takes the columns H^T as the sparse rows of H (near field and far-cluster
moments summed over the nonzeros of H), against
the several-column product of the same operator with the dense H^T
(fkf_cov_apply) and against the direct oracle.

Bars: 1e-12 relative (max abs / max abs) against the dense-H^T product in
FP64 (the two differ only in the rounding order of the moments); the
method's 1e-7 against the direct product; 1e-6 against the dense-H^T
product in the mixed mode, where both round the same moments to FP32 before
the couplings.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import direct

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _dense_ht(fkf, obs):
    import torch
    H = obs.csr().toarray()
    return H, torch.from_numpy(np.asfortranarray(H.T).T.copy()).cuda().t()


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def _rays_obs(fkf, shape, n_src, n_rcv, noise=1e-4, seed=0):
    wl = W.tiny(shape=shape, n_src=n_src, n_rcv=n_rcv, noise_var=noise, cfg_id=900 + seed)
    src, rcv = wl.rays()
    return fkf.Obs.from_rays(shape, src, rcv, noise)


def _random_obs(fkf, n, n_m, per_row, seed):
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for m in range(n_m):
        c = rng.choice(n, size=per_row, replace=False)
        rows += [m] * per_row
        cols += list(c)
        vals += list(rng.uniform(0.1, 1.0, per_row))
    H = sp.csr_matrix((vals, (rows, cols)), shape=(n_m, n))
    return fkf.Obs.from_csr(H, np.full(n_m, 1e-3))


CASES = {
    # rays on a grid with several levels of far clusters
    "rays-64x64": dict(pts=lambda: W.grid_points((64, 64)), nu=1.5, ell=0.2, theta=1e-4, leaf=64,
                       obs=lambda f: _rays_obs(f, (64, 64), 6, 5)),
    # ragged 16-point leaves
    "rays-leaf16-40x36": dict(pts=lambda: W.grid_points((40, 36)), nu=0.5, ell=0.3, theta=1.0,
                              leaf=16, obs=lambda f: _rays_obs(f, (40, 36), 4, 7, seed=1)),
    # irregular points, random sparse rows
    "random-irregular-3001": dict(pts=lambda: np.random.default_rng(7).uniform(0, 1, (3001, 2)),
                                  nu=2.5, ell=0.15, theta=2.0, leaf=64,
                                  obs=lambda f: _random_obs(f, 3001, 37, 40, 3)),
    # three dimensions (p^3 coefficients, more than one wavefront of lanes)
    "rays-3d-16": dict(pts=lambda: W.grid_points((16, 16, 16)), nu=0.5, ell=0.3, theta=1.0,
                       leaf=64, obs=None),
}


def _obs_3d(fkf, shape=(16, 16, 16), n_m=21, seed=5):
    rng = np.random.default_rng(seed)
    src = np.column_stack([np.zeros(n_m), rng.uniform(0.05, 0.95, (n_m, 2))])
    rcv = np.column_stack([np.ones(n_m), rng.uniform(0.05, 0.95, (n_m, 2))])
    return fkf.Obs.from_rays(shape, src, rcv, np.full(n_m, 1e-3))


@pytest.mark.parametrize("name", list(CASES))
def test_cross_cov_matches_dense_product_and_direct(name):
    import paper_1405_2276_amd as fkf
    c = CASES[name]
    pts = c["pts"]()
    cov = fkf.Cov(pts, nu=c["nu"], length=c["ell"], variance=c["theta"], leaf_size=c["leaf"])
    obs = c["obs"](fkf) if c["obs"] is not None else _obs_3d(fkf)
    H, Htd = _dense_ht(fkf, obs)
    _say(f"[xcov] case={name} n={len(pts)} n_m={H.shape[0]} nnz={obs.csr().nnz}")
    got = _host(obs.cross_cov(cov))
    dense = _host(cov.apply(Htd))
    want = direct.cov_matvec(pts, H.T, c["nu"], c["ell"], c["theta"])
    e_dense, e_direct = _rel(got, dense), _rel(got, want)
    _say(f"[xcov] case={name} vs dense-H^T product {e_dense:.2e}, vs direct {e_direct:.2e}")
    assert e_dense <= 1e-12
    assert e_direct <= 1e-7


def test_cross_cov_mixed_precision():
    import paper_1405_2276_amd as fkf
    c = CASES["rays-64x64"]
    pts = c["pts"]()
    cov = fkf.Cov(pts, nu=c["nu"], length=c["ell"], variance=c["theta"], leaf_size=c["leaf"],
                  precision="mixed")
    obs = c["obs"](fkf)
    H, Htd = _dense_ht(fkf, obs)
    got = _host(obs.cross_cov(cov))
    dense = _host(cov.apply(Htd))
    e = _rel(got, dense)
    _say(f"[xcov] mixed vs dense-H^T product {e:.2e}")
    assert e <= 1e-6


def test_cross_cov_column_blocks_under_workspace_bound():
    # a workspace bound that allows 7 columns per block (the sparse form keeps
    # two coefficient vectors per column): several blocks, the last one ragged
    import paper_1405_2276_amd as fkf
    c = CASES["rays-64x64"]
    pts = c["pts"]()
    cov0 = fkf.Cov(pts, nu=c["nu"], length=c["ell"], variance=c["theta"], leaf_size=c["leaf"])
    ncoef = cov0.info()["far_coef_per_rhs"]
    cov = fkf.Cov(pts, nu=c["nu"], length=c["ell"], variance=c["theta"], leaf_size=c["leaf"],
                  workspace_bytes=8 * 2 * ncoef * 7)
    obs = c["obs"](fkf)
    H, Htd = _dense_ht(fkf, obs)
    assert H.shape[0] % 7 != 0
    got = _host(obs.cross_cov(cov))
    dense = _host(cov0.apply(Htd))
    e = _rel(got, dense)
    _say(f"[xcov] blocks of 7 columns (n_m={H.shape[0]}) vs one block {e:.2e}")
    assert e <= 1e-12
    # a bound of n_m - 1 columns would leave a block of one column: the
    # blocks are shrunk so that none is
    n_m = H.shape[0]
    cov1 = fkf.Cov(pts, nu=c["nu"], length=c["ell"], variance=c["theta"], leaf_size=c["leaf"],
                   workspace_bytes=8 * 2 * ncoef * (n_m - 1))
    e1 = _rel(_host(obs.cross_cov(cov1)), dense)
    _say(f"[xcov] bound of {n_m - 1} columns vs one block {e1:.2e}")
    assert e1 <= 1e-12


def test_cross_cov_repeated_columns_are_summed():
    # a row listing the same cell twice is the operator with the two values
    # summed: the stored CSR, products with H and Gamma H^T all agree on it
    import torch
    import paper_1405_2276_amd as fkf
    pts = W.grid_points((32, 32))
    n = len(pts)
    cov = fkf.Cov(pts, nu=1.5, length=0.2, variance=1.0, leaf_size=64)
    rng = np.random.default_rng(9)
    rowptr = [0]
    col, val = [], []
    for m in range(9):
        c = list(rng.choice(n, size=30, replace=False))
        c = c + c[:5]                       # five cells twice
        v = list(rng.uniform(0.1, 1.0, len(c)))
        col += c[::-1]                      # unsorted
        val += v[::-1]
        rowptr.append(len(col))
    H = sp.csr_matrix((val, col, rowptr), shape=(9, n))   # sums duplicates when densified
    Hd = H.toarray()
    obs = fkf.Obs.from_csr(H, np.full(9, 1e-3))
    stored = obs.csr()
    assert stored.nnz == 9 * 30
    assert np.all(np.diff(stored.indices[stored.indptr[0]:stored.indptr[1]]) > 0)
    np.testing.assert_allclose(stored.toarray(), Hd, rtol=1e-15, atol=0)
    x = rng.standard_normal(n)
    hx = _host(obs.apply(torch.from_numpy(x).cuda()))
    np.testing.assert_allclose(hx, Hd @ x, rtol=1e-12)
    got = _host(obs.cross_cov(cov))
    want = direct.cov_matvec(pts, Hd.T, 1.5, 0.2, 1.0)
    e = _rel(got, want)
    _say(f"[xcov] repeated columns vs direct {e:.2e}")
    assert e <= 1e-7


def test_cross_cov_long_rows_take_dense_product():
    # rows beyond the sort size of the sparse moments: the dense-H^T product
    import paper_1405_2276_amd as fkf
    pts = W.grid_points((64, 64))
    n = len(pts)
    cov = fkf.Cov(pts, nu=0.5, length=0.3, variance=1.0, leaf_size=64)
    obs = _random_obs(fkf, n, 3, 2500, 4)
    H, Htd = _dense_ht(fkf, obs)
    got = _host(obs.cross_cov(cov))
    dense = _host(cov.apply(Htd))
    assert _rel(got, dense) <= 1e-15
    want = direct.cov_matvec(pts, H.T, 0.5, 0.3, 1.0)
    assert _rel(got, want) <= 1e-7


def test_cross_cov_argument_errors():
    import paper_1405_2276_amd as fkf
    cov = fkf.Cov(W.grid_points((32, 32)), nu=0.5, length=0.3, variance=1.0, leaf_size=64)
    obs = _rays_obs(fkf, (16, 16), 3, 3)
    with pytest.raises(fkf.FkfError) as e:      # cov has 1024 points, obs 256
        obs.cross_cov(cov)
    assert e.value.name == "FKF_E_ARG"
