"""GPU parity of the H-matrix covariance product against the direct oracle.

The bar is the one set for the method: relative error <= 1e-7 against the
direct (exact, O(N^2)) product in FP64.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import direct

pytestmark = pytest.mark.gpu

TOL = 1e-7


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.from_numpy(a.copy()).cuda()
    return torch.from_numpy(np.asfortranarray(a).T.copy()).cuda().t()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = {
    "exp-32x32": dict(pts=lambda: W.grid_points((32, 32)), nu=0.5, ell=0.3, theta=1.0, leaf=64),
    "m32-128x128": dict(pts=lambda: W.grid_points((128, 128)), nu=1.5, ell=0.2, theta=1e-4, leaf=64),
    "irregular-3001": dict(pts=lambda: np.random.default_rng(7).uniform(0, 1, (3001, 2)), nu=1.5,
                           ell=0.15, theta=2.0, leaf=64),
    "m52-jitter-40x31": dict(pts=lambda: W.grid_points((40, 31)) + np.random.default_rng(8).uniform(
        -0.004, 0.004, (1240, 2)), nu=2.5, ell=0.25, theta=1.0, leaf=48),
    "exp-3d-16": dict(pts=lambda: W.grid_points((16, 16, 16)), nu=0.5, ell=0.3, theta=1.0, leaf=64),
    "leaf16-20x30": dict(pts=lambda: W.grid_points((20, 30)), nu=1.5, ell=0.2, theta=1.0, leaf=16),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nrhs", [1, 3, 40])
def test_hmatvec_matches_direct(name, nrhs):
    import paper_1405_2276_amd as fkf
    c = CASES[name]
    pts = c["pts"]()
    _say(f"[hmat] case={name} nrhs={nrhs} n={len(pts)}")
    cov = fkf.Cov(pts, nu=c["nu"], length=c["ell"], variance=c["theta"], leaf_size=c["leaf"])
    X = np.random.default_rng(11).standard_normal((len(pts), nrhs))
    want = direct.cov_matvec(pts, X, c["nu"], c["ell"], c["theta"])
    got = _host(cov.apply(_dev(X if nrhs > 1 else X[:, 0])))
    got = got.reshape(want.shape)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    _say(f"[hmat] case={name} nrhs={nrhs} relerr={err:.3e} info={cov.info()['cheb_p']}")
    assert err <= TOL


@pytest.mark.parametrize("points", ["grid-96x72", "irregular-5000"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_stored_and_evaluated_couplings_agree(precision, points):
    # the far field with couplings stored at build (one matrix per distinct
    # geometry of an ordered pair: shared across most pairs on the grid, none
    # shared for random points) and evaluated in every product: the same
    # entries up to rounding, so the products agree to rounding
    import paper_1405_2276_amd as fkf
    pts = (W.grid_points((96, 72)) if points.startswith("grid")
           else np.random.default_rng(5).uniform(0, 1, (5000, 2)))
    kw = dict(nu=1.5, length=0.12, variance=1.0, precision=precision)
    c_st = fkf.Cov(pts, **kw)
    c_ev = fkf.Cov(pts, far_eval=True, **kw)
    inf = c_st.info()
    assert inf["far_bytes"] > 0 and c_ev.info()["far_bytes"] == 0
    assert inf["far_bytes"] == fkf.plan(pts, **kw)["far_bytes"]
    per = 4 if precision == "mixed" else 8
    shared = inf["far_bytes"] < 2 * per * inf["far_pair_entries"]
    _say(f"[hmat] {points}: {inf['far_bytes']} stored coupling bytes for "
         f"{inf['far_pair_entries']} pair entries")
    assert shared == points.startswith("grid")
    X = np.random.default_rng(21).standard_normal((len(pts), 5))
    for cols in (X[:, 0], X):
        a = _host(c_st.apply(_dev(cols)))
        b = _host(c_ev.apply(_dev(cols)))
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        _say(f"[hmat] stored vs evaluated couplings ({precision}) relerr={err:.2e}")
        assert err <= 1e-14


def test_hmatvec_evaluated_couplings_match_direct():
    import paper_1405_2276_amd as fkf
    for name in ("m32-128x128", "exp-3d-16"):
        c = CASES[name]
        pts = c["pts"]()
        cov = fkf.Cov(pts, nu=c["nu"], length=c["ell"], variance=c["theta"], leaf_size=c["leaf"],
                      far_eval=True)
        x = np.random.default_rng(12).standard_normal(len(pts))
        want = direct.cov_matvec(pts, x, c["nu"], c["ell"], c["theta"])
        got = _host(cov.apply(_dev(x)))
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        _say(f"[hmat] evaluated couplings case={name} relerr={err:.3e}")
        assert err <= TOL


def test_hmatvec_fixed_order_six_reports_error():
    # the 128x128 workload with Chebyshev order 6 at every level (no per-level
    # raise): measured, expected well above 1e-7 (see the order-selection rule)
    import paper_1405_2276_amd as fkf
    wl = W.MEDIUM
    pts = wl.points()
    cov = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance, cheb_order=6, block_tol=0)
    x = np.random.default_rng(3).standard_normal(len(pts))
    want = direct.cov_matvec(pts, x, wl.nu, wl.length, wl.variance)
    got = _host(cov.apply(_dev(x)))
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    _say(f"[hmat] fixed p=6 relerr={err:.3e}")
    assert 1e-9 < err < 1e-3


def test_hmatvec_headline_size_sampled_rows():
    import paper_1405_2276_amd as fkf
    wl = W.LARGE
    pts = wl.points()
    _say(f"[hmat] headline n={len(pts)}")
    cov = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance)
    info = cov.info()
    _say(f"[hmat] headline info {info}")
    X = np.random.default_rng(12).standard_normal((len(pts), 3))
    rows = np.random.default_rng(13).choice(len(pts), 256, replace=False)
    want = direct.cov_rows(pts, rows, X, wl.nu, wl.length, wl.variance)
    got1 = _host(cov.apply(_dev(X[:, 0])))
    got3 = _host(cov.apply(_dev(X)))
    e1 = np.linalg.norm(got1[rows] - want[:, 0]) / np.linalg.norm(want[:, 0])
    e3 = np.linalg.norm(got3[rows] - want) / np.linalg.norm(want)
    _say(f"[hmat] headline sampled relerr nrhs1={e1:.3e} nrhs3={e3:.3e}")
    assert e1 <= TOL and e3 <= TOL
    # the one- and multi-column paths agree
    np.testing.assert_allclose(got3[:, 0], got1, rtol=1e-12, atol=1e-12 * np.abs(got1).max())


def test_hmatvec_headline_size_every_row():
    # every row of Gamma x at N = 65536 against the oracle's direct product
    # (tests/golden/hmatvec_reference.npz, written by make_hmatvec_reference.py
    # from the oracle only), one column and both columns together, in the
    # configuration the benchmark times; bar 1e-7 relative as the 2-norm and
    # as the largest row error over the largest entry
    import os
    import paper_1405_2276_amd as fkf
    ref_path = os.path.join(os.path.dirname(__file__), "golden", "hmatvec_reference.npz")
    if not os.path.exists(ref_path):
        pytest.skip("reference file not generated")
    ref = np.load(ref_path)
    wl = W.LARGE
    pts = wl.points()
    _say(f"[hmat] headline every row n={len(pts)}")
    cov = fkf.Cov(pts, nu=wl.nu, length=wl.length, variance=wl.variance)
    x, want = ref["x"], ref["y"]
    got1 = _host(cov.apply(_dev(np.ascontiguousarray(x[:, 0]))))
    got2 = _host(cov.apply(_dev(x)))
    for tag, got, w in (("nrhs1", got1, want[:, 0]), ("nrhs2", got2, want)):
        e2 = np.linalg.norm(got - w) / np.linalg.norm(w)
        emax = np.abs(got - w).max() / np.abs(w).max()
        _say(f"[hmat] headline every row {tag} 2norm={e2:.3e} maxabs={emax:.3e}")
        assert e2 <= TOL and emax <= TOL


def test_hmatvec_deterministic_and_symmetric():
    import paper_1405_2276_amd as fkf
    pts = W.grid_points((64, 48))
    cov = fkf.Cov(pts, nu=1.5, length=0.2, variance=1.0)
    g = np.random.default_rng(5)
    x, y = g.standard_normal(len(pts)), g.standard_normal(len(pts))
    gx1 = _host(cov.apply(_dev(x)))
    gx2 = _host(cov.apply(_dev(x)))
    gy = _host(cov.apply(_dev(y)))
    assert np.array_equal(gx1, gx2)
    assert abs(y @ gx1 - x @ gy) <= 1e-12 * abs(y @ gx1)


def test_hmatvec_leading_dimensions_and_errors():
    import torch
    import paper_1405_2276_amd as fkf
    pts = W.grid_points((24, 24))
    cov = fkf.Cov(pts, nu=0.5, length=0.3)
    X = np.random.default_rng(2).standard_normal((576, 4))
    big = torch.zeros((4, 600), dtype=torch.float64, device="cuda")
    big[:, :576] = torch.from_numpy(X.T.copy()).cuda()
    Xv = big.t()[:576]           # ld 600
    out = torch.full((4, 610), 7.0, dtype=torch.float64, device="cuda")
    Yv = out.t()[:576]           # ld 610
    cov.apply(Xv, out=Yv)
    want = direct.cov_matvec(pts, X, 0.5, 0.3, 1.0)
    np.testing.assert_allclose(_host(Yv), want, rtol=1e-7, atol=1e-7 * np.abs(want).max())
    assert torch.all(out.t()[576:] == 7.0)
    with pytest.raises(ValueError):
        cov.apply(torch.zeros(10, dtype=torch.float64, device="cuda"))


def test_hmatvec_column_blocks_under_workspace_bound():
    # a small workspace bound makes the 40-column product run in blocks of a
    # few columns; every column must come out as in the one-block product
    import paper_1405_2276_amd as fkf
    pts = W.grid_points((40, 36))
    kw = dict(nu=1.5, length=0.2, variance=1.0, leaf_size=48)
    whole = fkf.Cov(pts, **kw)
    blocks = fkf.Cov(pts, workspace_bytes=300_000, **kw)
    X = np.random.default_rng(9).standard_normal((len(pts), 40))
    a, b = _host(whole.apply(_dev(X))), _host(blocks.apply(_dev(X)))
    err = np.abs(a - b).max() / np.abs(a).max()
    _say(f"[hmat] column blocks vs one block maxdiff={err:.2e}")
    assert err <= 1e-14
    want = direct.cov_matvec(pts, X, 1.5, 0.2, 1.0)
    assert np.linalg.norm(b - want) / np.linalg.norm(want) <= 1e-7
