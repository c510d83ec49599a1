"""fkf_cov_apply_noalloc (the product with its workspace in the library's
fixed per-device array, no device allocation) against fkf_cov_apply, the
existing entry point with the same kernels, on two calls in a row (the second
with a smaller operator and fewer columns), and against the direct oracle.

Bars: element by element against fkf_cov_apply at 1e-12 of the largest
entry (the same kernels in the same order: expected bitwise equal); against
the direct product 1e-7 relative, the matvec tolerance of the FP64 mode."""
import numpy as np
import pytest

import workloads as W
from oracle import direct

pytestmark = pytest.mark.gpu

CASES = [  # (grid, nu, length, columns): the first call is the larger one
    ((256, 256), 1.5, 0.1, 40),
    ((40, 36), 0.5, 0.3, 1),
]


def _say(msg):
    print(msg, flush=True)


def test_noalloc_product_matches_apply_on_consecutive_calls():
    import torch
    import paper_1405_2276_amd as fkf
    for call, (shape, nu, ell, nrhs) in enumerate(CASES):
        n = int(np.prod(shape))
        _say(f"[noalloc] call={call} grid={shape} n={n} nrhs={nrhs}")
        pts = W.grid_points(shape)
        cov = fkf.Cov(pts, nu=nu, length=ell, variance=1.0, leaf_size=64)
        x = W.normals(W.tiny(cfg_id=300 + call), W.STREAM_VECTORS, (n, nrhs))
        xd = fkf.to_device(x)
        want = cov.apply(xd)
        got = cov.apply_noalloc(xd, fkf.fortran_empty(n, nrhs))
        torch.cuda.synchronize()
        w = want.cpu().numpy().reshape(n, nrhs)
        g = got.cpu().numpy().reshape(n, nrhs)
        e_apply = np.abs(g - w).max() / np.abs(w).max()
        rows = np.sort(W.rng(300 + call, 7).choice(n, min(n, 256), replace=False))
        ref = direct.cov_rows(pts, rows, x, nu, ell, 1.0)
        e_dir = np.linalg.norm(g[rows] - ref) / np.linalg.norm(ref)
        _say(f"[noalloc] call={call} vs fkf_cov_apply {e_apply:.2e} vs direct {e_dir:.2e}")
        assert e_apply <= 1e-12
        assert e_dir <= 1e-7
        cov.close()


def test_noalloc_rejects_bad_arguments():
    import torch
    import paper_1405_2276_amd as fkf
    pts = W.grid_points((16, 16))
    cov = fkf.Cov(pts, nu=1.5, length=0.2, variance=1.0, leaf_size=64)
    x = torch.zeros(256, dtype=torch.float64, device="cuda")
    with pytest.raises(fkf.FkfError) as e:
        fkf._check(fkf._lib.fkf_cov_apply_noalloc(cov.handle, x.data_ptr(), 100, 1,
                                                   x.data_ptr(), 256, fkf._stream()))
    assert e.value.name == "FKF_E_ARG"
    # zero columns is a no-op
    fkf._check(fkf._lib.fkf_cov_apply_noalloc(cov.handle, None, 256, 0, None, 256,
                                               fkf._stream()))
    cov.close()
