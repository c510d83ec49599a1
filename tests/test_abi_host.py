"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, and its host logic (cluster tree, partition, ray tracer) is correct."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import rays as orays

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "fkf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fkf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import ctypes
    import paper_1405_2276_amd as fkf
    lib = ctypes.CDLL(fkf.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert "gfx950" in fkf.version()


@pytest.mark.parametrize("shape,leaf", [((32, 32), 64), ((128, 128), 64), ((37, 23), 64),
                                        ((16, 16, 16), 64), ((20, 30), 16)])
def test_partition_covers_every_entry_once(shape, leaf):
    import paper_1405_2276_amd as fkf
    pts = W.grid_points(shape)
    info = fkf.plan(pts, nu=1.5, length=0.2, leaf_size=leaf, block_tol=0, cheb_order=6)
    n = pts.shape[0]
    assert info["covered_entries"] == n * n
    assert info["n_leaves"] == -(-n // leaf)


def test_partition_irregular_points_and_orders():
    import paper_1405_2276_amd as fkf
    g = np.random.default_rng(1)
    pts = g.uniform(0, 1, (3001, 2))
    info = fkf.plan(pts, nu=0.5, length=0.3, leaf_size=64, block_tol=1e-7)
    assert info["covered_entries"] == 3001 * 3001
    assert all(6 <= p <= 16 for p in info["cheb_p"])


def test_headline_grid_partition_is_the_3x3_leaf_neighbourhood():
    import paper_1405_2276_amd as fkf
    wl = W.LARGE
    info = fkf.plan(wl.points(), nu=wl.nu, length=wl.length, variance=wl.variance)
    assert info["n_leaves"] == 1024
    # interior leaves have 9 near neighbours, edges 6, corners 4
    assert info["n_near_pairs"] == 30 * 30 * 9 + 4 * 30 * 6 + 4 * 4
    assert info["n_near_blocks"] == (info["n_near_pairs"] + 1024) // 2
    assert info["near_bytes"] == info["n_near_blocks"] * 64 * 64 * 8
    mixed = fkf.plan(wl.points(), nu=wl.nu, length=wl.length, variance=wl.variance,
                     precision="mixed")
    assert mixed["near_bytes"] * 2 == info["near_bytes"]
    assert mixed["cheb_p"] == info["cheb_p"]
    # coupling matrices: at least the smallest order's p^4 entries for every
    # unordered admissible pair; stored once per distinct geometry of an
    # ordered pair, which on this regular grid is a small fraction of them
    assert info["far_bytes"] == 2 * mixed["far_bytes"] > 0
    assert info["far_pair_entries"] >= (info["n_far_pairs"] // 2) * min(info["cheb_p"]) ** 4
    assert info["far_bytes"] < 8 * info["far_pair_entries"] // 10
    ev = fkf.plan(wl.points(), nu=wl.nu, length=wl.length, variance=wl.variance, far_eval=True)
    assert ev["far_bytes"] == 0 and ev["near_bytes"] == info["near_bytes"]


def test_plan_stores_every_coupling_of_irregular_points():
    # boxes of random points never repeat a geometry: one stored matrix per
    # ordered admissible pair (both orientations of every unordered one)
    import paper_1405_2276_amd as fkf
    pts = np.random.default_rng(3).uniform(0, 1, (6000, 2))
    info = fkf.plan(pts, nu=1.5, length=0.15, variance=1.0)
    assert info["n_far_pairs"] > 0
    assert info["far_bytes"] == 2 * 8 * info["far_pair_entries"]


@pytest.mark.parametrize("shape,nsrc,nrcv", [((32, 32), 8, 8), ((128, 128), 16, 15),
                                             ((256, 256), 24, 20), ((37, 23), 5, 7)])
def test_ray_tracer_matches_oracle_entrywise(shape, nsrc, nrcv):
    import paper_1405_2276_amd as fkf
    src, rcv = W.crosswell_2d(nsrc, nrcv)
    rp, col, val = fkf.rays_host(shape, src, rcv)
    n = int(np.prod(shape))
    H = sp.csr_matrix((val, col, rp), shape=(len(src), n)).toarray()
    Ho = orays.ray_operator(shape, src, rcv).toarray()
    np.testing.assert_allclose(H, Ho, rtol=0, atol=1e-14)


def test_ray_tracer_matches_oracle_3d_and_boundary_cases():
    import paper_1405_2276_amd as fkf
    src, rcv = W.crosswell_3d((2, 3), (3, 2))
    shape = (6, 5, 4)
    rp, col, val = fkf.rays_host(shape, src, rcv)
    H = sp.csr_matrix((val, col, rp), shape=(len(src), 120)).toarray()
    np.testing.assert_allclose(H, orays.ray_operator(shape, src, rcv).toarray(), atol=1e-14)
    # rays on grid lines / through corners
    src = np.array([[0, 0.5], [0, 0.25], [0, 0.0], [0, 0.0], [0.5, 0.0]])
    rcv = np.array([[1, 0.5], [1, 0.75], [1, 0.0], [1, 1.0], [0.5, 1.0]])
    rp, col, val = fkf.rays_host((4, 4), src, rcv)
    H = sp.csr_matrix((val, col, rp), shape=(5, 16)).toarray()
    np.testing.assert_allclose(H, orays.ray_operator((4, 4), src, rcv).toarray(), atol=1e-14)


def test_host_entry_points_reject_bad_arguments():
    import paper_1405_2276_amd as fkf
    with pytest.raises(fkf.FkfError) as e:
        fkf.plan(np.zeros((10, 2)), leaf_size=100)
    assert e.value.name == "FKF_E_ARG"
    with pytest.raises(ValueError):
        fkf.plan(np.zeros((10, 2)), precision="bf16")
    with pytest.raises(fkf.FkfError):
        fkf.rays_host((4, 4), np.array([[0.0, 2.0]]), np.array([[1.0, 0.5]]))
