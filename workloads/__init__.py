"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds geometry and random numbers only: cell-centred grid points,
crosswell source/receiver positions, Gaussian draws and a synthetic "truth"
field with its line-integral travel times.  It contains none of the filter's
arithmetic (no covariance kernel, no discretised ray operator, no Kalman
algebra), so both sides can consume it without sharing method code.

Workloads stand in for the paper's crosswell CO2 monitoring setup (Section 4.1:
sources on one well, receivers on the other, straight rays, travel-time data
every step).  The Frio-II reservoir simulation it used is not available; the
truth here is a growing smooth synthetic plume plus a random-walk drift.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROOT_SEED = 14052276

# Random streams (one child generator per (config, stream)).
STREAM_TRUTH = 0
STREAM_NOISE = 1
STREAM_SKETCH = 2
STREAM_DRAWS = 3
STREAM_VECTORS = 4


def rng(cfg_id: int, stream: int) -> np.random.Generator:
    """Independent generator for (config id, stream id), from one root seed."""
    ss = np.random.SeedSequence([ROOT_SEED, int(cfg_id), int(stream)])
    return np.random.default_rng(ss)


def grid_points(shape) -> np.ndarray:
    """Cell centres of a regular grid on the unit square/cube.

    Cell (i, j[, k]) has centre ((i+1/2)/nx, (j+1/2)/ny[, (k+1/2)/nz]) and flat
    index i + nx*(j + ny*k) (x fastest).  Returns an (N, d) float64 array.
    """
    shape = tuple(int(s) for s in shape)
    axes = [(np.arange(n, dtype=np.float64) + 0.5) / n for n in shape]
    mesh = np.meshgrid(*axes, indexing="ij")
    # x fastest: flatten in Fortran order of (i, j, k)
    return np.stack([m.ravel(order="F") for m in mesh], axis=1)


def crosswell_2d(n_src: int, n_rcv: int):
    """Sources on the left edge x=0, receivers on the right edge x=1.

    Source i at (0, (i+1/2)/n_src), receiver j at (1, (j+1/2)/n_rcv); ray m
    pairs source m // n_rcv with receiver m % n_rcv.  Returns (src, rcv) as
    (n_m, 2) arrays of ray start and end points.
    """
    ys = (np.arange(n_src) + 0.5) / n_src
    yr = (np.arange(n_rcv) + 0.5) / n_rcv
    src = np.array([[0.0, a] for a in ys for _ in yr])
    rcv = np.array([[1.0, b] for _ in ys for b in yr])
    return src, rcv


def crosswell_3d(src_lattice, rcv_lattice):
    """Sources on the face x=0, receivers on the face x=1 (3-D crosswell).

    A lattice (na, nb) places points at ((a+1/2)/na, (b+1/2)/nb) in (y, z).
    Every source is paired with every receiver.
    """
    def face(lat, x):
        na, nb = lat
        return np.array([[x, (a + 0.5) / na, (b + 0.5) / nb]
                         for a in range(na) for b in range(nb)])
    s, r = face(src_lattice, 0.0), face(rcv_lattice, 1.0)
    src = np.repeat(s, len(r), axis=0)
    rcv = np.tile(r, (len(s), 1))
    return src, rcv


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic filtering workload (grid, prior, rays, noise, steps)."""
    name: str
    cfg_id: int
    shape: tuple
    nu: float            # Matern smoothness (0.5, 1.5, 2.5)
    length: float        # Matern length scale
    variance: float      # Matern variance theta
    n_src: object        # int (2-D) or lattice tuple (3-D)
    n_rcv: object
    noise_var: float     # diagonal measurement-noise variance
    steps: int
    drift_sigma: float   # std of the per-step truth drift
    leaf_size: int = 64
    cheb_order: int = 6

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    @property
    def dim(self) -> int:
        return len(self.shape)

    def points(self) -> np.ndarray:
        return grid_points(self.shape)

    def rays(self):
        if self.dim == 2:
            return crosswell_2d(self.n_src, self.n_rcv)
        return crosswell_3d(self.n_src, self.n_rcv)

    @property
    def n_m(self) -> int:
        s, _ = self.rays()
        return len(s)


# The five workload shapes: a small exponential-kernel case, a 128^2 FP64 case,
# the 256^2 (N = 65536) headline case, and the 3-D 64^3 case.
SMALL = Workload("small-32x32", 1, (32, 32), 0.5, 0.3, 1.0, 8, 8, 1e-4, 5, 1.0)
MEDIUM = Workload("crosswell-128x128", 2, (128, 128), 1.5, 0.2, 1e-4, 16, 15, 1e-4, 20, 0.01)
LARGE = Workload("crosswell-256x256", 3, (256, 256), 1.5, 0.1, 1e-4, 24, 20, 1e-4, 50, 0.01)
CUBE = Workload("crosswell-64^3", 5, (64, 64, 64), 0.5, 0.15, 1e-4, (4, 8), (8, 4), 1e-4, 10, 0.01)

WORKLOADS = {w.name: w for w in (SMALL, MEDIUM, LARGE, CUBE)}


def crosswell_vertical(n_src: int, n_rcv: int):
    """Sources on the bottom edge y=0, receivers on the top edge y=1 (the
    crosswell geometry turned by a right angle): source i at ((i+1/2)/n_src, 0),
    receiver j at ((j+1/2)/n_rcv, 1), ray m pairs source m // n_rcv with
    receiver m % n_rcv."""
    xs = (np.arange(n_src) + 0.5) / n_src
    xr = (np.arange(n_rcv) + 0.5) / n_rcv
    src = np.array([[a, 0.0] for a in xs for _ in xr])
    rcv = np.array([[b, 1.0] for _ in xs for b in xr])
    return src, rcv


def batch(count: int = 64, steps: int = 10):
    """Independent filters of uneven size for the many-filter form: square
    grids with side uniform on {64, 72, ..., 256} (N = 4096 ... 65536),
    Matern nu in {1/2, 3/2} (fair coin), length uniform on [0.1, 0.3],
    variance 1e-4, crosswell rays with n_src uniform on {8..24} and n_rcv on
    {8..20} (64 ... 480 rays), R = 1e-4 I, `steps` steps each."""
    g = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 4, 0]))
    out = []
    for i in range(count):
        side = int(g.choice(np.arange(64, 257, 8)))
        nu = float(g.choice([0.5, 1.5]))
        ell = float(g.uniform(0.1, 0.3))
        ns, nr = int(g.integers(8, 25)), int(g.integers(8, 21))
        out.append(Workload(f"batch-{i}-{side}x{side}", 400 + i, (side, side), nu, ell, 1e-4,
                            ns, nr, 1e-4, steps, 0.01))
    return out


def tiny(shape=(8, 8), nu=0.5, length=0.3, variance=1.0, n_src=3, n_rcv=4,
         noise_var=1e-2, steps=4, drift_sigma=1.0, cfg_id=100, leaf_size=16,
         cheb_order=6) -> Workload:
    """A small custom workload for unit tests."""
    return Workload(f"tiny-{'x'.join(map(str, shape))}", cfg_id, tuple(shape), nu, length,
                    variance, n_src, n_rcv, noise_var, steps, drift_sigma, leaf_size,
                    cheb_order)


class _SmoothField:
    """Random smooth field: a sum of random cosines (random Fourier features).

    f(x) = sqrt(2/M) * sum_m a_m cos(w_m . x + phi_m), a_m ~ N(0,1),
    w_m ~ N(0, I/ell^2), phi_m ~ U[0, 2pi).  Its pointwise variance is 1.
    """

    def __init__(self, g: np.random.Generator, dim: int, ell: float, m: int = 64):
        self.w = g.standard_normal((m, dim)) / ell
        self.phi = g.uniform(0.0, 2 * math.pi, m)
        self.a = g.standard_normal(m) * math.sqrt(2.0 / m)

    def __call__(self, x: np.ndarray) -> np.ndarray:
        return np.cos(x @ self.w.T + self.phi) @ self.a


class Truth:
    """Synthetic time-lapse truth: growing plume plus random-walk drift.

    s_k(x) = A * min(k/K, 1) * exp(-|x - c|^2 / (2 w_k^2)) + sigma * sum_{j<=k} f_j(x)
    with f_j independent smooth random fields.  Travel time of a straight ray
    from a to b is the line integral of s_k, evaluated by Gauss-Legendre
    quadrature; measurement noise is added separately.
    """

    def __init__(self, wl: Workload, n_quad: int = 96):
        self.wl = wl
        g = rng(wl.cfg_id, STREAM_TRUTH)
        self.centre = np.full(wl.dim, 0.5) + 0.1 * g.uniform(-1, 1, wl.dim)
        self.amp = 3.0 * wl.drift_sigma
        self.fields = [_SmoothField(g, wl.dim, wl.length) for _ in range(wl.steps)]
        self.n_quad = n_quad

    def value(self, k: int, x: np.ndarray) -> np.ndarray:
        K = max(self.wl.steps, 1)
        w = 0.05 + 0.15 * min(k / K, 1.0)
        r2 = np.sum((x - self.centre) ** 2, axis=-1)
        s = self.amp * min(k / K, 1.0) * np.exp(-r2 / (2 * w * w))
        for j in range(min(k, len(self.fields))):
            s = s + self.wl.drift_sigma * self.fields[j](x)
        return s

    def cells(self, k: int) -> np.ndarray:
        return self.value(k, self.wl.points())

    def travel_times(self, k: int, src=None, rcv=None) -> np.ndarray:
        """Line integrals of s_k along the workload's rays, or along the
        straight rays src[m] -> rcv[m] when given."""
        if src is None:
            src, rcv = self.wl.rays()
        t, wq = np.polynomial.legendre.leggauss(self.n_quad)
        t = 0.5 * (t + 1.0)
        wq = 0.5 * wq
        seg = rcv - src
        L = np.linalg.norm(seg, axis=1)
        pts = src[:, None, :] + t[None, :, None] * seg[:, None, :]
        vals = self.value(k, pts.reshape(-1, self.wl.dim)).reshape(len(src), -1)
        return L * (vals @ wq)


def observations(wl: Workload, positive: bool = False) -> np.ndarray:
    """Noisy travel times y_k for k = 1..steps, shape (steps, n_m).

    Same values as Truth.travel_times(k) plus noise; the drift fields are
    evaluated once at the quadrature points and accumulated step by step.
    With positive=True the integrated field is exp(Truth.value), a strictly
    positive field around 1 (the truth for the non-negative observation
    model of the extended filter).
    """
    tr = Truth(wl)
    g = rng(wl.cfg_id, STREAM_NOISE)
    src, rcv = wl.rays()
    t, wq = np.polynomial.legendre.leggauss(tr.n_quad)
    t = 0.5 * (t + 1.0)
    wq = 0.5 * wq
    seg = rcv - src
    L = np.linalg.norm(seg, axis=1)
    pts = (src[:, None, :] + t[None, :, None] * seg[:, None, :]).reshape(-1, wl.dim)
    K = max(wl.steps, 1)
    r2 = np.sum((pts - tr.centre) ** 2, axis=-1)
    drift = np.zeros(len(pts))
    ys = []
    for k in range(1, wl.steps + 1):
        if k - 1 < len(tr.fields):
            drift = drift + wl.drift_sigma * tr.fields[k - 1](pts)
        w = 0.05 + 0.15 * min(k / K, 1.0)
        vals = tr.amp * min(k / K, 1.0) * np.exp(-r2 / (2 * w * w)) + drift
        if positive:
            vals = np.exp(vals)
        y = L * (vals.reshape(len(src), -1) @ wq)
        ys.append(y + math.sqrt(wl.noise_var) * g.standard_normal(len(y)))
    return np.array(ys)


def normals(wl: Workload, stream: int, shape) -> np.ndarray:
    """Standard normal draws from the (config, stream) generator."""
    return rng(wl.cfg_id, stream).standard_normal(shape)
