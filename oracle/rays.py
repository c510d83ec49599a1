"""Straight-ray travel-time operator (Section 4.1, eq. lineartomography).

Travel time along a ray is the integral of slowness along it; with slowness
constant in each grid cell it is sum_c (length of the ray inside cell c) * s_c,
so row m of H holds the lengths of ray m inside each cell.

Reading of the geometry (the paper defers it to other work): the domain is the
unit square/cube split into a regular grid with cell (i, j[, k]) at flat index
i + nx*(j + ny*k).  A ray is cut at every crossing with a grid line/plane, each
piece is assigned to the cell containing its midpoint, and a piece that lies
exactly on an interior grid line/plane is shared equally between the cells on
either side (on the outer boundary it belongs to the single adjacent cell).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def _ray_pieces(a, b, shape):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    d = b - a
    length = float(np.linalg.norm(d))
    ts = [0.0, 1.0]
    for ax, n in enumerate(shape):
        if d[ax] == 0.0:
            continue
        for k in range(n + 1):
            t = (k / n - a[ax]) / d[ax]
            if 0.0 < t < 1.0:
                ts.append(t)
    ts = np.unique(np.array(ts))
    out = {}
    for t0, t1 in zip(ts[:-1], ts[1:]):
        seg = (t1 - t0) * length
        if seg <= 1e-15 * max(length, 1.0):
            continue
        mid = a + 0.5 * (t0 + t1) * d
        choices = []
        for ax, n in enumerate(shape):
            u = mid[ax] * n
            ku = round(u)
            if d[ax] == 0.0 and abs(u - ku) <= 1e-9:
                # lies on grid plane ku: cells ku-1 and ku (those that exist)
                cand = [c for c in (ku - 1, ku) if 0 <= c < n]
            else:
                cand = [min(max(int(np.floor(u)), 0), n - 1)]
            choices.append(cand)
        combos = list(itertools.product(*choices))
        share = seg / len(combos)
        for idx in combos:
            flat = 0
            stride = 1
            for ax, n in enumerate(shape):
                flat += idx[ax] * stride
                stride *= n
            out[flat] = out.get(flat, 0.0) + share
    return out


def ray_operator(shape, src: np.ndarray, rcv: np.ndarray) -> sp.csr_matrix:
    """Sparse H (n_m x N): H[m, c] = length of ray m inside cell c."""
    shape = tuple(int(s) for s in shape)
    N = int(np.prod(shape))
    rows, cols, vals = [], [], []
    for m, (a, b) in enumerate(zip(src, rcv)):
        pieces = _ray_pieces(a, b, shape)
        for c in sorted(pieces):
            rows.append(m)
            cols.append(c)
            vals.append(pieces[c])
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(src), N))
