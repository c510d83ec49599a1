"""Gaussian sketch of the randomized generalized eigensolver (Appendix B).

The randomized algorithm of Appendix B draws a Gaussian matrix Omega.  The
library draws it on the GPU from a seed, so both sides implement the same
counter-based generator from its published definition and nothing random is
passed between them:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC 2011): a 128-bit counter and a 64-bit key, ten rounds
  of two 32 x 32 -> 64-bit multiplications (multipliers 0xD2511F53 and
  0xCD9E8D57) with the key bumped by the Weyl constants 0x9E3779B9 and
  0xBB67AE85 between rounds.
* Standard normals by the Box-Muller transform of two uniforms in (0, 1),
  each built from 53 bits of two output words.

Number e of a sketch (element (i, j) of an N x r column-major Omega is
e = i + N j) comes from the counter (q mod 2^32, q div 2^32, 0, 0),
q = e div 2, and the key (seed mod 2^32, seed div 2^32): with outputs
x0..x3, u1 = ((x0 >> 6) 2^27 + (x1 >> 5) + 1/2) 2^-53, u2 likewise from x2
and x3, rho = sqrt(-2 ln u1), and e even gives rho cos(2 pi u2), e odd
rho sin(2 pi u2).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32-10 of counters ctr (4 arrays of uint32 values) and key
    (2 ints); returns the 4 output words as uint64 arrays."""
    c = [np.asarray(x, dtype=np.uint64) for x in ctr]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for i in range(10):
        if i > 0:
            k0, k1 = (k0 + W0) & 0xFFFFFFFF, (k1 + W1) & 0xFFFFFFFF
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return c


def normals(seed: int, count: int) -> np.ndarray:
    """The first `count` standard normal numbers of the sketch stream `seed`."""
    npair = (count + 1) // 2
    q = np.arange(npair, dtype=np.uint64)
    zero = np.zeros(npair, dtype=np.uint64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    x = philox4x32_10((q & MASK, q >> np.uint64(32), zero, zero), (seed & 0xFFFFFFFF, seed >> 32))
    scale = 2.0 ** -53

    def unif(a, b):
        return (((a >> np.uint64(6)).astype(np.float64) * 2.0 ** 27
                 + (b >> np.uint64(5)).astype(np.float64) + 0.5) * scale)
    u1, u2 = unif(x[0], x[1]), unif(x[2], x[3])
    rho = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * npair)
    z[0::2] = rho * np.cos(2.0 * np.pi * u2)
    z[1::2] = rho * np.sin(2.0 * np.pi * u2)
    return z[:count]


def sketch(seed: int, n: int, r: int) -> np.ndarray:
    """Omega (n x r), element (i, j) = number i + n j of the stream."""
    return normals(seed, n * r).reshape(r, n).T
