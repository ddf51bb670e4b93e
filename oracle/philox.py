"""Counter-based Gaussian test matrices, FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper draws each Omega_k as a standard Gaussian matrix (section 2,
definition of a standard Gaussian matrix; Algorithms 2 and 3, the draw at the
top of each mode) without fixing a generator. Both sides of the parity check
therefore implement one published counter-based generator:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC 2011): a 4 x 32-bit counter, a 2 x 32-bit key, ten rounds of
  two 32x32->64 multiplies with the Weyl key schedule.
* Box-Muller (Box and Muller 1958): two uniforms (u_a, u_b) in (0,1) map to
  sqrt(-2 ln u_a) * (cos 2 pi u_b, sin 2 pi u_b).

Addressing of Omega_k[c, j] (mode k, row c, column j), all 0-based:
  counter = (c mod 2^32, c div 2^32, j div 4, k),  key = (seed mod 2^32, seed div 2^32)
  words (w0, w1, w2, w3) = Philox4x32-10(counter, key)
  pair  = (w0, w1) if (j div 2) is even else (w2, w3)
  u_a = (pair[0] + 1/2) * 2^-32,  u_b = (pair[1] + 1/2) * 2^-32
  Omega_k[c, j] = sqrt(-2 ln u_a) * (cos 2 pi u_b if j is even else sin 2 pi u_b)
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Ten Philox rounds on arrays of counters.

    ctr: tuple of four uint32-valued arrays (broadcastable); key: pair of ints.
    Returns four uint32 arrays.
    """
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in ctr)
    k0 = int(key[0]) & 0xFFFFFFFF
    k1 = int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0)
        if rnd < 9:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def gaussian_block(seed: int, mode: int, rows, cols) -> np.ndarray:
    """Omega_mode[rows][:, cols] in FP64 for integer index arrays rows (m,) and cols (l,)."""
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1, 1)
    cols = np.asarray(cols, dtype=np.uint64).reshape(1, -1)
    ctr = (rows & MASK32, rows >> np.uint64(32), cols >> np.uint64(2),
           np.full(cols.shape, mode, dtype=np.uint64))
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    first = ((cols >> np.uint64(1)) & np.uint64(1)) == 0
    wa = np.where(first, w[0], w[2]).astype(np.float64)
    wb = np.where(first, w[1], w[3]).astype(np.float64)
    ua = (wa + 0.5) * 2.0 ** -32
    ub = (wb + 0.5) * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(ua))
    even = (cols & np.uint64(1)) == 0
    return np.where(even, rad * np.cos(2.0 * np.pi * ub), rad * np.sin(2.0 * np.pi * ub))


def gaussian_omega(seed: int, mode: int, m: int, l: int, chunk: int = 1 << 18) -> np.ndarray:
    """The full m x l test matrix Omega_mode, FP64, built in row chunks."""
    out = np.empty((m, l))
    cols = np.arange(l)
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        out[r0:r1] = gaussian_block(seed, mode, np.arange(r0, r1), cols)
    return out
