"""Counter-based test matrices (Gaussian, uniform, Khatri-Rao), FP64 reference.

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

Other test matrices (section 5, comparison of random matrices: uniform entries
on [-1, 1], and Khatri-Rao products of Gaussian or uniform matrices, the
Khatri-Rao product of the preliminaries):
  stream tag t (the fourth counter word): t = k for the dense matrices of mode
  k; t = 4096 + 16 k + i for the Khatri-Rao factor of mode i (i != k) of mode k;
  uniform streams add 2^30 to t.
  uniform entry [c, j] of stream t = (w_(j mod 4) + 1/2) * 2^-31 - 1 with
  (w0..w3) = Philox4x32-10((c mod 2^32, c div 2^32, j div 4, t + 2^30), key).
  Khatri-Rao: Omega_k[c, j] = prod over the other modes i (increasing) of
  F_i[c_i, j], where (c_i) is c in row-major order over those modes (their
  sizes in increasing mode order), the column order of the mode-k unfolding.
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


UNIFORM_TAG = 1 << 30
KR_TAG = 4096

KINDS = ("gaussian", "uniform", "kr_gaussian", "kr_uniform")


def uniform_block(seed: int, tag: int, rows, cols) -> np.ndarray:
    """Uniform[-1, 1] entries [rows][:, cols] of stream `tag` (the uniform bit is added here)."""
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1, 1)
    cols = np.asarray(cols, dtype=np.uint64).reshape(1, -1)
    ctr = (rows & MASK32, rows >> np.uint64(32), cols >> np.uint64(2),
           np.full(cols.shape, (tag + UNIFORM_TAG) & 0xFFFFFFFF, dtype=np.uint64))
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    q = (cols & np.uint64(3))
    word = np.where(q == 0, w[0], np.where(q == 1, w[1], np.where(q == 2, w[2], w[3]))).astype(np.float64)
    return (word + 0.5) * 2.0 ** -31 - 1.0


def _factor(kind: str, seed: int, tag: int, m: int, l: int) -> np.ndarray:
    rows, cols = np.arange(m), np.arange(l)
    return gaussian_block(seed, tag, rows, cols) if kind == "gaussian" else uniform_block(seed, tag, rows, cols)


def omega_matrix(kind: str, seed: int, mode: int, other_dims, l: int) -> np.ndarray:
    """Omega_mode (m x l, m = prod(other_dims)) of one of the four kinds;
    other_dims are the sizes of the modes other than `mode`, in increasing
    mode order (the column order of the unfolding)."""
    other_dims = [int(x) for x in other_dims]
    m = int(np.prod(other_dims)) if other_dims else 1
    if kind == "gaussian":
        return gaussian_omega(seed, mode, m, l)
    if kind == "uniform":
        return _factor("uniform", seed, mode, m, l)
    if kind not in ("kr_gaussian", "kr_uniform"):
        raise ValueError("unknown test-matrix kind %r" % kind)
    base = "gaussian" if kind == "kr_gaussian" else "uniform"
    others = [i for i in range(len(other_dims) + 1) if i != mode]
    out = np.ones((1, l))
    for pos, i in enumerate(others):
        f = _factor(base, seed, KR_TAG + 16 * mode + i, other_dims[pos], l)
        # row-major over the modes taken so far: the new mode's index varies fastest
        out = (out[:, None, :] * f[None, :, :]).reshape(-1, l)
    return out
