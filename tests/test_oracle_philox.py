"""Pins for the oracle's Gaussian generator (Philox4x32-10 + Box-Muller)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle.philox import gaussian_block, gaussian_omega, philox4x32_10

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    out = philox4x32_10(tuple(np.array([c], dtype=np.uint64) for c in ctr), key)
    assert [int(o[0]) for o in out] == expect


def test_philox_vectorised_matches_scalar_calls():
    ctr = np.arange(100, dtype=np.uint64)
    vec = philox4x32_10((ctr, ctr * 3, ctr + 7, ctr ^ 5), (11, 13))
    for i in (0, 17, 99):
        one = philox4x32_10((np.uint64(i), np.uint64(3 * i), np.uint64(i + 7), np.uint64(i ^ 5)), (11, 13))
        assert [int(v[i]) for v in vec] == [int(x) for x in one]


def test_gaussian_is_standard_normal():
    om = gaussian_omega(seed=1, mode=0, m=20000, l=16)
    x = om.ravel()
    assert abs(x.mean()) < 5.0 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # every column and both halves of a Philox output are individually N(0,1)
    for j in range(16):
        assert stats.kstest(om[:, j], "norm").pvalue > 1e-4
    c = np.corrcoef(om.T)
    off = c[~np.eye(16, dtype=bool)]
    assert np.max(np.abs(off)) < 5.0 / np.sqrt(20000)


def test_gaussian_addressing():
    full = gaussian_omega(seed=7, mode=2, m=300, l=13)
    blk = gaussian_block(7, 2, np.arange(100, 140), np.arange(5, 11))
    np.testing.assert_array_equal(full[100:140, 5:11], blk)
    # chunked assembly gives the same matrix
    np.testing.assert_array_equal(gaussian_omega(7, 2, 300, 13, chunk=37), full)
    # mode, seed and 64-bit row index all change the draw
    assert not np.allclose(gaussian_omega(7, 1, 300, 13), full)
    assert not np.allclose(gaussian_omega(8, 2, 300, 13), full)
    hi = gaussian_block(7, 2, np.array([5 + (1 << 32)]), np.arange(13))
    assert not np.allclose(hi, full[5:6])


def test_gaussian_tail_and_extremes():
    # the uniforms sit strictly inside (0,1): the largest |value| is finite and
    # bounded by sqrt(-2 ln(2^-33)) ~ 6.77
    om = gaussian_omega(seed=3, mode=0, m=50000, l=8)
    assert np.all(np.isfinite(om))
    assert np.max(np.abs(om)) < np.sqrt(-2.0 * np.log(0.5 * 2.0 ** -32)) + 1e-12
