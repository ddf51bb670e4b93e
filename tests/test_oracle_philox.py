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


# --------------------------------------------------------------- other test matrices (section 5)

from oracle.philox import KR_TAG, omega_matrix, uniform_block  # noqa: E402


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_uniform_entries_are_the_known_answer_words(ctr, key, expect):
    """A uniform entry is (w + 1/2) 2^-31 - 1 of word j mod 4 of the Philox block
    addressed by (row, j div 4, tag + 2^30): on the known-answer counters the
    four entries are the four published output words, mapped."""
    c = ctr[0] + (ctr[1] << 32)
    tag = (ctr[3] - (1 << 30)) % (1 << 32)
    seed = key[0] + (key[1] << 32)
    got = uniform_block(seed, tag, [c], [4 * ctr[2] + q for q in range(4)])[0]
    want = [(w + 0.5) * 2.0 ** -31 - 1.0 for w in expect]
    assert list(got) == want


def test_uniform_is_uniform_on_the_open_interval():
    from scipy import stats
    u = omega_matrix("uniform", 17, 2, [400, 300], 16).ravel()
    assert -1.0 < u.min() and u.max() < 1.0
    assert abs(u.mean()) < 4.0 / np.sqrt(3.0 * u.size)
    assert abs(u.var() - 1.0 / 3.0) < 0.01
    assert stats.kstest(u, "uniform", args=(-1.0, 2.0)).pvalue > 1e-3


@pytest.mark.parametrize("kind", ["kr_gaussian", "kr_uniform"])
def test_khatri_rao_columns_are_rank_one(kind):
    """Each column of a Khatri-Rao test matrix, reshaped to the other modes'
    sizes (row-major), is an outer product: every unfolding has rank one."""
    dims = [5, 7, 6]  # mode 1 of a 4-way tensor: the others are modes 0, 2, 3
    om = omega_matrix(kind, 9, 1, dims, 10)
    assert om.shape == (5 * 7 * 6, 10)
    for j in range(10):
        t = om[:, j].reshape(dims)
        for ax in range(3):
            s = np.linalg.svd(np.moveaxis(t, ax, 0).reshape(dims[ax], -1), compute_uv=False)
            assert s[1] <= 1e-13 * s[0]


def test_khatri_rao_factor_streams_and_order():
    """Factor F_i of mode k is stream 4096 + 16 k + i; the last other mode's
    index varies fastest along the rows."""
    from oracle.philox import gaussian_block
    om = omega_matrix("kr_gaussian", 4, 0, [3, 4], 5)
    f1 = gaussian_block(4, KR_TAG + 0 + 1, np.arange(3), np.arange(5))
    f2 = gaussian_block(4, KR_TAG + 0 + 2, np.arange(4), np.arange(5))
    for a in range(3):
        for b in range(4):
            assert np.array_equal(om[a * 4 + b], f1[a] * f2[b])


@pytest.mark.parametrize("kind", ["gaussian", "uniform", "kr_gaussian", "kr_uniform"])
def test_every_kind_recovers_exact_tucker_rank(kind):
    """Any test matrix of full column rank on the range recovers a tensor of
    exact Tucker rank (Algorithm 3, q = 0 and 1)."""
    from oracle.rhosvd import randomized_hosvd, rel_error
    from workloads.generators import random_tucker
    a, _, _ = random_tucker((14, 12, 10), (3, 4, 2), 0.0, seed=41)
    dims = a.shape
    for q in (0, 1):
        def om(k, m, l):
            # ST-HOSVD: modes before k already hold their ranks
            cur = [(3, 4, 2)[i] if i < k else dims[i] for i in range(3)]
            return omega_matrix(kind, 5, k, [cur[i] for i in range(3) if i != k], l)
        res = randomized_hosvd(a, (3, 4, 2), 3, q, variant="st", seed=5, omega=om)
        assert rel_error(a, res) < 1e-12
