"""Pins for the oracle's tensor layout: unfolding and mode-k product by index loops."""
import itertools

import numpy as np
import pytest

from oracle.tensor import fold, frob2, mode_product, reconstruct, unfold
from workloads.generators import rng


def _loop_unfold(x, k):
    """A_(k)[i, col] with col the row-major index of the remaining indices (written out)."""
    dims = x.shape
    rest = [n for j, n in enumerate(dims) if j != k]
    out = np.zeros((dims[k], int(np.prod(rest))))
    for idx in itertools.product(*[range(n) for n in dims]):
        col = 0
        for j, n in enumerate(dims):
            if j == k:
                continue
            col = col * n + idx[j]
        out[idx[k], col] = x[idx]
    return out


def _loop_mode_product(x, b, k):
    """c_{..j..} = sum_{i_k} a_{..i_k..} b_{j i_k}, the paper's definition, by loops."""
    dims = list(x.shape)
    out_dims = dims.copy()
    out_dims[k] = b.shape[0]
    c = np.zeros(out_dims)
    for idx in itertools.product(*[range(n) for n in out_dims]):
        s = 0.0
        for ik in range(dims[k]):
            src = list(idx)
            src[k] = ik
            s += x[tuple(src)] * b[idx[k], ik]
        c[idx] = s
    return c


@pytest.mark.parametrize("dims", [(3, 4, 5), (2, 3, 4, 5)])
def test_unfold_matches_index_definition(dims):
    x = rng(0).standard_normal(dims)
    for k in range(len(dims)):
        np.testing.assert_array_equal(unfold(x, k), _loop_unfold(x, k))
        np.testing.assert_array_equal(fold(unfold(x, k), k, dims), x)


@pytest.mark.parametrize("dims", [(3, 4, 5), (2, 3, 4, 5)])
def test_inplace_view_column_order(dims):
    """A_(k)[i, p*S + s] = X[p, i, s] for the row-major view [P, n_k, S]."""
    x = rng(1).standard_normal(dims)
    for k in range(len(dims)):
        p_ = int(np.prod(dims[:k]))
        s_ = int(np.prod(dims[k + 1:]))
        v = x.reshape(p_, dims[k], s_)
        xk = unfold(x, k)
        for p in range(p_):
            for s in range(s_):
                np.testing.assert_array_equal(xk[:, p * s_ + s], v[p, :, s])


@pytest.mark.parametrize("dims", [(3, 4, 5), (2, 3, 4, 5)])
def test_mode_product_matches_definition(dims):
    g = rng(2)
    x = g.standard_normal(dims)
    for k in range(len(dims)):
        b = g.standard_normal((3, dims[k]))
        np.testing.assert_allclose(mode_product(x, b, k), _loop_mode_product(x, b, k), rtol=1e-13, atol=1e-13)
        # the unfolding form of the same product: (X x_k B)_(k) = B X_(k)
        np.testing.assert_allclose(unfold(mode_product(x, b, k), k), b @ unfold(x, k), rtol=1e-13, atol=1e-13)


def test_reconstruct_and_norm():
    g = rng(3)
    core = g.standard_normal((2, 3, 2))
    us = [np.linalg.qr(g.standard_normal((n, r)))[0] for n, r in zip((4, 5, 6), core.shape)]
    t = reconstruct(core, us)
    # orthonormal factors preserve the Frobenius norm
    assert abs(frob2(t) - frob2(core)) < 1e-12 * frob2(core)
    # and the entry formula of the Tucker format
    i, j, k = 3, 1, 5
    ref = sum(core[a, b, c] * us[0][i, a] * us[1][j, b] * us[2][k, c]
              for a in range(2) for b in range(3) for c in range(2))
    assert abs(t[i, j, k] - ref) < 1e-13
