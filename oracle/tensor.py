"""Dense tensor primitives in FP64: unfolding, folding, mode-k product.

TEST INFRASTRUCTURE ONLY (see the package header).

Conventions (section 2 of the paper, the mode-k product and the mode-k
unfolding A_(k) in R^{n_k x prod_{j != k} n_j}):

* Tensors are NumPy arrays in C order (last index fastest), modes 0-based.
* The paper leaves the column order of A_(k) open (its Kronecker identity for
  the Tucker form fits neither common convention). Reading taken here: the
  columns run over the remaining indices in row-major order, so that for the
  row-major view X = [P, n_k, S] (P = prod_{j<k} n_j, S = prod_{j>k} n_j)
  one has A_(k)[i, p*S + s] = X[p, i, s].
* mode_product(A, B, k) follows the paper's definition
  c_{i1..i(k-1) j i(k+1)..id} = sum_{ik} a_{i1..ik..id} b_{j ik}.
"""
from __future__ import annotations

import numpy as np


def unfold(x: np.ndarray, k: int) -> np.ndarray:
    """A_(k): n_k x (product of the other dims), columns in row-major order."""
    return np.moveaxis(x, k, 0).reshape(x.shape[k], -1)


def fold(mat: np.ndarray, k: int, dims) -> np.ndarray:
    """Inverse of unfold for a tensor of shape `dims` (dims[k] == mat.shape[0])."""
    dims = tuple(dims)
    rest = dims[:k] + dims[k + 1:]
    return np.moveaxis(mat.reshape((dims[k],) + rest), 0, k)


def mode_product(x: np.ndarray, b: np.ndarray, k: int) -> np.ndarray:
    """x x_k b for b of shape (J, n_k): replaces axis k by J."""
    out = np.tensordot(b, x, axes=([1], [k]))
    return np.ascontiguousarray(np.moveaxis(out, 0, k))


def frob2(x: np.ndarray) -> float:
    v = np.asarray(x, dtype=np.float64).ravel()
    return float(np.dot(v, v))


def reconstruct(g: np.ndarray, factors) -> np.ndarray:
    """G x_1 U_1 x_2 U_2 ... x_d U_d (the Tucker format)."""
    t = g
    for k, u in enumerate(factors):
        t = mode_product(t, u, k)
    return t
