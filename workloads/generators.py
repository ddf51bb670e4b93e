"""Seeded synthetic inputs for the randomized (S)T-HOSVD path.

This module builds test tensors and request streams only. It holds none of
the method's arithmetic (no sketch, no power step, no orthonormalisation, no
core contraction of A by its factors), so both the FP64 oracle and the GPU
path may take their inputs from here.

Every generator takes an explicit seed and uses NumPy's PCG64 stream, so a
tensor is reproducible bit for bit on any host. The large-tensor builders in
``build_on_device`` use torch on the GPU only to assemble inputs quickly; they
are not part of the method either.

Constructions (paper section 5.1):

* ``haar``: an n x r matrix with orthonormal columns, the Q factor of a
  Gaussian matrix with the signs of diag(R) folded in (Mezzadri 2007), which
  makes it Haar-distributed.
* ``tucker_tensor``: core x_1 U_1 ... x_d U_d (the Tucker format of the
  paper's preliminaries), expanded densely.
* ``add_noise``: A = T + eta * ||T||_F * E0 / ||E0||_F with E0 i.i.d. N(0,1).
* ``hilbert_tensor``: a_{i1..id} = 1 / (i1 + ... + id - d + 1), 1-based.
* ``superdiagonal``: the tendiag(v) tensor of the paper's tensor C.
* ``tensor_c``: tendiag(v) x_1 A_1 x_2 A_2 x_3 A_3 with A_n orthogonal n x n,
  with the three spectra (slow, fast, S-shaped) of section 5.1.
* ``sparse_cp_factors``: the sparse CP tensor of the processing-order study
  (section 3.2): sum_i w_i x_i o y_i o z_i with w_i = 1000/i for the first 50
  terms and 1/i for the others, every vector with a 0.05 fraction of nonzero
  entries, uniform on (0, 1), at positions drawn without replacement.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def haar(n: int, r: int, gen: np.random.Generator) -> np.ndarray:
    """n x r with orthonormal columns, Haar-distributed (Mezzadri 2007)."""
    g = gen.standard_normal((n, r))
    q, rr = np.linalg.qr(g)
    s = np.sign(np.diag(rr))
    s[s == 0] = 1.0
    return q * s[None, :]


def _expand_mode(t: np.ndarray, mat: np.ndarray, mode: int) -> np.ndarray:
    """Replace axis `mode` (size mat.shape[1]) by mat.shape[0]: sum_j mat[i, j] t[.., j, ..]."""
    out = np.tensordot(mat, t, axes=([1], [mode]))
    return np.moveaxis(out, 0, mode)


def tucker_tensor(core: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    t = core
    for k, u in enumerate(factors):
        t = _expand_mode(t, u, k)
    return np.ascontiguousarray(t)


def add_noise(t: np.ndarray, eta: float, gen: np.random.Generator) -> np.ndarray:
    if eta == 0.0:
        return t.copy()
    e0 = gen.standard_normal(t.shape)
    return t + (eta * np.linalg.norm(t.ravel()) / np.linalg.norm(e0.ravel())) * e0


def random_tucker(dims: Sequence[int], core_dims: Sequence[int], eta: float, seed: int,
                  core: np.ndarray | None = None) -> Tuple[np.ndarray, np.ndarray, List[np.ndarray]]:
    """Gaussian (or given) core times Haar factors plus scaled Gaussian noise. FP64."""
    gen = rng(seed)
    if core is None:
        core = gen.standard_normal(tuple(core_dims))
    factors = [haar(n, r, gen) for n, r in zip(dims, core_dims)]
    t = tucker_tensor(core, factors)
    return add_noise(t, eta, gen), core, factors


def hilbert_tensor(dims: Sequence[int]) -> np.ndarray:
    """a_{i1..id} = 1/(i1+...+id-d+1) with 1-based indices (1/(i+j+k-2) for d=3)."""
    d = len(dims)
    idx = np.meshgrid(*[np.arange(1, n + 1, dtype=np.float64) for n in dims], indexing="ij")
    s = sum(idx)
    return 1.0 / (s - d + 1.0)


def superdiagonal(v: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    t = np.zeros(tuple(dims))
    for i, x in enumerate(v):
        t[(i,) * len(dims)] = x
    return t


def spectrum_c(kind: str, n: int) -> np.ndarray:
    """The three diagonals of the paper's tensor C (section 5.1), 1-based i."""
    i = np.arange(1, n + 1, dtype=np.float64)
    if kind == "slow":
        return 1.0 / i ** 2
    if kind == "fast":
        return np.exp(-i / 7.0)
    if kind == "sshape":
        return 0.001 + 1.0 / (1.0 + np.exp(i - 29.0))
    raise ValueError(kind)


def tensor_c(kind: str, n: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """tendiag(v, [n,n,n]) x_1 A_1 x_2 A_2 x_3 A_3, A_k = orth of an n x n Gaussian.

    Every unfolding then has singular values exactly v (section 5.1).
    Built without the dense n^3 superdiagonal: T = sum_i v_i a1_i o a2_i o a3_i.
    """
    gen = rng(seed)
    v = spectrum_c(kind, n)
    a = [haar(n, n, gen) for _ in range(3)]
    t = np.einsum("i,ai,bi,ci->abc", v, a[0], a[1], a[2], optimize=True)
    return np.ascontiguousarray(t), v


def sparse_cp_factors(dims: Sequence[int], seed: int, nterms: int = 600, heavy: int = 50,
                      density: float = 0.05) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Weights w (nterms) and one n_k x nterms factor per mode whose columns are
    sparse vectors (round(density n_k) nonzeros, at least one)."""
    gen = rng(seed)
    i = np.arange(1, nterms + 1, dtype=np.float64)
    w = np.where(i <= heavy, 1000.0 / i, 1.0 / i)
    factors = []
    for n in dims:
        f = np.zeros((n, nterms))
        nnz = max(1, int(round(density * n)))
        for j in range(nterms):
            rows = gen.choice(n, size=nnz, replace=False)
            f[rows, j] = gen.uniform(0.0, 1.0, size=nnz)
        factors.append(f)
    return w, factors


def cp_tensor(w: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """Dense sum_i w_i f1_i o f2_i o ... (order 3)."""
    if len(factors) != 3:
        raise ValueError("order-3 CP tensors only")
    return np.ascontiguousarray(np.einsum("i,ai,bi,ci->abc", w, *factors, optimize=True))


# --------------------------------------------------------------------------
# Named workloads: the paper's section 5 test tensors at the sizes measured
# here (Hilbert, Tucker-plus-noise, tensor C, an order-4 Tucker tensor).
# Seeds: data seed 0, sketch seed 1.
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dims: Tuple[int, ...]
    ranks: Tuple[int, ...]
    p: int
    q: int
    variant: str          # "t" (T-HOSVD) or "st" (ST-HOSVD)
    storage: str          # "fp64" or "fp32"
    data_seed: int = 0
    sketch_seed: int = 1


WORKLOADS = {
    "tucker3_60_fp64": Workload("tucker3_60_fp64", (60, 60, 60), (10, 10, 10), 5, 1, "t", "fp64"),
    "hilbert3_400": Workload("hilbert3_400", (400, 400, 400), (30, 30, 30), 10, 3, "st", "fp32"),
    "tucker4_120": Workload("tucker4_120", (120, 120, 120, 120), (20, 20, 20, 20), 10, 2, "st", "fp32"),
    "tucker3_1000": Workload("tucker3_1000", (1000, 1000, 1000), (50, 50, 50), 10, 3, "st", "fp32"),
    "sparse_cp3_600": Workload("sparse_cp3_600", (600, 700, 800), (50, 50, 50), 10, 1, "st", "fp32"),
}


def make_tensor(name: str, dims: Sequence[int] | None = None) -> np.ndarray:
    """FP64 host tensor of a named workload (optionally at other dims, same recipe)."""
    w = WORKLOADS[name]
    dims = tuple(dims) if dims is not None else w.dims
    if name == "tucker3_60_fp64":
        a, _, _ = random_tucker(dims, (10,) * len(dims), 1e-3, w.data_seed)
        return a
    if name == "hilbert3_400":
        return hilbert_tensor(dims)
    if name == "tucker4_120":
        a, _, _ = random_tucker(dims, (20,) * len(dims), 1e-2, w.data_seed)
        return a
    if name == "tucker3_1000":
        r = 50
        core = superdiagonal(1.0 / np.arange(1, r + 1, dtype=np.float64), (r,) * len(dims))
        a, _, _ = random_tucker(dims, (r,) * len(dims), 1e-4, w.data_seed, core=core)
        return a
    if name == "sparse_cp3_600":
        return cp_tensor(*sparse_cp_factors(dims, w.data_seed))
    raise KeyError(name)


def build_on_device(name: str, device, dims: Sequence[int] | None = None, seed: int | None = None):
    """Same recipe as make_tensor, assembled with torch on `device` in FP64/FP32.

    For the 1000^3 tensor (4 GB in FP32) host assembly takes minutes; here the
    Haar factors and the core come from the host generator (so they match
    make_tensor) and only the dense expansion and the noise run on the device.
    The noise stream differs from the host one; the result follows the same
    recipe but is not bit-identical to make_tensor.
    """
    import torch

    w = WORKLOADS[name]
    dims = tuple(dims) if dims is not None else w.dims
    seed = w.data_seed if seed is None else seed
    if name == "hilbert3_400":
        return torch.from_numpy(hilbert_tensor(dims).astype(np.float32)).to(device)
    if name == "sparse_cp3_600":
        # factors from the host generator; the expansion (n_1 x (n_2 n_3) times
        # the terms) in FP64 on the device, one slab of mode-1 rows at a time
        wt, fs = sparse_cp_factors(dims, seed)
        x = torch.from_numpy(fs[0] * wt).to(device)
        y, z = (torch.from_numpy(f).to(device) for f in fs[1:])
        out = torch.empty(dims, dtype=torch.float32, device=device)
        for b0 in range(0, dims[1], 100):
            kr = (y[b0:b0 + 100, None, :] * z[None, :, :]).reshape(-1, x.shape[1])
            out[:, b0:b0 + 100, :] = (x @ kr.T).reshape(dims[0], -1, dims[2]).float()
        return out
    r = {"tucker3_60_fp64": 10, "tucker4_120": 20, "tucker3_1000": 50}[name]
    eta = {"tucker3_60_fp64": 1e-3, "tucker4_120": 1e-2, "tucker3_1000": 1e-4}[name]
    gen = rng(seed)
    if name == "tucker3_1000":
        core = superdiagonal(1.0 / np.arange(1, r + 1, dtype=np.float64), (r,) * len(dims))
    else:
        core = gen.standard_normal((r,) * len(dims))
    factors = [haar(n, r, gen) for n in dims]
    t = torch.from_numpy(core).to(device)
    for k, u in enumerate(factors):
        uu = torch.from_numpy(u).to(device)
        t = torch.movedim(torch.tensordot(uu, t, dims=([1], [k])), 0, k)
    t = t.contiguous()
    tn = torch.linalg.vector_norm(t)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) + 7919)
    out = torch.empty(dims, dtype=torch.float32, device=device)
    # noise added in slabs to bound the FP64 temporaries
    e_norm2 = 0.0
    slabs = []
    for i0 in range(0, dims[0], 64):
        e = torch.randn((min(64, dims[0] - i0),) + dims[1:], generator=g, device=device, dtype=torch.float32)
        e_norm2 += float(torch.sum(e.double() ** 2))
        slabs.append((i0, e))
    scale = eta * float(tn) / math.sqrt(e_norm2)
    for i0, e in slabs:
        out[i0:i0 + e.shape[0]] = (t[i0:i0 + e.shape[0]] + scale * e.double()).float()
    del slabs, t
    return out


# --------------------------------------------------------------------------
# Serving stream: order-3 requests with random dims and Tucker ranks.
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    dims: Tuple[int, int, int]
    ranks: Tuple[int, int, int]
    seed: int
    arrival_s: float


def request_stream(count: int, rate_per_s: float, seed: int = 0, n_lo: int = 32, n_hi: int = 256,
                   r_lo: int = 4, r_hi: int = 32) -> List[Request]:
    """Mode sizes U{n_lo..n_hi}, ranks U{r_lo..min(r_hi,n_k)} resampled until
    r_k <= prod_{j != k} r_j (a Tucker rank no unfolding can exceed), Poisson
    arrivals at `rate_per_s` (rate 0 or inf = all at t=0)."""
    gen = rng(seed)
    reqs = []
    t = 0.0
    for i in range(count):
        dims = tuple(int(x) for x in gen.integers(n_lo, n_hi + 1, size=3))
        while True:
            ranks = tuple(int(gen.integers(r_lo, min(r_hi, n) + 1)) for n in dims)
            if all(ranks[k] <= ranks[(k + 1) % 3] * ranks[(k + 2) % 3] for k in range(3)):
                break
        if rate_per_s and math.isfinite(rate_per_s):
            t += float(gen.exponential(1.0 / rate_per_s))
        reqs.append(Request(i, dims, ranks, seed * 1000003 + i, t))
    return reqs


def request_tensor(req: Request, eta: float = 1e-3) -> np.ndarray:
    a, _, _ = random_tucker(req.dims, req.ranks, eta, req.seed)
    return a


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 0) -> List[float]:
    """Arrival times (s) of a Poisson stream; rate 0 or inf: all at t = 0."""
    if not rate_per_s or not math.isfinite(rate_per_s):
        return [0.0] * count
    gen = rng(seed + 7)
    return [float(x) for x in np.cumsum(gen.exponential(1.0 / rate_per_s, size=count))]


def request_tensor_device(req: Request, device, eta: float = 1e-3):
    """The request's tensor (Gaussian core x Haar factors + eta noise), FP32 on
    `device`: core and factors from the request's host stream (as
    request_tensor), the expansion and the noise on the device."""
    import torch

    gen = rng(req.seed)
    core = gen.standard_normal(req.ranks)
    factors = [haar(n, r, gen) for n, r in zip(req.dims, req.ranks)]
    t = torch.from_numpy(core).to(device)
    for k, u in enumerate(factors):
        t = torch.movedim(torch.tensordot(torch.from_numpy(u).to(device), t, dims=([1], [k])), 0, k)
    g = torch.Generator(device=device)
    g.manual_seed(int(req.seed) + 104729)
    e = torch.randn(req.dims, generator=g, device=device, dtype=torch.float64)
    out = t + (eta * torch.linalg.vector_norm(t) / torch.linalg.vector_norm(e)) * e
    return out.float().contiguous()

