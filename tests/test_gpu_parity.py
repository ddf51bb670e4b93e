"""GPU parity: each C-ABI call against the FP64 oracle on the same seeded inputs.

Tolerances: FP64 1e-10 (about 1e6 unit roundoffs: summation error over
contractions of up to 1e6 terms, times the conditioning of the
orthonormalisation) and FP32 1e-5 (about 170 FP32 unit roundoffs; FP32
sums are blocked, so their error grows with the log of the length),
relative to the natural scale of each quantity (Cauchy-Schwarz scale for a
product entry, ||A|| for a reconstruction, Sigma_1 for a shift); subspace
sine distance <= 1e-4 where the oracle's spectral gap is at least 1e-2
(FP32) / 1e-6 (FP64) of Sigma_1.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import philox as orc_rng
from oracle import rhosvd as orc
from oracle.tensor import reconstruct, unfold
from workloads import generators as gen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_04840_amd import _lib
    return _lib


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _np(t):
    return t.detach().double().cpu().numpy()


DT = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.float32}


# --------------------------------------------------------------- generator

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fill_gaussian_matches_oracle(T, prec):
    for (seed, mode, row0, rows, cols) in [(1, 0, 0, 1000, 13), (7, 2, 12345, 257, 64), (3, 1, (1 << 32) - 5, 20, 5)]:
        g = _np(T.fill_gaussian(seed, mode, rows, cols, prec, row0=row0))
        o = orc_rng.gaussian_block(seed, mode, np.arange(row0, row0 + rows), np.arange(cols))
        err = np.abs(g - o)
        if prec == "fp64":
            assert err.max() < 1e-12
        else:
            # FP32 Box-Muller: relative 1e-6 except where u_a rounds near 1 (tiny values)
            assert np.all(err <= 2e-6 * np.abs(o) + 1e-3)
            assert np.mean(err) < 1e-6


# --------------------------------------------------------------- products

SHAPES = [
    ((60, 60, 60), 0, 15), ((60, 60, 60), 1, 15), ((60, 60, 60), 2, 15),
    ((37, 130, 29), 1, 33), ((37, 130, 29), 2, 29), ((131, 7, 45), 0, 64),
    ((5, 6, 7, 8), 2, 7), ((9, 10, 11, 12), 3, 12), ((300, 40), 0, 40), ((200,), 0, 1),
]


def _row_col_scale(xk, b):
    return np.sqrt(np.sum(xk ** 2, axis=1))[:, None] * np.sqrt(np.sum(b ** 2, axis=0))[None, :]


def _power_scale(xk, qa, alpha):
    """Per-entry scale of M = X_(k)(X_(k)^T Q) - alpha Q: entry (i, j) sums
    X_ic Z_cj over c with Z = X_(k)^T Q, so Cauchy-Schwarz bounds its rounding
    by the row norm of X_(k) times the column norm of Z, plus the shift term."""
    return _row_col_scale(xk, xk.T @ qa) + abs(alpha) * np.abs(qa)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,mode,l", SHAPES)
def test_sketch_matches_oracle(T, prec, dims, mode, l):
    a = gen.rng(3).standard_normal(dims)
    x = _dev(a, DT[prec])
    xa = _np(x)
    y = _np(T.sketch(x, mode, l, seed=11, precision=prec))
    xk = unfold(xa, mode)
    om = orc_rng.gaussian_omega(11, mode, xk.shape[1], l)
    ref = orc.sketch(xa, mode, om)
    assert np.all(np.abs(y - ref) <= TOL[prec] * _row_col_scale(xk, om))


def test_sketch_bf16_is_close(T):
    a = gen.rng(4).standard_normal((64, 50, 70))
    x = _dev(a, torch.float32)
    y = _np(T.sketch(x, 1, 40, seed=2, precision="bf16"))
    xa = _np(x)
    xk = unfold(xa, 1)
    ref = orc.sketch(xa, 1, orc_rng.gaussian_omega(2, 1, xk.shape[1], 40))
    # bf16 operands: ~2^-9 relative per product, random signs
    assert np.all(np.abs(y - ref) <= 2e-2 * _row_col_scale(xk, orc_rng.gaussian_omega(2, 1, xk.shape[1], 40)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,mode,l", SHAPES[:8])
def test_power_step_raw_matches_oracle(T, prec, dims, mode, l):
    g = gen.rng(5)
    a = g.standard_normal(dims)
    x = _dev(a, DT[prec])
    xa = _np(x)
    q0 = np.linalg.qr(g.standard_normal((dims[mode], l)))[0]
    q = _dev(q0, DT[prec])
    qa = _np(q)
    alpha = 0.37 * float(np.linalg.norm(a) ** 2) / dims[mode]
    al = torch.tensor([alpha], dtype=torch.float64, device="cuda")
    m = _np(T.shifted_power(x, mode, q, al, raw=True, precision=prec))
    ref = orc.shifted_power(xa, mode, qa, alpha)
    scale = _power_scale(unfold(xa, mode), qa, alpha)
    assert np.all(np.abs(m - ref) <= TOL[prec] * scale), np.max(np.abs(m - ref) / scale)


# Shapes of the one-pass power steps (S a multiple of 4): with FP32 products
# through the BF16 split, n > 256 takes the split one-pass kernel (32-column
# blocks) and n <= 256 the row contraction and column reduction; the FP32
# one-pass kernel (n <= 512, l <= 48) runs them with FP32 instructions in the
# solves below. Several rounds of blocks per workgroup (400 x 16640 columns),
# ragged row groups (n = 100, 44, 260), ragged last blocks (S = 1800, 100,
# 204), P > 1 (modes in the middle), n = 512, a row half with no group
# (n = 16) and widths of one to three 16-column tiles.
FUSED = [((400, 130, 128), 0, 40), ((100, 36, 50), 0, 17), ((30, 400, 100), 1, 48), ((8, 44, 68, 3), 1, 1),
         ((8, 44, 68, 3), 1, 44), ((512, 70, 40), 0, 48), ((16, 12, 64), 0, 16), ((260, 24, 20), 0, 33),
         # the split one-pass kernel's limits: 1024 rows with no padding and l = 64; 257 rows (one row past
         # a staged group), one 32-column block and l = 1; P > 1 with a 4-column last block
         ((1024, 36, 4), 0, 64), ((257, 8, 4), 0, 1), ((3, 260, 36), 1, 17)]


@pytest.mark.parametrize("dims,mode,l", FUSED)
def test_fused_power_step_matches_oracle(T, dims, mode, l):
    """The one-pass power step against the oracle's X_(k)(X_(k)^T Q) - alpha Q,
    element by element (FP32 operands, FP32 accumulation over at most the
    columns of one workgroup's blocks, FP64 sum of the workgroups)."""
    g = gen.rng(23)
    a = g.standard_normal(dims)
    x = _dev(a, torch.float32)
    xa = _np(x)
    q0 = np.linalg.qr(g.standard_normal((dims[mode], l)))[0]
    q = _dev(q0, torch.float32)
    qa = _np(q)
    alpha = 0.37 * float(np.linalg.norm(a) ** 2) / dims[mode]
    al = torch.tensor([alpha], dtype=torch.float64, device="cuda")
    print("fused power step", dims, mode, l, flush=True)
    m = _np(T.shifted_power(x, mode, q, al, raw=True, precision="fp32"))
    ref = orc.shifted_power(xa, mode, qa, alpha)
    # each entry sums m products of size |X_i| |Z_j| / m; FP32 rounding of Z
    # and of the sums: a few 2^-24 relative to the row and column scales
    xk = unfold(xa, mode)
    z = xk.T @ qa
    scale = np.sqrt(np.sum(xk ** 2, axis=1))[:, None] * np.sqrt(np.sum(z ** 2, axis=0))[None, :]
    assert np.all(np.abs(m - ref) <= 1e-5 * scale + 1e-5 * alpha * np.abs(qa)), np.max(np.abs(m - ref) / scale)


@pytest.mark.parametrize("dims", [(20, 64, 36), (300, 20, 36)])
def test_fused_power_step_at_an_unaligned_address(T, dims):
    """X and Q one element past an aligned address on the power-step paths
    (n = 20: the two split kernels; n = 300: the split one-pass kernel)."""
    mode, l = 0, 20
    g = gen.rng(29)
    a = g.standard_normal(dims)
    x = _dev_offset(a, torch.float32)
    assert x.data_ptr() % 16 != 0
    q = _dev_offset(np.linalg.qr(g.standard_normal((dims[mode], l)))[0], torch.float32)
    al = torch.tensor([0.5], dtype=torch.float64, device="cuda")
    m = _np(T.shifted_power(x, mode, q, al, raw=True, precision="fp32"))
    xa = _np(x)
    ref = orc.shifted_power(xa, mode, _np(q), 0.5)
    assert np.all(np.abs(m - ref) <= 1e-5 * _power_scale(unfold(xa, mode), _np(q), 0.5))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,mode,r", [((60, 60, 60), 0, 10), ((37, 130, 29), 1, 20), ((37, 130, 29), 2, 5),
                                         ((5, 6, 7, 8), 1, 3), ((9, 10, 11, 12), 3, 12), ((300, 40), 1, 33),
                                         ((100, 3, 70), 2, 64)])
def test_core_matches_oracle(T, prec, dims, mode, r):
    g = gen.rng(6)
    a = g.standard_normal(dims)
    u0 = np.linalg.qr(g.standard_normal((dims[mode], r)))[0] if r <= dims[mode] else g.standard_normal((dims[mode], r))
    x, u = _dev(a, DT[prec]), _dev(u0, DT[prec])
    out = _np(T.core(x, mode, u, precision=prec))
    ref = orc.core_step(_np(x), mode, _np(u))
    assert out.shape == ref.shape
    xk = unfold(_np(x), mode)
    scale = np.sqrt(np.sum(_np(u) ** 2, axis=0)).max() * np.sqrt(np.sum(xk ** 2, axis=0)).max()
    assert np.max(np.abs(out - ref)) <= TOL[prec] * scale


def _dev_offset(a, dtype):
    """`a` on the device at a base address one element past a 256-byte boundary."""
    a = np.ascontiguousarray(a)
    buf = torch.empty(a.size + 1, dtype=dtype, device="cuda")
    v = buf[1:].view(a.shape)
    v.copy_(torch.from_numpy(a).to(dtype=dtype))
    return v


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,mode,l", [((37, 130, 29), 1, 33), ((61, 45, 23), 0, 20), ((61, 45, 23), 2, 17),
                                         ((50, 33), 1, 7)])
def test_products_at_unaligned_addresses(T, prec, dims, mode, l):
    """Inputs and outputs that start one element past an aligned address, with
    odd row lengths: the wide loads and stores take any element address."""
    dt = DT[prec]
    g = gen.rng(17)
    a = g.standard_normal(dims)
    x = _dev_offset(a, dt)
    assert x.data_ptr() % 16 != 0
    xa = _np(x)
    xk = unfold(xa, mode)
    # sketch (column reduction)
    y = _np(T.sketch(x, mode, l, seed=5, precision=prec))
    om = orc_rng.gaussian_omega(5, mode, xk.shape[1], l)
    assert np.all(np.abs(y - orc.sketch(xa, mode, om)) <= TOL[prec] * _row_col_scale(xk, om))
    # raw power step (row contraction then column reduction), Q at an odd address
    q0 = np.linalg.qr(g.standard_normal((dims[mode], l)))[0]
    q = _dev_offset(q0, dt)
    al = torch.tensor([0.25], dtype=torch.float64, device="cuda")
    m = _np(T.shifted_power(x, mode, q, al, raw=True, precision=prec))
    ref = orc.shifted_power(xa, mode, _np(q), 0.25)
    assert np.all(np.abs(m - ref) <= TOL[prec] * _power_scale(xk, _np(q), 0.25))
    # core step with U and the output at odd addresses
    r = min(l, dims[mode])
    u = _dev_offset(np.linalg.qr(g.standard_normal((dims[mode], r)))[0], dt)
    od = list(dims)
    od[mode] = r
    out = _dev_offset(np.zeros(od), dt)
    sh = T._shape(x.shape)
    T._check(T.lib.tucker_core(ctypes.byref(sh), mode, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(u.data_ptr()), r,
                               T._PREC[prec], ctypes.c_void_p(out.data_ptr()), T._stream(x.device)))
    torch.cuda.synchronize()
    refc = orc.core_step(xa, mode, _np(u))
    scale = np.sqrt(np.sum(_np(u) ** 2, axis=0)).max() * np.sqrt(np.sum(xk ** 2, axis=0)).max()
    assert np.max(np.abs(_np(out) - refc)) <= TOL[prec] * scale


# --------------------------------------------------------------- svd econ

def _matrix_with_spectrum(n, l, s, seed, turn=True):
    g = gen.rng(seed)
    u = np.linalg.qr(g.standard_normal((n, l)))[0]
    v = np.linalg.qr(g.standard_normal((l, l)))[0] if turn else np.eye(l)
    return (u * s[None, :]) @ v.T


# "orthogonal": columns already orthogonal with graded lengths (the shape of a
# power step's turned iterate without a shift), so the scaled first pass is
# orthonormal to rounding and the second and third passes leave at once
@pytest.mark.parametrize("n,l,kind", [(60, 15, "flat"), (400, 40, "graded"), (1000, 60, "graded"), (130, 64, "flat"),
                                      (77, 33, "severe"), (256, 40, "deficient"), (50, 50, "graded"),
                                      (90, 20, "zero_tail"), (400, 40, "orthogonal"), (1000, 60, "orthogonal"),
                                      (60, 15, "orthogonal")])
def test_orth_matches_lapack(T, n, l, kind):
    if kind == "orthogonal":
        s = np.logspace(0, -6, l)
    elif kind == "flat":
        s = np.linspace(2.0, 1.0, l)
    elif kind == "graded":
        s = np.logspace(0, -6, l)
    elif kind == "severe":
        s = np.logspace(0, -14, l)
    elif kind == "deficient":
        s = np.concatenate([np.logspace(0, -3, l - 7), np.zeros(7)])
    else:
        s = np.concatenate([np.logspace(0, -2, l - 3), np.zeros(3)])
    y = _matrix_with_spectrum(n, l, s, seed=n + l, turn=kind != "orthogonal")
    q, sig = T.orth(_dev(y, torch.float64), "fp64")
    q, sig = _np(q), _np(sig)
    s_ref = np.linalg.svd(y, compute_uv=False)
    # orthonormal columns, descending values, values within u-level of Sigma_1
    assert np.max(np.abs(q.T @ q - np.eye(l))) < 1e-12
    assert np.all(np.diff(sig) <= 1e-15 * sig[0])
    assert np.max(np.abs(sig - s_ref)) < 1e-12 * s_ref[0]
    # range: Y = Q Q^T Y
    assert np.linalg.norm(y - q @ (q.T @ y)) < 1e-12 * np.linalg.norm(y)
    # leading singular vectors match LAPACK up to sign where separated
    u_ref = np.linalg.svd(y, full_matrices=False)[0]
    for j in range(l - 1):
        gap = min(abs(s_ref[j] - s_ref[j + 1]), abs(s_ref[j - 1] - s_ref[j]) if j else np.inf)
        if gap > 1e-6 * s_ref[0] and s_ref[j] > 1e-8 * s_ref[0]:
            c = abs(float(q[:, j] @ u_ref[:, j]))
            assert c > 1 - 1e-8, (j, c)


# --------------------------------------------------------------- whole solves

SIGN_TOL = {"fp64": 1e-8, "fp32": 1e-4}


def _check_signed_factors(us, res, ranks, prec, gap_need):
    """The factors as returned, column by column, against the oracle's: both
    sides apply the sign rule of reading A5 (each column's largest-magnitude
    entry positive, the lowest row on ties), and nothing is aligned here, so a
    wrong sign on either side puts that column 2 away. Checked where the
    column's singular value is separated from its neighbours (else any
    rotation is correct) and where the rule's pick is not within rounding of
    the runner-up entry (else either sign is). Returns (columns checked, every
    column of every mode checked)."""
    stol = SIGN_TOL["fp64" if prec == "fp64" else "fp32"]
    checked, complete = 0, True
    for k, lg in enumerate(res.logs):
        s, r, uo = lg.sigmas[-1], ranks[k], res.factors[k]
        for j in range(r):
            lo = abs(s[j] - s[j + 1]) if j + 1 < len(s) else np.inf
            hi = abs(s[j - 1] - s[j]) if j > 0 else np.inf
            a = np.sort(np.abs(uo[:, j]))[::-1]
            if min(lo, hi) < gap_need * s[0] or (len(a) > 1 and a[0] - a[1] <= 10 * stol):
                complete = False
                continue
            err = np.max(np.abs(us[k][:, j] - uo[:, j]))
            assert err <= stol, (k, j, err)
            checked += 1
    return checked, complete


def _compare_solve(a_dev, a64, ranks, p, q, shift, variant, prec, seed=1, check_core=True, order=None,
                   fp32_products="split"):
    from paper_2506_04840_amd import _lib as T
    fn = T.rsthosvd if variant == "st" else T.rthosvd
    G, U, info = fn(a_dev, ranks, p=p, q=q, shift=shift, seed=seed, precision=prec, order=order,
                    fp32_products=fp32_products)
    torch.cuda.synchronize()
    g, us = _np(G), [_np(u) for u in U]
    oo = orc.decreasing_order(a64.shape) if order == "decreasing" else order
    res = orc.randomized_hosvd(a64, ranks, p, q, shift=shift, variant=variant, seed=seed, order=oo)
    tol = TOL["fp64" if prec == "fp64" else "fp32"]
    na = np.linalg.norm(a64)
    # (i) reconstruction
    d_rec = np.linalg.norm(reconstruct(g, us) - reconstruct(res.core, res.factors)) / na
    assert d_rec <= tol, d_rec
    # orthonormal factors
    for u in us:
        assert np.max(np.abs(u.T @ u - np.eye(u.shape[1]))) < (1e-12 if prec == "fp64" else 1e-5)
    gap_need = 1e-6 if prec == "fp64" else 1e-2
    for k, lg in enumerate(res.logs):
        s = lg.sigmas[-1]
        r = ranks[k]
        # (iii) shifts and Sigma(l,l), in units of Sigma_1
        for t in range(q + 1):
            assert abs(info["alpha"][k][t] - lg.alphas[t]) <= tol * lg.sigmas[t][0], (k, t)
            assert abs(info["sigma_l"][k][t] - lg.sigmas[t][-1]) <= tol * lg.sigmas[t][0], (k, t)
            assert abs(info["sigma_1"][k][t] - lg.sigmas[t][0]) <= tol * lg.sigmas[t][0], (k, t)
        assert info["l"][k] == lg.l
        # (ii) subspace where the gap allows
        if r < len(s) and (s[r - 1] - s[r]) >= gap_need * s[0]:
            uo = res.factors[k]
            sin = np.linalg.norm(us[k] - uo @ (uo.T @ us[k]), 2)
            assert sin <= 1e-4, (k, sin)
    # (iv) the factors column by column and the core entrywise with the signs
    # both sides chose (the sign rule, nothing aligned), where they are unique
    checked, complete = _check_signed_factors(us, res, ranks, prec, gap_need)
    if check_core and complete:
        assert np.max(np.abs(g - res.core)) <= 10 * tol * np.linalg.norm(res.core)
    # the norms and the identity-based relative error the solve reports (section 5,
    # and the orthogonal-projection identity of section 2.2)
    _check_info_norms(info, a64 if prec == "fp64" else _np(a_dev), g, res, prec)
    return G, U, info, res


def _check_info_norms(info, a_stored, g, res, prec):
    """info.normA2 is ||A||^2 of the stored tensor (FP64 sums of exactly
    representable squares: a few units of FP64 rounding); info.normG2 is the
    returned core's ||G||^2 (summed here from the core as returned), and within the
    solve's tolerance of the oracle core's; info.rel_error is the identity form
    sqrt(1 - ||G||^2/||A||^2) of both reported norms, and matches the oracle's
    identity-form error within the tolerance in RE^2."""
    tol = TOL["fp64" if prec == "fp64" else "fp32"]
    na2 = orc.frob2(a_stored)
    assert abs(info["normA2"] - na2) <= 1e-12 * na2, (info["normA2"], na2)
    assert abs(info["normG2"] - float(np.dot(g.ravel(), g.ravel()))) <= 1e-12 * na2
    assert abs(info["normG2"] - orc.frob2(res.core)) <= 4 * tol * na2
    re_id = np.sqrt(max(info["normA2"] - info["normG2"], 0.0) / info["normA2"]) if na2 > 0 else 0.0
    assert abs(info["rel_error"] - re_id) <= 1e-15 + 1e-12 * re_id
    re_o = orc.rel_error_identity(a_stored, res.core)
    assert abs(info["rel_error"] ** 2 - re_o ** 2) <= 4 * tol, (info["rel_error"], re_o)


def test_solve_tucker3_60_fp64_thosvd(T):
    a = gen.make_tensor("tucker3_60_fp64")
    x = _dev(a, torch.float64)
    _, _, info, res = _compare_solve(x, a, (10, 10, 10), 5, 1, "adaptive", "t", "fp64")
    re = orc.rel_error(a, res)
    assert 0.5e-3 < re < 2e-3


@pytest.mark.parametrize("variant", ["t", "st"])
@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_solve_fp64_small_all_q(T, variant, q):
    a, _, _ = gen.random_tucker((33, 45, 28), (5, 6, 4), 0.05, seed=21)
    _compare_solve(_dev(a, torch.float64), a, (5, 6, 4), 6, q, "adaptive", variant, "fp64")


@pytest.mark.parametrize("shift", ["adaptive", "none"])
@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_solve_hilbert_fp32(T, shift, q):
    a = gen.hilbert_tensor((96, 96, 96)).astype(np.float32)
    x = _dev(a, torch.float32)
    _compare_solve(x, a.astype(np.float64), (30, 30, 30), 10, q, shift, "st", "fp32")


def test_solve_order4_fp32(T):
    a, _, _ = gen.random_tucker((24, 26, 22, 25), (5, 5, 5, 5), 1e-2, seed=8)
    a32 = a.astype(np.float32)
    _compare_solve(_dev(a32, torch.float32), a32.astype(np.float64), (5, 5, 5, 5), 10, 2, "adaptive", "st", "fp32")


def test_solve_bf16_reports_close_error(T):
    a, _, _ = gen.random_tucker((40, 44, 36, 30), (6, 6, 6, 6), 1e-2, seed=9)
    a32 = a.astype(np.float32)
    G, U, info = T.rsthosvd(_dev(a32, torch.float32), (6, 6, 6, 6), p=10, q=2, precision="bf16")
    re_g = np.linalg.norm(a32 - reconstruct(_np(G), [_np(u) for u in U])) / np.linalg.norm(a32)
    res = orc.randomized_hosvd(a32.astype(np.float64), (6, 6, 6, 6), 10, 2, variant="st", seed=1)
    re_o = orc.rel_error(a32.astype(np.float64), res)
    assert re_g <= re_o * 1.05


def test_exact_rank_recovery_and_deficiency(T):
    a, _, _ = gen.random_tucker((30, 32, 34), (4, 5, 3), 0.0, seed=12)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        x = _dev(a, DT[prec])
        for q in (0, 2):
            G, U, info = T.rsthosvd(x, (4, 5, 3), p=6, q=q, precision=prec)
            xa = _np(x)
            re = np.linalg.norm(xa - reconstruct(_np(G), [_np(u) for u in U])) / np.linalg.norm(xa)
            assert re < tol, (prec, q, re)
            for u in U:
                uu = _np(u)
                assert np.max(np.abs(uu.T @ uu - np.eye(uu.shape[1]))) < 1e-5


def test_deterministic_bitwise(T):
    a = gen.hilbert_tensor((70, 80, 90)).astype(np.float32)
    x = _dev(a, torch.float32)
    r1 = T.rsthosvd(x, (12, 12, 12), p=8, q=3)
    r2 = T.rsthosvd(x, (12, 12, 12), p=8, q=3)
    assert torch.equal(r1[0], r2[0])
    for u1, u2 in zip(r1[1], r2[1]):
        assert torch.equal(u1, u2)


def test_q_le_1_shift_invariance_bitwise(T):
    a, _, _ = gen.random_tucker((50, 40, 45), (5, 5, 5), 0.1, seed=2)
    x = _dev(a.astype(np.float32), torch.float32)
    for q in (0, 1):
        ra = T.rsthosvd(x, (5, 5, 5), p=5, q=q, shift="adaptive")
        rn = T.rsthosvd(x, (5, 5, 5), p=5, q=q, shift="none")
        assert torch.equal(ra[0], rn[0])


def test_edge_shapes(T):
    # order 1 and 2, n = r, clamped l, tiny modes, ragged tails
    cases = [((200,), (1,), 3, 1), ((64, 48), (10, 10), 4, 2), ((16, 17, 18), (16, 3, 2), 5, 1),
             ((3, 100, 5), (3, 9, 5), 10, 2), ((129, 2, 257), (7, 2, 11), 4, 1)]
    for dims, ranks, p, q in cases:
        a, _, _ = gen.random_tucker(dims, tuple(min(r + 1, n) for r, n in zip(ranks, dims)), 0.05, seed=len(dims))
        _compare_solve(_dev(a, torch.float64), a, ranks, p, q, "adaptive", "st", "fp64", check_core=False)


@pytest.mark.parametrize("fp32_products,dims", [("native", (64, 68, 72)), ("split", (300, 264, 32))])
def test_fp32_t_hosvd_with_concurrent_fused_power_steps(T, fp32_products, dims):
    """FP32 T-HOSVD where modes 0 (S = n1 n2) and 1 (P = n0, S = n2) both take
    a one-pass power step, on their own streams at the same time (each with
    its own chunk counters), two power steps each, against the FP64 oracle;
    mode 2 (S = 1) runs the two-kernel products. FP32 instructions take the
    FP32 one-pass kernel (n <= 512); products through the BF16 split take the
    split one-pass kernel, which needs n > 256. Then the same solve again:
    each mode zeroes its counter at its start, and every launch takes its base
    (the fetches of the launches before it) from the host."""
    a, _, _ = gen.random_tucker(dims, (8, 9, 10), 1e-2, seed=43)
    a32 = a.astype(np.float32)
    x = _dev(a32, torch.float32)
    for _ in range(2):
        _compare_solve(x, a32.astype(np.float64), (8, 9, 10), 10, 2, "adaptive", "t", "fp32",
                       fp32_products=fp32_products)


@pytest.mark.parametrize("variant", ["t", "st"])
def test_solve_largest_order_and_width(T, variant):
    """The limits: order 8 (TUCKER_MAX_ORDER), and a mode whose sketch width is
    l = 64 (TUCKER_MAX_L), both against the oracle in FP64."""
    a, _, _ = gen.random_tucker((3, 4, 3, 5, 3, 2, 3, 4), (2, 2, 2, 3, 2, 2, 2, 2), 0.05, seed=41)
    _compare_solve(_dev(a, torch.float64), a, (2, 2, 2, 3, 2, 2, 2, 2), 1, 1, "adaptive", variant, "fp64",
                   check_core=False)
    a, _, _ = gen.random_tucker((100, 90, 80), (54, 50, 40), 0.05, seed=42)
    _, _, info, _ = _compare_solve(_dev(a, torch.float64), a, (54, 50, 40), 10, 1, "adaptive", variant, "fp64",
                                   check_core=False)
    assert info["l"][0] == 64


@pytest.mark.parametrize("q", [0, 2])
def test_solve_bf16_reaches_fp32_error(T, q):
    """BF16 operands: the last step's products run on FP32 operands, so the
    final subspace, the reconstruction and the relative error match the FP64
    oracle to the FP32 tolerance although the earlier passes round to BF16."""
    a, _, _ = gen.random_tucker((150, 140, 130), (12, 12, 12), 1e-4, seed=7)
    x = _dev(a, torch.float32)
    a32 = _np(x)
    res = orc.randomized_hosvd(a32, (12, 12, 12), 8, q, shift="adaptive", variant="st", seed=3)
    re_o = orc.rel_error(a32, res)
    G, U, info = T.rsthosvd(x, (12, 12, 12), p=8, q=q, seed=3, precision="bf16")
    torch.cuda.synchronize()
    g, us = _np(G), [_np(u) for u in U]
    rec = reconstruct(g, us)
    na = np.linalg.norm(a32)
    assert np.linalg.norm(rec - reconstruct(res.core, res.factors)) / na <= 1e-5
    assert abs(np.linalg.norm(a32 - rec) / na - re_o) <= 1e-6


# --------------------------------------------------------------- Algorithm 4 (PVE-controlled q)

def _pve_ratios(res, ranks):
    """Per mode, the tol each power step needed to stop there (from the oracle's
    logs): max_{i<r} |sigma_t(i) - sigma_{t-1}(i)| / sigma_t(r + 1)."""
    out = []
    for k, lg in enumerate(res.logs):
        r = ranks[k]
        prev = np.zeros(lg.l)
        rat = []
        for t in range(1, len(lg.sigmas)):
            sig = lg.sigmas[t] + lg.alphas[t - 1]
            rat.append(np.max(np.abs(sig[:r] - prev[:r])) / sig[min(r, lg.l - 1)])
            prev = sig
        out.append(rat)
    return out


@pytest.mark.parametrize("variant", ["st", "t"])
@pytest.mark.parametrize("target", ["zero", "mid", "inf"])
def test_solve_pve_fp64_matches_oracle(T, target, variant):
    """Algorithm 4 in FP64 against the oracle (and its T-HOSVD form, the
    paper's Algorithm 2-v3): the same power counts q_k (tol chosen away from
    every step's threshold, where rounding could flip the decision) and the
    reconstruction within 1e-10."""
    a, _, _ = gen.random_tucker((33, 45, 28), (5, 6, 4), 0.05, seed=21)
    ranks, p, qmax = (5, 6, 4), 6, 12
    if target == "zero":
        tol = 0.0
    elif target == "inf":
        tol = float("inf")
    else:
        probe = orc.randomized_sthosvd_pve(a, ranks, p, qmax, 0.0, seed=1, variant=variant)
        rats = _pve_ratios(probe, ranks)
        tol = float(np.sqrt(rats[0][1] * rats[0][2]))  # mode 1 stops at its third step
        for _ in range(20):
            res = orc.randomized_sthosvd_pve(a, ranks, p, qmax, tol, seed=1, variant=variant)
            if all(abs(x / tol - 1.0) > 1e-6 for rr in _pve_ratios(res, ranks) for x in rr):
                break
            tol *= 1.37
    res = orc.randomized_sthosvd_pve(a, ranks, p, qmax, tol, seed=1, variant=variant)
    fn = T.rsthosvd_pve if variant == "st" else T.rthosvd_pve
    G, U, info, qs = fn(_dev(a, torch.float64), ranks, p=p, q_max=qmax, tol=tol, seed=1, precision="fp64")
    torch.cuda.synchronize()
    assert qs == res.qs, (qs, res.qs, tol)
    na = np.linalg.norm(a)
    d = np.linalg.norm(reconstruct(_np(G), [_np(u) for u in U]) - reconstruct(res.core, res.factors)) / na
    assert d <= 1e-10, d
    for k, lg in enumerate(res.logs):
        for t in range(min(qs[k], 16) + 1):
            assert abs(info["alpha"][k][t] - lg.alphas[t]) <= 1e-10 * lg.sigmas[t][0], (k, t)


def test_solve_pve_fp32_reaches_oracle_error(T):
    """FP32 storage, tol = 0.5 (the paper's recommended setting). Estimate
    changes below the FP32 iterate's rounding level count as none, so a mode
    may stop before the FP64 oracle does (never more than one step later); the
    relative error is the oracle's."""
    a, _, _ = gen.random_tucker((60, 50, 40), (8, 7, 6), 1e-3, seed=22)
    a32 = a.astype(np.float32).astype(np.float64)
    res = orc.randomized_sthosvd_pve(a32, (8, 7, 6), 8, 20, 0.5, seed=4)
    G, U, info, qs = T.rsthosvd_pve(_dev(a32, torch.float32), (8, 7, 6), p=8, q_max=20, tol=0.5, seed=4)
    torch.cuda.synchronize()
    assert all(1 <= x <= y + 1 for x, y in zip(qs, res.qs)), (qs, res.qs)
    rec = reconstruct(_np(G), [_np(u) for u in U])
    assert abs(np.linalg.norm(a32 - rec) / np.linalg.norm(a32) - orc.rel_error(a32, res)) <= 1e-6


# --------------------------------------------------------------- other test matrices (section 5)

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["gaussian", "uniform", "kr_gaussian", "kr_uniform"])
def test_fill_test_matrix_matches_oracle(T, kind, prec):
    dims, mode, l = (7, 9, 5, 6), 2, 13
    m = 7 * 9 * 6
    g = _np(T.fill_test_matrix(kind, 11, mode, dims, m, l, prec))
    o = orc_rng.omega_matrix(kind, 11, mode, [7, 9, 6], l)
    err = np.abs(g - o)
    if prec == "fp64":
        assert np.all(err <= 1e-12 * np.maximum(1.0, np.abs(o)))
    elif kind == "uniform":
        assert np.all(err <= 6e-8)  # one rounding of the exact FP64 value
    else:
        # FP32 Box-Muller (relative 1e-6 but for tiny values), one factor per other mode
        assert np.all(err <= 1e-5 * np.abs(o) + 3e-3)
        assert np.median(err / np.maximum(np.abs(o), 1e-3)) < 3e-6
    # a row window addresses the same entries
    gw = _np(T.fill_test_matrix(kind, 11, mode, dims, 50, l, prec, row0=100))
    assert np.array_equal(gw, g[100:150])


@pytest.mark.parametrize("variant", ["t", "st"])
@pytest.mark.parametrize("kind", ["uniform", "kr_gaussian", "kr_uniform"])
def test_solve_with_other_test_matrices(T, kind, variant):
    """Whole FP64 solves drawing each kind of test matrix: the oracle, given
    the same matrices (the unfolding's other sizes; ST: ranks of the modes
    already processed), reaches the same reconstruction to 1e-10."""
    a, _, _ = gen.random_tucker((26, 30, 22), (5, 6, 4), 0.05, seed=23)
    ranks, p, q = (5, 6, 4), 5, 1

    def om(k, m, l):
        cur = [ranks[i] if (variant == "st" and i < k) else a.shape[i] for i in range(3)]
        return orc_rng.omega_matrix(kind, 3, k, [cur[i] for i in range(3) if i != k], l)

    res = orc.randomized_hosvd(a, ranks, p, q, variant=variant, seed=3, omega=om)
    fn = T.rsthosvd if variant == "st" else T.rthosvd
    G, U, info = fn(_dev(a, torch.float64), ranks, p=p, q=q, seed=3, precision="fp64", omega=kind)
    torch.cuda.synchronize()
    d = np.linalg.norm(reconstruct(_np(G), [_np(u) for u in U]) - reconstruct(res.core, res.factors))
    assert d / np.linalg.norm(a) <= 1e-10


# --------------------------------------------------------------- processing order (Sections 2.2, 3.2)

@pytest.mark.parametrize("order", [(2, 0, 1), (1, 2, 0), (2, 1, 0), "decreasing"])
@pytest.mark.parametrize("q", [0, 2])
def test_solve_st_in_processing_order_fp64(T, order, q):
    """ST-HOSVD in a given processing order matches the oracle run in the same
    order (reconstruction, shifts and Sigma logs per mode, subspaces, core)."""
    a, _, _ = gen.random_tucker((33, 45, 28), (5, 6, 4), 0.05, seed=21)
    _compare_solve(_dev(a, torch.float64), a, (5, 6, 4), 6, q, "adaptive", "st", "fp64", order=order)


def test_solve_st_in_processing_order_fp32_order4(T):
    a, _, _ = gen.random_tucker((20, 44, 12, 36), (4, 7, 3, 6), 0.02, seed=27)
    a32 = a.astype(np.float32)
    for order in ("decreasing", (3, 0, 2, 1)):
        print("order", order, flush=True)
        _compare_solve(_dev(a32, torch.float32), a32.astype(np.float64), (4, 7, 3, 6), 5, 1, "adaptive", "st",
                       "fp32", order=order)


def test_solve_t_does_not_depend_on_the_order(T):
    a, _, _ = gen.random_tucker((33, 45, 28), (5, 6, 4), 0.05, seed=21)
    x = _dev(a, torch.float64)
    G0, U0, _ = T.rthosvd(x, (5, 6, 4), p=6, q=1, seed=2, precision="fp64")
    G1, U1, _ = T.rthosvd(x, (5, 6, 4), p=6, q=1, seed=2, precision="fp64", order=(2, 0, 1))
    torch.cuda.synchronize()
    assert torch.equal(G0, G1)
    for u, v in zip(U0, U1):
        assert torch.equal(u, v)


def test_solve_st_in_processing_order_with_khatri_rao(T):
    """The test matrix of each mode is drawn for its current sizes, which the
    order decides (modes processed before k have size r)."""
    a, _, _ = gen.random_tucker((26, 30, 22), (5, 6, 4), 0.05, seed=23)
    ranks, p, q, order = (5, 6, 4), 5, 1, (2, 0, 1)

    def om(k, m, l):
        before = order[:order.index(k)]
        cur = [ranks[i] if i in before else a.shape[i] for i in range(3)]
        return orc_rng.omega_matrix("kr_gaussian", 3, k, [cur[i] for i in range(3) if i != k], l)

    res = orc.randomized_hosvd(a, ranks, p, q, variant="st", seed=3, omega=om, order=order)
    G, U, _ = T.rsthosvd(_dev(a, torch.float64), ranks, p=p, q=q, seed=3, precision="fp64", omega="kr_gaussian",
                         order=order)
    torch.cuda.synchronize()
    d = np.linalg.norm(reconstruct(_np(G), [_np(u) for u in U]) - reconstruct(res.core, res.factors))
    assert d / np.linalg.norm(a) <= 1e-10


# --------------------------------------------------------------- holistic variants (Appendices A, B)

def _compare_holistic(a_dev, a64, ranks, p, q, shift, variant, prec, seed=1, order=None, tol=None):
    fn = T_mod().rsthosvd if variant == "st" else T_mod().rthosvd
    G, U, info = fn(a_dev, ranks, p=p, q=q, shift=shift, seed=seed, precision=prec, order=order, holistic=True)
    torch.cuda.synchronize()
    g, us = _np(G), [_np(u) for u in U]
    oo = orc.decreasing_order(a64.shape) if order == "decreasing" else order
    res = orc.randomized_hosvd_holistic(a64, ranks, p, q, shift=shift, variant=variant, seed=seed, order=oo)
    tol = TOL["fp64" if prec == "fp64" else "fp32"] if tol is None else tol
    na = np.linalg.norm(a64)
    d_rec = np.linalg.norm(reconstruct(g, us) - reconstruct(res.core, res.factors)) / na
    assert d_rec <= tol, d_rec
    for u in us:
        assert np.max(np.abs(u.T @ u - np.eye(u.shape[1]))) < (1e-12 if prec == "fp64" else 1e-5)
    for k, lg in enumerate(res.logs):
        assert info["l"][k] == lg.l
        for t in range(q + 1):
            assert abs(info["alpha"][k][t] - lg.alphas[t]) <= tol * lg.sigmas[t][0], (k, t)
            assert abs(info["sigma_1"][k][t] - lg.sigmas[t][0]) <= tol * lg.sigmas[t][0], (k, t)
    # the factors themselves where the small tensor's spectrum separates r_k
    if prec == "fp64":
        for k in range(len(ranks)):
            assert np.max(np.abs(us[k] - res.factors[k])) < 1e-6 or _gap_small(res, a64, k, ranks), k
    return G, U, info, res


def T_mod():
    from paper_2506_04840_amd import _lib
    return _lib


def _gap_small(res, a64, k, ranks):
    s = np.linalg.svd(orc.unfold(a64, k), compute_uv=False)
    r = ranks[k]
    return r < len(s) and (s[r - 1] - s[r]) < 1e-6 * s[0]


@pytest.mark.parametrize("variant", ["t", "st"])
@pytest.mark.parametrize("q,shift", [(0, "adaptive"), (1, "adaptive"), (2, "adaptive"), (2, "none")])
def test_holistic_fp64_matches_oracle(T, variant, q, shift):
    a, _, _ = gen.random_tucker((33, 45, 28), (5, 6, 4), 0.05, seed=21)
    _compare_holistic(_dev(a, torch.float64), a, (5, 6, 4), 6, q, shift, variant, "fp64")


def test_holistic_fp32_hilbert(T):
    a = gen.hilbert_tensor((96, 96, 96)).astype(np.float32)
    _compare_holistic(_dev(a, torch.float32), a.astype(np.float64), (30, 30, 30), 10, 1, "adaptive", "st", "fp32")


@pytest.mark.parametrize("order", [(2, 0, 1), "decreasing"])
def test_holistic_in_processing_order(T, order):
    a, _, _ = gen.random_tucker((20, 44, 31), (4, 6, 5), 0.05, seed=29)
    _compare_holistic(_dev(a, torch.float64), a, (4, 6, 5), 5, 1, "adaptive", "st", "fp64", order=order)


@pytest.mark.parametrize("variant", ["t", "st"])
def test_holistic_exact_rank_and_wide_small_unfolding(T, variant):
    """Exact Tucker rank is recovered. In the ST form the last mode's unfolding
    of the small tensor is 13 x 4 (fewer columns than rows, rank 3): its left
    singular vectors come from the unfolding itself rather than from its
    transpose, through the rank-deficient CholeskyQR."""
    a, _, _ = gen.random_tucker((5, 5, 100), (2, 2, 3), 0.0, seed=31)
    G, U, info, res = _compare_holistic(_dev(a, torch.float64), a, (2, 2, 3), 10, 1, "adaptive", variant, "fp64")
    rec = reconstruct(_np(G), [_np(u) for u in U])
    assert np.linalg.norm(a - rec) / np.linalg.norm(a) < 1e-12


# --------------------------------------------------------------- graph replay of whole solves

@pytest.mark.parametrize("variant,q,holistic", [("st", 2, False), ("t", 1, False), ("st", 1, True), ("t", 1, True)])
def test_solve_graph_replay_equals_eager(T, variant, q, holistic):
    """A captured solve (side streams joined through events) replayed three
    times, with eager work and new tensor contents between replays, gives the
    eager result bitwise each time."""
    a, _, _ = gen.random_tucker((40, 36, 30), (5, 6, 4), 0.05, seed=37)
    b, _, _ = gen.random_tucker((40, 36, 30), (5, 6, 4), 0.05, seed=38)
    dev = torch.device("cuda:0")
    s = T.Solver(a.shape, (5, 6, 4), 6, q, "adaptive", 3, "fp32", variant == "st", dev, holistic=holistic)
    A = torch.from_numpy(a.astype(np.float32)).to(dev)
    ref = {}
    for name, src in (("a", a), ("b", b)):
        A.copy_(torch.from_numpy(src.astype(np.float32)))
        G, U = s.run(A)
        torch.cuda.synchronize()
        ref[name] = (G.clone(), [u.clone() for u in U])
    A.copy_(torch.from_numpy(a.astype(np.float32)))
    s.capture(A)
    for rep, name in enumerate(("a", "b", "a")):
        A.copy_(torch.from_numpy((a if name == "a" else b).astype(np.float32)))
        _ = torch.ones(4096, device=dev).sum().item()  # eager work between replays
        G, U = s.replay()
        torch.cuda.synchronize()
        print("replay", rep, name, flush=True)
        assert torch.equal(G, ref[name][0])
        for u, v in zip(U, ref[name][1]):
            assert torch.equal(u, v)


def test_t_hosvd_capture_runs_modes_in_sequence(T):
    """Under stream capture a T-HOSVD runs its modes one after another on the
    capturing stream (the eager call runs them on concurrent streams): an
    order-4 FP64 solve with q = 2, captured and replayed twice, equals the
    eager concurrent solve bitwise, and the eager call after the capture still
    does."""
    a, _, _ = gen.random_tucker((18, 16, 14, 12), (3, 4, 3, 2), 0.02, seed=41)
    dev = torch.device("cuda:0")
    s = T.Solver(a.shape, (3, 4, 3, 2), 4, 2, "adaptive", 5, "fp64", False, dev)
    A = torch.from_numpy(a).to(dev)
    G, U = s.run(A)
    torch.cuda.synchronize()
    ref = (G.clone(), [u.clone() for u in U])
    s.capture(A)
    for rep in range(2):
        G.zero_()
        G, U = s.replay()
        torch.cuda.synchronize()
        print("replay", rep, flush=True)
        assert torch.equal(G, ref[0])
        for u, v in zip(U, ref[1]):
            assert torch.equal(u, v)
    G, U = s.run(A)
    torch.cuda.synchronize()
    assert torch.equal(G, ref[0])


# --------------------------------------------------------------- degenerate inputs

@pytest.mark.parametrize("variant", ["st", "t"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_tensor(T, variant, prec):
    """A = 0: every column of every iterate is dependent. The core is exactly
    zero, the factors are orthonormal (completed by the fixed pseudo-random
    directions), the shift stays at 0 and the deficiency flag is raised."""
    x = torch.zeros((30, 28, 26), dtype=DT[prec], device="cuda")
    fn = T.rsthosvd if variant == "st" else T.rthosvd
    G, U, info = fn(x, (4, 5, 3), p=5, q=2, precision=prec)
    torch.cuda.synchronize()
    assert torch.count_nonzero(G).item() == 0
    for u in U:
        uu = _np(u)
        assert np.all(np.isfinite(uu))
        assert np.max(np.abs(uu.T @ uu - np.eye(uu.shape[1]))) < (1e-12 if prec == "fp64" else 1e-6)
    assert all(a == 0.0 for row in info["alpha"][:3] for a in row)
    assert info["flags"] & T.INFO_DEFICIENT


def test_ranks_above_the_true_rank_and_unit_modes(T):
    """Ranks above the tensor's exact Tucker rank (the extra columns are
    completion directions: orthonormal, the reconstruction still exact), and a
    mode of size 1, against the oracle."""
    a, _, _ = gen.random_tucker((24, 22, 20), (2, 3, 2), 0.0, seed=43)
    G, U, info = T.rsthosvd(_dev(a, torch.float64), (5, 6, 4), p=4, q=1, precision="fp64")
    torch.cuda.synchronize()
    rec = reconstruct(_np(G), [_np(u) for u in U])
    assert np.linalg.norm(a - rec) / np.linalg.norm(a) < 1e-12
    for u in U:
        uu = _np(u)
        assert np.max(np.abs(uu.T @ uu - np.eye(uu.shape[1]))) < 1e-12
    b, _, _ = gen.random_tucker((1, 30, 40), (1, 5, 5), 0.05, seed=44)
    for variant in ("st", "t"):
        _compare_solve(_dev(b, torch.float64), b, (1, 5, 5), 4, 1, "adaptive", variant, "fp64", check_core=False)


# --------------------------------------------------------------- norms, relative error, sign rule

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("numel", [1, 7, 4096, 100003, 3 * 1024 * 1024 + 5])
def test_norm2_matches_oracle(T, prec, numel):
    """tucker_norm2: ||X||_F^2 with FP64 accumulation against the oracle's frob2
    of the same stored values (a sum of exactly representable squares)."""
    x = _dev(gen.rng(numel).standard_normal(numel), DT[prec])
    got = float(T.norm2(x).item())
    ref = orc.frob2(_np(x))
    assert abs(got - ref) <= 1e-13 * ref, (got, ref)


@pytest.mark.parametrize("case", ["st_first_mode_s1", "order1", "t_concurrent", "bf16", "holistic", "pve",
                                  "fp64_odd_stage"])
def test_info_norms_on_every_path(T, case):
    """info.normA2 / normG2 / rel_error on the paths that carry ||A||^2 in the
    first sketch (S > 1 and each edge form) and on those that take a pass of
    their own (the first mode processed has S == 1): normA2 is the oracle's
    frob2 of the stored tensor, rel_error the identity form of section 2.2,
    matching the oracle's identity-form error in RE^2 within the tolerance."""
    a, _, _ = gen.random_tucker((33, 45, 28), (5, 6, 4), 0.05, seed=51)
    ranks, p, q = (5, 6, 4), 6, 2
    kw = {}
    prec, variant = "fp32", "st"
    if case == "st_first_mode_s1":
        kw["order"] = (2, 0, 1)
    elif case == "order1":
        a = gen.rng(52).standard_normal(300)
        ranks, p, q = (1,), 3, 1
    elif case == "t_concurrent":
        variant = "t"
    elif case == "bf16":
        prec = "bf16"
    elif case == "holistic":
        kw["holistic"] = True
    elif case == "fp64_odd_stage":
        prec = "fp64"
        a, _, _ = gen.random_tucker((21, 19, 23), (4, 4, 4), 0.05, seed=53)  # S = 437 and 23: odd edge stages
        ranks = (4, 4, 4)
    x = _dev(a, DT[prec])
    xa = _np(x)
    if case == "pve":
        G, U, info, qs = T.rsthosvd_pve(x, ranks, p=p, q_max=6, tol=0.5, seed=1)
        res = orc.randomized_sthosvd_pve(xa, ranks, p, 6, 0.5, seed=1)
    else:
        fn = T.rsthosvd if variant == "st" else T.rthosvd
        G, U, info = fn(x, ranks, p=p, q=q, seed=1, precision=prec, **kw)
        oo = kw.get("order")
        if kw.get("holistic"):
            res = orc.randomized_hosvd_holistic(xa, ranks, p, q, variant=variant, seed=1)
        else:
            res = orc.randomized_hosvd(xa, ranks, p, q, variant=variant, seed=1, order=oo)
    torch.cuda.synchronize()
    print("norms", case, info["normA2"], info["normG2"], info["rel_error"], flush=True)
    _check_info_norms(info, xa, _np(G), res, "fp64" if prec == "fp64" else "fp32")
    assert not info["flags"] & T.INFO_INTERNAL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", ["t", "st"])
def test_sign_rule_factors_and_core(T, prec, variant):
    """Every factor column and the core against the oracle with no sign
    alignment at all, on a tensor whose unfoldings have well separated
    singular values (superdiagonal core 4, 3.2, 2.5, ... times Haar factors,
    plus noise): every column is unique up to its sign, and the sign rule
    fixes the sign, so both sides must return the same vectors."""
    g = gen.rng(61)
    v = 4.0 * 0.8 ** np.arange(6)
    dims, r = (40, 36, 32), 6
    core = gen.superdiagonal(v, (r, r, r))
    a, _, _ = gen.random_tucker(dims, (r, r, r), 1e-3, seed=62, core=core)
    x = _dev(a, DT[prec])
    G, U, info, res = _compare_solve(x, _np(x), (r, r, r), 6, 2, "adaptive", variant, prec)
    checked, complete = _check_signed_factors([_np(u) for u in U], res, (r, r, r), prec,
                                              1e-6 if prec == "fp64" else 1e-2)
    assert complete and checked == 3 * r, (checked, complete)
    assert np.max(np.abs(_np(G) - res.core)) <= 10 * TOL[prec] * np.linalg.norm(res.core)


def test_nonfinite_input_is_flagged(T):
    """A NaN in the tensor: every iterate's Gram is non-finite, the
    orthonormalisation takes every column as dependent (bounded loops, no
    hang), the solve completes with TUCKER_INFO_NONFINITE set, orthonormal
    finite factors and a core that carries the NaN."""
    a, _, _ = gen.random_tucker((30, 28, 26), (4, 4, 4), 0.05, seed=63)
    a[3, 4, 5] = np.nan
    for prec in ("fp64", "fp32"):
        G, U, info = T.rsthosvd(_dev(a, DT[prec]), (4, 4, 4), p=4, q=2, precision=prec)
        torch.cuda.synchronize()
        assert info["flags"] & T.INFO_NONFINITE, info["flags"]
        for u in U:
            uu = _np(u)
            assert np.all(np.isfinite(uu))
            assert np.max(np.abs(uu.T @ uu - np.eye(uu.shape[1]))) < 1e-5
        assert not bool(torch.isfinite(G).all())


@pytest.mark.parametrize("fp32_products,dims", [("native", (96, 80, 72)), ("split", (288, 48, 40))])
def test_fused_power_steps_without_rezeroing(T, fp32_products, dims):
    """Four FP32 power steps through a one-pass kernel in one mode (the FP32
    one with FP32 instructions, the split one, n > 256, with products through
    the BF16 split): the chunk counter is zeroed once at the mode's start and
    every later launch takes its base from the host. Each step's iterate (its
    Sigma(1,1), Sigma(l,l) and shift) matches the oracle's, on a tensor whose
    unfolding spectra decay as 0.9^i (slowly enough that the steps' iterates
    differ), and no launch flags its counter out of step."""
    core = gen.superdiagonal(0.9 ** np.arange(40), (40, 40, 40))
    a, _, _ = gen.random_tucker(dims, (40, 40, 40), 1e-2, seed=64, core=core)
    a32 = a.astype(np.float32)
    x = _dev(a32, torch.float32)
    G, U, info, res = _compare_solve(x, a32.astype(np.float64), (12, 12, 12), 8, 4, "adaptive", "st", "fp32",
                                     check_core=False, fp32_products=fp32_products)
    assert not info["flags"] & T.INFO_INTERNAL
    lg = res.logs[0]
    # the iterates of consecutive steps really differ (a stale partial would repeat one)
    assert len({round(s[-1] / s[0], 6) for s in lg.sigmas[1:]}) == len(lg.sigmas) - 1


# --------------------------------------------------------------- FP32 products through BF16 splits

def test_split_products_match_their_definitions(T):
    """FP32 power step and core contraction at a size where both product
    kernels take the three-piece BF16 split (mode 0 of 64 x 300000: 4688 tiles
    of 64 columns): every entry within 1e-5 of its Cauchy-Schwarz scale of
    the FP64 definitions X_(0)(X_(0)^T Q) and U^T X_(0) (the split keeps 24
    significant bits of each operand; measured about 3e-8 and 2e-7), and
    within the same bound of the FP32-instruction path's result."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    X = torch.randn((64, 300000), generator=g, device=dev, dtype=torch.float32)
    Q = torch.linalg.qr(torch.randn((64, 40), generator=g, device=dev, dtype=torch.float64))[0].float().contiguous()
    alpha = torch.zeros(1, dtype=torch.float64, device=dev)
    M = T.shifted_power(X, 0, Q, alpha, raw=True)
    U = Q[:, :30].contiguous()
    C = T.core(X, 0, U).double()
    X64 = X.double()
    Z = X64.T @ Q.double()
    sc = torch.linalg.vector_norm(X64, dim=1)[:, None] * torch.linalg.vector_norm(Z, dim=0)[None, :]
    err = ((M - X64 @ Z).abs() / sc).max().item()
    print("split power step: max error / scale %.3e" % err, flush=True)
    assert err <= 1e-5
    Cref = U.double().T @ X64
    sc2 = torch.linalg.vector_norm(U.double(), dim=0)[:, None] * torch.linalg.vector_norm(X64, dim=0)[None, :]
    err2 = ((C - Cref).abs() / sc2).max().item()
    print("split core: max error / scale %.3e" % err2, flush=True)
    assert err2 <= 1e-5


@pytest.mark.parametrize("fp32_products", ["split", "native"])
def test_fp32_solve_at_split_sizes_matches_oracle(T, fp32_products):
    """A whole FP32 ST-HOSVD whose mode-0 products run through the BF16 split
    (48 x 96 x 3000: 4500 tiles of 64 columns), and the same solve on the FP32
    instructions only, each against the FP64 oracle on the same tensor and
    test matrices: reconstruction within 1e-5, shifts and singular values,
    subspaces, signed factors and core (the checks of every solve test)."""
    a, _, _ = gen.random_tucker((48, 96, 3000), (6, 8, 10), 1e-3, seed=51)
    a32 = a.astype(np.float32)
    _compare_solve(_dev(a32, torch.float32), a32.astype(np.float64), (6, 8, 10), 6, 2, "adaptive", "st", "fp32",
                   seed=4, fp32_products=fp32_products)


# Shapes that reach the BF16-matrix-core product kernels (FP32 split pieces and
# BF16 operands) on their awkward paths: mode-k views [P, n, S] with a partial
# 32-row batch or n < 32, 32-column tiles cut by S, S a multiple of 32, of 4
# but not 32, and odd; sketch widths of one to four 16-column tiles. Each view
# has at least 4096 tiles of 64 columns, so the row contraction takes the
# split kernel (the column reduction takes it for any S > 1).
_AWKWARD = [
    ((4096, 33, 40), 1, 8), ((4096, 33, 40), 1, 33),
    ((2048, 70, 67), 1, 24), ((2048, 70, 67), 1, 60),
    ((1, 20, 270000), 1, 17),
    ((100, 262208), 0, 60),
    # n > 256: the one-pass power step on the BF16 matrix cores at each staged
    # row count (512, 768, 1024 rows), ragged rows and last blocks, P > 1
    ((300, 40, 36), 0, 24), ((700, 37, 12), 0, 60), ((6, 1000, 44), 1, 40), ((1024, 36, 4), 0, 64),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("dims,mode,l", _AWKWARD)
def test_product_kernels_at_awkward_shapes(T, prec, dims, mode, l):
    """Sketch, raw power step and core contraction against the oracle entry by
    entry, each within its Cauchy-Schwarz scale: FP32 split pieces at the
    FP32 tolerance; BF16 operands (each rounded with relative error at most
    2^-9) within 2^-8 for one product, and for the power step within
    2^-8 (2 + sqrt(n)), the bound for its second product run on a rounded
    first one when X is Gaussian and Q has unit columns."""
    g = gen.rng(21)
    a = g.standard_normal(dims).astype(np.float32)
    x = _dev(a, torch.float32)
    xa = _np(x)
    xk = unfold(xa, mode)
    n = dims[mode]
    one = TOL["fp32"] if prec == "fp32" else 2.0 ** -8
    two = TOL["fp32"] if prec == "fp32" else 2.0 ** -8 * (2.0 + np.sqrt(n))
    print("case", prec, dims, mode, l, flush=True)
    # sketch
    y = _np(T.sketch(x, mode, l, seed=9, precision=prec))
    om = orc_rng.gaussian_omega(9, mode, xk.shape[1], l)
    err = np.abs(y - orc.sketch(xa, mode, om)) / _row_col_scale(xk, om)
    print("  sketch max err/scale %.3e" % err.max(), flush=True)
    assert err.max() <= one
    # raw power step (no shift)
    q0 = np.linalg.qr(g.standard_normal((n, l)))[0]
    q = _dev(q0, torch.float32)
    qa = _np(q)
    al = torch.zeros(1, dtype=torch.float64, device="cuda")
    m = _np(T.shifted_power(x, mode, q, al, raw=True, precision=prec))
    err = np.abs(m - orc.shifted_power(xa, mode, qa, 0.0)) / _power_scale(xk, qa, 0.0)
    print("  power max err/scale %.3e" % err.max(), flush=True)
    assert err.max() <= two
    # core contraction (FP32 products for both: the BF16 path contracts on FP32 operands)
    r = min(l, n)
    u = _dev(q0[:, :r], torch.float32)
    out = _np(T.core(x, mode, u, precision=prec))
    ref = orc.core_step(xa, mode, _np(u))
    ck = unfold(out, mode)
    err = np.abs(ck - unfold(ref, mode)) / _row_col_scale(_np(u).T, xk)
    print("  core max err/scale %.3e" % err.max(), flush=True)
    assert err.max() <= TOL["fp32"]
