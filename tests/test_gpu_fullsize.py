"""Parity at the benchmark's full sizes, through the C ABI, in the launch
configuration the benchmark times (the same entry points, split policies and
grids as the solves' own products):

* the products of the first mode (sketch, raw shifted power step, core
  contraction) at 400^3 FP32, 1000^3 FP32 and 120^4 with BF16 operands, on
  sampled outputs that the oracle's definitions compute one by one;
* whole solves: the 400^3 Hilbert solve against the FP64 oracle's solve of the
  same tensor and test matrices; the 1000^3 and 120^4 Tucker-plus-noise solves
  against what their construction fixes at any size (orthonormal factors, and a
  relative error equal to the noise level eta, since the signal has exactly the
  requested Tucker rank);
* one full serving batch (256 requests of the serving distribution) against
  one-request solves and, for a sample, the oracle.
"""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from oracle import philox as orc_rng  # noqa: E402
from oracle import rhosvd as orc  # noqa: E402
from oracle.tensor import reconstruct  # noqa: E402
from workloads import generators as gen  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_04840_amd import _lib
    return _lib


def _say(*a):
    print(*a, flush=True)


def _np(t):
    return t.detach().double().cpu().numpy()


def _orthonormal(n, r, seed, dtype):
    q = np.linalg.qr(gen.rng(seed).standard_normal((n, r)))[0]
    return torch.from_numpy(q).to(device="cuda", dtype=dtype)


def _row_col_scale(xr, b):
    """Cauchy-Schwarz scale of the entries of xr @ b: row norms times column norms."""
    return np.sqrt(np.sum(xr ** 2, axis=1))[:, None] * np.sqrt(np.sum(b ** 2, axis=0))[None, :]


def _sampled_products(T, A, l, rows, cols, prec, tol, om_full=None):
    """Mode-0 sketch and core of A (device, row-major) on sampled outputs."""
    n = A.shape[0]
    m = A.numel() // n
    x_rows = A.reshape(n, m)[rows].double().cpu().numpy()
    _say("sketch", tuple(A.shape), "l", l, prec)
    y = _np(T.sketch(A, 0, l, seed=1, precision=prec))
    om = om_full[:, cols] if om_full is not None else orc_rng.gaussian_block(1, 0, np.arange(m), cols)
    ref = x_rows @ om
    scale = np.sqrt(np.sum(x_rows ** 2, axis=1))[:, None] * np.sqrt(np.sum(om ** 2, axis=0))[None, :]
    got = y[np.ix_(rows, cols)]
    assert np.all(np.abs(got - ref) <= tol * scale), np.max(np.abs(got - ref) / scale)
    # core: out(j, s) = sum_i U(i, j) X(i, s) at sampled s, all j
    r = min(l, n)
    U = _orthonormal(n, r, 7, A.dtype if A.dtype != torch.bfloat16 else torch.float32)
    _say("core", tuple(A.shape), "r", r)
    out = T.core(A, 0, U, precision=prec if prec != "bf16" else "fp32")
    ss = np.array([0, 1, m // 3, m - 2, m - 1])
    x_cols = A.reshape(n, m)[:, torch.from_numpy(ss).to("cuda")].double().cpu().numpy()
    u = _np(U)
    ref_c = u.T @ x_cols
    got_c = _np(out.reshape(r, m)[:, torch.from_numpy(ss).to("cuda")])
    scale_c = np.sqrt(np.sum(x_cols ** 2, axis=0))[None, :]
    assert np.all(np.abs(got_c - ref_c) <= 1e-5 * scale_c), np.max(np.abs(got_c - ref_c) / scale_c)


def test_hilbert3_400_products_sampled(T):
    """400^3 FP32, mode 0, l = 40: sketch, core, and the raw shifted power step
    (whose inner product X^T Q the oracle forms in full)."""
    A = gen.build_on_device("hilbert3_400", torch.device("cuda:0"))
    rows = np.array([0, 1, 57, 200, 398, 399])
    om = orc_rng.gaussian_omega(1, 0, 400 * 400, 40)
    _sampled_products(T, A, 40, rows, np.arange(40), "fp32", 1e-5, om_full=om)
    _say("power step 400^3")
    Q = _orthonormal(400, 40, 5, torch.float32)
    alpha = 0.25
    al = torch.tensor([alpha], dtype=torch.float64, device="cuda")
    m = _np(T.shifted_power(A, 0, Q, al, raw=True, precision="fp32"))
    xk = A.reshape(400, -1).double().cpu().numpy()
    qa = _np(Q)
    z = xk.T @ qa
    ref = xk[rows] @ z - alpha * qa[rows]
    scale = _row_col_scale(xk[rows], z) + alpha * np.abs(qa[rows])
    assert np.all(np.abs(m[rows] - ref) <= 1e-5 * scale), np.max(np.abs(m[rows] - ref) / scale)


def test_hilbert3_400_solve_matches_oracle(T):
    """The benchmark's default solve (ST, r = 30, p = 10, q = 3, adaptive, FP32)
    against the FP64 oracle on the same tensor and test matrices."""
    A = gen.build_on_device("hilbert3_400", torch.device("cuda:0"))
    _say("solve hilbert3_400")
    s = T.Solver(A.shape, (30, 30, 30), 10, 3, "adaptive", 1, "fp32", True, A.device)
    G, U = s.run(A)
    torch.cuda.synchronize()
    a = A.double().cpu().numpy()
    res = orc.randomized_hosvd(a, (30, 30, 30), 10, 3, shift="adaptive", variant="st", seed=1)
    g, us = _np(G), [_np(u) for u in U]
    na = np.linalg.norm(a)
    assert np.linalg.norm(reconstruct(g, us) - reconstruct(res.core, res.factors)) / na <= 1e-5
    for u in us:
        assert np.max(np.abs(u.T @ u - np.eye(30))) < 1e-5


def _explicit_rel_error(A, G, U):
    """||A - G x_1 U_1 ... x_d U_d|| / ||A||, formed explicitly on the device in
    FP64 slabs of mode 0 (measurement of a result, not part of the oracle)."""
    Gd, Ud = G.double(), [u.double() for u in U]
    core12 = Gd
    for k in range(1, len(Ud)):
        core12 = torch.movedim(torch.tensordot(Ud[k], core12, dims=([1], [k])), 0, k)
    num = den = 0.0
    for i0 in range(0, A.shape[0], 100):
        i1 = min(A.shape[0], i0 + 100)
        ahat = torch.tensordot(Ud[0][i0:i1], core12, dims=([1], [0]))
        slab = A[i0:i1].double()
        num += float(torch.sum((slab - ahat) ** 2))
        den += float(torch.sum(slab ** 2))
    return (num / den) ** 0.5


def _noise_level_solve(T, name, ranks, p, q, prec, eta, re_tol):
    A = gen.build_on_device(name, torch.device("cuda:0"))
    _say("solve", name, prec)
    s = T.Solver(A.shape, ranks, p, q, "adaptive", 1, prec, True, A.device)
    G, U = s.run(A)
    torch.cuda.synchronize()
    for u in U:
        ud = u.double()
        assert float(torch.max(torch.abs(ud.T @ ud - torch.eye(ud.shape[1], device=ud.device, dtype=ud.dtype)))) < 1e-5
    assert bool(torch.isfinite(G).all())
    re = _explicit_rel_error(A, G, U)
    _say(name, "RE", re)
    assert abs(re - eta) <= re_tol * eta, re


def test_tucker3_1000_products_sampled(T):
    A = gen.build_on_device("tucker3_1000", torch.device("cuda:0"))
    _sampled_products(T, A, 60, np.array([0, 499, 999]), np.array([0, 17, 59]), "fp32", 1e-5)


def test_tucker3_1000_solve_reaches_the_noise_level(T):
    """1000^3 FP32, r = 50, p = 10, q = 3: the signal has Tucker rank 50, so the
    relative error equals eta = 1e-4 (to 1 %)."""
    _noise_level_solve(T, "tucker3_1000", (50, 50, 50), 10, 3, "fp32", 1e-4, 0.01)


def test_tucker4_120_products_sampled_bf16(T):
    """120^4, mode 0, l = 30, BF16 operands with FP32 accumulation: within the
    BF16 rounding of both operands (2^-8 each, relative to the row and column
    norms)."""
    A = gen.build_on_device("tucker4_120", torch.device("cuda:0"))
    n = 120
    m = A.numel() // n
    rows, cols = np.array([0, 60, 119]), np.array([0, 29])
    _say("sketch bf16 120^4")
    y = _np(T.sketch(A, 0, 30, seed=1, precision="bf16"))
    x_rows = A.reshape(n, m)[rows].double().cpu().numpy()
    om = orc_rng.gaussian_block(1, 0, np.arange(m), cols)
    ref = x_rows @ om
    scale = np.sqrt(np.sum(x_rows ** 2, axis=1))[:, None] * np.sqrt(np.sum(om ** 2, axis=0))[None, :]
    assert np.all(np.abs(y[np.ix_(rows, cols)] - ref) <= 2 * 2.0 ** -8 * scale)


def test_tucker3_1000_power_step_sampled(T):
    """1000^3 FP32, mode 0, l = 60: the raw shifted power step the solve runs
    at n = 1000, on sampled rows, against the oracle's definition
    X_(0)(X_(0)^T Q) - alpha Q with X_(0)^T Q formed in full (FP64, in column
    slabs), per entry within 1e-5 of the row norm of X_(0) times the column
    norm of X_(0)^T Q."""
    A = gen.build_on_device("tucker3_1000", torch.device("cuda:0"))
    n, l, alpha = 1000, 60, 3e-3
    Q = _orthonormal(n, l, 9, torch.float32)
    al = torch.tensor([alpha], dtype=torch.float64, device="cuda")
    _say("power step 1000^3")
    got = _np(T.shifted_power(A, 0, Q, al, raw=True, precision="fp32"))
    qa = _np(Q)
    rows = np.array([0, 1, 333, 500, 998, 999])
    X = A.reshape(n, -1)
    m = X.shape[1]
    xr = X[torch.from_numpy(rows).to("cuda")].double().cpu().numpy()
    acc = np.zeros((len(rows), l))
    zn2 = np.zeros(l)
    for c0 in range(0, m, 100000):
        xs = X[:, c0:c0 + 100000].double().cpu().numpy()
        z = xs.T @ qa
        acc += xr[:, c0:c0 + 100000] @ z
        zn2 += np.sum(z ** 2, axis=0)
    ref = acc - alpha * qa[rows]
    scale = np.sqrt(np.sum(xr ** 2, axis=1))[:, None] * np.sqrt(zn2)[None, :] + alpha * np.abs(qa[rows])
    err = np.abs(got[rows] - ref)
    assert np.all(err <= 1e-5 * scale), np.max(err / scale)


def _recon_distance(g1, u1, g2, u2):
    """||G1 x_k U1_k - G2 x_k U2_k||_F from the cores and factors (FP64): the
    squared norms and the inner product are contractions in the core space,
    <A1, A2> = <G1, G2 x_k (U1_k^T U2_k)>."""
    def inner(ga, ua, gb, ub):
        t = gb
        for k in range(len(ua)):
            t = np.moveaxis(np.tensordot(ua[k].T @ ub[k], t, axes=([1], [k])), 0, k)
        return float(np.sum(ga * t))
    d2 = inner(g1, u1, g1, u1) + inner(g2, u2, g2, u2) - 2.0 * inner(g1, u1, g2, u2)
    return max(d2, 0.0) ** 0.5


def test_tucker4_120_bf16_solve_matches_oracle(T):
    """120^4 with BF16 operands (r = 20, p = 10, q = 2): the FP64 oracle's solve
    of the same stored tensor and test matrices. The last step runs on FP32
    operands, so the approximation matches the oracle's to the FP32
    tolerance: reconstruction within 1e-5 of ||A||, relative error within 1e-6,
    and the solve's own norms and identity-form error match the oracle's."""
    A = gen.build_on_device("tucker4_120", torch.device("cuda:0"))
    ranks = (20, 20, 20, 20)
    _say("solve tucker4_120 bf16")
    G, U, info = T.rsthosvd(A, ranks, p=10, q=2, seed=1, precision="bf16")
    torch.cuda.synchronize()
    a = A.double().cpu().numpy()
    _say("oracle tucker4_120")
    res = orc.randomized_hosvd(a, ranks, 10, 2, shift="adaptive", variant="st", seed=1)
    g, us = _np(G), [_np(u) for u in U]
    na2 = orc.frob2(a)
    d = _recon_distance(g, us, res.core, res.factors) / na2 ** 0.5
    _say("reconstruction distance", d)
    assert d <= 1e-5, d
    re_o = orc.rel_error(a, res)
    del a
    re_g = _explicit_rel_error(A, G, U)
    _say("RE gpu", re_g, "oracle", re_o, "info", info["rel_error"])
    assert abs(re_g - re_o) <= 1e-6, (re_g, re_o)
    assert abs(info["normA2"] - na2) <= 1e-12 * na2
    assert abs(info["rel_error"] ** 2 - (1.0 - orc.frob2(res.core) / na2)) <= 4e-5


def test_tucker4_120_solve_reaches_the_noise_level(T):
    """120^4, r = 20, p = 10, q = 2, BF16 operands (the last step on FP32
    operands): the relative error equals eta = 1e-2 (to 0.5 %)."""
    _noise_level_solve(T, "tucker4_120", (20, 20, 20, 20), 10, 2, "bf16", 1e-2, 0.005)


def test_serving_full_batch(T):
    """One batch at the serving capacity (256 requests of the serving
    distribution): every request's relative error equals its one-request solve's
    to 1e-6 relative, and a sample matches the FP64 oracle."""
    from paper_2506_04840_amd import serve
    reqs = gen.request_stream(256, 0.0, seed=0, n_lo=32, n_hi=256, r_lo=4, r_hi=32)
    dev = torch.device("cuda:0")
    jobs = [serve.Job(r.rid, gen.request_tensor_device(r, dev), r.ranks, r.seed, 0.0).prepare(8, 1) for r in reqs]
    _say("batch of", len(jobs))
    solver = T.BatchSolver(256, 3, 1, 8, 48, 4 << 30, "adaptive", "cuda:0")
    solver.plan([j.item for j in jobs])
    solver.step()
    torch.cuda.synchronize()

    def rel(A, G, U):
        Ad = A.double()
        ahat = G.double()
        for k, u in enumerate(U):
            ahat = torch.movedim(torch.tensordot(u.double(), ahat, dims=([1], [k])), 0, k)
        return float(torch.linalg.vector_norm(Ad - ahat) / torch.linalg.vector_norm(Ad))

    for i, j in enumerate(jobs):
        Gs, Us, _ = T.rsthosvd(j.A, j.ranks, p=8, q=1, shift="adaptive", seed=j.seed, precision="fp32")
        rb, rs = rel(j.A, j.G, j.U), rel(j.A, Gs, Us)
        assert abs(rb - rs) <= 1e-6 * rs + 1e-9, (i, rb, rs)
    for i in (0, 77, 255):
        j = jobs[i]
        _say("oracle request", i, tuple(j.A.shape), j.ranks)
        a = j.A.double().cpu().numpy()
        res = orc.randomized_hosvd(a, j.ranks, 8, 1, shift="adaptive", variant="st", seed=j.seed)
        rec = reconstruct(_np(j.G), [_np(u) for u in j.U])
        assert np.linalg.norm(rec - reconstruct(res.core, res.factors)) / np.linalg.norm(a) <= 1e-5
