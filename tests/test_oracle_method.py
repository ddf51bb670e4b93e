"""Pins for the oracle's method against what the paper and the mathematics fix.

Each test names the fact it checks. A plausible slip in the oracle (a dropped
-alpha Q term, a flipped sign, alpha_t used in place of alpha_{t-1}, Sigma(1,1)
in place of Sigma(l,l), X^T X in place of X X^T, a transposed unfolding, the
wrong tensor fed to ST-HOSVD) fails at least one of them.
"""
import os

import numpy as np
import pytest

from oracle.philox import gaussian_omega
from oracle.rhosvd import (hosvd_full, randomized_hosvd, rel_error, rel_error_identity, sign_fix,
                           svd_econ)
from oracle.tensor import frob2, mode_product, reconstruct, unfold
from workloads.generators import random_tucker, rng, spectrum_c, tensor_c

TABLE3 = os.path.join(os.path.dirname(__file__), "golden", "table3_tensor_c_fast.txt")


def _tail2(x, k, r):
    s = np.linalg.svd(unfold(x, k), compute_uv=False)
    return float(np.sum(s[r:] ** 2))


# ---------------------------------------------------------------- Algorithm 1

@pytest.mark.parametrize("variant", ["t", "st"])
def test_hosvd_tail_bound(variant):
    """Theorem 2.1: ||A - Ahat||^2 <= sum_k sum_{i>r_k} sigma_i(A_(k))^2 (both variants)."""
    for seed in range(4):
        a = rng(seed).standard_normal((7, 8, 9))
        ranks = (3, 4, 2)
        res = hosvd_full(a, ranks, variant)
        err2 = frob2(a - reconstruct(res.core, res.factors))
        bound = sum(_tail2(a, k, ranks[k]) for k in range(3))
        assert err2 <= bound * (1 + 1e-12)
        # Eckart-Young per mode is a lower bound on any Tucker approximation
        assert err2 >= max(_tail2(a, k, ranks[k]) for k in range(3)) * (1 - 1e-12)


# ------------------------------------------------- randomized, exact structure

@pytest.mark.parametrize("variant", ["t", "st"])
@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("shift", ["adaptive", "none"])
def test_exact_tucker_rank_is_recovered(variant, q, shift):
    """rank(A_(k)) <= r_k for an exact Tucker tensor: with l_k >= r_k the method is exact."""
    a, _, _ = random_tucker((12, 10, 11), (3, 4, 2), 0.0, seed=5)
    res = randomized_hosvd(a, (3, 4, 2), p=3, q=q, shift=shift, variant=variant, seed=9)
    assert rel_error(a, res) < 1e-12
    for u in res.factors:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-13)


@pytest.mark.parametrize("variant", ["t", "st"])
def test_identity_and_orthonormal_factors(variant):
    """Ahat is an orthogonal projection of A: ||A - Ahat||^2 = ||A||^2 - ||G||^2."""
    a, _, _ = random_tucker((14, 12, 13), (4, 4, 4), 0.3, seed=6)
    res = randomized_hosvd(a, (4, 3, 5), p=4, q=2, variant=variant, seed=2)
    for u in res.factors:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-13)
    e_explicit = rel_error(a, res)
    e_ident = rel_error_identity(a, res.core)
    assert abs(e_explicit ** 2 - e_ident ** 2) < 1e-13
    # G = A x_1 U_1^T ... x_d U_d^T for both variants
    g = a
    for k, u in enumerate(res.factors):
        g = mode_product(g, u.T, k)
    np.testing.assert_allclose(res.core, g, atol=1e-12)


@pytest.mark.parametrize("variant", ["t", "st"])
@pytest.mark.parametrize("q", [1, 2])
def test_full_width_sketch_equals_deterministic_hosvd(variant, q):
    """l_k = n_k and q >= 1: Q spans R^{n_k} and the iterate's left singular vectors
    are those of X_(k) X_(k)^T, so the method returns Algorithm 1's factors."""
    a = rng(11).standard_normal((5, 6, 7))
    ranks = (2, 3, 2)
    res = randomized_hosvd(a, ranks, p=10, q=q, variant=variant, seed=4)
    ref = hosvd_full(a, ranks, variant)
    for k in range(3):
        if res.logs[k].l == a.shape[k]:
            np.testing.assert_allclose(res.factors[k], ref.factors[k], atol=1e-9)
    if all(res.logs[k].l == a.shape[k] for k in range(3)):
        np.testing.assert_allclose(res.core, ref.core, atol=1e-9)


def test_full_width_shift_closed_form():
    """With l = n the shifted iterate (X X^T - alpha I) Q has singular values
    lambda_i - alpha_{t-1} (lambda = eigenvalues of X X^T), so the midpoint rule
    gives alpha_1 = lambda_n / 2 and then stays there (up to rounding)."""
    a = rng(12).standard_normal((6, 7, 8))
    res = randomized_hosvd(a, (2, 2, 2), p=10, q=4, variant="t", shift="adaptive", seed=3)
    for k in range(3):
        lam = np.sort(np.linalg.eigvalsh(unfold(a, k) @ unfold(a, k).T))[::-1]
        log = res.logs[k]
        assert log.l == a.shape[k]
        assert log.alphas[0] == 0.0
        for t in range(1, 5):
            np.testing.assert_allclose(log.sigmas[t], lam - log.alphas[t - 1], rtol=0, atol=1e-11 * lam[0])
            assert abs(log.alphas[t] - lam[-1] / 2) <= 1e-11 * lam[0]


def test_shift_invariants():
    """alpha_t is nondecreasing and stays in [0, sigma_l(X_(k))^2 / 2] (section 3.1 (a)-(c))."""
    a, _, _ = random_tucker((30, 28, 26), (6, 6, 6), 0.05, seed=13)
    for variant in ("t", "st"):
        res = randomized_hosvd(a, (5, 5, 5), p=5, q=6, variant=variant, seed=8)
        g = a
        for k in range(3):
            x = a if variant == "t" else g
            s = np.linalg.svd(unfold(x, k), compute_uv=False)
            log = res.logs[k]
            al = np.array(log.alphas)
            assert al[0] == 0.0
            assert np.all(np.diff(al) >= 0)
            assert np.all(al <= s[log.l - 1] ** 2 / 2 * (1 + 1e-12))
            assert al[-1] > 0
            g = mode_product(g, res.factors[k].T, k)


@pytest.mark.parametrize("variant", ["t", "st"])
def test_q_le_1_shift_has_no_effect(variant):
    """alpha_0 = 0, so with q <= 1 the adaptive and unshifted runs are bitwise equal."""
    a, _, _ = random_tucker((16, 15, 14), (4, 4, 4), 0.1, seed=14)
    for q in (0, 1):
        r1 = randomized_hosvd(a, (4, 4, 4), p=5, q=q, variant=variant, shift="adaptive", seed=5)
        r2 = randomized_hosvd(a, (4, 4, 4), p=5, q=q, variant=variant, shift="none", seed=5)
        np.testing.assert_array_equal(r1.core, r2.core)
        for u1, u2 in zip(r1.factors, r2.factors):
            np.testing.assert_array_equal(u1, u2)


def test_q_ge_2_shift_changes_the_iterate():
    a, _, _ = random_tucker((16, 15, 14), (4, 4, 4), 0.3, seed=14)
    r1 = randomized_hosvd(a, (4, 4, 4), p=5, q=3, variant="st", shift="adaptive", seed=5)
    r2 = randomized_hosvd(a, (4, 4, 4), p=5, q=3, variant="st", shift="none", seed=5)
    assert np.max(np.abs(r1.core - r2.core)) > 1e-12
    assert all(lg.alphas[-1] > 0 for lg in r1.logs)
    assert all(all(x == 0 for x in lg.alphas) for lg in r2.logs)


def test_unshifted_is_plain_subspace_iteration():
    """Algorithm A.1: with alpha = 0, range(Q_q) = range((X X^T)^q X Omega)."""
    a = rng(15).standard_normal((9, 10, 11))
    q, p, ranks = 2, 3, (3, 3, 3)
    res = randomized_hosvd(a, ranks, p=p, q=q, variant="t", shift="none", seed=6)
    for k in range(3):
        xk = unfold(a, k)
        l = res.logs[k].l
        om = gaussian_omega(6, k, xk.shape[1], l)
        b = xk @ om
        for _ in range(q):
            b = xk @ (xk.T @ b)
        qb = np.linalg.qr(b)[0]
        # the oracle's final Q (all l columns) spans the same space: compare projectors
        qq = _final_q(a, k, ranks[k], p, q, 6)
        assert np.linalg.norm(qb @ qb.T - qq @ qq.T, 2) < 1e-8


def _final_q(a, k, r, p, q, seed):
    xk = unfold(a, k)
    l = min(r + p, xk.shape[0], xk.shape[1])
    qm, _ = svd_econ(xk @ gaussian_omega(seed, k, xk.shape[1], l))
    for _ in range(q):
        qm, _ = svd_econ(xk @ (xk.T @ qm))
    return qm


def test_sign_rule():
    u = np.array([[0.1, -0.9], [-0.8, 0.2], [0.3, 0.9]])
    f = sign_fix(u)
    np.testing.assert_array_equal(f[:, 0], -u[:, 0])       # largest |.| is -0.8 -> flip
    np.testing.assert_array_equal(f[:, 1], -u[:, 1])       # tie |-0.9| = |0.9|: first row wins -> flip


def test_infeasible_rank_rejected():
    a = rng(1).standard_normal((4, 4, 32))
    with pytest.raises(ValueError):
        randomized_hosvd(a, (4, 4, 17), p=2, q=1, variant="t")   # r_3 > n_1 n_2 = 16


def test_sketch_width_clamp():
    a = rng(1).standard_normal((6, 5, 40))
    res = randomized_hosvd(a, (3, 3, 8), p=10, q=1, variant="st", seed=2)
    assert [lg.l for lg in res.logs] == [6, 5, 9]            # n_1, n_2, then m_3 = r_1 r_2 = 9


@pytest.mark.parametrize("variant", ["t", "st"])
def test_soft_tail_bound_randomized(variant):
    """The randomized result with a clear gap stays within 1% of Theorem 2.1's bound."""
    a, _, _ = random_tucker((40, 40, 40), (6, 6, 6), 1e-3, seed=16)
    res = randomized_hosvd(a, (6, 6, 6), p=5, q=1, variant=variant, seed=1)
    err2 = frob2(a - reconstruct(res.core, res.factors))
    bound = sum(_tail2(a, k, 6) for k in range(3))
    assert err2 <= 1.01 * bound
    assert err2 >= max(_tail2(a, k, 6) for k in range(3)) * (1 - 1e-9)
    assert 0.5e-3 < rel_error(a, res) < 2e-3


def _table3():
    out = []
    for line in open(TABLE3):
        line = line.strip()
        if line and not line.startswith("#"):
            r, v = line.split()
            out.append((int(r), v))
    return out


def _matches_print(x, printed):
    """x rounds to the printed three-significant-digit value."""
    mant, exp = printed.split("e")
    scale = 10.0 ** int(exp)
    return abs(x - float(printed)) <= 0.5 * 10 ** -(len(mant.split(".")[1])) * scale + 1e-15


def test_table3_fast_decay_closed_form():
    """Every unfolding of tensor C has singular values v: the optimum RE is a closed form,
    and it is what Table 3 prints for the fast-decay rows."""
    v = spectrum_c("fast", 600)
    for r, printed in _table3():
        re_opt = np.sqrt(np.sum(v[r:] ** 2) / np.sum(v ** 2))
        assert _matches_print(re_opt, printed), (r, re_opt, printed)


def test_table3_fast_decay_reproduced_by_method():
    """Algorithm 3 (s = 10, q = 2) on tensor C (fast decay) reproduces Table 3's RE.
    n = 160 instead of 600: the truncated tail exp(-2*160/7) is far below print precision."""
    a, _ = tensor_c("fast", 160, seed=0)
    for r, printed in _table3():
        res = randomized_hosvd(a, (r, r, r), p=10, q=2, variant="st", shift="adaptive", seed=1)
        re = rel_error(a, res)
        assert _matches_print(re, printed), (r, re, printed)


def test_table3_tensor_c_singular_values():
    """The construction gives unfoldings with singular values exactly v."""
    a, v = tensor_c("sshape", 40, seed=3)
    for k in range(3):
        s = np.linalg.svd(unfold(a, k), compute_uv=False)
        np.testing.assert_allclose(s, v, rtol=0, atol=1e-13)


# --------------------------------------------------------------- Algorithm 4 (PVE-controlled q)

from oracle.rhosvd import pve_converged, randomized_sthosvd_pve  # noqa: E402


def test_pve_stopping_test_by_hand():
    """The stopping test on numbers worked out by hand: r = 2 estimates, the
    third is the reference (tol times sigma_t(r + 1))."""
    sig_t = np.array([10.0, 5.0, 1.0, 0.2])
    sig_hat = np.array([9.9, 5.05, 0.5, 0.1])
    # largest change among the first two estimates: |10 - 9.9| = 0.1; reference sigma_t(3) = 1.0
    assert pve_converged(sig_t, sig_hat, 2, 0.1 + 1e-15)
    assert not pve_converged(sig_t, sig_hat, 2, 0.09)
    # the third estimate (change 0.5) is not among the first r = 2
    assert pve_converged(sig_t, sig_hat, 2, 0.11)
    # l = r: the last estimate stands in for the reference
    assert pve_converged(sig_t[:2], sig_hat[:2], 2, 0.1 / 5.0 + 1e-15)
    assert not pve_converged(sig_t[:2], sig_hat[:2], 2, 0.019)
    # sigma-hat = 0 (first step) passes only when tol >= sigma_1 / sigma_{r+1}
    assert not pve_converged(sig_t, np.zeros(4), 2, 9.99)
    assert pve_converged(sig_t, np.zeros(4), 2, 10.0)


@pytest.mark.parametrize("variant", ["st", "t"])
@pytest.mark.parametrize("shift", ["adaptive", "none"])
def test_pve_tol_zero_is_algorithm_3_with_q_max(shift, variant):
    """tol = 0 never stops early (the estimates of a noisy tensor keep moving):
    q_k = q_max and every result equals Algorithm 3 (the T form: Algorithm 2)
    with q = q_max."""
    a, _, _ = random_tucker((24, 22, 20), (4, 5, 3), 1e-2, seed=31)
    res = randomized_sthosvd_pve(a, (4, 5, 3), 4, 4, 0.0, shift=shift, seed=2, variant=variant)
    ref = randomized_hosvd(a, (4, 5, 3), 4, 4, shift=shift, variant=variant, seed=2)
    assert res.qs == [4, 4, 4]
    assert np.array_equal(res.core, ref.core)
    for u, v in zip(res.factors, ref.factors):
        assert np.array_equal(u, v)
    for lp, lr in zip(res.logs, ref.logs):
        assert lp.alphas == lr.alphas


@pytest.mark.parametrize("variant", ["st", "t"])
def test_pve_unbounded_tol_is_algorithm_3_with_one_step(variant):
    """tol = inf stops after the first power step: q_k = 1 and the result
    equals Algorithm 3 (Algorithm 2) with q = 1."""
    a, _, _ = random_tucker((24, 22, 20), (4, 5, 3), 1e-2, seed=32)
    res = randomized_sthosvd_pve(a, (4, 5, 3), 4, 6, np.inf, seed=2, variant=variant)
    ref = randomized_hosvd(a, (4, 5, 3), 4, 1, variant=variant, seed=2)
    assert res.qs == [1, 1, 1]
    assert np.array_equal(res.core, ref.core)


def test_pve_first_mode_steps_fall_with_tol():
    """Mode 1 runs the same iteration for every tol (only the stop differs), so
    its power count cannot grow as tol grows; a tighter tol never lowers the RE
    reached by much."""
    a, _, _ = random_tucker((40, 36, 32), (6, 6, 6), 5e-2, seed=33)
    prev = None
    for tol in (1e-4, 1e-3, 1e-2, 1e-1, 0.5, 2.0):
        res = randomized_sthosvd_pve(a, (6, 6, 6), 3, 40, tol, seed=5)
        if prev is not None:
            assert res.qs[0] <= prev
        prev = res.qs[0]
        assert 1 <= min(res.qs) and max(res.qs) <= 40


def test_pve_t_form_modes_are_independent():
    """In the T form every mode reads A: mode 3's power count and factor are the
    same whatever ranks the other modes ask for (in the ST form they are not,
    since mode 3 then works on a tensor the other factors contracted)."""
    a, _, _ = random_tucker((20, 18, 16), (4, 3, 5), 5e-2, seed=35)
    r1 = randomized_sthosvd_pve(a, (4, 3, 5), 3, 30, 0.05, seed=9, variant="t")
    r2 = randomized_sthosvd_pve(a, (2, 6, 5), 3, 30, 0.05, seed=9, variant="t")
    assert r1.qs[2] == r2.qs[2]
    assert np.array_equal(r1.factors[2], r2.factors[2])
    s1 = randomized_sthosvd_pve(a, (4, 3, 5), 3, 30, 0.05, seed=9, variant="st")
    s2 = randomized_sthosvd_pve(a, (2, 6, 5), 3, 30, 0.05, seed=9, variant="st")
    assert not np.array_equal(s1.factors[2], s2.factors[2])


def test_pve_reaches_the_q_max_error():
    """With a clear gap, tol = 0.5 stops after few steps at the relative error
    of q_max steps (the paper's observation for its tensors)."""
    a, _, _ = random_tucker((40, 36, 32), (6, 6, 6), 1e-3, seed=34)
    res = randomized_sthosvd_pve(a, (6, 6, 6), 4, 20, 0.5, seed=7)
    full = randomized_hosvd(a, (6, 6, 6), 4, 20, variant="st", seed=7)
    assert max(res.qs) <= 5
    assert abs(rel_error(a, res) - rel_error(a, full)) <= 1e-6 * rel_error(a, full)


# --------------------------------------------------------------- processing order

def test_t_hosvd_does_not_depend_on_the_order():
    """T-HOSVD computes every factor from A itself: any processing order gives
    the same factors and core, bit for bit."""
    a, _, _ = random_tucker((18, 16, 14), (4, 3, 5), 1e-2, seed=51)
    ref = randomized_hosvd(a, (4, 3, 5), 3, 1, variant="t", seed=2)
    res = randomized_hosvd(a, (4, 3, 5), 3, 1, variant="t", seed=2, order=(2, 0, 1))
    assert np.array_equal(res.core, ref.core)
    for u, v in zip(res.factors, ref.factors):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 1, 0), (1, 2, 0), (2, 0, 1)])
def test_st_hosvd_bound_holds_in_every_order(order):
    """ST-HOSVD's error bound ||A - Ahat||^2 <= sum_k sum_{i > r_k}
    sigma_i(A_(k))^2 (the tails of A's own unfoldings) holds whatever the
    processing order; here with a full-width sketch (the deterministic method)."""
    a, _, _ = random_tucker((12, 10, 9), (3, 4, 2), 0.3, seed=52)
    ranks = (3, 4, 2)
    tails = sum(np.sum(np.linalg.svd(unfold(a, k), compute_uv=False)[ranks[k]:] ** 2) for k in range(3))
    res = randomized_hosvd(a, ranks, 20, 0, variant="st", seed=3, order=order)
    err2 = frob2(a - reconstruct(res.core, res.factors))
    assert err2 <= tails * (1 + 1e-12)
    assert res.core.shape == ranks


def test_exact_rank_is_recovered_in_a_permuted_order():
    a, _, _ = random_tucker((14, 12, 10), (3, 4, 2), 0.0, seed=53)
    res = randomized_hosvd(a, (3, 4, 2), 2, 1, variant="st", seed=4, order=(1, 2, 0))
    assert rel_error(a, res) < 1e-12


def test_bad_order_rejected():
    a, _, _ = random_tucker((6, 5, 4), (2, 2, 2), 0.0, seed=54)
    with pytest.raises(ValueError):
        randomized_hosvd(a, (2, 2, 2), 1, 0, order=(0, 0, 1))


def test_decreasing_order():
    from oracle.rhosvd import decreasing_order
    assert decreasing_order((60, 12, 40)) == [0, 2, 1]
    assert decreasing_order((5, 7, 7, 5)) == [1, 2, 0, 3]
    assert decreasing_order((3,)) == [0]
    shape = (9, 30, 30, 2, 31)
    o = decreasing_order(shape)
    assert sorted(o) == list(range(5)) and all(shape[o[i]] >= shape[o[i + 1]] for i in range(4))


# --------------------------------------------------------------- holistic variants (Appendices A, B)

from oracle.rhosvd import randomized_hosvd_holistic  # noqa: E402


@pytest.mark.parametrize("variant", ["t", "st"])
@pytest.mark.parametrize("q,shift", [(0, "adaptive"), (2, "adaptive"), (2, "none")])
def test_holistic_full_width_is_the_deterministic_hosvd(variant, q, shift):
    """With l_k = n_k the range finder spans everything (B is A rotated mode by
    mode), so the holistic result is Algorithm 1's: the same factors after the
    sign rule and the same core."""
    a, _, _ = random_tucker((9, 8, 7), (3, 4, 2), 0.3, seed=61)
    ranks = (3, 4, 2)
    ref = hosvd_full(a, ranks, variant)
    res = randomized_hosvd_holistic(a, ranks, 50, q, shift=shift, variant=variant, seed=5)
    assert [lg.l for lg in res.logs] == [9, 8, 7]
    for u, v in zip(res.factors, ref.factors):
        assert np.max(np.abs(u - v)) < 1e-10
    assert np.max(np.abs(res.core - ref.core)) < 1e-10 * np.linalg.norm(a)


@pytest.mark.parametrize("variant", ["t", "st"])
@pytest.mark.parametrize("shift", ["adaptive", "none"])
def test_holistic_recovers_exact_rank(variant, shift):
    a, _, _ = random_tucker((20, 18, 16), (3, 5, 4), 0.0, seed=62)
    res = randomized_hosvd_holistic(a, (3, 5, 4), 4, 1, shift=shift, variant=variant, seed=6)
    assert rel_error(a, res) < 1e-12
    for u in res.factors:
        assert np.max(np.abs(u.T @ u - np.eye(u.shape[1]))) < 1e-12


def test_holistic_unshifted_spans_as_orth_iteration():
    """Algorithm A.2 orthonormalises every iterate with a QR factorisation; with
    alpha = 0 the SVD-based steps span the same columns. In the T-HOSVD form
    every mode reads A, so the Q_k differ only by a rotation inside their span,
    which phase 2 absorbs: an independent QR form of phase 1 followed by
    Algorithm 1 of the small tensor gives the same approximation. (In the
    ST-HOSVD form the rotation of Q_k changes the coordinates the next mode's
    test matrix multiplies, so only the distribution agrees.)"""
    a, _, _ = random_tucker((16, 14, 12), (4, 3, 5), 0.1, seed=63)
    ranks, p, q = (4, 3, 5), 3, 2
    res = randomized_hosvd_holistic(a, ranks, p, q, shift="none", variant="t", seed=7)
    from oracle.philox import gaussian_omega
    from oracle.tensor import mode_product
    qs = []
    for k in range(3):
        xk = unfold(a, k)
        l_k = min(ranks[k] + p, xk.shape[0], xk.shape[1])
        qm, _ = np.linalg.qr(xk @ gaussian_omega(7, k, xk.shape[1], l_k))
        for _ in range(q):
            qm, _ = np.linalg.qr(xk @ (xk.T @ qm))
        qs.append(qm)
    b = a
    for k in range(3):
        b = mode_product(b, qs[k].T, k)
    small = hosvd_full(b, ranks, "t")
    ahat_qr = reconstruct(small.core, [qm @ v for qm, v in zip(qs, small.factors)])
    assert np.linalg.norm(reconstruct(res.core, res.factors) - ahat_qr) < 1e-10 * np.linalg.norm(a)


def test_holistic_projection_identity_and_order():
    a, _, _ = random_tucker((15, 13, 11), (4, 3, 3), 0.05, seed=64)
    res = randomized_hosvd_holistic(a, (4, 3, 3), 4, 1, variant="st", seed=8, order=(2, 0, 1))
    assert abs(rel_error(a, res) - rel_error_identity(a, res.core)) < 1e-10
    t0 = randomized_hosvd_holistic(a, (4, 3, 3), 4, 1, variant="t", seed=8)
    t1 = randomized_hosvd_holistic(a, (4, 3, 3), 4, 1, variant="t", seed=8, order=(1, 2, 0))
    assert np.array_equal(t0.core, t1.core)
