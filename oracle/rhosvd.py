"""The method, step by step in FP64: shifted randomized T-HOSVD / ST-HOSVD.

TEST INFRASTRUCTURE ONLY (see the package header).

Follows, in the paper's order and notation:
  * Algorithm 1 (deterministic T-HOSVD / ST-HOSVD): ``hosvd_full``.
  * Algorithm 2 (shifted randomized T-HOSVD) and Algorithm 3 (shifted
    randomized ST-HOSVD): ``randomized_hosvd`` with variant "t" / "st" and
    shift "adaptive".
  * Appendix Algorithm A.1 (the unshifted randomized model): the same routine
    with shift "none" (alpha stays 0).
  * Algorithm 4 (Algorithm 3 with the power count of each mode chosen by the
    per-vector-error criterion): ``randomized_sthosvd_pve``.
  * Appendix Algorithms A.2 and B.1 (the holistic variants: range finders
    kept at width l_k, then a deterministic HOSVD of the small tensor):
    ``randomized_hosvd_holistic``.

Per mode k, on X = A (variant t) or X = the partially contracted core
(variant st, dims r_1..r_{k-1}, n_k..n_d):
  l_k   = min(r_k + p, n_k, m_k)             (oversampling p; clamp, see below)
  Y     = X_(k) Omega_k ;  [Q, Sigma] = svd(Y, econ) ;  alpha_0 = 0
  for t = 1..q:
      M = X_(k) (X_(k)^T Q) - alpha_{t-1} Q ; [Q, Sigma] = svd(M, econ)
      if Sigma(l_k, l_k) > alpha_{t-1}: alpha_t = (Sigma(l_k, l_k) + alpha_{t-1}) / 2
      else alpha_t = alpha_{t-1}
  U_k = Q(:, 1:r_k) ;  G <- G x_k U_k^T

Readings where the paper is silent or loose:
  * Algorithm 3 writes the shift in the power step without its subscript; it
    is alpha_{t-1}, as in Algorithm 2.
  * The else-branch of the shift update is not written: alpha_t = alpha_{t-1}.
  * Sigma(l, l) is the l-th (smallest) singular value of the shifted iterate M.
  * q = 0 is allowed (no power step; U_k from svd(X_(k) Omega_k)).
  * l_k is clamped to min(r_k + p, n_k, m_k): the paper assumes l_k below both.
  * svd returns singular values in descending order; U_k's column signs are
    fixed by ``sign_fix`` (largest-magnitude entry of each column positive,
    ties to the lowest row index).
  * Processing order (1, ..., d), as in the paper's experiments.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import numpy as np

from .philox import gaussian_omega
from .tensor import frob2, mode_product, reconstruct, unfold


def svd_econ(y: np.ndarray):
    """[Q, Sigma, ~] = svd(Y, 'econ'), descending Sigma (LAPACK)."""
    q, s, _ = np.linalg.svd(y, full_matrices=False)
    return q, s


def column_signs(u: np.ndarray) -> np.ndarray:
    """Sign of each column's largest-|.| entry (first on ties; +1 for a zero column)."""
    idx = np.argmax(np.abs(u), axis=0)
    s = np.sign(u[idx, np.arange(u.shape[1])])
    s[s == 0] = 1.0
    return s


def sign_fix(u: np.ndarray) -> np.ndarray:
    """Flip columns so each column's largest-|.| entry is positive (first on ties)."""
    u = np.array(u, dtype=np.float64, copy=True)
    if u.size == 0:
        return u
    return u * column_signs(u)[None, :]


def sketch_width(r: int, p: int, n: int, m: int) -> int:
    return int(min(r + p, n, m))


def sketch(x: np.ndarray, k: int, omega: np.ndarray) -> np.ndarray:
    """Y = X_(k) Omega_k."""
    return unfold(x, k) @ omega


def shifted_power(x: np.ndarray, k: int, q_mat: np.ndarray, alpha: float) -> np.ndarray:
    """M = X_(k) (X_(k)^T Q) - alpha Q."""
    xk = unfold(x, k)
    return xk @ (xk.T @ q_mat) - alpha * q_mat


def shift_update(alpha: float, sigma_l: float) -> float:
    """Midpoint rule: move alpha halfway to Sigma(l,l) when that is larger."""
    return (sigma_l + alpha) / 2.0 if sigma_l > alpha else alpha


def core_step(x: np.ndarray, k: int, u: np.ndarray) -> np.ndarray:
    """X x_k U^T."""
    return mode_product(x, u.T, k)


@dataclasses.dataclass
class ModeLog:
    l: int
    m: int
    alphas: List[float]            # alpha_0 .. alpha_q
    sigmas: List[np.ndarray]       # Sigma after the sketch svd and after each power step


@dataclasses.dataclass
class Result:
    core: np.ndarray
    factors: List[np.ndarray]
    logs: List[ModeLog]


OmegaProvider = Callable[[int, int, int], np.ndarray]


def decreasing_order(shape: Sequence[int]) -> List[int]:
    """The processing order of the cost count in Section 3.2: the modes by
    decreasing size n_{p_1} >= ... >= n_{p_d}; equal sizes keep increasing mode."""
    return sorted(range(len(shape)), key=lambda k: -int(shape[k]))


def randomized_hosvd(a: np.ndarray, ranks: Sequence[int], p: int, q: int, *,
                     shift: str = "adaptive", variant: str = "st", seed: int = 1,
                     omega: Optional[OmegaProvider] = None, order: Optional[Sequence[int]] = None) -> Result:
    """Algorithm 2 (variant 't') / Algorithm 3 (variant 'st'); shift 'none' = Algorithm A.1.
    `order` is the processing order (a permutation of the modes; default
    1..d): ST-HOSVD contracts the modes in that order, T-HOSVD is unaffected.
    Factors and logs stay indexed by mode; Omega_k is mode k's whatever the order."""
    if shift not in ("adaptive", "none") or variant not in ("t", "st"):
        raise ValueError("bad shift or variant")
    a = np.asarray(a, dtype=np.float64)
    d = a.ndim
    order = list(range(d)) if order is None else [int(k) for k in order]
    if sorted(order) != list(range(d)):
        raise ValueError("order must be a permutation of the modes")
    g = a.copy()
    factors: List[Optional[np.ndarray]] = [None] * d
    logs: List[Optional[ModeLog]] = [None] * d
    for k in order:
        x = a if variant == "t" else g
        n_k = x.shape[k]
        m_k = x.size // n_k
        r_k = int(ranks[k])
        if not (1 <= r_k <= n_k and r_k <= m_k):
            raise ValueError("infeasible rank at mode %d" % k)
        l_k = sketch_width(r_k, p, n_k, m_k)
        om = omega(k, m_k, l_k) if omega is not None else gaussian_omega(seed, k, m_k, l_k)
        qm, s = svd_econ(sketch(x, k, om))
        alpha = 0.0
        alphas, sigmas = [alpha], [s]
        for _t in range(q):
            qm, s = svd_econ(shifted_power(x, k, qm, alpha))
            if shift == "adaptive":
                alpha = shift_update(alpha, s[l_k - 1])
            alphas.append(alpha)
            sigmas.append(s)
        u_k = sign_fix(qm[:, :r_k])
        factors[k] = u_k
        if variant == "st":
            g = core_step(g, k, u_k)
        logs[k] = ModeLog(l_k, m_k, alphas, sigmas)
    if variant == "t":  # the core of T-HOSVD: A x_k U_k^T over the modes in order
        g = a
        for k in range(d):
            g = core_step(g, k, factors[k])
    return Result(g, factors, logs)


@dataclasses.dataclass
class PveResult(Result):
    qs: List[int] = dataclasses.field(default_factory=list)   # power steps taken per mode


def pve_converged(sig_t: np.ndarray, sig_hat: np.ndarray, r: int, tol: float) -> bool:
    """Algorithm 4's stopping test: the largest change of the first r_k
    estimates sigma_t(i) = Sigma(i,i) + alpha_{t-1} since the previous step is
    at most tol times the (r_k+1)-th estimate (the l_k-th when l_k = r_k)."""
    ref = sig_t[min(r, len(sig_t) - 1)]
    return float(np.max(np.abs(sig_t[:r] - sig_hat[:r]))) <= tol * ref


def randomized_sthosvd_pve(a: np.ndarray, ranks: Sequence[int], p: int, q_max: int, tol: float, *,
                           shift: str = "adaptive", seed: int = 1,
                           omega: Optional[OmegaProvider] = None, variant: str = "st") -> PveResult:
    """Algorithm 4: shifted randomized ST-HOSVD whose power count q_k per mode
    stops at the first t <= q_max that passes ``pve_converged`` (the test comes
    before the shift update; sigma-hat starts at zero, so t = 1 passes only for
    an unbounded tol). shift "none" keeps alpha at zero. variant "t" is the
    T-HOSVD form the paper names Algorithm 2-v3 (details omitted there): every
    mode from A, the core A x_1 U_1^T ... x_d U_d^T at the end.

    Readings: the printed test's right-hand side is garbled; it is read as tol
    times sigma_t(r_k + 1), the first discarded estimate, and sigma_t(l_k) stands
    in when l_k = r_k. q_max >= 1."""
    if shift not in ("adaptive", "none") or variant not in ("t", "st"):
        raise ValueError("bad shift or variant")
    if q_max < 1:
        raise ValueError("q_max must be at least 1")
    a = np.asarray(a, dtype=np.float64)
    g = a.copy()
    factors: List[np.ndarray] = []
    logs: List[ModeLog] = []
    qs: List[int] = []
    for k in range(a.ndim):
        x = a if variant == "t" else g
        n_k = x.shape[k]
        m_k = x.size // n_k
        r_k = int(ranks[k])
        if not (1 <= r_k <= n_k and r_k <= m_k):
            raise ValueError("infeasible rank at mode %d" % k)
        l_k = sketch_width(r_k, p, n_k, m_k)
        om = omega(k, m_k, l_k) if omega is not None else gaussian_omega(seed, k, m_k, l_k)
        qm, s = svd_econ(sketch(x, k, om))
        alpha = 0.0
        sig_hat = np.zeros(l_k)
        alphas, sigmas = [alpha], [s]
        q_k = 0
        for _t in range(q_max):
            q_k += 1
            qm, s = svd_econ(shifted_power(x, k, qm, alpha))
            sig_t = s + alpha
            sigmas.append(s)
            if pve_converged(sig_t, sig_hat, r_k, tol):
                alphas.append(alpha)
                break
            if shift == "adaptive":
                alpha = shift_update(alpha, s[l_k - 1])
            alphas.append(alpha)
            sig_hat = sig_t
        u_k = sign_fix(qm[:, :r_k])
        factors.append(u_k)
        g = core_step(g, k, u_k)   # T-HOSVD: the same contractions of A, in mode order
        logs.append(ModeLog(l_k, m_k, alphas, sigmas))
        qs.append(q_k)
    return PveResult(g, factors, logs, qs)


def hosvd_full(a: np.ndarray, ranks: Sequence[int], variant: str = "st") -> Result:
    """Algorithm 1: U_k from the full econ SVD of A_(k) (T) or G_(k) (ST)."""
    a = np.asarray(a, dtype=np.float64)
    g = a.copy()
    factors, logs = [], []
    for k in range(a.ndim):
        x = a if variant == "t" else g
        qm, s = svd_econ(unfold(x, k))
        u_k = sign_fix(qm[:, :int(ranks[k])])
        factors.append(u_k)
        g = core_step(g, k, u_k)
        logs.append(ModeLog(qm.shape[1], x.size // x.shape[k], [0.0], [s]))
    return Result(g, factors, logs)


def randomized_hosvd_holistic(a: np.ndarray, ranks: Sequence[int], p: int, q: int, *,
                              shift: str = "adaptive", variant: str = "st", seed: int = 1,
                              omega: Optional[OmegaProvider] = None,
                              order: Optional[Sequence[int]] = None) -> Result:
    """The holistic variants of Appendices A and B: Algorithm B.1 (variant 'st',
    shift 'adaptive'), its unshifted model Algorithm A.2 (shift 'none'), and the
    T-HOSVD analogue the paper names but does not print (variant 't').

    Phase 1, per mode k in the processing order, on X = A (variant t) or on the
    partially contracted tensor B (variant st, modes processed before k have
    size l_j): the range finder of Algorithms 2 / 3 with l_k = min(r_k + p, n_k,
    m_k) columns, all kept, with the sign rule: Q_k (n_k x l_k). Variant st contracts
    B <- B x_k Q_k^T at once; variant t forms B = A x_1 Q_1^T ... x_d Q_d^T
    after the loop.
    Phase 2, on the small tensor B (l_1 x ... x l_d): the deterministic
    ST-HOSVD (variant st) or T-HOSVD (variant t, the revision the paper allows
    for that step) with ranks r, in the same processing order: V_k = the
    leading r_k left singular vectors of C_(k) (C = B for t, B contracted by
    the V_j of the modes before k for st); U_k = Q_k V_k with the sign rule,
    V_k's columns flipped with U_k's; G = B x_1 V_1^T ... x_d V_d^T.

    Readings: Algorithm B.1 orthonormalises the sketch without an SVD and
    starts from alpha_0 = 0; an SVD spans the same columns and, for q >= 1,
    the last step's SVD fixes Q_k whatever basis the earlier steps used, so
    the first step here is the one of Algorithms 2 / 3. Algorithm A.2 takes
    every Q_k from an orthonormalisation; here Q_k is the last iterate's left
    singular vectors (the same span; in the ST form another basis changes the
    coordinates the next mode's test matrix multiplies, so the two agree in
    distribution). For the same reason Q_k takes the sign rule before the
    contraction: its column signs set the next test matrix's coordinates, and
    the sign rule makes them independent of the SVD routine. Logs are those of
    phase 1."""
    if shift not in ("adaptive", "none") or variant not in ("t", "st"):
        raise ValueError("bad shift or variant")
    a = np.asarray(a, dtype=np.float64)
    d = a.ndim
    order = list(range(d)) if order is None else [int(k) for k in order]
    if sorted(order) != list(range(d)):
        raise ValueError("order must be a permutation of the modes")
    b = a.copy()
    qs: List[Optional[np.ndarray]] = [None] * d
    logs: List[Optional[ModeLog]] = [None] * d
    for k in order:
        x = a if variant == "t" else b
        n_k = x.shape[k]
        m_k = x.size // n_k
        r_k = int(ranks[k])
        if not (1 <= r_k <= n_k and r_k <= m_k):
            raise ValueError("infeasible rank at mode %d" % k)
        l_k = sketch_width(r_k, p, n_k, m_k)
        om = omega(k, m_k, l_k) if omega is not None else gaussian_omega(seed, k, m_k, l_k)
        qm, s = svd_econ(sketch(x, k, om))
        alpha = 0.0
        alphas, sigmas = [alpha], [s]
        for _t in range(q):
            qm, s = svd_econ(shifted_power(x, k, qm, alpha))
            if shift == "adaptive":
                alpha = shift_update(alpha, s[l_k - 1])
            alphas.append(alpha)
            sigmas.append(s)
        qs[k] = sign_fix(qm)
        if variant == "st":
            b = core_step(b, k, qs[k])
        logs[k] = ModeLog(l_k, m_k, alphas, sigmas)
    if variant == "t":
        for k in range(d):
            b = core_step(b, k, qs[k])
    # phase 2: the deterministic (S)T-HOSVD of B
    c = b.copy()
    factors: List[Optional[np.ndarray]] = [None] * d
    vs: List[Optional[np.ndarray]] = [None] * d
    for k in order:
        x = b if variant == "t" else c
        r_k = int(ranks[k])
        if r_k > min(x.shape[k], x.size // x.shape[k]):
            raise ValueError("infeasible rank at mode %d in the small tensor" % k)
        vm, _ = svd_econ(unfold(x, k))
        v_k = vm[:, :r_k]
        u_k = qs[k] @ v_k
        sg = column_signs(u_k)
        factors[k] = u_k * sg[None, :]
        vs[k] = v_k * sg[None, :]
        if variant == "st":
            c = core_step(c, k, vs[k])
    if variant == "t":
        c = b
        for k in range(d):
            c = core_step(c, k, vs[k])
    return Result(c, factors, logs)


def rel_error(a: np.ndarray, res: Result) -> float:
    """RE = ||A - Ahat|| / ||A|| with Ahat = G x_1 U_1 ... x_d U_d, formed explicitly."""
    ahat = reconstruct(res.core, res.factors)
    return float(np.sqrt(frob2(a - ahat) / frob2(a)))


def rel_error_identity(a: np.ndarray, core: np.ndarray) -> float:
    """RE via ||A - Ahat||^2 = ||A||^2 - ||G||^2 (orthonormal factors)."""
    na, ng = frob2(a), frob2(core)
    return float(np.sqrt(max(na - ng, 0.0) / na))
