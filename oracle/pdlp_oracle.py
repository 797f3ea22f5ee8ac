"""Plain FP64 CPU oracle of the PDLP path (Applegate et al., "Practical Large-Scale Linear
Programming using Primal-Dual Hybrid Gradient").

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct reference the HIP
solver is checked against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does.  It shares no code with the HIP
solver: everything here is written from the paper with NumPy / SciPy.sparse in float64.

Every function names the passage it follows.  Where the paper is silent or inconsistent the
reading taken is stated in the docstring with a short tag (Zn / Rn) that the design notes list.

Parity status (what pins each part, other than this code itself):
  * kkt()                    - vertex enumeration, HiGHS optimum + marginals, hand-made LPs.
  * precondition()           - Ruiz norm convergence, Pock-Chambolle spectral bound, same optimum.
  * normalized_gap()         - closed form when the ball lies inside the box, zero at an optimum,
                               brute-force sampling on tiny cases, independent bisection.
  * pdhg step / adaptive rule- a hand-worked 2x2 step with its Eq. (5) limit and Algorithm 2
                               proposals (k = 1, 7, both branches) worked in exact decimals,
                               the optimum as a fixed point, eta_bar >= 1/||K||_2 on every
                               attempt.
  * power_iteration_norm()   - numpy.linalg.norm(., 2) of the dense matrix, the closed forms of
                               diagonal and rank-one matrices, monotone and bounded estimates.
  * restart / primal weight  - table-driven cases with hand-written gap sequences, closed form.
  * solve()                  - optimum matches vertex enumeration and HiGHS, KKT <= tol,
                               scale invariance (Proposition 1), PageRank fixed point.
  * the first-100-iterate trajectory itself is parity unpinned by the paper (it prints no
    iterates); only the pins above constrain it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

OPTIMAL = 0
ITERATION_LIMIT = 1
NUMERICAL_ERROR = 2

# restart reasons, as a bit mask (Section 3.2, criteria (i)-(iii))
RESTART_SUFFICIENT = 1
RESTART_NECESSARY = 2
RESTART_ARTIFICIAL = 4


@dataclass
class Options:
    """Solver options; defaults are the paper's PDLP settings (Section 3 and Appendix C)."""
    ruiz_iters: int = 10                 # Section 3.5: 10 Ruiz passes ...
    pock_chambolle: bool = True          # ... then one Pock-Chambolle pass
    pc_alpha: float = 1.0                # alpha = 1
    step_policy: str = "adaptive"        # Algorithm 2; "constant" = eta 0.9/||K||_2 (Section 2 baseline);
                                         # "malitsky_pock" = the line search of Appendix C
    mp_breaking_factor: float = 1.0      # Malitsky-Pock hyperparameters, the paper's best setting
    mp_downscaling: float = 0.5
    mp_interpolation: float = 0.4
    restarts: bool = True                # Section 3.2 adaptive restarts
    pw_power_of_two: bool = False        # with restarts off: Appendix C "no restart" mode, the
                                         # primal weight still updated at k = 2, 4, 8, ... (R10)
    restart_to_current: bool = True      # False: the candidate is always the average
                                         # (Appendix C "adaptive restart (theory)")
    beta_sufficient: float = 0.1         # reading R4: the printed 0.9 / 0.1 are transposed
    beta_necessary: float = 0.9
    beta_artificial: float = 0.5
    primal_weight_update: bool = True    # Algorithm 3
    theta: float = 0.5                   # smoothing in Algorithm 3
    primal_importance: float = 1.0       # multiplies the initial primal weight
    eps_zero: float = 1e-10              # "small nonzero tolerance" (reading Z4)
    check_every: int = 40                # restart / termination evaluation cadence (Section 3)
    max_retries: int = 100               # cap of Algorithm 2's retry loop (reading Z19)
    power_iters: int = 200               # for the constant-step baseline


@dataclass
class Trace:
    attempts: list = field(default_factory=list)   # (k, eta, eta_bar, accepted)
    iterates: list = field(default_factory=list)   # (k, x_scaled, y_scaled) after accepted steps
    checks: list = field(default_factory=list)     # dicts, one per restart/termination check
    states: list = field(default_factory=list)     # full solver state before each step (if asked)
    trace_iters: int = 0


@dataclass
class Result:
    status: int
    x: np.ndarray            # unscaled primal output
    y: np.ndarray            # unscaled dual output
    kkt: dict
    k: int                   # accepted PDHG steps
    attempts: int
    restarts: int
    omega: float
    eta_hat: float
    kkt_passes: float
    x_scaled: np.ndarray
    y_scaled: np.ndarray
    D1: np.ndarray
    D2: np.ndarray
    trace: Trace | None = None


# ------------------------------------------------------------------------------------------
# Problem pieces (Section 2)
# ------------------------------------------------------------------------------------------

def project_lambda(g: np.ndarray, l: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Projection onto Lambda (Section 2, definition of Lambda_i by which bounds are finite):
    {0} if both bounds are infinite, R^- if only u is finite, R^+ if only l is finite, R else."""
    lf = np.isfinite(l)
    uf = np.isfinite(u)
    lam = g.copy()
    lam[~lf & ~uf] = 0.0
    only_u = ~lf & uf
    lam[only_u] = np.minimum(g[only_u], 0.0)
    only_l = lf & ~uf
    lam[only_l] = np.maximum(g[only_l], 0.0)
    return lam


def dual_objective(q, y, l, u, lam) -> float:
    """Dual objective of problem (1): q^T y + sum l_i lam_i^+ + sum u_i min(lam_i, 0).

    Reading R1: the paper writes "- u^T lambda^-" while defining v^- = min(0, v); with that
    definition the minus sign breaks weak duality (a box-constrained LP min -x, 0<=x<=1
    would get dual value +1 > -1).  The term that keeps weak duality is u_i * min(lam_i, 0),
    i.e. lambda^- read as the magnitude max(0, -lam).  A term whose bound is infinite
    contributes 0, since Lambda forces that part of lambda to 0 (reading Z16)."""
    lam_pos = np.maximum(lam, 0.0)
    lam_neg = np.minimum(lam, 0.0)
    lf = np.isfinite(l)
    uf = np.isfinite(u)
    return float(q @ y + l[lf] @ lam_pos[lf] + u[uf] @ lam_neg[uf])


def kkt(c, K, q, l, u, n_eq, x, y) -> dict:
    """Relative KKT error of (x, y) for problem (1): the termination criteria of Section 4.1
    (Eq. (6a)-(6c)) with lambda = proj_Lambda(c - K^T y).  Returns the three relative errors
    and their max (reading Z22: one scalar <= eps iff all three criteria hold at eps)."""
    K = sp.csr_matrix(K)
    m = K.shape[0]
    m1 = m - n_eq
    Kx = K @ x
    g = c - K.T @ y
    lam = project_lambda(g, l, u)
    pobj = float(c @ x)
    dobj = dual_objective(q, y, l, u, lam)
    e_gap = abs(dobj - pobj) / (1.0 + abs(dobj) + abs(pobj))
    r = np.empty(m)
    r[m1:] = Kx[m1:] - q[m1:]                     # A x - b
    r[:m1] = np.maximum(q[:m1] - Kx[:m1], 0.0)    # (h - G x)^+
    e_pri = float(np.linalg.norm(r)) / (1.0 + float(np.linalg.norm(q)))
    e_dual = float(np.linalg.norm(g - lam)) / (1.0 + float(np.linalg.norm(c)))
    return dict(e_gap=e_gap, e_pri=e_pri, e_dual=e_dual, kkt=max(e_gap, e_pri, e_dual),
                pobj=pobj, dobj=dobj)


# ------------------------------------------------------------------------------------------
# Diagonal preconditioning (Section 3.5)
# ------------------------------------------------------------------------------------------

def _row_norms(A: sp.csr_matrix, kind: str) -> np.ndarray:
    A = sp.csr_matrix(A)
    absA = abs(A)
    if kind == "inf":
        r = np.asarray(absA.max(axis=1).todense()).ravel()
    elif kind == "1":
        r = np.asarray(absA.sum(axis=1)).ravel()
    else:
        raise ValueError(kind)
    return r


def precondition(K, c, q, l, u, ruiz_iters=10, pock_chambolle=True, pc_alpha=1.0):
    """Section 3.5: K~ = D1 K D2 with c~ = D2 c, q~ = D1 q, l~ = l / D2, u~ = u / D2.

    Default: ruiz_iters Ruiz passes, then one Pock-Chambolle pass with alpha = 1.
    Reading Z2: the printed (D1)_jj = sqrt(||K_j,.||) is the norm the pass divides by; the
    multiplier that equilibrates is its reciprocal (the only choice under which Ruiz's
    row/column infinity norms tend to 1).  Ruiz uses the row and column infinity norms of the
    current K~, both taken before that pass rescales.  Pock-Chambolle with alpha = 1 uses
    row and column 1-norms (||.||_{2-alpha} = ||.||_alpha = ||.||_1).  A zero norm (empty row
    or column) leaves that scale factor at 1 (reading Z17).
    Returns (K~, c~, q~, l~, u~, D1, D2)."""
    Kt = sp.csr_matrix(K, dtype=np.float64, copy=True)
    m, n = Kt.shape
    D1 = np.ones(m)
    D2 = np.ones(n)

    def rescale(kind):
        nonlocal Kt, D1, D2
        r = _row_norms(Kt, kind)
        s = _row_norms(Kt.T.tocsr(), kind)
        r = np.where(r > 0.0, r, 1.0)
        s = np.where(s > 0.0, s, 1.0)
        dr = 1.0 / np.sqrt(r)
        ds = 1.0 / np.sqrt(s)
        Kt = sp.csr_matrix(sp.diags(dr) @ Kt @ sp.diags(ds))
        D1 = D1 * dr
        D2 = D2 * ds

    for _ in range(ruiz_iters):
        rescale("inf")
    if pock_chambolle:
        if pc_alpha != 1.0:
            raise NotImplementedError("only alpha = 1 (the paper's default) is implemented")
        rescale("1")
    Kt.sort_indices()
    return Kt, D2 * c, D1 * q, l / D2, u / D2, D1, D2


# ------------------------------------------------------------------------------------------
# Normalized duality gap (Section 3.2)
# ------------------------------------------------------------------------------------------

def weighted_norm(dx, dy, omega) -> float:
    """||z||_omega = sqrt(omega ||x||^2 + ||y||^2 / omega) (Section 2)."""
    return math.sqrt(omega * float(dx @ dx) + float(dy @ dy) / omega)


def trust_region_linear_max(a: np.ndarray, lo: np.ndarray, hi: np.ndarray, r: float):
    """max a^T e over {lo <= e <= hi, ||e||_2 <= r}, with lo <= 0 <= hi (0 is feasible).

    The Lagrangian of the ball constraint is separable, so the maximiser is
    e(s) = clip(s a, lo, hi) for the smallest s >= 0 with ||e(s)|| = r (s = inf if the
    whole box corner lies inside the ball).  ||e(s)||^2 is piecewise quadratic in s with
    breakpoints t_i = hi_i / a_i (a_i > 0) or lo_i / a_i (a_i < 0); sort them and solve the
    quadratic on the piece where the norm crosses r.  Returns (value, s)."""
    nz = a != 0.0
    aa = np.abs(a[nz])
    b = np.where(a[nz] > 0.0, hi[nz], -lo[nz])         # distance to the bound along sign(a)
    t = b / aa                                          # breakpoints, may be +inf or 0
    order = np.argsort(t, kind="stable")
    t_s, a2_s, b2_s = t[order], aa[order] ** 2, b[order] ** 2
    # suffix sums of a^2 (still linear at s) and prefix sums of b^2 (already clipped)
    A_suf = np.concatenate([np.cumsum(a2_s[::-1])[::-1], [0.0]])
    B_pre = np.concatenate([[0.0], np.cumsum(np.where(np.isfinite(b2_s), b2_s, 0.0))])
    r2 = r * r
    # f at each finite breakpoint t_k: t_k^2 * sum_{j>=k} a_j^2 + sum_{j<k} b_j^2
    fin = np.isfinite(t_s)
    nfin = int(fin.sum())
    f_at = t_s[:nfin] ** 2 * A_suf[:nfin] + B_pre[:nfin]
    hit = np.flatnonzero(f_at >= r2)
    k = int(hit[0]) if hit.size else nfin               # first breakpoint with f >= r^2
    A = A_suf[k]
    B = B_pre[k]
    if k == nfin and A == 0.0:
        s = math.inf
    else:
        s = math.sqrt(max(r2 - B, 0.0) / A)
    if math.isinf(s):
        e_abs = b
    else:
        e_abs = np.minimum(s * aa, b)
    return float(aa @ e_abs), s


def normalized_gap(x, y, x_ref, y_ref, omega, g_x, g_y, l, u, m1) -> float:
    """mu(z, z_ref): the normalized duality gap rho_r(z) with r = ||z - z_ref||_omega
    (Section 3.2).  With g_x = c - K^T y and g_y = q - K x,
        L(x, y^) - L(x^, y) = (y^ - y)^T g_y - (x^ - x)^T g_x.
    Substituting e_x = sqrt(omega)(x^ - x), e_y = (y^ - y)/sqrt(omega) turns the omega-ball
    into the Euclidean ball of radius r, the objective into a^T e with
    a = (-g_x / sqrt(omega), sqrt(omega) g_y), and Z into the box
    e_x in [sqrt(omega)(l - x), sqrt(omega)(u - x)], e_y,i >= -y_i/sqrt(omega) (i < m1).
    The paper cites a linear-time method without giving it; this is the exact solve above.
    Reading Z12: r = 0 gives mu = 0.  Reading R2: the box is widened to contain 0 when z
    lies outside Z by rounding (lo = min(lo, 0), hi = max(hi, 0))."""
    r = weighted_norm(x - x_ref, y - y_ref, omega)
    if r == 0.0:
        return 0.0
    sw = math.sqrt(omega)
    a = np.concatenate([-g_x / sw, sw * g_y])
    lo_x = sw * (l - x)
    hi_x = sw * (u - x)
    m = y.shape[0]
    lo_y = np.full(m, -np.inf)
    lo_y[:m1] = -y[:m1] / sw
    hi_y = np.full(m, np.inf)
    lo = np.minimum(np.concatenate([lo_x, lo_y]), 0.0)
    hi = np.maximum(np.concatenate([hi_x, hi_y]), 0.0)
    val, _ = trust_region_linear_max(a, lo, hi, r)
    return val / r


# ------------------------------------------------------------------------------------------
# Primal weight (Section 3.3, Algorithm 3) and restart rules (Section 3.2)
# ------------------------------------------------------------------------------------------

def initial_primal_weight(c, q, eps_zero) -> float:
    """InitializePrimalWeight(c, q) = ||c||/||q|| if both norms exceed eps_zero, else 1."""
    nc = float(np.linalg.norm(c))
    nq = float(np.linalg.norm(q))
    if nc > eps_zero and nq > eps_zero:
        return nc / nq
    return 1.0


def primal_weight_update(dx_norm, dy_norm, omega_prev, theta, eps_zero) -> float:
    """Algorithm 3: exp(theta log(dy/dx) + (1-theta) log(omega_prev)) when both distances
    exceed eps_zero, otherwise omega_prev."""
    if dx_norm > eps_zero and dy_norm > eps_zero:
        return math.exp(theta * math.log(dy_norm / dx_norm) + (1.0 - theta) * math.log(omega_prev))
    return omega_prev


def restart_mask(mu_c, mu_anchor, mu_prev, t, k, n_outer, opts: Options) -> int:
    """Restart criteria (i)-(iii) of Section 3.2 as a bit mask.

    Reading R4: the paper prints beta_sufficient = 0.9 > beta_necessary = 0.1, yet calls the
    first inequality of (ii) a safeguard for its second; with beta_necessary < beta_sufficient
    (ii) implies (i) and can never decide a restart.  (ii) only acts when
    beta_necessary > beta_sufficient, so the defaults are read transposed: (i) needs the gap to
    fall to 0.1 of the anchor's, (ii) to 0.9 of it plus no progress since the previous check.
    The paper's own text supports this: Appendix C describes its "adaptive restart (theory)"
    variant, with both parameters set to exp(-1), as the default with criterion (ii) taken
    away.  That distinction is only real if (ii) can decide a restart under the defaults,
    i.e. if beta_necessary exceeds beta_sufficient there.

    Reading Z9: mu(z^{n,0}, z^{n-1,0}) is undefined in the first outer loop (n = 0), so
    (i) and (ii) are false there; (iii) t >= beta_art * k holds anyway because t = k.
    Reading Z11: the "previous candidate" in (ii) is the candidate's gap at the previous
    check of this outer loop (+inf at the first check after a restart)."""
    mask = 0
    if n_outer > 0:
        if mu_c <= opts.beta_sufficient * mu_anchor:
            mask |= RESTART_SUFFICIENT
        if mu_c <= opts.beta_necessary * mu_anchor and mu_c > mu_prev:
            mask |= RESTART_NECESSARY
    if t >= opts.beta_artificial * k:
        mask |= RESTART_ARTIFICIAL
    return mask


# ------------------------------------------------------------------------------------------
# PDHG step (Eq. (3) with tau = eta/omega, sigma = eta*omega; Algorithm 2)
# ------------------------------------------------------------------------------------------

def pdhg_step(x, y, eta, omega, c, K, KT, q, l, u, m1):
    """One PDHG step, Eq. (3):  x' = proj_X(x - tau (c - K^T y)),
    y' = proj_Y(y + sigma (q - K(2x' - x))),  tau = eta/omega, sigma = eta*omega."""
    xp = np.clip(x - (eta / omega) * (c - KT @ y), l, u)
    yp = y + (eta * omega) * (q - K @ (2.0 * xp - x))
    yp[:m1] = np.maximum(yp[:m1], 0.0)
    return xp, yp


def step_size_limit(dx, dy, omega, K) -> float:
    """The largest step Eq. (5) allows: ||dz||_omega^2 / (2 dy^T K dx).

    Reading Z5: the denominator is taken in absolute value, and a zero denominator gives
    +inf (accept); this is what makes 'eta_bar >= 1/||K||_2 always' true."""
    num = omega * float(dx @ dx) + float(dy @ dy) / omega
    den = 2.0 * abs(float(dy @ (K @ dx)))
    if den == 0.0:
        return math.inf
    return num / den


def next_step_size(eta_bar, eta, k) -> float:
    """eta' = min((1 - (k+1)^-0.3) eta_bar, (1 + (k+1)^-0.6) eta) (Algorithm 2).

    Reading R3 (replaces Z6): Algorithm 1 starts its counter at k = 0 and passes it to
    Algorithm 2, which then gives eta' = min(0 * eta_bar, 2 eta) = 0 after the first step, and
    every later step has eta = 0.  The counter is therefore read as 1-based: k is the number
    of the step being taken (accepted steps so far + 1), so the first step uses 2^-0.3."""
    k1 = float(k + 1)
    return min((1.0 - k1 ** -0.3) * eta_bar, (1.0 + k1 ** -0.6) * eta)


def power_iteration_norm(K, iters) -> float:
    """||K||_2 estimated by power iteration on K^T K (Section 2, baseline PDHG), started
    from the all-ones vector (a deterministic start both implementations share)."""
    K = sp.csr_matrix(K)
    v = np.ones(K.shape[1])
    v /= np.linalg.norm(v)
    sigma = 0.0
    for _ in range(iters):
        w = K.T @ (K @ v)
        nw = float(np.linalg.norm(w))
        if nw == 0.0:
            return 0.0
        sigma = math.sqrt(nw)
        v = w / nw
    return sigma


# ------------------------------------------------------------------------------------------
# PDLP driver (Algorithm 1)
# ------------------------------------------------------------------------------------------

def mp_candidate(eta, theta, interpolation):
    """Malitsky-Pock line search (Appendix C), the first candidate step for iteration k+1:
    eta^ = eta_k + interpolation (sqrt(1 + theta_k) - 1) eta_k, theta^ = eta_k / eta^, with
    theta_k = eta_{k-1} / eta_k as the appendix defines it (reading R6: the reciprocal of
    Malitsky and Pock's own ratio; the printed definition is followed)."""
    eta_hat = eta + interpolation * (math.sqrt(1.0 + theta) - 1.0) * eta
    return eta_hat, eta / eta_hat


def mp_dual_trial(x, xp, y, eta_hat, theta_hat, omega, K, q, m1):
    """Candidate dual iterate of the line search: proj_Y(y + omega eta^ (q - K(x' + theta^ (x' - x))))."""
    yh = y + (omega * eta_hat) * (q - K @ (xp + theta_hat * (xp - x)))
    yh[:m1] = np.maximum(yh[:m1], 0.0)
    return yh


def mp_accepts(eta_hat, dy, KTdy, breaking_factor) -> bool:
    """The line-search test eta^ ||K^T (y^ - y)|| <= breaking_factor ||y^ - y|| (reading R7:
    the step in front of the norm is the candidate eta^ the trial was computed with)."""
    return eta_hat * float(np.linalg.norm(KTdy)) <= breaking_factor * float(np.linalg.norm(dy))


def solve(c, K, q, l, u, n_eq, tol=1e-8, iter_limit=100000, opts: Options | None = None,
          trace_iters: int = 0, record_trace: bool = False, record_states: int = 0) -> Result:
    """Algorithm 1 after preconditioning: adaptive steps (Algorithm 2), eta-weighted
    averages, restart candidate, restart criteria, primal weight updates (Algorithm 3).
    step_policy "constant" takes the fixed step of the baseline PDHG (Section 2) and
    "malitsky_pock" the line search of Appendix C in place of Algorithm 2.

    Evaluation cadence (Section 3): restart/termination checks only when the number of
    accepted steps k is a positive multiple of check_every, plus a termination check before
    the first step (reading Z8).  At a check the candidate z_c is tested for termination
    and returned if it passes (reading Z14).  Termination uses the unscaled problem
    (reading Z15).  eta_hat is carried across restarts (Z7).  The average covers the
    iterates accepted since the last restart, weighted by the step each was taken with (Z20).
    After a restart mu_anchor = mu(z^{n,0}, z^{n-1,0}) is computed with the updated primal
    weight (Z10).  At the iteration limit the current iterate is returned.

    record_states = K keeps, for k = 0..K, the complete state the loop holds before taking
    step k + 1 (iterate, anchor, weighted sums, step size, primal weight, counters, gap
    memory), so a single step can be replayed from it."""
    opts = opts or Options()
    K = sp.csr_matrix(K, dtype=np.float64)
    m, n = K.shape
    m1 = m - n_eq
    c = np.asarray(c, np.float64)
    q = np.asarray(q, np.float64)
    l = np.asarray(l, np.float64)
    u = np.asarray(u, np.float64)

    Kt, ct, qt, lt, ut, D1, D2 = precondition(K, c, q, l, u, opts.ruiz_iters,
                                              opts.pock_chambolle, opts.pc_alpha)
    KtT = Kt.T.tocsr()
    tr = Trace(trace_iters=trace_iters) if (record_trace or trace_iters > 0 or record_states) else None

    def unscaled_kkt(xs, ys):
        return kkt(c, K, q, l, u, n_eq, D2 * xs, D1 * ys)

    # initial point (Section 4.1 'Initialization', reading Z18) and scalars
    x = np.clip(np.zeros(n), lt, ut)
    y = np.zeros(m)
    omega = initial_primal_weight(ct, qt, opts.eps_zero) * opts.primal_importance
    maxabs = float(np.max(np.abs(Kt.data))) if Kt.nnz else 0.0
    eta_hat = 1.0 / maxabs if maxabs > 0.0 else 1.0   # 1/||K~||_inf, entrywise max (Z3)
    if opts.step_policy == "constant":
        nrm = power_iteration_norm(Kt, opts.power_iters)
        eta_hat = 0.9 / nrm if nrm > 0.0 else 1.0
    k = 0
    t = 0
    n_outer = 0
    attempts = 0
    kkt_passes = 0.0
    xa, ya = x.copy(), y.copy()                # anchor z^{n,0}
    Sx = np.zeros(n)
    Sy = np.zeros(m)
    Seta = 0.0
    mu_prev = math.inf
    mu_anchor = math.inf
    mp_theta = 1.0                              # Malitsky-Pock theta_k (1 at the start, R8)
    pw_done = 0                                 # k of the last "no restart" weight update
    kty = KtT @ y                               # K~^T y of the current y

    def finish(status, xs, ys):
        kk = unscaled_kkt(xs, ys)
        return Result(status=status, x=D2 * xs, y=D1 * ys, kkt=kk, k=k, attempts=attempts,
                      restarts=n_outer, omega=omega, eta_hat=eta_hat, kkt_passes=kkt_passes,
                      x_scaled=xs.copy(), y_scaled=ys.copy(), D1=D1, D2=D2, trace=tr)

    if unscaled_kkt(x, y)["kkt"] <= tol:
        return finish(OPTIMAL, x, y)

    while True:
        if k >= 2 and (k & (k - 1)) == 0 and k != pw_done and not opts.restarts and opts.pw_power_of_two:
            # "no restart" mode (Appendix C, reading R10): at k = 2^j the weight is updated as an
            # artificial restart would, from the distance of the current iterate to the iterate
            # of the previous update, and that anchor moves; iterate and averages stay
            pw_done = k
            if opts.primal_weight_update:
                omega = primal_weight_update(float(np.linalg.norm(x - xa)), float(np.linalg.norm(y - ya)),
                                             omega, opts.theta, opts.eps_zero)
            xa, ya = x.copy(), y.copy()
            n_outer += 1
            mp_theta = 1.0
        if tr is not None and k <= record_states and (not tr.states or tr.states[-1]["k"] != k):
            tr.states.append(dict(k=k, t=t, n_outer=n_outer, x=x.copy(), y=y.copy(), xa=xa.copy(),
                                  ya=ya.copy(), Sx=Sx.copy(), Sy=Sy.copy(), Seta=Seta,
                                  eta_hat=eta_hat, omega=omega, mu_prev=mu_prev,
                                  mu_anchor=mu_anchor))
        if k >= iter_limit:
            return finish(ITERATION_LIMIT, x, y)
        if opts.step_policy == "malitsky_pock":
            # ---- Malitsky-Pock line search (Appendix C) ----
            xp = np.clip(x - (eta_hat / omega) * (ct - kty), lt, ut)
            eta, th = mp_candidate(eta_hat, mp_theta, opts.mp_interpolation)
            retries = 0
            while True:
                yp = mp_dual_trial(x, xp, y, eta, th, omega, Kt, qt, m1)
                kty_p = KtT @ yp
                attempts += 1
                kkt_passes += 1.0
                dy = yp - y
                kdy = kty_p - kty
                nk = float(np.linalg.norm(kdy))
                eta_bar = opts.mp_breaking_factor * float(np.linalg.norm(dy)) / nk if nk > 0.0 else math.inf
                ok = bool(np.all(np.isfinite(xp)) and np.all(np.isfinite(yp)))
                accepted = bool(ok and mp_accepts(eta, dy, kdy, opts.mp_breaking_factor))
                if tr is not None:
                    tr.attempts.append((k, eta, eta_bar, accepted))
                if not ok:
                    st = OPTIMAL if unscaled_kkt(x, y)["kkt"] <= tol else NUMERICAL_ERROR
                    return finish(st, x, y)
                if accepted:
                    break
                eta = opts.mp_downscaling * eta
                th = eta_hat / eta
                retries += 1
                if retries >= opts.max_retries:
                    st = OPTIMAL if unscaled_kkt(x, y)["kkt"] <= tol else NUMERICAL_ERROR
                    return finish(st, x, y)
            x, y, kty = xp, yp, kty_p
            Sx += eta * x                       # weight: the accepted step (reading R9)
            Sy += eta * y
            Seta += eta
            eta_hat, mp_theta = eta, th
            k += 1
            t += 1
            if tr is not None and k <= trace_iters:
                tr.iterates.append((k, x.copy(), y.copy()))
            if k % opts.check_every != 0:
                continue
        else:
            # ---- AdaptiveStepOfPDHG (Algorithm 2) ----
            eta = eta_hat
            retries = 0
            while True:
                xp, yp = pdhg_step(x, y, eta, omega, ct, Kt, KtT, qt, lt, ut, m1)
                attempts += 1
                kkt_passes += 1.0
                if opts.step_policy == "constant":
                    eta_bar = math.inf
                    eta_next = eta
                else:
                    eta_bar = step_size_limit(xp - x, yp - y, omega, Kt)
                    eta_next = next_step_size(eta_bar, eta, k + 1)
                ok = np.isfinite(eta_next) and np.all(np.isfinite(xp)) and np.all(np.isfinite(yp))
                accepted = bool(ok and eta <= eta_bar)
                if tr is not None:
                    tr.attempts.append((k, eta, eta_bar, accepted))
                if not ok:
                    st = OPTIMAL if unscaled_kkt(x, y)["kkt"] <= tol else NUMERICAL_ERROR
                    return finish(st, x, y)
                if accepted:
                    break
                eta = eta_next
                retries += 1
                if retries >= opts.max_retries:
                    st = OPTIMAL if unscaled_kkt(x, y)["kkt"] <= tol else NUMERICAL_ERROR
                    return finish(st, x, y)
            x, y = xp, yp
            Sx += eta * x
            Sy += eta * y
            Seta += eta
            eta_hat = eta_next
            k += 1
            t += 1
            if tr is not None and k <= trace_iters:
                tr.iterates.append((k, x.copy(), y.copy()))
            if k % opts.check_every != 0:
                continue
        # ---- restart / termination check (Algorithm 1, Section 3.2) ----
        xbar = Sx / Seta
        ybar = Sy / Seta
        kkt_passes += 1.0 if opts.restarts else 0.0
        gx_cur = ct - KtT @ y
        gy_cur = qt - Kt @ x
        if opts.restarts:
            gx_avg = ct - KtT @ ybar
            gy_avg = qt - Kt @ xbar
            mu_cur = normalized_gap(x, y, xa, ya, omega, gx_cur, gy_cur, lt, ut, m1)
            mu_avg = normalized_gap(xbar, ybar, xa, ya, omega, gx_avg, gy_avg, lt, ut, m1)
            # GetRestartCandidate, tie -> average; "theory" mode always takes the average
            use_avg = (not (mu_cur < mu_avg)) or not opts.restart_to_current
        else:
            mu_cur = mu_avg = math.nan
            use_avg = False
        if use_avg:
            xc, yc, mu_c, gxc, gyc = xbar, ybar, mu_avg, gx_avg, gy_avg
        else:
            xc, yc, mu_c, gxc, gyc = x, y, mu_cur, gx_cur, gy_cur
        kc = unscaled_kkt(xc, yc)
        rec = dict(k=k, mu_cur=mu_cur, mu_avg=mu_avg, use_avg=use_avg, kkt=kc["kkt"],
                   mask=0, omega_before=omega)
        if tr is not None:
            tr.checks.append(rec)
        if kc["kkt"] <= tol:
            rec["terminated"] = True
            return finish(OPTIMAL, xc, yc)
        if not opts.restarts:
            rec["omega_after"] = omega
            continue
        mask = restart_mask(mu_c, mu_anchor, mu_prev, t, k, n_outer, opts)
        rec["mask"] = mask
        if mask:
            dxn = float(np.linalg.norm(xc - xa))
            dyn = float(np.linalg.norm(yc - ya))
            if opts.primal_weight_update:
                omega = primal_weight_update(dxn, dyn, omega, opts.theta, opts.eps_zero)
            mu_anchor = normalized_gap(xc, yc, xa, ya, omega, gxc, gyc, lt, ut, m1)
            xa, ya = xc.copy(), yc.copy()
            x, y = xc.copy(), yc.copy()
            if opts.step_policy == "malitsky_pock":
                kty = KtT @ y
                mp_theta = 1.0                  # the line search restarts with theta = 1 (R8)
            Sx[:] = 0.0
            Sy[:] = 0.0
            Seta = 0.0
            t = 0
            n_outer += 1
            mu_prev = math.inf
            rec["mu_anchor"] = mu_anchor
        else:
            mu_prev = mu_c
        rec["omega_after"] = omega


def solve_lp(lp, tol=1e-8, iter_limit=100000, opts=None, trace_iters=0, record_trace=False,
             record_states=0):
    """solve() on a workloads.lpgen.LP."""
    return solve(lp.c, lp.K(), lp.q, lp.l, lp.u, lp.n_eq, tol, iter_limit, opts,
                 trace_iters, record_trace, record_states)


# ------------------------------------------------------------------------------------------
# Unrolled PDHG and its adjoint (differentiation through a fixed number of steps of Eq. (3))
# ------------------------------------------------------------------------------------------

def unroll_forward(Kt, ct, qt, lt, ut, m1, eta, omega, T):
    """T steps of Eq. (3) with fixed tau = eta/omega, sigma = eta*omega on the preconditioned
    problem, from x0 = proj_X(0), y0 = 0 (Section 4.1 initialisation).  The dual step uses
    K~(2x' - x) as printed.  Returns the lists of iterates x_0..x_T, y_0..y_T."""
    Kt = sp.csr_matrix(Kt)
    KT = Kt.T.tocsr()
    tau, sigma = eta / omega, eta * omega
    x = np.clip(np.zeros(Kt.shape[1]), lt, ut)
    y = np.zeros(Kt.shape[0])
    xs, ys = [x], [y]
    for _ in range(T):
        xn = np.clip(x - tau * (ct - KT @ y), lt, ut)
        yn = y + sigma * (qt - Kt @ (2.0 * xn - x))
        yn[:m1] = np.maximum(yn[:m1], 0.0)
        x, y = xn, yn
        xs.append(x)
        ys.append(y)
    return xs, ys


def unroll_backward(Kt, lt, ut, m1, eta, omega, xs, ys, gx_T, gy_T=None):
    """Reverse mode of unroll_forward: given dL/dx_T (and dL/dy_T, default 0), returns
    (dL/dc~, dL/dq~).

    Step t maps (x_t, y_t) to x_{t+1} = clip(u), u = x_t - tau (c~ - K~^T y_t), and
    y_{t+1} = proj_Y(v), v = y_t + sigma (q~ - K~ (2 x_{t+1} - x_t)).  The Jacobian of the
    clip is 1 where l < x_{t+1} < u and 0 elsewhere; that of proj_Y is 1 on the equality rows
    and where y_{t+1} > 0.  Going backwards with adjoints (xb, yb) of (x_{t+1}, y_{t+1}):
      vb  = mask_y * yb                      ;  qb += sigma vb
      xb' = xb - 2 sigma K~^T vb              (x_{t+1} also enters v)
      ub  = mask_x * xb'                     ;  cb -= tau ub
      xb <- ub + sigma K~^T vb                (adjoint of x_t)
      yb <- vb + tau K~ ub                    (adjoint of y_t)"""
    Kt = sp.csr_matrix(Kt)
    KT = Kt.T.tocsr()
    tau, sigma = eta / omega, eta * omega
    m = Kt.shape[0]
    xb = np.array(gx_T, dtype=np.float64)
    yb = np.zeros(m) if gy_T is None else np.array(gy_T, dtype=np.float64)
    cb = np.zeros(Kt.shape[1])
    qb = np.zeros(m)
    T = len(xs) - 1
    for t in range(T - 1, -1, -1):
        x1, y1 = xs[t + 1], ys[t + 1]
        mask_y = np.ones(m)
        mask_y[:m1] = (y1[:m1] > 0.0).astype(np.float64)
        vb = mask_y * yb
        qb += sigma * vb
        g = KT @ vb
        mask_x = ((x1 > lt) & (x1 < ut)).astype(np.float64)
        ub = mask_x * (xb - 2.0 * sigma * g)
        cb -= tau * ub
        xb = ub + sigma * g
        yb = vb + tau * (Kt @ ub)
    return cb, qb


def unroll_user(K, c, q, l, u, m1, x_tgt, T, eta=None, omega=None, gy_T=None):
    """The unrolled map in the user's variables and its gradient, for the loss
    ||x_T - x_tgt||^2 (+ <gy_T, y_T> when gy_T is given).

    D1, D2 come from K alone (Section 3.5), so they, eta and omega are constants of the map:
    c~ = D2 c, q~ = D1 q, x_T = D2 x~_T, y_T = D1 y~_T, hence dL/dc = D2 dL/dc~,
    dL/dq = D1 dL/dq~ and dL/dx~_T = D2 dL/dx_T.  eta defaults to 0.9 / ||K~||_2 (power
    iteration), omega to the initial primal weight of Section 3.3 computed from the LP's own
    c~, q~.  Returns dict(x_T, y_T, loss, gc, gq, eta, omega)."""
    Kt, ct, qt, lt, ut, D1, D2 = precondition(K, c, q, l, u)
    if eta is None:
        eta = 0.9 / power_iteration_norm(Kt, 200)
    if omega is None:
        omega = initial_primal_weight(ct, qt, 1e-10)
    xs, ys = unroll_forward(Kt, ct, qt, lt, ut, m1, eta, omega, T)
    x_T = D2 * xs[-1]
    y_T = D1 * ys[-1]
    r = x_T - x_tgt
    loss = float(r @ r)
    gy_s = None
    if gy_T is not None:
        loss += float(np.asarray(gy_T) @ y_T)
        gy_s = D1 * np.asarray(gy_T)
    cb, qb = unroll_backward(Kt, lt, ut, m1, eta, omega, xs, ys, D2 * (2.0 * r), gy_s)
    return dict(x_T=x_T, y_T=y_T, loss=loss, gc=D2 * cb, gq=D1 * qb, eta=eta, omega=omega)

