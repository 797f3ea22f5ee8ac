"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics (CPU only).

Each test checks the oracle against something other than itself: brute-force vertex
enumeration, HiGHS (a library LP solver) and its marginals, hand-worked values, closed forms,
independent bisection, invariants (Ruiz convergence, the Pock-Chambolle spectral bound,
Proposition 1 scale invariance, the PageRank fixed point).
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

from oracle import pdlp_oracle as O
from workloads import lpgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _highs(lp):
    K = lp.K()
    m1 = lp.m1
    res = linprog(lp.c, A_ub=-K[:m1] if m1 else None, b_ub=-lp.q[:m1] if m1 else None,
                  A_eq=K[m1:] if lp.n_eq else None, b_eq=lp.q[m1:] if lp.n_eq else None,
                  bounds=list(zip(np.where(np.isfinite(lp.l), lp.l, None),
                                  np.where(np.isfinite(lp.u), lp.u, None))),
                  method="highs", options=dict(primal_feasibility_tolerance=1e-10,
                                               dual_feasibility_tolerance=1e-10))
    assert res.status == 0
    y = np.zeros(lp.m)
    if m1:
        y[:m1] = -res.ineqlin.marginals
    if lp.n_eq:
        y[m1:] = res.eqlin.marginals
    return res.fun, res.x, y


def _vertex_enumeration(lp):
    """min c^T x over {Gx >= h, Ax = b, l <= x <= u} by trying every basis of active
    constraints (all equalities plus n - n_eq of the inequality rows and bounds)."""
    K = lp.K().toarray()
    m1, n = lp.m1, lp.n
    rows = [(K[i], lp.q[i]) for i in range(m1)]
    rows += [(np.eye(n)[j], lp.l[j]) for j in range(n)]
    rows += [(np.eye(n)[j], lp.u[j]) for j in range(n)]
    eq = [(K[i], lp.q[i]) for i in range(m1, lp.m)]
    best = math.inf
    for sub in itertools.combinations(range(len(rows)), n - len(eq)):
        A = np.array([r[0] for r in eq] + [rows[s][0] for s in sub])
        b = np.array([r[1] for r in eq] + [rows[s][1] for s in sub])
        if abs(np.linalg.det(A)) < 1e-9:
            continue
        x = np.linalg.solve(A, b)
        if np.all(K[:m1] @ x >= lp.q[:m1] - 1e-9) and np.allclose(K[m1:] @ x, lp.q[m1:], atol=1e-9) \
                and np.all(x >= lp.l - 1e-9) and np.all(x <= lp.u + 1e-9):
            best = min(best, float(lp.c @ x))
    return best


# ------------------------------------------------------------------------------------------
# the final answer: optimum, KKT evaluator, certificates
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_vertex_enumeration_matches_oracle(seed):
    lp = lpgen.tiny_box_lp(seed, m=4, n=5, n_eq=1)
    opt = _vertex_enumeration(lp)
    r = O.solve_lp(lp, tol=1e-9, iter_limit=200000)
    assert r.status == O.OPTIMAL
    assert r.kkt["kkt"] <= 1e-9
    assert abs(r.kkt["pobj"] - opt) <= 1e-7 * (1 + abs(opt))


def test_highs_optimum_tiny_lp():
    lp = lpgen.tiny_lp()
    fun, _, _ = _highs(lp)
    r = O.solve_lp(lp, tol=1e-8)
    assert r.status == O.OPTIMAL and r.kkt["kkt"] <= 1e-8
    assert abs(r.kkt["pobj"] - fun) <= 1e-7 * abs(fun)
    # strong duality with the bound terms (reading Z24): the oracle's dual value too
    assert abs(r.kkt["dobj"] - fun) <= 1e-7 * abs(fun)


def test_kkt_evaluator_at_highs_solution():
    """At HiGHS's primal/dual optimum the relative KKT error is at round-off level, and it
    grows when the point is perturbed (pins the sign conventions of kkt())."""
    lp = lpgen.tiny_lp()
    fun, x, y = _highs(lp)
    k = O.kkt(lp.c, lp.K(), lp.q, lp.l, lp.u, lp.n_eq, x, y)
    assert k["kkt"] < 1e-8
    assert abs(k["pobj"] - fun) < 1e-9 * abs(fun)
    k2 = O.kkt(lp.c, lp.K(), lp.q, lp.l, lp.u, lp.n_eq, x + 1e-3, y)
    assert k2["e_pri"] > 1e-6
    k3 = O.kkt(lp.c, lp.K(), lp.q, lp.l, lp.u, lp.n_eq, x, y * 1.01)
    assert k3["kkt"] > 1e-5


def test_dual_objective_upper_bound_term_sign():
    """min -x1 - x2 s.t. x1 + x2 >= 0, 0 <= x <= 1: optimum -2 at x = (1,1), y = 0,
    lambda = c = (-1,-1).  Weak duality forces the dual value -2 (reading R1)."""
    K = sp.csr_matrix(np.array([[1.0, 1.0]]))
    c = np.array([-1.0, -1.0])
    k = O.kkt(c, K, np.array([0.0]), np.zeros(2), np.ones(2), 0, np.ones(2), np.zeros(1))
    assert k["pobj"] == -2.0 and k["dobj"] == -2.0 and k["kkt"] == 0.0


def test_reduced_cost_projection_sets():
    """Lambda_i is {0}, R^-, R^+ or R by which bounds are finite (Section 2)."""
    g = np.array([1.0, -1.0, 1.0, -1.0, 1.0, -1.0, 1.0, -1.0])
    inf = np.inf
    l = np.array([-inf, -inf, -inf, -inf, 0.0, 0.0, 0.0, 0.0])
    u = np.array([inf, inf, 1.0, 1.0, inf, inf, 1.0, 1.0])
    lam = O.project_lambda(g, l, u)
    assert lam.tolist() == [0.0, 0.0, 0.0, -1.0, 1.0, 0.0, 1.0, -1.0]


@pytest.mark.parametrize("maker", [lpgen.tiny_lp, lambda: lpgen.large_plain(7, 300, 600)])
def test_generator_certificates(maker):
    """x0 is feasible and (y0, lambda = s) dual feasible, so dual bound <= optimum <= c^T x0."""
    lp = maker()
    K = lp.K()
    m1 = lp.m1
    assert np.all(K[:m1] @ lp.x0 >= lp.q[:m1] - 1e-9)
    assert np.allclose(K[m1:] @ lp.x0, lp.q[m1:], atol=1e-9)
    assert np.all(lp.x0 >= lp.l) and np.all(lp.x0 <= lp.u)
    assert np.all(lp.y0[:m1] >= 0)
    lam = lp.c - K.T @ lp.y0
    np.testing.assert_allclose(O.project_lambda(lam, lp.l, lp.u), lam, atol=1e-12)
    fun, _, _ = _highs(lp)
    dual_bound = O.dual_objective(lp.q, lp.y0, lp.l, lp.u, lam)
    assert dual_bound <= fun + 1e-7 * abs(fun) and fun <= float(lp.c @ lp.x0) + 1e-7 * abs(fun)


def test_tiny_lp_generator_is_deterministic():
    a, b = lpgen.tiny_lp(), lpgen.tiny_lp()
    assert a.sha256() == b.sha256()
    assert a.m == 200 and a.n == 500 and a.nnz == 2500 and a.n_eq == 120
    assert np.all(np.diff(a.row_ptr) >= 0)


# ------------------------------------------------------------------------------------------
# the PDHG step and the step-size rule
# ------------------------------------------------------------------------------------------

def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_pdhg_step_hand_worked():
    g = _golden("pdhg_step_2x2.txt")
    K = sp.csr_matrix(np.array([[1.0, 2.0], [3.0, 4.0]]))
    xp, yp = O.pdhg_step(np.array([1.0, 1.0]), np.array([0.5, -1.0]), 0.1, 2.0,
                         np.array([1.0, 1.0]), K, K.T.tocsr(), np.array([1.0, 2.0]),
                         np.zeros(2), np.full(2, 10.0), 1)
    np.testing.assert_allclose(xp, [g["x_next_0"], g["x_next_1"]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(yp, [g["y_next_0"], g["y_next_1"]], rtol=0, atol=1e-15)


def test_pdhg_projection_onto_dual_cone():
    """Only the first m1 dual entries are clipped at 0 (Y = {y : y_{1:m1} >= 0})."""
    K = sp.csr_matrix(np.eye(2))
    _, yp = O.pdhg_step(np.zeros(2), np.zeros(2), 1.0, 1.0, np.zeros(2), K, K.T.tocsr(),
                        np.array([-3.0, -3.0]), np.full(2, -1.0), np.full(2, 1.0), 1)
    assert yp.tolist() == [0.0, -3.0]


def test_optimum_is_fixed_point_of_pdhg():
    lp = lpgen.tiny_lp()
    _, x, y = _highs(lp)
    K = lp.K()
    xp, yp = O.pdhg_step(x, y, 0.1, 1.0, lp.c, K, K.T.tocsr(), lp.q, lp.l, lp.u, lp.m1)
    assert np.max(np.abs(xp - x)) < 1e-8 and np.max(np.abs(yp - y)) < 1e-8


def test_eta_bar_at_least_inverse_spectral_norm():
    """Algorithm 2: eta_bar >= 1/||K~||_2 on every attempt; every accepted eta <= eta_bar."""
    lp = lpgen.tiny_lp()
    Kt = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)[0]
    nrm = np.linalg.norm(Kt.toarray(), 2)
    r = O.solve_lp(lp, tol=1e-8, iter_limit=3000, record_trace=True)
    for (_, eta, eta_bar, acc) in r.trace.attempts:
        assert eta_bar >= (1.0 - 1e-12) / nrm
        if acc:
            assert eta <= eta_bar


def _step_2x2():
    """The hand-worked 2x2 step of pdhg_step_2x2.txt: (dx, dy, omega, K)."""
    K = sp.csr_matrix(np.array([[1.0, 2.0], [3.0, 4.0]]))
    x, y = np.array([1.0, 1.0]), np.array([0.5, -1.0])
    xp, yp = O.pdhg_step(x, y, 0.1, 2.0, np.array([1.0, 1.0]), K, K.T.tocsr(), np.array([1.0, 2.0]),
                         np.zeros(2), np.full(2, 10.0), 1)
    return xp - x, yp - y, 2.0, K


def test_step_size_limit_hand_worked():
    """Eq. (5): eta_bar = ||dz||_omega^2 / (2 |dy^T K dx|), against the value worked by hand in
    exact decimals (tests/golden/step_size_rule_2x2.txt)."""
    g = _golden("step_size_rule_2x2.txt")
    dx, dy, omega, K = _step_2x2()
    assert O.step_size_limit(dx, dy, omega, K) == pytest.approx(g["eta_bar"], rel=1e-14, abs=0)
    # the same limit with the roles of the two updates exchanged (dy^T K dx is symmetric in
    # the pair only through K; a transposed operand changes it)
    assert O.step_size_limit(dx, dy, omega, sp.csr_matrix(K.T)) != pytest.approx(g["eta_bar"], rel=1e-3)


def test_next_step_size_hand_worked():
    """Algorithm 2's proposal eta' at steps k = 1 and k = 7 (both branches of the min), against
    values worked by hand in exact decimals."""
    g = _golden("step_size_rule_2x2.txt")
    eb = g["eta_bar"]
    assert O.next_step_size(eb, 0.1, 1) == pytest.approx(g["eta_next_k1"], rel=1e-14, abs=0)
    assert O.next_step_size(eb, 0.1, 7) == pytest.approx(g["eta_next_k7"], rel=1e-14, abs=0)
    assert O.next_step_size(1.0, 0.1, 7) == pytest.approx(g["eta_next_k7_cap"], rel=1e-14, abs=0)
    # first step never collapses to zero (reading R3)
    assert O.next_step_size(3.0, 1.0, 1) > 0.0


def test_step_rule_pins_reject_planted_mistakes():
    """The hand-worked values above tell apart the plausible slips in Algorithm 2: each variant
    below plants one in a copy of the rule, and must miss a golden value by far more than the
    tolerance the pins use."""
    g = _golden("step_size_rule_2x2.txt")
    dx, dy, omega, K = _step_2x2()
    nx, ny, cross = float(dx @ dx), float(dy @ dy), float(dy @ (K @ dx))
    limits = {
        "omega swapped": (nx / omega + ny * omega) / (2 * abs(cross)),
        "factor 2 dropped": (omega * nx + ny / omega) / abs(cross),
        "unweighted norm": (nx + ny) / (2 * abs(cross)),
    }
    for name, v in limits.items():
        assert abs(v - g["eta_bar"]) > 1e-6 * g["eta_bar"], name
    eb = g["eta_bar"]

    def rule(eta_bar, eta, k, e1, e2, shift):
        k1 = float(k + shift)
        return min((1.0 - k1 ** -e1) * eta_bar, (1.0 + k1 ** -e2) * eta)

    variants = {
        "exponents swapped": lambda eb_, eta, k: rule(eb_, eta, k, 0.6, 0.3, 1),
        "0-based counter": lambda eb_, eta, k: rule(eb_, eta, k, 0.3, 0.6, 0) if k > 0 else 0.0,
        "counter one ahead": lambda eb_, eta, k: rule(eb_, eta, k, 0.3, 0.6, 2),
    }
    for name, f in variants.items():
        miss = [abs(f(eb, 0.1, 1) - g["eta_next_k1"]) / g["eta_next_k1"],
                abs(f(eb, 0.1, 7) - g["eta_next_k7"]) / g["eta_next_k7"],
                abs(f(1.0, 0.1, 7) - g["eta_next_k7_cap"]) / g["eta_next_k7_cap"]]
        assert max(miss) > 1e-6, name


def test_power_iteration_norm_against_numpy():
    """||K~||_2 by power iteration (the constant step of the baseline PDHG, Section 2) against
    numpy.linalg.norm(., 2) of the dense matrix; the estimate never exceeds the norm (it is
    sqrt(||K^T K v||) with ||v|| = 1) and does not decrease from one iteration to the next."""
    lp = lpgen.tiny_lp()
    K = lp.K()
    Kt = O.precondition(K, lp.c, lp.q, lp.l, lp.u)[0]
    for A, iters, rel in ((K, 200, 1e-10), (Kt, 1000, 1e-9)):
        ref = float(np.linalg.norm(A.toarray(), 2))
        est = O.power_iteration_norm(A, iters)
        assert abs(est - ref) <= rel * ref, (est, ref)
        prev = 0.0
        for it in (1, 2, 5, 20, 100):
            e = O.power_iteration_norm(A, it)
            assert prev <= e * (1 + 1e-15) and e <= ref * (1 + 1e-14)
            prev = e
    # diagonal and rank-one matrices: the norm is known in closed form
    D = sp.csr_matrix(np.diag([0.5, -3.0, 2.0]))
    assert O.power_iteration_norm(D, 200) == pytest.approx(3.0, rel=1e-12)
    # (rank one: the second iterate is already the top right singular vector v / ||v||)
    u, v = np.array([1.0, 2.0, 2.0]), np.array([3.0, 4.0])
    assert O.power_iteration_norm(sp.csr_matrix(np.outer(u, v)), 2) == pytest.approx(15.0, rel=1e-14)


# ------------------------------------------------------------------------------------------
# normalized duality gap
# ------------------------------------------------------------------------------------------

def _bisection_trust_region(a, lo, hi, r, iters=400):
    """Independent solve of max a^T e over box and ball: bisection on the multiplier."""
    def e_of(s):
        return np.clip(s * a, lo, hi)
    far = e_of(1e300)
    far = np.where(a == 0, 0.0, far)
    if np.all(np.isfinite(far)) and float(far @ far) <= r * r:
        return float(a @ far)
    s_lo, s_hi = 0.0, 1.0
    while float(np.sum(e_of(s_hi) ** 2)) < r * r:
        s_hi *= 2.0
    for _ in range(iters):
        mid = 0.5 * (s_lo + s_hi)
        if float(np.sum(e_of(mid) ** 2)) < r * r:
            s_lo = mid
        else:
            s_hi = mid
    return float(a @ e_of(s_hi))


def test_trust_region_against_bisection_and_sampling():
    rng = np.random.default_rng(0)
    for _ in range(300):
        N = int(rng.integers(1, 8))
        a = rng.standard_normal(N)
        a[rng.random(N) < 0.1] = 0.0
        lo = -rng.exponential(1.0, N)
        hi = rng.exponential(1.0, N)
        lo[rng.random(N) < 0.3] = -np.inf
        hi[rng.random(N) < 0.3] = np.inf
        lo[rng.random(N) < 0.1] = 0.0
        r = float(rng.exponential(1.0)) + 1e-3
        v, _ = O.trust_region_linear_max(a, lo, hi, r)
        vb = _bisection_trust_region(a, lo, hi, r)
        assert abs(v - vb) <= 1e-10 * (1 + abs(v))
        # random feasible points never beat it
        e = rng.standard_normal((2000, N))
        e *= (r * rng.random((2000, 1)) ** (1.0 / N)) / np.linalg.norm(e, axis=1, keepdims=True)
        e = np.clip(e, lo, hi)
        assert np.max(e @ a) <= v + 1e-12


def test_normalized_gap_ball_inside_box():
    """Small radius around an interior point: the box is inactive and
    mu = ||a|| = sqrt(||g_x||^2/omega + omega ||g_y||^2)."""
    rng = np.random.default_rng(1)
    n, m, m1 = 6, 4, 2
    x = rng.uniform(2, 3, n)
    y = np.concatenate([rng.uniform(2, 3, m1), rng.standard_normal(m - m1)])
    gx, gy = rng.standard_normal(n), rng.standard_normal(m)
    omega = 0.7
    xr = x + 1e-3 * rng.standard_normal(n)
    yr = y + 1e-3 * rng.standard_normal(m)
    mu = O.normalized_gap(x, y, xr, yr, omega, gx, gy, np.zeros(n), np.full(n, 5.0), m1)
    expect = math.sqrt(gx @ gx / omega + omega * gy @ gy)
    assert abs(mu - expect) <= 1e-13 * expect


def test_normalized_gap_zero_at_optimum():
    lp = lpgen.tiny_lp()
    _, x, y = _highs(lp)
    K = lp.K()
    gx = lp.c - K.T @ y
    gy = lp.q - K @ x
    scale = float(np.linalg.norm(lp.c)) + float(np.linalg.norm(lp.q))
    for r_off in (1e-2, 1.0, 10.0):
        xr = x + r_off
        mu = O.normalized_gap(x, y, xr, y, 1.3, gx, gy, lp.l, lp.u, lp.m1)
        assert mu <= 1e-7 * scale


def test_normalized_gap_zero_radius():
    x = np.ones(3)
    y = np.ones(2)
    assert O.normalized_gap(x, y, x, y, 1.0, np.ones(3), np.ones(2), np.zeros(3), np.full(3, 2.0), 1) == 0.0


# ------------------------------------------------------------------------------------------
# restart rules and primal weight
# ------------------------------------------------------------------------------------------

def test_restart_mask_table():
    opts = O.Options()
    assert (opts.beta_sufficient, opts.beta_necessary, opts.beta_artificial) == (0.1, 0.9, 0.5)
    with open(os.path.join(GOLDEN, "restart_table.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            mu_c, mu_a, mu_p, t, k, n_out, expect = line.split()
            got = O.restart_mask(float(mu_c), float(mu_a), float(mu_p), int(t), int(k),
                                 int(n_out), opts)
            assert got == int(expect), line


def test_primal_weight_update_closed_form():
    # theta = 1/2: omega_new = sqrt(omega_prev * dy/dx)
    assert math.isclose(O.primal_weight_update(2.0, 8.0, 9.0, 0.5, 1e-10), 6.0, rel_tol=1e-15)
    assert O.primal_weight_update(0.0, 8.0, 9.0, 0.5, 1e-10) == 9.0
    assert O.primal_weight_update(2.0, 1e-12, 9.0, 0.5, 1e-10) == 9.0
    assert math.isclose(O.primal_weight_update(2.0, 8.0, 9.0, 1.0, 1e-10), 4.0, rel_tol=1e-15)
    assert O.initial_primal_weight(np.array([3.0, 4.0]), np.array([0.0, 2.0]), 1e-10) == 2.5
    assert O.initial_primal_weight(np.zeros(2), np.array([0.0, 2.0]), 1e-10) == 1.0


def test_first_checks_restart_artificially():
    """In the first outer loop t = k, so criterion (iii) restarts at k = 40; at k = 80,
    t = 40 >= 0.5 * 80 restarts again (reading Z9)."""
    r = O.solve_lp(lpgen.tiny_lp(), tol=1e-8, iter_limit=80, record_trace=True)
    ch = r.trace.checks
    assert [c["k"] for c in ch] == [40, 80]
    assert ch[0]["mask"] & O.RESTART_ARTIFICIAL and ch[1]["mask"] & O.RESTART_ARTIFICIAL
    assert r.restarts == 2


# ------------------------------------------------------------------------------------------
# preconditioning
# ------------------------------------------------------------------------------------------

def test_ruiz_norms_converge_to_one():
    lp = lpgen.large_plain(3, 300, 600)
    spreads = []
    for it in (1, 2, 4, 8, 16, 32):
        Kt = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u, ruiz_iters=it, pock_chambolle=False)[0]
        A = abs(Kt)
        rn = np.asarray(A.max(axis=1).todense()).ravel()
        cn = np.asarray(A.max(axis=0).todense()).ravel()
        spreads.append(max(abs(np.log(rn)).max(), abs(np.log(cn)).max()))
    assert all(b <= a + 1e-12 for a, b in zip(spreads, spreads[1:]))
    assert spreads[-1] < 1e-3


def test_pock_chambolle_spectral_bound_and_same_optimum():
    lp = lpgen.tiny_lp()
    Kt, ct, qt, lt, ut, D1, D2 = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)
    assert np.linalg.norm(Kt.toarray(), 2) <= 1.0 + 1e-12
    np.testing.assert_allclose(Kt.toarray(), np.diag(D1) @ lp.K().toarray() @ np.diag(D2), rtol=1e-13)
    sc = lpgen.from_csr(Kt, ct, qt, lt, ut, lp.n_eq)
    f0, _, _ = _highs(lp)
    f1, _, _ = _highs(sc)
    assert abs(f0 - f1) <= 1e-8 * abs(f0)


def test_scaling_keeps_infinite_bounds_and_empty_rows():
    lp = lpgen.add_empty_row_and_column(lpgen.large_plain(5, 100, 200))
    Kt, ct, qt, lt, ut, D1, D2 = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)
    assert D1[0] == 1.0 and D2[-1] == 1.0
    assert np.array_equal(np.isinf(lt), np.isinf(lp.l)) and np.array_equal(np.isinf(ut), np.isinf(lp.u))
    r = O.solve_lp(lp, tol=1e-8, iter_limit=100000)
    assert r.status == O.OPTIMAL
    fun, _, _ = _highs(lp)
    assert abs(r.kkt["pobj"] - fun) <= 1e-6 * (1 + abs(fun))


# ------------------------------------------------------------------------------------------
# Proposition 1 (Appendix A) and the PageRank fixed point (Appendix D)
# ------------------------------------------------------------------------------------------

def _scaled_lp(lp, gamma, ax, ay):
    return lpgen.from_csr(gamma * lp.K(), gamma * ay * lp.c, gamma * ax * lp.q, ax * lp.l,
                          ax * lp.u, lp.n_eq)


def test_scale_invariance_constant_step_bitwise():
    """Proposition 1 with powers of two: x^ = a_x x and y^ = a_y y exactly for the baseline
    PDHG (constant step, omega = InitializePrimalWeight, no scaling, no restarts)."""
    lp = lpgen.tiny_lp()
    g, ax, ay = 4.0, 2.0, 8.0
    opts = O.Options(ruiz_iters=0, pock_chambolle=False, step_policy="constant", restarts=False,
                     power_iters=100)
    a = O.solve_lp(lp, 1e-30, 60, opts, trace_iters=60)
    b = O.solve_lp(_scaled_lp(lp, g, ax, ay), 1e-30, 60, opts, trace_iters=60)
    for (k1, x1, y1), (k2, x2, y2) in zip(a.trace.iterates, b.trace.iterates):
        assert np.array_equal(ax * x1, x2) and np.array_equal(ay * y1, y2), k1


def test_scale_invariance_full_pdlp():
    """The same invariance for full PDLP (scaling, adaptive steps, restarts, primal weight):
    bitwise before the first primal-weight update; after it the log/exp of Algorithm 3 round
    differently on the two problems and the trajectories agree to round-off amplified by the
    iteration (1e-9 relative over 200 steps)."""
    lp = lpgen.tiny_lp()
    g, ax, ay = 4.0, 2.0, 8.0
    a = O.solve_lp(lp, 1e-30, 200, trace_iters=200)
    b = O.solve_lp(_scaled_lp(lp, g, ax, ay), 1e-30, 200, trace_iters=200)
    for (k1, x1, y1), (k2, x2, y2) in zip(a.trace.iterates, b.trace.iterates):
        # Ruiz maps gamma*K (gamma = 4) to the same K~ with D1, D2 halved, so the scaled
        # problems are related by x~^ = 4 x~ and y~^ = 16 y~
        if k1 < 40:
            assert np.array_equal(4.0 * x1, x2) and np.array_equal(16.0 * y1, y2), k1
        else:
            np.testing.assert_allclose(4.0 * x1, x2, rtol=1e-9, atol=1e-9 * np.abs(x2).max())
            np.testing.assert_allclose(16.0 * y1, y2, rtol=1e-9, atol=1e-9 * np.abs(y2).max())
    np.testing.assert_allclose(ax * a.x, b.x, rtol=1e-8, atol=1e-8)


def test_pagerank_solution_is_the_stationary_vector():
    N = 2000
    lp = lpgen.pagerank_lp(2, N)
    r = O.solve_lp(lp, tol=1e-8, iter_limit=100000)
    assert r.status == O.OPTIMAL
    K = lp.K()
    S = -(K[:N, :N] - sp.eye(N)) / 0.85          # recover S' from the rows
    assert np.allclose(np.asarray(S.sum(axis=0)).ravel(), 1.0)
    pi = np.full(N, 1.0 / N)
    for _ in range(400):
        pi = 0.85 * (S @ pi) + 0.15 / N
    assert np.abs(r.x - pi).sum() < 1e-6
    assert abs(r.kkt["pobj"]) == 0.0


# ------------------------------------------------------------------------------------------
# unrolled PDHG adjoint: reverse mode vs central finite differences of the forward map
# ------------------------------------------------------------------------------------------

def test_unroll_adjoint_matches_finite_differences():
    lp = lpgen.tiny_plain(9, 60, 120, 24, 4)
    Kt, ct, qt, lt, ut, D1, D2 = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)
    eta = 0.9 / O.power_iteration_norm(Kt, 200)
    omega = O.initial_primal_weight(ct, qt, 1e-10)
    T = 30
    rng = np.random.default_rng(0)
    x_tgt = rng.uniform(0, 5, lp.n)

    def loss(c_t, q_t):
        xs, _ = O.unroll_forward(Kt, c_t, q_t, lt, ut, lp.m1, eta, omega, T)
        return float(np.sum((xs[-1] - x_tgt) ** 2))

    xs, ys = O.unroll_forward(Kt, ct, qt, lt, ut, lp.m1, eta, omega, T)
    gc, gq = O.unroll_backward(Kt, lt, ut, lp.m1, eta, omega, xs, ys, 2.0 * (xs[-1] - x_tgt))
    h = 1e-6
    for j in rng.choice(lp.n, 12, replace=False):
        e = np.zeros(lp.n)
        e[j] = h
        fd = (loss(ct + e, qt) - loss(ct - e, qt)) / (2 * h)
        assert abs(fd - gc[j]) <= 1e-6 * (1 + abs(fd)), (j, fd, gc[j])
    for i in rng.choice(lp.m, 12, replace=False):
        e = np.zeros(lp.m)
        e[i] = h
        fd = (loss(ct, qt + e) - loss(ct, qt - e)) / (2 * h)
        assert abs(fd - gq[i]) <= 1e-6 * (1 + abs(fd)), (i, fd, gq[i])


def test_unroll_one_step_closed_form():
    # T = 1 from x0 = proj(0), y0 = 0: x1 = clip(x0 - tau c~), so with x~ the only path,
    # dL/dc~ = -tau * mask * dL/dx~_1 and dL/dq~ = 0 for a loss on x_1 alone.
    lp = lpgen.tiny_plain(5, 30, 70, 12, 4)
    Kt, ct, qt, lt, ut, D1, D2 = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)
    eta, omega = 0.3, 1.7
    xs, ys = O.unroll_forward(Kt, ct, qt, lt, ut, lp.m1, eta, omega, 1)
    x0 = np.clip(np.zeros(lp.n), lt, ut)
    assert np.array_equal(xs[1], np.clip(x0 - (eta / omega) * ct, lt, ut))
    g = np.random.default_rng(1).standard_normal(lp.n)
    gc, gq = O.unroll_backward(Kt, lt, ut, lp.m1, eta, omega, xs, ys, g)
    inside = (xs[1] > lt) & (xs[1] < ut)
    assert np.allclose(gc, -(eta / omega) * inside * g, rtol=0, atol=1e-15)
    assert np.all(gq == 0.0)


def test_unroll_user_units_gradient_matches_finite_differences():
    # the full map (c, q) -> ||x_T - x_tgt||^2 + <gy, y_T> in the user's units, on an LP with
    # free, one-sided and boxed columns; D1, D2 depend on K only, eta and omega are held fixed.
    lp = lpgen.tiny_plain(11, 40, 90, 16, 4)
    rng = np.random.default_rng(2)
    l = lp.l.copy()
    u = lp.u.copy()
    l[:20] = -np.inf
    u[:20] = np.inf                 # free
    u[20:40] = np.inf               # [0, inf)
    x_tgt = rng.uniform(0, 5, lp.n)
    gy = rng.standard_normal(lp.m)
    K = lp.K()
    base = O.unroll_user(K, lp.c, lp.q, l, u, lp.m1, x_tgt, 25, gy_T=gy)
    eta, omega = base["eta"], base["omega"]

    def loss(c, q):
        return O.unroll_user(K, c, q, l, u, lp.m1, x_tgt, 25, eta, omega, gy_T=gy)["loss"]

    h = 1e-6
    for j in rng.choice(lp.n, 10, replace=False):
        e = np.zeros(lp.n)
        e[j] = h
        fd = (loss(lp.c + e, lp.q) - loss(lp.c - e, lp.q)) / (2 * h)
        assert abs(fd - base["gc"][j]) <= 1e-6 * (1 + abs(fd)), (j, fd, base["gc"][j])
    for i in rng.choice(lp.m, 10, replace=False):
        e = np.zeros(lp.m)
        e[i] = h
        fd = (loss(lp.c, lp.q + e) - loss(lp.c, lp.q - e)) / (2 * h)
        assert abs(fd - base["gq"][i]) <= 1e-6 * (1 + abs(fd)), (i, fd, base["gq"][i])


# ------------------------------------------------------------------------------------------
# Malitsky-Pock line search (Appendix C)
# ------------------------------------------------------------------------------------------

def test_malitsky_pock_without_interpolation_is_fixed_step_pdhg():
    # interpolation 0 keeps eta^ = eta_k and theta^ = 1, so the trial is the extrapolation
    # 2x' - x of Eq. (3); with eta <= 1/||K~||_2 the test eta ||K^T dy|| <= ||dy|| always
    # holds, so the line search accepts every first trial and follows fixed-step PDHG.
    lp = lpgen.tiny_plain(21, 50, 110, 20, 4)
    Kt, ct, qt, lt, ut, D1, D2 = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)
    KT = Kt.T.tocsr()
    eta = 0.9 / np.linalg.norm(Kt.toarray(), 2)
    omega = 1.3
    x = np.clip(np.zeros(lp.n), lt, ut)
    y = np.zeros(lp.m)
    xr, yr = x.copy(), y.copy()
    theta = 1.0
    for _ in range(60):
        xp = np.clip(x - (eta / omega) * (ct - KT @ y), lt, ut)
        eh, th = O.mp_candidate(eta, theta, 0.0)
        assert eh == eta and th == 1.0
        yp = O.mp_dual_trial(x, xp, y, eh, th, omega, Kt, qt, lp.m1)
        assert O.mp_accepts(eh, yp - y, KT @ (yp - y), 1.0)
        x, y, theta = xp, yp, th
        xr, yr = O.pdhg_step(xr, yr, eta, omega, ct, Kt, KT, qt, lt, ut, lp.m1)
        assert np.allclose(x, xr, rtol=1e-12, atol=1e-12) and np.allclose(y, yr, rtol=1e-12, atol=1e-12)


def test_malitsky_pock_candidate_range():
    # eta^ lies in [eta_k, sqrt(1 + theta_k) eta_k], at the ends for interpolation 0 and 1
    for theta in (0.25, 1.0, 3.0):
        lo, _ = O.mp_candidate(2.0, theta, 0.0)
        hi, th = O.mp_candidate(2.0, theta, 1.0)
        assert lo == 2.0 and abs(hi - 2.0 * math.sqrt(1.0 + theta)) < 1e-15 and abs(th - 2.0 / hi) < 1e-16
        mid, _ = O.mp_candidate(2.0, theta, 0.4)
        assert lo < mid < hi


def test_malitsky_pock_solves_to_highs_objective():
    lp = lpgen.tiny_lp()
    opts = O.Options(step_policy="malitsky_pock")
    r = O.solve_lp(lp, tol=1e-8, iter_limit=60000, opts=opts, record_trace=True)
    assert r.status == O.OPTIMAL and r.kkt["kkt"] <= 1e-8
    ref, _, _ = _highs(lp)
    assert abs(float(lp.c @ r.x) - ref) <= 1e-6 * max(1.0, abs(ref))
    # every logged trial obeys the acceptance rule it reports
    rejected = 0
    for (k, eta, eta_bar, acc) in r.trace.attempts:
        rejected += not acc
        if math.isinf(eta_bar):
            assert acc
        elif abs(eta - eta_bar) > 1e-12 * eta:
            assert acc == (eta < eta_bar)
    assert rejected > 0          # the line search did shrink steps on this LP


def test_no_restart_mode_updates_weight_at_powers_of_two():
    # Appendix C "no restart": restarts off, primal weight still updated at k = 2, 4, 8, ...
    lp = lpgen.tiny_plain(4, 60, 140, 24, 4)
    opts = O.Options(restarts=False, pw_power_of_two=True)
    r = O.solve_lp(lp, tol=1e-30, iter_limit=300, opts=opts, record_states=300)
    states = r.trace.states
    changed = [s["k"] for a, s in zip(states, states[1:]) if s["omega"] != a["omega"]]
    assert changed == [2, 4, 8, 16, 32, 64, 128, 256]
    # the anchor is the iterate of the previous update; iterates and averages are not reset
    for st in states:
        if st["k"] in (64, 128):
            assert np.array_equal(st["xa"], st["x"]) and st["t"] == st["k"]
    assert r.restarts == 8
    # without the mode, restarts off keeps the initial weight
    r0 = O.solve_lp(lp, tol=1e-30, iter_limit=300, opts=O.Options(restarts=False), record_states=300)
    assert len({s["omega"] for s in r0.trace.states}) == 1
