"""GPU parity of the HIP solver against the CPU oracle (run on an MI355X).

Every case prints what it runs before touching the GPU.  The bars:
  * preconditioning D1, D2 and the products: relative 1e-13 (round-off of sums in another order);
  * the first 100 accepted iterates: relative 1e-11 per iterate, separately for x and y, and
    identical accept/reject, candidate and restart decisions;
  * a full solve: the oracle's own KKT evaluation of the GPU's answer <= 1e-8 and the
    objective matching HiGHS;
  * integer-like outcomes (status, counts, decisions): exact.
"""
import math
import sys

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import paper_2106_04756_amd as P
from oracle import pdlp_oracle as O
from workloads import lpgen
from replay import rel, replay_steps, row_bound, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def make(lp, **kw):
    return P.Solver.from_lp(lp, **kw)


# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("panels,order,sub", [(0, 0, -1), (1, 0, -1), (1, 1, -1), (1, 0, 3), (1, 1, 2)])
def test_spmv_matches_scipy_on_ragged_shapes(panels, order, sub):
    """Unscaled products (no preconditioning) on every schedule path: lane-group rows of
    every width, one-workgroup rows, split giant rows, empty rows/columns; in the plain row
    layout and in XCD column panels, whole or cut into sub-panels."""
    import torch
    rng = np.random.default_rng(5)
    m, n = 3000, 70000
    lens = np.concatenate([rng.poisson(3, m - 6), [0, 600, 5000, 16385, 40000, 70000]])
    rows, cols = [], []
    for i, ln in enumerate(lens):
        cs = rng.choice(n, size=min(ln, n), replace=False)
        rows.append(np.full(cs.size, i))
        cols.append(cs)
    K = sp.csr_matrix((rng.standard_normal(int(lens.sum())), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, n))
    K.sort_indices()
    lp = lpgen.from_csr(K, np.ones(n), np.zeros(m), np.zeros(n), np.full(n, 1.0), n_eq=0)
    say("spmv ragged", m, n, K.nnz, "panels", panels, "order", order, "sub-panels", sub)
    kw = dict(xcd_panels=panels, column_order=order)
    if sub > 0:
        kw.update(lds_gather=0, xcd_subpanels=sub)
    s = make(lp, ruiz_iters=0, pock_chambolle=0, **kw)
    if sub > 0:
        assert (s.info()["panels_K"], s.info()["panels_KT"]) == (8 * sub, 8 * sub)
    for trial in range(2):
        x = rng.standard_normal(n)
        y = rng.standard_normal(m)
        out = torch.empty(m, dtype=torch.float64, device="cuda")
        s.spmv(torch.from_numpy(x).cuda(), out)
        ref = K @ x
        scale = abs(K) @ np.abs(x)
        assert np.all(np.abs(out.cpu().numpy() - ref) <= 1e-13 * scale + 1e-300)
        outT = torch.empty(n, dtype=torch.float64, device="cuda")
        s.spmv(torch.from_numpy(y).cuda(), outT, transpose=True)
        refT = K.T @ y
        scaleT = abs(K.T) @ np.abs(y)
        assert np.all(np.abs(outT.cpu().numpy() - refT) <= 1e-13 * scaleT + 1e-300)


LDS_MODES = {
    # one panel per 64-column slice, every gather from LDS
    "slices": dict(xcd_panels=1, lds_gather=1, lds_entries=64),
    # XCD panels, hot columns first, each panel's first 50 columns staged, the rest from memory
    "xcd_stage": dict(xcd_panels=1, column_order=1, lds_gather=2, lds_entries=50),
}


@pytest.mark.parametrize("mode", sorted(LDS_MODES))
def test_spmv_with_lds_stage_matches_scipy(mode):
    """Products with the gathered operand staged in LDS: rows of every lane width up to the
    512-entry limit of the LDS path, empty rows and columns, several tasks per segment."""
    import torch
    rng = np.random.default_rng(9)
    m, n = 2500, 9000
    lens = np.concatenate([rng.poisson(6, m - 8), [0, 0, 1, 64, 65, 200, 511, 512]])
    rows, cols = [], []
    for i, ln in enumerate(lens):
        cs = rng.choice(n - 3, size=ln, replace=False)       # the last 3 columns stay empty
        rows.append(np.full(cs.size, i))
        cols.append(cs)
    K = sp.csr_matrix((rng.standard_normal(int(lens.sum())), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, n))
    K.sort_indices()
    lp = lpgen.from_csr(K, np.ones(n), np.zeros(m), np.zeros(n), np.full(n, 1.0), n_eq=0)
    say("spmv lds", mode, m, n, K.nnz)
    s = make(lp, ruiz_iters=0, pock_chambolle=0, **LDS_MODES[mode])
    for trial in range(2):
        x = rng.standard_normal(n)
        y = rng.standard_normal(m)
        out = torch.empty(m, dtype=torch.float64, device="cuda")
        s.spmv(torch.from_numpy(x).cuda(), out)
        assert np.all(np.abs(out.cpu().numpy() - K @ x) <= row_bound(K, x))
        outT = torch.empty(n, dtype=torch.float64, device="cuda")
        s.spmv(torch.from_numpy(y).cuda(), outT, transpose=True)
        KT = K.T.tocsr()
        assert np.all(np.abs(outT.cpu().numpy() - KT @ y) <= row_bound(KT, y))


@pytest.mark.parametrize("panels", [0, 1])
def test_preconditioning_matches_oracle(panels):
    for lp in (lpgen.tiny_lp(), lpgen.large_plain(11, 2000, 4000), lpgen.pagerank_lp(2, 30000)):
        say("scaling", lp.name, lp.m, lp.n, lp.nnz, "panels", panels)
        s = make(lp, xcd_panels=panels)
        D1, D2 = s.scaling()
        _, _, _, _, _, oD1, oD2 = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)
        assert np.max(np.abs(D1 / oD1 - 1)) < 1e-13
        assert np.max(np.abs(D2 / oD2 - 1)) < 1e-13


def _trajectory_parity(lp, iters=100, opts=None, calibrate=False, **kw):
    """Free-running: the GPU's first `iters` iterates against the oracle's, 1e-11 relative per
    iterate, the step sizes, decisions and checks beside them.  calibrate=True widens every
    bar to 10 times the oracle's own divergence at that point when only the order of its sums
    over the columns changes (_calibration), where the trajectory amplifies round-off beyond the
    fixed bars; decisions must still be identical."""
    opts = opts or O.Options()
    say("trajectory", lp.name, lp.m, lp.n, lp.nnz, kw, "calibrated" if calibrate else "")
    s = make(lp, trace_iters=iters, **kw)
    st = s.solve(1e-30, iters)
    assert st == P.ITERATION_LIMIT
    tr = s.trace()
    ref = O.solve_lp(lp, tol=1e-30, iter_limit=iters, opts=opts, trace_iters=iters)
    assert tr["n_iter"] == iters == len(ref.trace.iterates)
    cal = _calibration(lp, ref, iters, opts) if calibrate else None
    worst = 0.0
    for k in range(iters):
        kk, xo, yo = ref.trace.iterates[k]
        ex = rel(tr["xs"][k], xo)
        ey = rel(tr["ys"][k], yo) if lp.m else 0.0
        bar = max(1e-11, 10 * cal["iterate"][k]) if cal else 1e-11
        worst = max(worst, ex / bar, ey / bar)
        assert ex <= bar and ey <= bar, (k + 1, ex, ey, bar)
    ga = tr["attempts"]
    oa = ref.trace.attempts
    assert len(ga) == len(oa)
    for i, (g, o) in enumerate(zip(ga, oa)):
        assert g[0] == o[0] and g[3] == o[3]
        # the step tried is the previous proposal of Algorithm 2, min((1 - (k+1)^-0.3) eta_bar,
        # (1 + (k+1)^-0.6) eta): eta_bar's denominator 2 |dy^T K dx| cancels, so it carries the
        # last-bit differences of the dot products (summed in another order on the GPU) with a
        # gain of ~1e2 along a free-running trajectory; the iterates themselves stay at 1e-11
        assert abs(g[1] - o[1]) <= max(1e-10, 10 * cal["eta"][i] if cal else 0.0) * o[1]
        if math.isfinite(o[2]):
            assert abs(g[2] - o[2]) <= max(1e-9, 10 * cal["eta_bar"][i] if cal else 0.0) * o[2]
    gc, oc = tr["checks"], ref.trace.checks
    assert len(gc) == len(oc)
    for j, (g, o) in enumerate(zip(gc, oc)):
        assert g["k"] == o["k"] and g["use_avg"] == o["use_avg"] and g["mask"] == o["mask"]
        tol = max(1e-11, 10 * cal["omega_after"][j] if cal else 0.0)
        assert abs(g["omega_after"] - o["omega_after"]) <= tol * o["omega_after"]
        for key in ("mu_cur", "mu_avg"):
            if math.isfinite(o[key]):
                tol = max(1e-9, 10 * cal[key][j] if cal else 0.0)
                assert abs(g[key] - o[key]) <= tol * max(abs(o[key]), 1e-300), key
    return worst


def _calibration(lp, ref, iters, opts, seeds=(5, 6, 7)):
    """The oracle's own sensitivity along this trajectory: the oracle run again on the same LP
    with its columns in a random order (every sum over the columns taken in another order,
    nothing else changed), for three orders, and the largest relative difference of each
    iterate, each attempt's step and step limit, and each check's gaps and primal weight (one
    order alone can understate it by 10 times at some steps).  Its decisions must match the
    first run's, which is what makes the comparison point by point."""
    out = {"iterate": np.zeros(iters)}
    oa, oc = ref.trace.attempts, ref.trace.checks
    out["eta"] = np.zeros(len(oa))
    out["eta_bar"] = np.zeros(len(oa))
    for key in ("omega_after", "mu_cur", "mu_avg"):
        out[key] = np.zeros(len(oc))
    for seed in seeds:
        perm = np.random.default_rng(seed).permutation(lp.n)
        K = lp.K()[:, perm].tocsr()
        K.sort_indices()
        lp2 = lpgen.from_csr(K, lp.c[perm], lp.q, lp.l[perm], lp.u[perm], lp.n_eq, name=lp.name + " permuted")
        r2 = O.solve_lp(lp2, tol=1e-30, iter_limit=iters, opts=opts, trace_iters=iters)
        for k in range(iters):
            _, x1, y1 = ref.trace.iterates[k]
            _, x2, y2 = r2.trace.iterates[k]
            xb = np.empty_like(x2)
            xb[perm] = x2
            out["iterate"][k] = max(out["iterate"][k], rel(xb, x1), rel(y2, y1) if lp.m else 0.0)
        pa, pc = r2.trace.attempts, r2.trace.checks
        assert len(oa) == len(pa) and all(o[0] == q[0] and o[3] == q[3] for o, q in zip(oa, pa))
        for i, (o, q) in enumerate(zip(oa, pa)):
            out["eta"][i] = max(out["eta"][i], abs(q[1] - o[1]) / o[1])
            if math.isfinite(o[2]) and math.isfinite(q[2]):
                out["eta_bar"][i] = max(out["eta_bar"][i], abs(q[2] - o[2]) / o[2])
        assert len(oc) == len(pc) and all(o["k"] == q["k"] and o["use_avg"] == q["use_avg"] and
                                          o["mask"] == q["mask"] for o, q in zip(oc, pc))
        for key in ("omega_after", "mu_cur", "mu_avg"):
            for j, (o, q) in enumerate(zip(oc, pc)):
                if math.isfinite(o[key]):
                    out[key][j] = max(out[key][j], abs(q[key] - o[key]) / max(abs(o[key]), 1e-300))
    return out


def test_trajectory_parity_tiny_lp():
    """Free-running: the GPU's first 100 iterates against the oracle's, 1e-11 per iterate."""
    _trajectory_parity(lpgen.tiny_lp())


def test_trajectory_parity_tiny_lp_reordered_columns():
    """The same with the internal column order (dense columns first in each XCD panel): every
    n-vector of the trace comes back in the user's order."""
    _trajectory_parity(lpgen.tiny_lp(), xcd_panels=1, column_order=1)


@pytest.mark.parametrize("seed", [21, 22])
@pytest.mark.parametrize("kw", [dict(), dict(xcd_panels=1, column_order=1)])
def test_trajectory_parity_400x900(seed, kw):
    """Free-running on two 400 x 900 LPs of the large-LP recipe over the first 100 steps (two
    restart checks): each iterate within 1e-11, or within 10 times the oracle's own divergence
    at that step when only the order of its column sums changes, where this trajectory
    amplifies round-off beyond 1e-11 (seed 22: 5e-11 at k = 57, 2e-10 at k = 100); the step
    sizes and gaps likewise; accept/reject and restart decisions identical."""
    worst = _trajectory_parity(lpgen.large_plain(seed, 400, 900), iters=100, calibrate=True, **kw)
    say("worst error / bar", worst)


@pytest.mark.parametrize("maker", [lambda: lpgen.pagerank_lp(2, 20000), lambda: lpgen.batched_instance(1)],
                         ids=["pagerank_2e4", "batched_member_1"])
def test_trajectory_parity_calibrated(maker):
    """The calibrated free-running comparison (see test_trajectory_parity_400x900) on the
    PageRank LP on 2e4 nodes, whose trajectory amplifies round-off most (the oracle moves
    itself by up to 5e-9 per iterate and 7e-6 in the step limit within 100 steps), and on a
    member of the batched workload, in the default layout."""
    worst = _trajectory_parity(maker(), iters=100, calibrate=True)
    say("worst error / bar", worst)


def _replay_parity(lp, steps=100, opts=None, **kw):
    """Replayed steps: for k = 0..steps-1 the GPU is put in the oracle's exact state before
    step k+1 and must land on the oracle's state after it (replay.replay_steps).  This tests
    every step's arithmetic without the amplification of round-off that a free-running PDLP
    trajectory shows (the step-size ratio of Algorithm 2 is ill-conditioned, so last-bit
    differences grow along a trajectory)."""
    ref = O.solve_lp(lp, tol=1e-30, iter_limit=steps, opts=opts, record_states=steps,
                     trace_iters=steps, record_trace=True)
    o = opts or O.Options()
    Kt, ct, qt = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u, ruiz_iters=o.ruiz_iters,
                                pock_chambolle=o.pock_chambolle)[:3]
    say("replay", lp.name, lp.m, lp.n, lp.nnz, kw)
    replay_steps(make(lp, **kw), ref, Kt, range(steps), ct, qt)


@pytest.mark.parametrize("maker", [
    lpgen.tiny_lp,
    lambda: lpgen.large_plain(21, 400, 900),
    lambda: lpgen.large_plain(22, 400, 900),
    lambda: lpgen.add_empty_row_and_column(lpgen.tiny_plain(1, 150, 300, 60, 4)),
    lambda: lpgen.pagerank_lp(2, 20000),
])
def test_replayed_step_parity(maker):
    _replay_parity(maker())


@pytest.mark.parametrize("maker", [
    lpgen.tiny_lp,
    lambda: lpgen.large_plain(21, 400, 900),
    lambda: lpgen.pagerank_lp(2, 20000),
])
def test_replayed_step_parity_xcd_panels(maker):
    _replay_parity(maker(), xcd_panels=1)


@pytest.mark.parametrize("maker", [
    lambda: lpgen.large_plain(21, 400, 900),
    lambda: lpgen.pagerank_lp(2, 20000),
])
def test_replayed_step_parity_xcd_subpanels(maker):
    """Both copies in XCD panels cut into two sub-panels each, taken one after another."""
    _replay_parity(maker(), xcd_panels=1, lds_gather=0, xcd_subpanels=2)


def test_trajectory_parity_tiny_lp_xcd_subpanels():
    _trajectory_parity(lpgen.tiny_lp(), xcd_panels=1, lds_gather=0, xcd_subpanels=3)


@pytest.mark.parametrize("mode", sorted(LDS_MODES))
@pytest.mark.parametrize("maker", [lpgen.tiny_lp, lambda: lpgen.large_plain(21, 400, 900)])
def test_replayed_step_parity_lds_stage(maker, mode):
    _replay_parity(maker(), **LDS_MODES[mode])


@pytest.mark.parametrize("mode", sorted(LDS_MODES))
def test_trajectory_parity_tiny_lp_lds_stage(mode):
    _trajectory_parity(lpgen.tiny_lp(), **LDS_MODES[mode])


@pytest.mark.parametrize("maker", [lpgen.tiny_lp, lambda: lpgen.large_plain(21, 400, 900)])
def test_replayed_step_parity_reordered_columns(maker):
    """Checkpoints in and out (x, anchor, weighted sums) cross the interface in the user's
    order while the solver keeps its own column order."""
    _replay_parity(maker(), xcd_panels=1, column_order=1)


# the paper's ablation switches (Appendix C): same option on both sides
ABLATIONS = {
    "constant_step": (dict(step_policy="constant"), dict(step_policy=1)),
    "no_restarts": (dict(restarts=False), dict(adaptive_restarts=0)),
    "restart_theory": (dict(beta_sufficient=0.37, beta_necessary=0.37, restart_to_current=False),
                       dict(beta_sufficient=0.37, beta_necessary=0.37, restart_to_current=0)),
    "fixed_weight": (dict(primal_weight_update=False, primal_importance=0.1),
                     dict(primal_weight_update=0, primal_importance=0.1)),
    "no_scaling": (dict(ruiz_iters=0, pock_chambolle=False), dict(ruiz_iters=0, pock_chambolle=0)),
    "ruiz_only": (dict(pock_chambolle=False), dict(pock_chambolle=0)),
    "pock_chambolle_only": (dict(ruiz_iters=0), dict(ruiz_iters=0)),
    "no_restart_weight_at_2j": (dict(restarts=False, pw_power_of_two=True),
                                dict(adaptive_restarts=0, pw_power_of_two=1)),
}


@pytest.mark.parametrize("name", sorted(ABLATIONS))
def test_ablation_switches_replay(name):
    o_kw, g_kw = ABLATIONS[name]
    _replay_parity(lpgen.large_plain(21, 400, 900), steps=90, opts=O.Options(**o_kw), **g_kw)


def test_constant_step_uses_power_iteration_norm():
    lp = lpgen.tiny_lp()
    say("constant step size")
    s = make(lp, step_policy=1)
    Kt = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)[0]
    eta = 0.9 / O.power_iteration_norm(Kt, 200)
    assert abs(s.get_state()["eta_hat"] - eta) <= 1e-12 * eta
    # power iteration approaches ||K~||_2 from below
    sigma_est, sigma = 0.9 / eta, np.linalg.norm(Kt.toarray(), 2)
    assert 0.99 * sigma <= sigma_est <= sigma * (1 + 1e-12)


def test_solve_tiny_lp_to_1e8():
    lp = lpgen.tiny_lp()
    say("solve tiny_lp")
    s = make(lp)
    st = s.solve(1e-8, 100000)
    assert st == P.OPTIMAL
    x, y, kkt = s.get()
    k = O.kkt(lp.c, lp.K(), lp.q, lp.l, lp.u, lp.n_eq, x, y)
    assert k["kkt"] <= 1e-8
    assert abs(k["kkt"] - kkt[3]) <= 1e-10
    K = lp.K()
    res = linprog(lp.c, A_ub=-K[:lp.m1], b_ub=-lp.q[:lp.m1], A_eq=K[lp.m1:], b_eq=lp.q[lp.m1:],
                  bounds=list(zip(lp.l, lp.u)), method="highs")
    assert abs(k["pobj"] - res.fun) <= 1e-7 * abs(res.fun)
    ref = O.solve_lp(lp, tol=1e-8)
    info = s.info()
    # beyond the first iterates the two trajectories may part on a near-tie; the work to
    # reach 1e-8 stays of the same size
    assert 0.5 * ref.k <= info["iterations"] <= 2 * ref.k


@pytest.mark.parametrize("panels", [0, 1])
def test_malitsky_pock_trajectory_parity(panels):
    """The line search of Appendix C (step_policy 2): the first 100 iterates, every trial's
    step and acceptance, and the checks against the oracle, free-running, in the plain row
    layout and in forced XCD panels."""
    worst = _trajectory_parity(lpgen.tiny_lp(), opts=O.Options(step_policy="malitsky_pock"), step_policy=2,
                               xcd_panels=panels)
    say("malitsky-pock worst iterate error / 1e-11", worst)


@pytest.mark.parametrize("panels", [0, 1])
def test_malitsky_pock_trajectory_parity_400x900(panels):
    """The line search on a 400 x 900 LP of the large-LP recipe, free-running over 100
    iterations, calibrated as in test_trajectory_parity_400x900 (on this LP the oracle's own
    divergence stays below 1e-13, so the bar is 1e-11 throughout)."""
    worst = _trajectory_parity(lpgen.large_plain(21, 400, 900), opts=O.Options(step_policy="malitsky_pock"),
                               calibrate=True, step_policy=2, xcd_panels=panels, column_order=panels)
    say("malitsky-pock 400x900 worst error / bar", worst)


def test_malitsky_pock_solve_to_1e8():
    lp = lpgen.tiny_lp()
    say("solve tiny_lp malitsky-pock")
    s = make(lp, step_policy=2)
    st = s.solve(1e-8, 100000)
    assert st == P.OPTIMAL
    x, y, kkt = s.get()
    k = O.kkt(lp.c, lp.K(), lp.q, lp.l, lp.u, lp.n_eq, x, y)
    assert k["kkt"] <= 1e-8
    ref = O.solve_lp(lp, tol=1e-8, opts=O.Options(step_policy="malitsky_pock"))
    info = s.info()
    assert 0.5 * ref.k <= info["iterations"] <= 2 * ref.k
    # each iteration forms K~ x' once and K~^T y^ once per trial
    assert info["spmv_K"] >= info["iterations"] and info["spmv_KT"] >= info["attempts"]


def test_solve_pagerank_matches_stationary_vector():
    N = 20000
    lp = lpgen.pagerank_lp(2, N)
    say("solve pagerank", N)
    s = make(lp)
    assert s.solve(1e-8, 200000) == P.OPTIMAL
    x, y, kkt = s.get()
    K = lp.K()
    assert O.kkt(lp.c, K, lp.q, lp.l, lp.u, lp.n_eq, x, y)["kkt"] <= 1e-8
    S = -(K[:N, :N] - sp.eye(N)) / 0.85
    pi = np.full(N, 1.0 / N)
    for _ in range(400):
        pi = 0.85 * (S @ pi) + 0.15 / N
    assert np.abs(x - pi).sum() < 1e-6


@pytest.mark.parametrize("panels", [0, 1])
def test_two_runs_are_bitwise_equal_and_resume_is_seamless(panels):
    lp = lpgen.large_plain(31, 3000, 7000)
    say("determinism", lp.nnz, "panels", panels)
    a = make(lp, xcd_panels=panels)
    b = make(lp, xcd_panels=panels)
    a.solve(1e-30, 300)
    b.solve(1e-30, 120)
    b.solve(1e-30, 300)          # resume from k = 120
    xa, ya = a.iterate()
    xb, yb = b.iterate()
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    ia, ib = a.info(), b.info()
    assert ia["iterations"] == ib["iterations"] == 300 and ia["omega"] == ib["omega"]


def test_host_thread_count_does_not_change_the_solve():
    """pdlp_create prepares the LP (internal column order, transpose, layouts, interleaved
    entries) on 1 or on all host threads: above 2^20 nonzeros the parallel chunks are taken, and
    the scaling vectors and 80 steps through two restart checks are bitwise the same.  XCD
    panels and the internal column order forced: K~ in XCD panels with the hot stage, K~^T in
    LDS slices."""
    lp = lpgen.large_plain(32, 30000, 60000)
    assert lp.nnz > (1 << 20)
    say("host threads", lp.nnz)
    runs = []
    try:
        for th in (1, 0):
            P.set_host_threads(th)
            s = make(lp, xcd_panels=1, column_order=1)
            inf = s.info()
            s.solve(1e-30, 80)
            x, y = s.iterate()
            D1, D2 = s.scaling()
            runs.append((x, y, D1, D2, inf["layout_K"], inf["layout_KT"], s.info()["omega"]))
            s.close()
    finally:
        P.set_host_threads(0)
    a, b = runs
    assert a[4:6] == b[4:6] and a[4] > 0 and a[5] > 0, (a[4:6], b[4:6])
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)
    assert a[6] == b[6]


@pytest.mark.parametrize("kw", [dict(), dict(xcd_panels=1), dict(step_policy=2),
                                dict(LDS_MODES["slices"]), dict(LDS_MODES["xcd_stage"], step_policy=2)])
def test_graph_replay_equals_kernel_by_kernel(kw):
    """Blocks replayed as captured HIP graphs give bit-identical iterates, counters and every
    attempt and check record (each block's replay is compared) as launching kernel by kernel,
    with host synchronisation between the blocks as in every solve."""
    lp = lpgen.tiny_lp()
    say("graph replay vs eager", kw)
    out = []
    for graphs in (1, 0):
        s = make(lp, use_graphs=graphs, **kw)
        st = s.solve(1e-8, 2000)
        st2 = s.solve(1e-8, 100000)          # a second call continues with the same graphs
        x, y, kkt = s.get()
        info = s.info()
        tr = s.trace()
        out.append((st, st2, x, y, kkt, info, tr))
        s.close()
    a, b = out
    assert a[0] == b[0] and a[1] == b[1] == P.OPTIMAL
    for i in (2, 3, 4):
        assert np.array_equal(a[i], b[i])
    for key in ("iterations", "attempts", "restarts", "checks", "spmv_K", "spmv_KT", "omega", "eta_hat"):
        assert a[5][key] == b[5][key], key
    assert a[6]["attempts"] == b[6]["attempts"]
    assert len(a[6]["checks"]) == len(b[6]["checks"])
    for ca, cb in zip(a[6]["checks"], b[6]["checks"]):
        for key in ca:       # NaN (no anchor gap without a restart) compares as equal to NaN
            va, vb = ca[key], cb[key]
            assert va == vb or (isinstance(va, float) and math.isnan(va) and math.isnan(vb)), key


@pytest.mark.parametrize("kw", [dict(), dict(LDS_MODES["slices"])])
def test_kernel_timing_counts_the_slots_that_ran(kw):
    """With kernel timing the solver runs one block at a time, cuts a block at the iteration
    limit instead of idling, and counts the attempt slots that ran, in each of the four
    passes; the iterates equal those of a graph-replayed solve bit for bit."""
    lp = lpgen.tiny_lp()
    say("kernel timing counts", kw)
    a = make(lp, time_kernels=1, **kw)
    b = make(lp, **kw)
    for lim in (5, 25, 40, 41, 97, 160):        # inside a block, at and across checks
        a.reset_kernel_times()
        ia0, ib0 = a.info(), b.info()
        a.solve(1e-30, lim)
        b.solve(1e-30, lim)
        ia1, ib1 = a.info(), b.info()
        assert ia1["iterations"] == ib1["iterations"] == lim
        d = ia1["attempts"] - ia0["attempts"]
        assert d == ib1["attempts"] - ib0["attempts"] and d >= lim - ia0["iterations"]
        t, c = a.pass_times()
        assert list(c) == [d] * 4 and np.all(t >= 0), (lim, c, d)
        tk, ck = a.kernel_times()
        assert list(ck) == [d, d] and np.allclose(tk, [t[0] + t[1], t[2] + t[3]])
    a.set_kernel_timing(False)                  # graphs again from here on
    a.solve(1e-30, 240)
    b.solve(1e-30, 240)
    xa, ya = a.iterate()
    xb, yb = b.iterate()
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    assert a.info()["checks"] == b.info()["checks"] >= 6


def test_edge_cases():
    # no constraints at all: min c^T x over a box
    n = 7
    c = np.array([1.0, -2.0, 0.5, -0.1, 3.0, -4.0, 0.0])
    lp = lpgen.LP(m=0, n=n, n_eq=0, c=c, row_ptr=np.zeros(1, np.int64), col_idx=np.zeros(0, np.int32),
                  val=np.zeros(0), q=np.zeros(0), l=-np.ones(n), u=2 * np.ones(n))
    say("edge m=0")
    s = make(lp)
    assert s.solve(1e-10, 10000) == P.OPTIMAL
    x, _, kkt = s.get()
    np.testing.assert_allclose(x, np.where(c > 0, -1.0, np.where(c < 0, 2.0, x)), atol=1e-9)
    # only equalities, and only inequalities
    base = lpgen.tiny_plain(3, 60, 150, 0, 4)
    say("edge all equalities")
    s = make(base)
    assert s.solve(1e-8, 200000) == P.OPTIMAL
    base2 = lpgen.tiny_plain(4, 60, 150, 60, 4)
    say("edge all inequalities")
    s = make(base2)
    assert s.solve(1e-8, 200000) == P.OPTIMAL
    # iteration limit 0 and tolerance 0
    say("edge limits")
    s = make(lpgen.tiny_lp())
    assert s.solve(1e-8, 0) == P.ITERATION_LIMIT
    assert s.info()["iterations"] == 0
    assert s.solve(0.0, 57) == P.ITERATION_LIMIT
    assert s.info()["iterations"] == 57
    _, _, kkt = s.get()
    assert np.all(np.isfinite(kkt))


@pytest.mark.parametrize("panels", [0, 1])
def test_product_over_a_copy_without_columns(panels):
    """K~^T y of an LP without constraints (m = 0): every row of K~^T is empty and the product
    is exactly zero, whatever the caller's buffer holds (here one NaN)."""
    import torch
    n = 300
    lp = lpgen.LP(m=0, n=n, n_eq=0, c=np.ones(n), row_ptr=np.zeros(1, np.int64), col_idx=np.zeros(0, np.int32),
                  val=np.zeros(0), q=np.zeros(0), l=np.zeros(n), u=np.ones(n))
    say("product with no rows", "panels", panels)
    s = make(lp, ruiz_iters=0, pock_chambolle=0, xcd_panels=panels)
    y = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    out = torch.full((n,), 5.0, dtype=torch.float64, device="cuda")
    s.spmv(y, out, transpose=True)
    assert torch.equal(out.cpu(), torch.zeros(n, dtype=torch.float64))


def test_get_before_solve_and_device_outputs():
    import torch
    lp = lpgen.tiny_lp()
    say("api states")
    s = make(lp)
    with pytest.raises(P.PdlpError):
        s.get()
    s.solve(1e-8, 200)
    x, y, _ = s.get()
    xd = torch.empty(lp.n, dtype=torch.float64, device="cuda")
    yd = torch.empty(lp.m, dtype=torch.float64, device="cuda")
    s.get_into(xd, yd)
    assert np.array_equal(xd.cpu().numpy(), x) and np.array_equal(yd.cpu().numpy(), y)
    # device-pointer inputs give the same solver
    t = {k: torch.from_numpy(np.asarray(getattr(lp, k))).cuda() for k in
         ("c", "row_ptr", "col_idx", "val", "q", "l", "u")}
    s2 = P.Solver(lp.m, lp.n, lp.n_eq, t["c"], t["row_ptr"], t["col_idx"], t["val"], t["q"], t["l"], t["u"])
    s2.solve(1e-8, 200)
    x2, y2, _ = s2.get()
    assert np.array_equal(x, x2) and np.array_equal(y, y2)


# ------------------------------------------------------------------------------------------
# batched solve (one workgroup per LP)
# ------------------------------------------------------------------------------------------

def test_batched_solve_matches_oracle_and_single_solver():
    members = [lpgen.batched_instance(i) for i in (2, 3, 5, 7)] + [lpgen.tiny_lp(1)] + \
              [lpgen.add_empty_row_and_column(lpgen.tiny_plain(3, 60, 150, 20, 4))]
    say("batch", [lp.m for lp in members])
    b = P.Batch(members)
    b.solve(1e-8, 100000)
    xs, ys, st, it, kkt = b.get()
    for k, lp in enumerate(members):
        ref = O.solve_lp(lp, tol=1e-8, iter_limit=100000)
        assert st[k] == ref.status == O.OPTIMAL, (k, st[k], ref.status)
        kk = O.kkt(lp.c, lp.K(), lp.q, lp.l, lp.u, lp.n_eq, xs[k], ys[k])
        assert kk["kkt"] <= 1e-8, (k, kk)
        assert abs(kk["kkt"] - kkt[k, 3]) <= 1e-10
        assert abs(kk["pobj"] - ref.kkt["pobj"]) <= 1e-6 * (1 + abs(ref.kkt["pobj"]))
        assert 0.5 * ref.k <= it[k] <= 2 * ref.k, (k, it[k], ref.k)


def test_batched_first_steps_match_oracle():
    """Iteration limit 40: every member's returned point (the current iterate) after one
    check equals the oracle's at the iterate tolerance."""
    members = [lpgen.batched_instance(i) for i in range(8)]
    b = P.Batch(members)
    b.solve(1e-30, 40)
    xs, ys, st, it, _ = b.get()
    for k, lp in enumerate(members):
        ref = O.solve_lp(lp, tol=1e-30, iter_limit=40)
        assert st[k] == P.ITERATION_LIMIT and it[k] == 40
        assert rel(xs[k], ref.x) <= 1e-11 and rel(ys[k], ref.y) <= 1e-11, k


@pytest.mark.parametrize("sched", P.Batch.SCHEDULES)
def test_batched_schedules_match_oracle(sched):
    """Every schedule the tuner can pick for a size class (threads per member x rows per thread
    in flight): after 40 steps every member's iterate equals the oracle's at the iterate
    tolerance, and a full solve is certified by the oracle's KKT evaluation.  The members span
    three size classes."""
    members = [lpgen.batched_instance(i) for i in (0, 2, 6, 9)] + \
              [lpgen.add_empty_row_and_column(lpgen.tiny_plain(3, 60, 150, 20, 4))]
    say("batch schedule", sched, [lp.nnz for lp in members])
    b = P.Batch(members)
    b.set_schedule([sched] * P.Batch.BATCH_CLASSES)
    assert b.schedule()[0] == [sched] * P.Batch.BATCH_CLASSES
    assert sum(b.schedule()[1]) == len(members)
    b.solve(1e-30, 40)
    xs, ys, st, it, _ = b.get()
    for k, lp in enumerate(members):
        ref = O.solve_lp(lp, tol=1e-30, iter_limit=40)
        assert st[k] == P.ITERATION_LIMIT and it[k] == 40
        assert rel(xs[k], ref.x) <= 1e-11 and rel(ys[k], ref.y) <= 1e-11, k
    b.solve(1e-8, 100000)                    # a second solve starts again from the data
    xs, ys, st, it, kkt = b.get()
    for k, lp in enumerate(members):
        assert st[k] == P.OPTIMAL, (k, st[k])
        kk = O.kkt(lp.c, lp.K(), lp.q, lp.l, lp.u, lp.n_eq, xs[k], ys[k])
        assert kk["kkt"] <= 1e-8 and abs(kk["kkt"] - kkt[k, 3]) <= 1e-10, (k, kk["kkt"])


def test_batched_tune_then_solve_repeats_bitwise():
    """The tuner's choice is one of the schedules, its timing runs leave no solve behind, and
    two solves of the same batch give bit-identical points, also under another schedule
    (every schedule sums each row in the same order)."""
    members = [lpgen.batched_instance(i) for i in range(12)]
    say("batch tune")
    b = P.Batch(members)
    sched = b.tune(30)
    assert all(q in P.Batch.SCHEDULES for q in sched) and b.schedule()[0] == sched
    with pytest.raises(P.PdlpError):
        b.get()
    b.solve(1e-8, 3000)
    x1, y1, st1, it1, k1 = b.get()
    b.solve(1e-8, 3000)
    x2, y2, st2, it2, k2 = b.get()
    for k in range(len(members)):
        assert np.array_equal(x1[k], x2[k]) and np.array_equal(y1[k], y2[k])
    assert np.array_equal(it1, it2) and np.array_equal(k1, k2)
    for t in (128, 256, 512):                  # the same threads with 1 or 2 rows in flight
        pts = []
        for rows in (1, 2):
            b.set_schedule([(t, rows)] * P.Batch.BATCH_CLASSES)
            b.solve(1e-8, 3000)
            pts.append(b.get())
        for k in range(len(members)):
            assert np.array_equal(pts[0][0][k], pts[1][0][k]) and np.array_equal(pts[0][1][k], pts[1][1][k])
        assert np.array_equal(pts[0][3], pts[1][3])


def test_batched_rejects_bad_member():
    lps = [lpgen.batched_instance(0), lpgen.tiny_lp()]
    lps[1].l = lps[1].l.copy()
    lps[1].l[3] = 20.0
    with pytest.raises(P.PdlpError, match="member 1"):
        P.Batch(lps)
