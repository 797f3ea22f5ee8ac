"""Shared check of the GPU tests: replayed PDLP steps against the oracle's recorded states."""
import math
import sys

import numpy as np

EPS = np.finfo(np.float64).eps


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def row_bound(A, v):
    """Largest difference between two float64 sums of row i of A v in any orders: each is
    within (len_i - 1) u (|A||v|)_i of the exact value (u = eps / 2), so their difference is
    within len_i eps (|A||v|)_i; never below 1e-13 of (|A||v|)_i."""
    lens = np.diff(A.indptr).astype(np.float64)
    return np.maximum(1e-13, lens * EPS) * (abs(A) @ np.abs(v)) + 1e-300


def _step_bounds(Kt, KtT, ct, qt, a, xp, yp, eta, omega):
    """Elementwise bounds on the difference between two float64 evaluations of one PDHG step
    (Eq. (3)) from the same state a with step eta and weight omega, whose products sum in
    different orders.  A product row of length len differs by at most len eps (|K||v|)_i
    between two orders; every other operation adds a few roundings of its operands; clipping
    and projection do not enlarge differences.  Returns (bound on x', bound on y')."""
    x, y = a["x"], a["y"]
    lens, lensT = np.diff(Kt.indptr), np.diff(KtT.indptr)
    absK, absKT = abs(Kt), abs(KtT)
    aKTy = absKT @ np.abs(y)
    ex = (eta / omega) * (lensT * EPS * aKTy + 2 * EPS * (np.abs(ct) + aKTy)) \
        + 2 * EPS * (np.abs(x) + np.abs(xp))
    aKxp, aKx = absK @ np.abs(xp), absK @ np.abs(x)
    eKxp = lens * EPS * aKxp + absK @ ex
    eKx = lens * EPS * aKx
    ey = eta * omega * (2 * eKxp + eKx + 4 * EPS * (np.abs(qt) + 2 * aKxp + aKx)) \
        + 2 * EPS * (np.abs(y) + np.abs(yp))
    return ex, ey


def replay_steps(s, ref, Kt, ks, ct, qt):
    """For each k in ks the GPU solver s is put in the oracle's exact state before step k+1
    (pdlp_set_state) and must land on the oracle's state after it, including the restart
    check when k+1 is a multiple of the check period.  ref: an oracle result with
    record_states and trace_iters >= max(ks) + 1; Kt, ct, qt: the oracle's preconditioned
    K, c and q.

    Tolerances: every vector (iterate, anchor, weighted sum) within max(1e-12 |b|, 2 |e|) in
    2-norm, where e bounds the elementwise difference of two evaluations of the step
    (_step_bounds), carried through the weighted sums and, after a restart, the average; the
    proposed step eta_hat within the conditioning of the denominator 2 dy^T K dx of
    Algorithm 2, which the GPU forms as dy^T (K x' - K x): its error is bounded by
    2 eps sum_i |dy_i| len_i ((|K||x'|)_i + (|K||x|)_i)."""
    absK = abs(Kt)
    KtT = Kt.T.tocsr()
    rowlen = np.diff(Kt.indptr).astype(np.float64)
    states = ref.trace.states
    att_by_k = {}
    for a in ref.trace.attempts:
        att_by_k.setdefault(a[0], []).append(a)
    for k in ks:
        a, b = states[k], states[k + 1]
        assert a["k"] == k and b["k"] == k + 1
        s.set_state(a)
        s.solve(1e-30, k + 1)
        g = s.get_state()
        assert (g["k"], g["t"], g["n_outer"]) == (b["k"], b["t"], b["n_outer"]), k
        _, xp, yp = ref.trace.iterates[k]
        eta = [t[1] for t in att_by_k[k] if t[3]][-1]          # the accepted attempt's step
        ex, ey = _step_bounds(Kt, KtT, ct, qt, a, xp, yp, eta, a["omega"])
        eSx = eta * ex + 2 * EPS * (np.abs(a["Sx"]) + eta * np.abs(xp))
        eSy = eta * ey + 2 * EPS * (np.abs(a["Sy"]) + eta * np.abs(yp))
        bound = {"x": ex, "y": ey, "Sx": eSx, "Sy": eSy, "xa": 0.0 * ex, "ya": 0.0 * ey}
        if b["n_outer"] > a["n_outer"]:
            # restarted to the current iterate or to the average S / (S_eta + eta)
            seta = a["Seta"] + eta
            for key, e, eS in (("x", ex, eSx), ("y", ey, eSy)):
                bound[key] = e + eS / seta + 2 * EPS * np.abs(b[key])
                bound[key[0] + "a"] = bound[key]
        for key in ("x", "y", "xa", "ya", "Sx", "Sy"):
            diff = np.linalg.norm(g[key] - b[key])
            bar = max(1e-12 * np.linalg.norm(b[key]), 2 * np.linalg.norm(bound[key]))
            assert diff <= bar, (k, key, rel(g[key], b[key]), bar)
        assert abs(g["Seta"] - b["Seta"]) <= 1e-15 * b["Seta"], k
        assert abs(g["omega"] - b["omega"]) <= 1e-13 * b["omega"], k
        for key in ("mu_prev", "mu_anchor"):
            if math.isfinite(b[key]):
                assert abs(g[key] - b[key]) <= 1e-9 * abs(b[key]), (k, key)
            else:
                assert g[key] == b[key], (k, key)
        # conditioning of eta_bar on the accepted attempt
        dx, dy = xp - a["x"], yp - a["y"]
        den = abs(float(dy @ (Kt @ dx)))
        err_den = 2 * EPS * float(np.abs(dy) @ (rowlen * (absK @ np.abs(xp) + absK @ np.abs(a["x"]))))
        tol = 1e-13 + (4 * err_den / den if den > 0 else 0.0)
        if len(att_by_k[k]) > 1:
            tol = max(tol, 1e-9)            # a rejected attempt chains two step proposals
        assert abs(g["eta_hat"] - b["eta_hat"]) <= tol * b["eta_hat"], (k, g["eta_hat"], b["eta_hat"], tol)
