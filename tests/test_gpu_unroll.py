"""GPU parity of the unrolled PDHG and its hand-written adjoint (run on an MI355X).

The map: T fixed steps of Eq. (3) (frozen eta, omega, D1, D2; no restarts or rejections) from
x0 = proj(0), y0 = 0; the adjoint gives d loss / d(c, q).  Bars:
  * x_T, y_T and the gradients against the oracle's unroll: elementwise within 1e-10 of the
    vector's largest entry (fixed-step PDHG is nonexpansive, so round-off does not grow
    geometrically; the masks agree unless a pre-projection value sits within round-off of a
    bound, which these seeded inputs avoid);
  * checkpoint segment lengths: bit-identical gradients (the recomputation replays the same
    deterministic kernels);
  * finite differences of the GPU's own forward map, h = 1e-6, on 64 coordinates of (c, q) at
    the full unroll size, one-sided and central, with kinks of the piecewise-affine map told
    apart (see that test).
"""
import sys

import numpy as np
import pytest

import paper_2106_04756_amd as P
from oracle import pdlp_oracle as O
from workloads import lpgen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def close(a, b, tol):
    scale = max(1.0, float(np.abs(b).max()) if b.size else 1.0)
    err = float(np.abs(a - b).max()) if b.size else 0.0
    assert err <= tol * scale, (err, scale)


def oracle_case(lp, x_tgt, T, gy=None, l=None, u=None):
    l = lp.l if l is None else l
    u = lp.u if u is None else u
    return O.unroll_user(lp.K(), lp.c, lp.q, l, u, lp.m1, x_tgt, T, gy_T=gy)


def gpu_grad(s, lp, x_tgt, T, segment, eta, omega, gy=None):
    x, y = s.unroll_forward(lp.c, lp.q, T, segment, eta, omega)
    gc, gq = s.unroll_backward(2.0 * (x - x_tgt), gy)
    return x, y, gc, gq


@pytest.mark.parametrize("segment,kw", [(0, {}), (7, {}), (7, dict(xcd_panels=1, column_order=1)),
                                        (7, dict(xcd_panels=1, lds_gather=1, lds_entries=64))])
def test_unroll_matches_oracle_small(segment, kw):
    lp = lpgen.tiny_lp()
    rng = np.random.default_rng(40)
    x_tgt = rng.uniform(0, 5, lp.n)
    gy = rng.standard_normal(lp.m)
    T = 60
    say("unroll small", lp.name, "T", T, "segment", segment, kw)
    ref = oracle_case(lp, x_tgt, T, gy)
    with P.Solver.from_lp(lp, **kw) as s:
        x, y, gc, gq = gpu_grad(s, lp, x_tgt, T, segment, ref["eta"], ref["omega"], gy)
        info = s.unroll_info()
    close(x, ref["x_T"], 1e-10)
    close(y, ref["y_T"], 1e-10)
    close(gc, ref["gc"], 1e-10)
    close(gq, ref["gq"], 1e-10)
    assert info["steps"] == T and info["ready"] == 1
    if segment == 7:
        assert info["checkpoints"] == 9 and info["recomputed_steps"] == 56


def test_unroll_segments_are_bit_identical():
    lp = lpgen.tiny_lp()
    rng = np.random.default_rng(41)
    x_tgt = rng.uniform(0, 5, lp.n)
    gy = rng.standard_normal(lp.m)
    T = 45
    say("unroll segments", lp.name, "T", T)
    with P.Solver.from_lp(lp) as s:
        outs = {}
        for seg in (0, 1, 7, 45, 1000):
            outs[seg] = gpu_grad(s, lp, x_tgt, T, seg, 0.0, 0.0, gy)
        # a second backward after the masks of the first segment were recomputed
        gc2, gq2 = s.unroll_backward(2.0 * (outs[1000][0] - x_tgt), gy)
    for seg, o in outs.items():
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b), seg
    assert np.array_equal(gc2, outs[0][2]) and np.array_equal(gq2, outs[0][3])


def test_unroll_default_step_and_weight():
    lp = lpgen.tiny_lp()
    say("unroll defaults", lp.name)
    Kt, ct, qt, lt, ut, D1, D2 = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)
    eta = 0.9 / O.power_iteration_norm(Kt, 200)
    omega = O.initial_primal_weight(ct, qt, 1e-10)
    with P.Solver.from_lp(lp) as s:
        s.unroll_forward(None, None, 3, 0)
        info = s.unroll_info()
    assert abs(info["eta"] - eta) <= 1e-12 * eta
    assert abs(info["omega"] - omega) <= 1e-12 * omega


def test_unroll_edge_cases():
    lp = lpgen.add_empty_row_and_column(lpgen.tiny_plain(6, 120, 260, 50, 4))
    rng = np.random.default_rng(42)
    x_tgt = rng.uniform(0, 5, lp.n)
    l = lp.l.copy()
    u = lp.u.copy()
    l[:30] = -np.inf
    u[:30] = np.inf
    u[30:60] = np.inf
    lp2 = lpgen.from_csr(lp.K(), lp.c, lp.q, l, u, n_eq=lp.n_eq, name="edge LP")
    for panels in (0, 1):
        with P.Solver.from_lp(lp2, xcd_panels=panels) as s:
            for T in (0, 1, 33):
                say("unroll edge", lp2.name, "panels", panels, "T", T)
                ref = oracle_case(lp2, x_tgt, T)
                x, y, gc, gq = gpu_grad(s, lp2, x_tgt, T, 4, ref["eta"], ref["omega"])
                close(x, ref["x_T"], 1e-10)
                close(y, ref["y_T"], 1e-10)
                close(gc, ref["gc"], 1e-10)
                close(gq, ref["gq"], 1e-10)
                if T == 0:
                    assert np.all(gc == 0.0) and np.all(gq == 0.0)


def test_unroll_errors():
    lp = lpgen.tiny_lp()
    say("unroll errors")
    with P.Solver.from_lp(lp) as s:
        with pytest.raises(P.PdlpError, match="no forward pass"):
            s.unroll_backward(np.zeros(lp.n))
        with pytest.raises(P.PdlpError, match="steps >= 0"):
            s.unroll_forward(None, None, -1, 0)
        with pytest.raises(P.PdlpError, match="finite eta"):
            s.unroll_forward(None, None, 5, 0, float("nan"))


def test_unroll_full_size_matches_oracle():
    lp, x_tgt = lpgen.unroll_lp()
    T = 500
    say("unroll full size", lp.name, "T", T, "segment 50")
    ref = oracle_case(lp, x_tgt, T)
    with P.Solver.from_lp(lp) as s:
        x, y, gc, gq = gpu_grad(s, lp, x_tgt, T, 50, ref["eta"], ref["omega"])
        info = s.unroll_info()
    assert info["checkpoints"] == 10 and info["recomputed_steps"] == 450
    close(x, ref["x_T"], 1e-10)
    close(y, ref["y_T"], 1e-10)
    close(gc, ref["gc"], 1e-10)
    close(gq, ref["gq"], 1e-10)


def test_unroll_full_size_finite_differences():
    """64 coordinates of (c, q): differences of the GPU forward map (same frozen eta, omega),
    h = 1e-6.  The map (c, q) -> x_T is piecewise affine (affine while no projection mask
    changes), so with w = 2 (x_T - x_tgt) the one-sided quotients (x_T(c + h e) - x_T(c)) . w / h
    and (x_T(c) - x_T(c - h e)) . w / h both equal dL/dc_j up to round-off unless a mask
    changes inside the interval; then the side without the kink still does.  Every coordinate
    must match on at least one side; kink-free ones on both sides and centrally."""
    lp, x_tgt = lpgen.unroll_lp()
    T = 500
    rng = np.random.default_rng(44)
    say("unroll FD", lp.name, "T", T)
    with P.Solver.from_lp(lp) as s:
        x0, y, gc, gq = gpu_grad(s, lp, x_tgt, T, 50, 0.0, 0.0)
        info = s.unroll_info()
        eta, omega = info["eta"], info["omega"]
        w = 2.0 * (x0 - x_tgt)

        def xT(c, q):
            return s.unroll_forward(c, q, T, 50, eta, omega)[0]

        h = 1e-6
        kinks = 0
        cases = [("c", j) for j in rng.choice(lp.n, 32, replace=False)] + \
                [("q", i) for i in rng.choice(lp.m, 32, replace=False)]
        for which, k in cases:
            e = np.zeros(lp.n if which == "c" else lp.m)
            e[k] = h
            if which == "c":
                xp, xm, g = xT(lp.c + e, lp.q), xT(lp.c - e, lp.q), gc[k]
            else:
                xp, xm, g = xT(lp.c, lp.q + e), xT(lp.c, lp.q - e), gq[k]
            gp = float((xp - x0) @ w) / h
            gm = float((x0 - xm) @ w) / h
            tol = 5e-5 + 1e-7 * abs(g)
            assert min(abs(gp - g), abs(gm - g)) <= tol, (which, k, g, gp, gm)
            if abs(gp - gm) > 10 * tol:
                kinks += 1
            else:
                assert abs(gp - g) <= tol and abs(gm - g) <= tol, (which, k, g, gp, gm)
                assert abs(0.5 * (gp + gm) - g) <= tol, (which, k, g, gp, gm)
        say("coordinates with a mask change within h:", kinks, "of", len(cases))
        assert kinks <= len(cases) // 2


def test_unroll_autograd_function():
    import torch
    from paper_2106_04756_amd.unroll import unrolled_pdhg
    lp = lpgen.tiny_lp()
    rng = np.random.default_rng(45)
    x_tgt = rng.uniform(0, 5, lp.n)
    T = 40
    say("unroll autograd", lp.name, "T", T)
    with P.Solver.from_lp(lp) as s:
        dev = torch.device("cuda:0")
        c = torch.tensor(lp.c, device=dev, requires_grad=True)
        q = torch.tensor(lp.q, device=dev, requires_grad=True)
        tgt = torch.tensor(x_tgt, device=dev)
        x, y = unrolled_pdhg(s, c, q, steps=T, segment=8)
        loss = ((x - tgt) ** 2).sum() + y.sum()
        # another forward on the same solver before backward: the Function replays its own
        c2 = torch.tensor(lp.c * 1.5, device=dev)
        unrolled_pdhg(s, c2, q.detach(), steps=T, segment=8)
        loss.backward()
        xr, yr = s.unroll_forward(lp.c, lp.q, T, 8)
        gc, gq = s.unroll_backward(2.0 * (xr - x_tgt), np.ones(lp.m))
        assert np.array_equal(x.detach().cpu().numpy(), xr)
        assert np.array_equal(c.grad.cpu().numpy(), gc)
        assert np.array_equal(q.grad.cpu().numpy(), gq)
