"""GPU parity at the full workload sizes, in the launch configuration that bench.py times:
options at their defaults (XCD panels and the internal column order chosen automatically from
the sparsity pattern) and every step kernel timed with HIP events.

Workloads: the 1e6 x 2e6 LP with 1.35e8 nonzeros (the bench workload, seed 1), the PageRank LP
on 5e6 nodes (one 5e6-long row, reduced in chunks) and the 1e6 x 2e6 LP with column counts
truncated to [1, 190] (2.1e7 nonzeros).

The oracle's preconditioning of the two largest matrices takes minutes on one host core, so
those run unscaled (no Ruiz or Pock-Chambolle pass).  The layout and the launch grids depend
on the sparsity pattern only, so the kernels and grids are those of the scaled solve.  The
2.1e7-nonzero LP runs with the preconditioning on: its scaling vectors and a replayed restart
check are compared at full size.

Bars: the products element by element against scipy within max(1e-13, len eps) of |K||x| per
row (two sums of the same terms in different orders); replayed steps as in
replay.replay_steps (1e-12 relative on every vector, or the bound that the products' summation
order gives where that is larger: the 5e6-long row of the PageRank LP)."""
import numpy as np
import pytest

import paper_2106_04756_amd as P
from oracle import pdlp_oracle as O
from replay import replay_steps, row_bound, say
from workloads import lpgen

pytestmark = pytest.mark.gpu

UNSCALED = dict(ruiz_iters=0, pock_chambolle=0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def _products(s, K, seed):
    """K x and K^T y of the solver's (unscaled) matrix against scipy, element by element."""
    import torch
    rng = np.random.default_rng(seed)
    m, n = K.shape
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    out = torch.empty(m, dtype=torch.float64, device="cuda")
    s.spmv(torch.from_numpy(x).cuda(), out)
    assert np.all(np.abs(out.cpu().numpy() - K @ x) <= row_bound(K, x))
    outT = torch.empty(n, dtype=torch.float64, device="cuda")
    s.spmv(torch.from_numpy(y).cuda(), outT, transpose=True)
    KT = K.T.tocsr()
    assert np.all(np.abs(outT.cpu().numpy() - KT @ y) <= row_bound(KT, y))


def _unscaled_case(lp, steps=2):
    say("full size", lp.name, lp.m, lp.n, lp.nnz, "unscaled, bench launch configuration")
    opts = O.Options(ruiz_iters=0, pock_chambolle=False)
    ref = O.solve_lp(lp, tol=1e-30, iter_limit=steps, opts=opts, record_states=steps,
                     trace_iters=steps, record_trace=True)
    say("oracle done")
    K = lp.K()
    s = P.Solver.from_lp(lp, time_kernels=1, **UNSCALED)
    say("solver created")
    _products(s, K, 7)
    say("products ok")
    replay_steps(s, ref, K, range(steps), lp.c, lp.q)
    say("replayed steps ok")
    s.close()


def test_large_lp_full_size_unscaled():
    """The bench workload itself: 1.35e8 nonzeros in XCD panels, hot columns first."""
    _unscaled_case(lpgen.large_lp(1))


def test_pagerank_full_size_unscaled():
    """5e6 nodes: the sum(x) = 1 row of 5e6 nonzeros is reduced in chunks and combined."""
    _unscaled_case(lpgen.pagerank_5m())


def test_truncated_large_lp_full_size_scaled_through_restart_check():
    """2.1e7 nonzeros with the default preconditioning: D1, D2 at 1e-13 and steps 1, 2 and
    the restart check at k = 40 (normalized gaps, candidate, primal weight) replayed."""
    lp = lpgen.large_lp_truncated(1)
    say("full size", lp.name, lp.m, lp.n, lp.nnz, "scaled, bench launch configuration")
    steps = 40
    ref = O.solve_lp(lp, tol=1e-30, iter_limit=steps, record_states=steps, trace_iters=steps,
                     record_trace=True)
    oD1, oD2 = ref.D1, ref.D2
    K = lp.K()
    # |K~| for the tolerance of the step proposal only
    Kt = K.copy()
    Kt.data = K.data * oD1[np.repeat(np.arange(lp.m), np.diff(K.indptr))] * oD2[K.indices]
    say("oracle done")
    s = P.Solver.from_lp(lp, time_kernels=1)
    D1, D2 = s.scaling()
    assert np.max(np.abs(D1 / oD1 - 1)) < 1e-13
    assert np.max(np.abs(D2 / oD2 - 1)) < 1e-13
    say("scaling ok")
    replay_steps(s, ref, Kt, [0, 1, steps - 1], oD2 * lp.c, oD1 * lp.q)
    assert len(ref.trace.checks) >= 1 and ref.trace.checks[-1]["k"] == steps
    say("replayed steps and check ok")
    s.close()
