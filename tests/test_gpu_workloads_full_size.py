"""GPU parity at the full workload sizes, in the launch configuration that bench.py times:
options at their defaults (XCD panels or LDS slices and the internal column order chosen
automatically from the sparsity pattern).

Workloads: the 1e6 x 2e6 LP with 1.35e8 nonzeros (the bench workload, seed 1), the PageRank LP
on 5e6 nodes (one 5e6-long row) and the 1e6 x 2e6 LP with column counts truncated to [1, 190]
(2.1e7 nonzeros).  Each runs with the default preconditioning (10 Ruiz passes, then
Pock-Chambolle): D1 and D2 against the oracle's at 1e-13, both products of the scaled matrix
element by element, and steps 1, 2 and 40 replayed, step 40 with its restart check (normalized
gaps, candidate, restart criteria, primal-weight update).  The oracle's preconditioning and
40 steps of the largest LP take a few minutes of one host core.

Bars: the products element by element against scipy on the oracle's K~ = D1 K D2 within
max(1e-13, len eps) of |K~||x| per row (two sums of the same terms in different orders) plus
3 max|D/D_oracle - 1| |K~||x| (the scaling vectors differ in their last bits); replayed steps as
in replay.replay_steps (1e-12 relative on every vector, or the bound that the products'
summation order gives where that is larger: the 5e6-long row of the PageRank LP)."""
import numpy as np
import pytest

import paper_2106_04756_amd as P
from oracle import pdlp_oracle as O
from replay import replay_steps, row_bound, say
from workloads import lpgen

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def _products(s, K, seed, extra=0.0):
    """K x and K^T y of the solver's matrix against scipy's K, element by element."""
    import torch
    rng = np.random.default_rng(seed)
    m, n = K.shape
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    out = torch.empty(m, dtype=torch.float64, device="cuda")
    s.spmv(torch.from_numpy(x).cuda(), out)
    assert np.all(np.abs(out.cpu().numpy() - K @ x) <= row_bound(K, x) + extra * (abs(K) @ np.abs(x)))
    outT = torch.empty(n, dtype=torch.float64, device="cuda")
    s.spmv(torch.from_numpy(y).cuda(), outT, transpose=True)
    KT = K.T.tocsr()
    assert np.all(np.abs(outT.cpu().numpy() - KT @ y) <= row_bound(KT, y) + extra * (abs(KT) @ np.abs(y)))


def _scaled_case(lp, steps=40, panels=None):
    """Default options: scaling vectors, products of K~ and steps 1, 2 and `steps` (with its
    restart check) replayed against the oracle.  panels: the (K~, K~^T) panel counts the
    automatic layout choice must make."""
    say("full size", lp.name, lp.m, lp.n, lp.nnz, "scaled, bench launch configuration")
    ref = O.solve_lp(lp, tol=1e-30, iter_limit=steps, record_states=steps, trace_iters=steps,
                     record_trace=True)
    oD1, oD2 = ref.D1, ref.D2
    K = lp.K()
    Kt = K.copy()
    Kt.data = K.data * oD1[np.repeat(np.arange(lp.m), np.diff(K.indptr))] * oD2[K.indices]
    del K
    say("oracle done")
    s = P.Solver.from_lp(lp)
    inf = s.info()
    say("layouts", inf["layout_K"], inf["layout_KT"], "panels", inf["panels_K"], inf["panels_KT"])
    if panels is not None:
        assert (inf["panels_K"], inf["panels_KT"]) == panels
    D1, D2 = s.scaling()
    dmax = max(float(np.max(np.abs(D1 / oD1 - 1))), float(np.max(np.abs(D2 / oD2 - 1))))
    assert dmax < 1e-13, dmax
    say("scaling ok", dmax)
    _products(s, Kt, 7, extra=3 * dmax)
    say("products ok")
    replay_steps(s, ref, Kt, [0, 1, steps - 1], oD2 * lp.c, oD1 * lp.q)
    assert len(ref.trace.checks) >= 1 and ref.trace.checks[-1]["k"] == steps
    say("replayed steps and check ok")
    s.close()


@pytest.mark.timeout(1200)
def test_large_lp_full_size_scaled_through_restart_check():
    """The bench workload itself: 1.35e8 nonzeros, K~ in XCD panels with a hot LDS stage, K~^T
    in LDS slices."""
    _scaled_case(lpgen.large_lp(1))


@pytest.mark.timeout(900)
def test_pagerank_full_size_scaled_through_restart_check():
    """5e6 nodes: the sum(x) = 1 row of 5e6 nonzeros.  K~ has no hot columns and that row
    rules out the LDS kernel, so its 8 XCD panels (4.8 MiB of x each) are cut into 6
    sub-panels each; K~^T stays in the plain layout."""
    _scaled_case(lpgen.pagerank_5m(), panels=(48, 1))


@pytest.mark.timeout(900)
def test_truncated_large_lp_full_size_scaled_through_restart_check():
    """2.1e7 nonzeros."""
    _scaled_case(lpgen.large_lp_truncated(1))
