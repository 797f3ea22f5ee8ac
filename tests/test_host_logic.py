"""Host-side checks that need no GPU: the C-ABI library loads and exports every entry point
declared in include/pdlp.h, the SpMV row schedule covers every row exactly once within the
kernels' LDS and lane limits, and input validation rejects malformed LPs before any device
work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2106_04756_amd as P
from paper_2106_04756_amd import pdlp as B
from workloads import lpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdlp.h")

ELEMS_PER_LANE, WAVE_MAX, VEC_MAX, CHUNK, ROUNDS = 8, 512, 16384, 16384, 4


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdlp_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared_functions() == sorted(B.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = P.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_struct_layouts_match_header():
    # pdlp_options: 10 int32 + 6 double + 4 int32 + 3 double + 5 int32 and 4 bytes of tail
    # padding (8-byte alignment); pdlp_info and the records
    assert ctypes.sizeof(B.Options) == 10 * 4 + 6 * 8 + 4 * 4 + 3 * 8 + 5 * 4 + 4
    assert ctypes.sizeof(B.AttemptRec) == 32
    assert ctypes.sizeof(B.CheckRec) == 8 + 5 * 8 + 4 * 4
    assert ctypes.sizeof(B.Info) == 2 * 4 + 10 * 8 + 2 * 8 + 4 * 8 + 3 * 8 + 4 * 4
    assert ctypes.sizeof(B.UnrollInfo) == 4 * 8 + 5 * 8 + 2 * 4


def test_default_options_are_the_papers():
    o = P.default_options()
    assert (o.ruiz_iters, o.pock_chambolle, o.adaptive_restarts, o.primal_weight_update) == (10, 1, 1, 1)
    assert o.check_every == 40 and o.theta == 0.5 and o.beta_artificial == 0.5
    assert (o.beta_sufficient, o.beta_necessary) == (0.1, 0.9)
    assert o.eps_zero == 1e-10 and o.primal_importance == 1.0
    assert (o.step_policy, o.restart_to_current, o.power_iters, o.xcd_panels) == (0, 1, 200, -1)
    assert (o.mp_breaking_factor, o.mp_downscaling, o.mp_interpolation) == (1.0, 0.5, 0.4)
    assert o.use_graphs == 1 and o.column_order == -1
    assert (o.lds_gather, o.lds_entries, o.xcd_subpanels) == (-1, 0, -1)


def _check_schedule(row_ptr):
    desc, nsplit, perm = P.schedule(row_ptr)
    nrows = row_ptr.size - 1
    lens = np.diff(row_ptr)
    seen = np.zeros(nrows, dtype=np.int64)
    chunks = {}
    perm_used = np.zeros(perm.size, dtype=np.int64)
    for a, b, kl, aux in desc:
        kind, lg = kl & 0xFF, kl >> 8
        if kind == 0:
            L = 1 << lg
            assert 1 <= b <= (64 // L) * ROUNDS
            rows = perm[a:a + b]
            perm_used[a:a + b] += 1
            assert np.all(lens[rows] <= ELEMS_PER_LANE * L)
            # entries per lane: enough for the task's longest row, and no more
            assert 1 <= aux <= ELEMS_PER_LANE and np.all(lens[rows] <= aux * L)
            assert aux == 1 or lens[rows].max() > (aux - 1) * L
            if lg > 0:
                assert np.all(lens[rows] > ELEMS_PER_LANE * L // 2)
            seen[rows] += 1
        elif kind == 1:
            assert WAVE_MAX < lens[a] <= VEC_MAX
            seen[a] += 1
        else:
            assert kind == 2
            chunks.setdefault((a, aux), []).append(b)
    for (row, sid), cs in chunks.items():
        assert lens[row] > VEC_MAX
        assert sorted(cs) == list(range(-(-lens[row] // CHUNK)))
        seen[row] += 1
    assert len({sid for (_, sid) in chunks}) == nsplit
    assert np.all(seen == 1)
    short = int((lens <= WAVE_MAX).sum())
    assert np.all(perm_used[:short] == 1)
    return desc, nsplit


@pytest.mark.parametrize("lens", [
    [],
    [0],
    [0, 0, 0, 5, 0],
    [1] * 1000,
    [8, 9, 16, 17, 512, 513, 16384, 16385, 0, 3],
    [40000, 1, 2, 100000, 0],
])
def test_schedule_covers_rows(lens):
    rp = np.concatenate([[0], np.cumsum(np.asarray(lens, dtype=np.int64))]).astype(np.int64)
    _check_schedule(rp)


def test_schedule_on_workload_shapes():
    rng = np.random.default_rng(0)
    # Zipf-like column counts (rows of the transposed copy) and Poisson rows
    for lens in (np.minimum(rng.zipf(1.5, 20000), 2000), rng.poisson(136, 5000), rng.poisson(12.5, 3000)):
        rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        _check_schedule(rp)
    lp = lpgen.pagerank_lp(2, 50000)
    desc, nsplit = _check_schedule(lp.row_ptr)
    assert nsplit == 1          # the normalisation row sum(x) = 1


def _create(lp, **kw):
    return P.Solver(lp.m, lp.n, lp.n_eq, lp.c, lp.row_ptr, lp.col_idx, lp.val, lp.q, lp.l, lp.u, **kw)


@pytest.mark.parametrize("mutate,needle", [
    (lambda d: d.__setitem__("c", np.where(np.arange(d["c"].size) == 3, np.nan, d["c"])), "c["),
    (lambda d: d.__setitem__("l", np.where(np.arange(d["l"].size) == 2, 11.0, d["l"])), "l > u"),
    (lambda d: d.__setitem__("u", np.where(np.arange(d["u"].size) == 2, np.nan, d["u"])), "NaN"),
    (lambda d: d.__setitem__("col_idx", np.where(np.arange(d["col_idx"].size) == 0, 10**6, d["col_idx"])), "out of range"),
    (lambda d: d.__setitem__("val", np.where(np.arange(d["val"].size) == 7, np.inf, d["val"])), "non-finite matrix"),
    (lambda d: d.__setitem__("q", np.where(np.arange(d["q"].size) == 1, np.inf, d["q"])), "q["),
    (lambda d: d.__setitem__("n_eq", 201), "n_eq"),
    (lambda d: d.__setitem__("l", np.full(d["l"].size, np.inf)), None),
])
def test_create_rejects_invalid_input(mutate, needle):
    lp = lpgen.tiny_lp()
    d = dict(m=lp.m, n=lp.n, n_eq=lp.n_eq, c=lp.c.copy(), row_ptr=lp.row_ptr.copy(),
             col_idx=lp.col_idx.copy(), val=lp.val.copy(), q=lp.q.copy(), l=lp.l.copy(), u=lp.u.copy())
    mutate(d)
    with pytest.raises(P.PdlpError) as ei:
        P.Solver(d["m"], d["n"], d["n_eq"], d["c"], d["row_ptr"], d["col_idx"], d["val"], d["q"],
                 d["l"], d["u"])
    assert ei.value.code == B.ERR_INVALID_ARGUMENT
    if needle:
        assert needle in str(ei.value)


def test_create_rejects_unsorted_columns():
    lp = lpgen.tiny_lp()
    ci = lp.col_idx.copy()
    s, e = lp.row_ptr[5], lp.row_ptr[6]
    ci[s:e] = ci[s:e][::-1]
    with pytest.raises(P.PdlpError, match="strictly increasing"):
        P.Solver(lp.m, lp.n, lp.n_eq, lp.c, lp.row_ptr, ci, lp.val, lp.q, lp.l, lp.u)


def test_create_rejects_bad_sizes_and_options():
    lp = lpgen.tiny_lp()
    with pytest.raises(P.PdlpError, match="sizes"):
        P.Solver(lp.m, 0, lp.n_eq, lp.c, lp.row_ptr, lp.col_idx, lp.val, lp.q, lp.l, lp.u)
    with pytest.raises(P.PdlpError, match="options"):
        _create(lp, check_every=0)
    with pytest.raises(P.PdlpError, match="options"):      # needs restarts off
        _create(lp, pw_power_of_two=1)
    with pytest.raises(P.PdlpError, match="options"):
        _create(lp, step_policy=3)
    for bad in (dict(lds_gather=3), dict(lds_gather=-2), dict(lds_entries=-1), dict(lds_entries=19457),
                dict(xcd_subpanels=-2), dict(xcd_subpanels=9)):
        with pytest.raises(P.PdlpError, match="options"):
            _create(lp, **bad)


def test_schedule_rounds_follow_matrix_size():
    # small matrices: one row per lane group per task (more, shorter tasks); large ones: up to
    # four rounds per task once every wavefront of a full grid has several tasks
    for nrows, want in ((1000, 64), (8192 * 64, 64), (8192 * 64 * 3, 192), (2_000_000, 256)):
        rp = np.arange(nrows + 1, dtype=np.int64)           # rows of one nonzero: 64 per round
        desc, _, _ = P.schedule(rp)
        assert desc[:, 1].max() == want, (nrows, desc[:, 1].max())


def test_batch_create_checks_the_options_of_pdlp_create():
    # the batched solver accepts the option ranges of pdlp_create, with the adaptive step policy
    # and without the "no restart" weight events (rejected before any device work)
    lps = [lpgen.tiny_lp()]
    for bad in (dict(adaptive_restarts=0, pw_power_of_two=1), dict(step_policy=1), dict(beta_sufficient=0.0),
                dict(beta_artificial=-1.0), dict(check_every=0), dict(lds_entries=19457)):
        with pytest.raises(P.PdlpError, match="options") as ei:
            P.Batch(lps, **bad)
        assert ei.value.code == B.ERR_INVALID_ARGUMENT, bad


def test_outputs_must_be_writable_float64_in_place():
    # an output the library cannot write in place is refused, not silently copied
    with pytest.raises(ValueError):
        B._out_ptr(np.zeros(4, dtype=np.float32))
    with pytest.raises(ValueError):
        B._out_ptr(np.zeros(8)[::2])
    ro = np.zeros(4)
    ro.setflags(write=False)
    with pytest.raises(ValueError):
        B._out_ptr(ro)
    a = np.zeros(4)
    assert B._out_ptr(a).value == a.ctypes.data
    import torch
    with pytest.raises(ValueError):
        B._out_ptr(torch.zeros(4, dtype=torch.float32))
    t = torch.zeros(4, dtype=torch.float64)
    assert B._out_ptr(t).value == t.data_ptr()
