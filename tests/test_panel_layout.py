"""Host-only checks of the column-panel layout the products read (pdlp_build_panel_layout):
the panel rows, their slots, the wavefront tasks, the interleaved entries and the LDS
workgroups' segments, each against what it must hold, recomputed here in NumPy from the input
CSR matrix.  No GPU is needed."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2106_04756_amd as P


def _matrix(seed, m, n):
    """Rows of every class: empty, 1..8 (one lane), up to 512 (a wavefront), one longer (a
    workgroup task), with empty columns at the end."""
    rng = np.random.default_rng(seed)
    lens = rng.choice([0, 1, 2, 3, 5, 9, 17, 40, 130, 512], size=m,
                      p=[.05, .25, .15, .15, .1, .1, .08, .07, .04, .01])
    lens[rng.integers(m)] = min(n - 5, 900)
    rows, cols = [], []
    for i, ln in enumerate(lens):
        cs = rng.choice(n - 5, size=min(ln, n - 5), replace=False)
        rows.append(np.full(cs.size, i))
        cols.append(cs)
    K = sp.csr_matrix((rng.standard_normal(int(sum(c.size for c in cols))),
                       (np.concatenate(rows), np.concatenate(cols))), shape=(m, n))
    K.sort_indices()
    return K


def _check(K, L, npanel, groups, aligned, cuts=None, emax=8):
    m, n = K.shape
    rp, ci, v = K.indptr.astype(np.int64), K.indices, K.data
    nnz = K.nnz
    cut = L["cut"]
    assert cut[0] == 0 and cut[-1] == n and np.all(np.diff(cut) >= 0)
    if cuts is not None:
        assert np.array_equal(cut, cuts)
    # every nonzero once; each panel row a run of one row inside one panel
    src = L["src"]
    assert np.array_equal(np.sort(src), np.arange(nnz))
    pp, prow_row = L["prow_ptr"], L["prow_row"]
    assert pp[0] == 0 and pp[-1] == nnz and np.all(np.diff(pp) > 0)
    nprow = prow_row.size
    panel_of = np.empty(nprow, dtype=np.int64)
    for k in range(nprow):
        e = src[pp[k]:pp[k + 1]]
        r = prow_row[k]
        assert np.all((e >= rp[r]) & (e < rp[r + 1])) and np.all(np.diff(e) == 1)
        p = np.searchsorted(cut, ci[e[0]], side="right") - 1
        assert np.all((ci[e] >= cut[p]) & (ci[e] < cut[p + 1]))
        panel_of[k] = p
    assert np.all(np.diff(panel_of) >= 0)                       # stored panel after panel
    # slots: row r's panel rows in panel order, covering the row
    sptr, sidx = L["slot_ptr"], L["slot_idx"]
    assert sptr[-1] == nprow and np.array_equal(np.sort(sidx), np.arange(nprow))
    piece = 512 if emax == 16 else None            # LDS layouts cut longer runs into pieces
    for r in range(m):
        ks = sidx[sptr[r]:sptr[r + 1]]
        assert np.all(prow_row[ks] == r) and np.all(np.diff(panel_of[ks]) >= 0)
        assert (pp[ks + 1] - pp[ks]).sum() == rp[r + 1] - rp[r]
        # the row's entries in order: each panel row starts where the previous one ended
        if ks.size:
            starts = src[pp[ks]]
            assert starts[0] == rp[r] and np.array_equal(starts[1:], src[pp[ks[:-1] + 1] - 1] + 1)
        same = np.diff(panel_of[ks]) == 0
        if piece is None:
            assert not same.any()
        else:
            # pieces of one run: all but the run's last hold exactly 512 entries
            assert np.all((pp[ks[:-1][same] + 1] - pp[ks[:-1][same]]) == piece)
    # wavefront tasks: inside their panel, E L >= every row, every short panel row once
    wave, wb = L["wave"], L["wave_begin"]
    lens = np.diff(pp)
    cov = np.zeros(nprow, dtype=np.int64)
    for p in range(npanel):
        for t in range(wb[p], wb[p + 1]):
            a, b, kl, E = wave[t]
            lanes = 1 << (kl >> 8)
            assert 1 <= E <= emax and np.all(panel_of[a:a + b] == p)
            assert np.all(lens[a:a + b] <= E * lanes)
            # the fewest lanes that reach each row with at most emax entries per lane
            assert lanes == 1 or np.all(lens[a:a + b] > emax * (lanes // 2))
            cov[a:a + b] += 1
    assert np.array_equal(cov, (lens <= 512).astype(np.int64))
    long_ = lens[lens > 512]                        # a workgroup task each, chunks of 16384 beyond
    assert L["nblock"] == int(np.where(long_ > 16384, -(-long_ // 16384), 1).sum())
    if piece is not None:                           # runs beyond 16384 entries stay whole
        assert np.all((lens <= piece) | (lens > 16384))
    # interleaved entries, walked as the kernel reads them
    off, cis, vs = L["task_off"], L["cis"], L["vs"]
    assert off[0] == 0 and off[-1] == cis.size
    civ = ci[src]
    vv = v[src]
    seen = np.zeros(nnz, dtype=np.int64)
    for t in range(wave.shape[0]):
        a, b, kl, E = wave[t]
        lg = kl >> 8
        lanes, per_round = 1 << lg, 64 >> lg
        rounds = -(-b // per_round)
        assert off[t + 1] - off[t] == rounds * 64 * E
        for i in range(rounds):
            for j in range(64):
                slot, lane = i * per_round + (j >> lg), j & (lanes - 1)
                for k in range(E):
                    pos = off[t] + 64 * E * i + 64 * k + j
                    assert 0 <= cis[pos] < n
                    e = k * lanes + lane
                    if slot < b and e < lens[a + slot]:
                        q = pp[a + slot] + e
                        assert cis[pos] == civ[q] and vs[pos] == vv[q]
                        seen[q] += 1
                    else:
                        assert vs[pos] == 0.0
    short = np.repeat(lens <= 512, lens)
    assert np.array_equal(seen, short.astype(np.int64))
    # LDS segments: every wavefront task once, inside its panel; aligned: group b on b mod P
    sp_, seg = L["seg_ptr"], L["seg"]
    tcov = np.zeros(wave.shape[0], dtype=np.int64)
    for g in range(groups):
        for s in range(sp_[g], sp_[g + 1]):
            p, tb, te, _ = seg[s]
            assert wb[p] <= tb < te <= wb[p + 1]
            if aligned:
                assert p == g % npanel
            tcov[tb:te] += 1
    assert np.all(tcov == 1)


@pytest.mark.parametrize("emax", [8, 16])
@pytest.mark.parametrize("npanel,groups,aligned", [(1, 7, False), (3, 24, True), (8, 256, True),
                                                   (17, 5, False)])
def test_panel_layout_equal_nonzero_cuts(npanel, groups, aligned, emax):
    K = _matrix(npanel, 400, 1500)
    L = P.panel_layout(K.indptr, K.indices, K.data, K.shape[1], npanel, groups=groups, aligned=aligned,
                       emax=emax)
    _check(K, L, npanel, groups, aligned, emax=emax)


@pytest.mark.parametrize("emax", [8, 16])
def test_panel_layout_width_slices(emax):
    """Cuts every 128 columns: the slices the LDS-staged products use."""
    K = _matrix(11, 300, 1000)
    W = 128
    npanel = -(-K.shape[1] // W)
    cuts = np.minimum(np.arange(npanel + 1) * W, K.shape[1]).astype(np.int32)
    L = P.panel_layout(K.indptr, K.indices, K.data, K.shape[1], npanel, cuts=cuts, groups=9, emax=emax)
    _check(K, L, npanel, 9, False, cuts=cuts, emax=emax)


@pytest.mark.parametrize("sub", [2, 6])
def test_panel_layout_sub_panel_cuts(sub):
    """8 column ranges of equal nonzero count, each cut into `sub` ranges of equal width: the
    sub-panels an XCD takes one after another."""
    K = _matrix(13, 400, 1500)
    counts = np.bincount(K.indices, minlength=K.shape[1])
    pref = np.concatenate([[0], np.cumsum(counts)])
    xcd = np.searchsorted(pref, np.arange(9) * (K.nnz / 8), side="left").clip(0, K.shape[1])
    xcd[0], xcd[-1] = 0, K.shape[1]
    cuts = [int(xcd[p] + (xcd[p + 1] - xcd[p]) * k // sub) for p in range(8) for k in range(sub)]
    cuts = np.array(cuts + [K.shape[1]], dtype=np.int32)
    assert np.all(np.diff(cuts) >= 0)
    npanel = 8 * sub
    L = P.panel_layout(K.indptr, K.indices, K.data, K.shape[1], npanel, cuts=cuts, groups=8 * 32)
    _check(K, L, npanel, 8 * 32, False, cuts=cuts)


@pytest.mark.parametrize("npanel", [1, 3])
def test_lds_layout_cuts_long_runs_into_pieces(npanel):
    """Rows of 513 .. 2600 nonzeros inside one panel: the LDS layouts (16 entries per lane) hold
    them as consecutive pieces of 512 entries, so they need no workgroup task."""
    rng = np.random.default_rng(7)
    m, n = 40, 3000
    lens = rng.choice([1, 7, 600, 1100, 2600], size=m)
    rows, cols = [], []
    for i, ln in enumerate(lens):
        cs = rng.choice(n, size=ln, replace=False)
        rows.append(np.full(cs.size, i))
        cols.append(cs)
    K = sp.csr_matrix((rng.standard_normal(int(lens.sum())), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, n))
    K.sort_indices()
    L = P.panel_layout(K.indptr, K.indices, K.data, n, npanel, groups=6, emax=16)
    assert L["nblock"] == 0
    _check(K, L, npanel, 6, False, emax=16)
    L8 = P.panel_layout(K.indptr, K.indices, K.data, n, npanel, groups=6, emax=8)
    assert L8["nblock"] > 0
    _check(K, L8, npanel, 6, False, emax=8)


def test_lds_layout_keeps_giant_runs_whole():
    """A run of more than 16384 entries in one panel stays one workgroup task (its pieces would
    serialize the combine); the shorter runs around it are cut."""
    rng = np.random.default_rng(8)
    m, n = 6, 20000
    lens = [3, 17000, 700, 1, 16384, 40]
    rows, cols = [], []
    for i, ln in enumerate(lens):
        cs = rng.choice(n, size=ln, replace=False)
        rows.append(np.full(cs.size, i))
        cols.append(cs)
    K = sp.csr_matrix((rng.standard_normal(int(sum(lens))), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, n))
    K.sort_indices()
    L = P.panel_layout(K.indptr, K.indices, K.data, n, 1, groups=2, emax=16)
    assert L["nblock"] == 2                          # the 17000-entry run in two chunks
    _check(K, L, 1, 2, False, emax=16)


def test_panel_layout_rejects_bad_arguments():
    K = _matrix(2, 50, 200)
    with pytest.raises(P.PdlpError):
        P.panel_layout(K.indptr, K.indices, K.data, K.shape[1], 3, groups=7, aligned=True)
    with pytest.raises(P.PdlpError):
        P.panel_layout(K.indptr, K.indices, K.data, K.shape[1], 3, emax=12)
    bad = K.indices.copy()
    bad[0] = K.shape[1]                                       # a column out of range
    with pytest.raises(P.PdlpError):
        P.panel_layout(K.indptr, bad, K.data, K.shape[1], 3)
    with pytest.raises(P.PdlpError):                           # cuts not ending at ncols
        P.panel_layout(K.indptr, K.indices, K.data, K.shape[1], 2, cuts=np.array([0, 50, 100], np.int32))


def test_layouts_do_not_depend_on_the_host_thread_count():
    """Above 2^20 nonzeros the host preparation runs in parallel chunks (rows, tasks, column
    ranges); every array of the layout must be the same for 1, 3 and 8 threads."""
    rng = np.random.default_rng(12)
    m, n = 70000, 50000
    lens = rng.choice([0, 1, 3, 9, 20, 60, 300, 700], size=m, p=[.05, .2, .2, .2, .15, .15, .04, .01])
    cols = np.concatenate([rng.choice(n, size=ln, replace=False) for ln in lens])
    rows = np.repeat(np.arange(m), lens)
    K = sp.csr_matrix((rng.standard_normal(cols.size), (rows, cols)), shape=(m, n))
    K.sort_indices()
    assert K.nnz > (1 << 20)
    W = 4096
    npanel = -(-n // W)
    cuts = np.minimum(np.arange(npanel + 1) * W, n).astype(np.int32)
    out = {}
    try:
        for th in (1, 3, 8):
            P.set_host_threads(th)
            out[th] = (P.panel_layout(K.indptr, K.indices, K.data, n, 8, groups=256, aligned=True, emax=16),
                       P.panel_layout(K.indptr, K.indices, K.data, n, npanel, cuts=cuts, groups=64, emax=16),
                       P.schedule(K.indptr))
    finally:
        P.set_host_threads(0)
    for th in (3, 8):
        for a, b in zip(out[1][:2], out[th][:2]):
            assert a.keys() == b.keys()
            for k in a:
                assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (th, k)
        for a, b in zip(out[1][2], out[th][2]):
            assert np.array_equal(np.asarray(a), np.asarray(b)), th
