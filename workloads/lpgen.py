"""Seeded synthetic LP instances shared by the oracle tests, the GPU tests and bench.py.

This module only *builds* problem data (a constraint matrix, right-hand sides, costs and
bounds).  It contains none of the solver's arithmetic: no PDHG step, no scaling, no
restart logic.  Both the CPU oracle and the HIP path read the very same arrays from here.

Problem form (Section 2, problem (1)):  min c^T x  s.t.  G x >= h,  A x = b,  l <= x <= u,
with K = [G; A] stored as one CSR matrix whose first m1 = m - n_eq rows are the ">=" rows
and whose last n_eq rows are the equalities, and q = [h; b].

Instances that are built as "<=" rows (the workload recipes) are negated into the ">="
form before they are returned.  Every recipe is feasible and bounded by construction:
x0 is a feasible point and (y0, lambda = s) is a dual-feasible point, so
    dual_bound <= optimum <= c^T x0.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

INF = np.inf


@dataclass
class LP:
    """One LP in the form above, CSR of K with int64 row pointers and int32 columns."""
    m: int
    n: int
    n_eq: int
    c: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    q: np.ndarray
    l: np.ndarray
    u: np.ndarray
    name: str = ""
    x0: np.ndarray | None = None        # feasible primal point (certificate)
    y0: np.ndarray | None = None        # dual point, y0[:m1] >= 0
    s: np.ndarray | None = None         # c - K^T y0, lies in the reduced-cost set
    extra: dict = field(default_factory=dict)

    @property
    def m1(self) -> int:
        return self.m - self.n_eq

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def K(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.m, self.n))

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.c, self.row_ptr, self.col_idx, self.val, self.q, self.l, self.u):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(np.int64([self.m, self.n, self.n_eq]).tobytes())
        return h.hexdigest()


def from_csr(K: sp.csr_matrix, c, q, l, u, n_eq, name="") -> LP:
    K = sp.csr_matrix(K)
    K.sort_indices()
    m, n = K.shape
    return LP(m=m, n=n, n_eq=int(n_eq), c=np.asarray(c, np.float64).copy(),
              row_ptr=K.indptr.astype(np.int64), col_idx=K.indices.astype(np.int32),
              val=K.data.astype(np.float64), q=np.asarray(q, np.float64).copy(),
              l=np.asarray(l, np.float64).copy(), u=np.asarray(u, np.float64).copy(), name=name)


# ----------------------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------------------

def _distinct_rows_per_column(rng, counts: np.ndarray, m: int) -> np.ndarray:
    """For column j draw counts[j] distinct rows uniformly from [0, m).

    Returns the keys col*m + row sorted ascending (so column-major, rows ascending).
    Duplicates drawn with replacement are redrawn until none remain.
    """
    n = counts.shape[0]
    cols = np.repeat(np.arange(n, dtype=np.int64), counts)
    key = cols * m + rng.integers(0, m, size=cols.shape[0], dtype=np.int64)
    del cols
    key.sort()
    while True:
        dup = np.flatnonzero(key[1:] == key[:-1]) + 1
        if dup.size == 0:
            return key
        dcols = key[dup] // m
        key[dup] = dcols * m + rng.integers(0, m, size=dup.size, dtype=np.int64)
        # re-sort the complete segments of the touched columns (they occupy the same slots)
        touched = np.zeros(n, dtype=bool)
        touched[dcols] = True
        sel = touched[key // m]
        sub = key[sel]
        sub.sort()
        key[sel] = sub


def _csc_to_lp_csr(key: np.ndarray, vals: np.ndarray, m: int, n: int) -> sp.csr_matrix:
    cols = (key // m).astype(np.int64)
    rows = (key % m).astype(np.int32)
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=n), out=colptr[1:])
    del cols
    csc = sp.csc_matrix((vals, rows, colptr), shape=(m, n))
    csr = csc.tocsr()
    csr.sort_indices()
    return csr


def _finish_plain_lp(rng, K_le_form: sp.csr_matrix, m_le: int, x0, l, u, free_cols, name,
                     slack_hi=1.0) -> LP:
    """Given K whose first m_le rows are '<=' rows and the rest equalities, draw slack, y0, s
    (in this order) and return the '>=' form with the certificates attached."""
    m, n = K_le_form.shape
    Kx0 = K_le_form @ x0
    slack = rng.uniform(0.0, slack_hi, size=m_le)
    q_le = Kx0.copy()
    q_le[:m_le] += slack
    # negate the "<=" rows:  -K_le x >= -q_le
    sign = np.ones(m)
    sign[:m_le] = -1.0
    K = sp.diags(sign) @ K_le_form
    K = sp.csr_matrix(K)
    K.sort_indices()
    q = sign * q_le
    y0 = rng.standard_normal(m)
    y0[:m_le] = np.abs(y0[:m_le])
    s = rng.uniform(0.0, 1.0, size=n)
    if free_cols is not None:
        s[free_cols] = 0.0
    c = K.T @ y0 + s
    lp = from_csr(K, c, q, l, u, n_eq=m - m_le, name=name)
    lp.x0, lp.y0, lp.s = x0, y0, s
    return lp


# ----------------------------------------------------------------------------------------
# workload recipes
# ----------------------------------------------------------------------------------------

def tiny_plain(seed: int = 0, m: int = 200, n: int = 500, n_le: int = 80, per_col: int = 5,
               name="tiny plain LP") -> LP:
    """Small plain LP: per_col nonzeros per column at distinct uniform rows, N(0,1) values,
    rows [0, n_le) are '<=' rows (negated to '>='), the rest equalities, bounds [0, 10],
    q = K x0 (+U[0,1] slack on the inequality rows) with x0 ~ U[0,5], c = K^T y0 + s."""
    rng = np.random.default_rng(seed)
    key = _distinct_rows_per_column(rng, np.full(n, per_col, dtype=np.int64), m)
    vals = rng.standard_normal(key.shape[0])
    K = _csc_to_lp_csr(key, vals, m, n)
    x0 = rng.uniform(0.0, 5.0, size=n)
    l = np.zeros(n)
    u = np.full(n, 10.0)
    return _finish_plain_lp(rng, K, n_le, x0, l, u, None, name)


def tiny_lp(seed: int = 0) -> LP:
    """Tiny plain LP: m=200 (80 '<=' rows, 120 equalities), n=500, 5 nonzeros per column."""
    return tiny_plain(seed, 200, 500, 80, 5, name="tiny plain LP m=200 n=500 nnz=2500")


def large_plain(seed: int = 1, m: int = 1_000_000, n: int = 2_000_000, eq_frac: float = 0.3,
                zipf_a: float = 1.5, max_col: int = 2000, big_frac: float = 0.01,
                name="large plain LP", truncate: bool = False) -> LP:
    """Large plain LP: column nonzero counts min(Zipf(a), max_col) at distinct uniform rows,
    N(0,1) values with big_frac of the columns multiplied by 1e3, the last eq_frac of the rows
    equalities, mixed column bounds (50% [0,inf), 30% [l,u] with l~U[-5,0], u~U[0,5], 20% free).
    x0: U[l,u] on boxed, U[0,5] on [0,inf), U[-5,5] on free columns.  s = 0 on free columns.
    truncate=True draws the counts from Zipf(a) conditioned on <= max_col (redrawing larger
    values) instead of clipping them."""
    rng = np.random.default_rng(seed)
    if truncate:
        counts = rng.zipf(zipf_a, size=n)
        while True:
            bad = counts > max_col
            if not bad.any():
                break
            counts[bad] = rng.zipf(zipf_a, size=int(bad.sum()))
        counts = np.minimum(counts, m).astype(np.int64)
    else:
        counts = np.minimum(rng.zipf(zipf_a, size=n), min(max_col, m)).astype(np.int64)
    key = _distinct_rows_per_column(rng, counts, m)
    vals = rng.standard_normal(key.shape[0])
    big = rng.choice(n, size=int(round(big_frac * n)), replace=False)
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=colptr[1:])
    colscale = np.ones(n)
    colscale[big] = 1e3
    vals *= np.repeat(colscale, counts)
    K = _csc_to_lp_csr(key, vals, m, n)
    del key, vals
    m_le = m - int(round(eq_frac * m))
    perm = rng.permutation(n)
    n_pos, n_box = int(round(0.5 * n)), int(round(0.3 * n))
    pos_cols, box_cols, free_cols = perm[:n_pos], perm[n_pos:n_pos + n_box], perm[n_pos + n_box:]
    l = np.full(n, -INF)
    u = np.full(n, INF)
    l[pos_cols] = 0.0
    lb = rng.uniform(-5.0, 0.0, size=box_cols.size)
    ub = rng.uniform(0.0, 5.0, size=box_cols.size)
    l[box_cols], u[box_cols] = lb, ub
    x0 = np.empty(n)
    x0[pos_cols] = rng.uniform(0.0, 5.0, size=pos_cols.size)
    x0[box_cols] = rng.uniform(lb, ub)
    x0[free_cols] = rng.uniform(-5.0, 5.0, size=free_cols.size)
    lp = _finish_plain_lp(rng, K, m_le, x0, l, u, free_cols, name)
    lp.extra["col_counts"] = counts
    return lp


def large_lp(seed: int = 1) -> LP:
    """Large plain LP m=1e6, n=2e6, Zipf(1.5) column counts clipped to [1,2000] (nnz ~1.36e8)."""
    return large_plain(seed, name="large plain LP m=1e6 n=2e6 Zipf(1.5) columns")


def large_lp_truncated(seed: int = 1) -> LP:
    """Large plain LP m=1e6, n=2e6 with about 2.1e7 nonzeros: as large_lp, with the column
    counts Zipf(1.5) truncated to [1, 190] (mean ~10.6)."""
    return large_plain(seed, max_col=190, truncate=True,
                       name="large plain LP m=1e6 n=2e6 Zipf(1.5) columns truncated to [1,190]")


def preferential_attachment_graph(seed: int, n_nodes: int, out_deg: int = 8):
    """Directed preferential-attachment graph: nodes 0..out_deg form a complete directed seed
    graph; every later node v links to out_deg distinct earlier nodes, drawn with probability
    proportional to (in-degree + 1).  Nodes join in batches of at most 1% of the current graph
    size; a batch draws from the degree pool as it stood when the batch started.
    Returns (src, dst) int64 edge arrays (edge src -> dst)."""
    rng = np.random.default_rng(seed)
    d = out_deg
    s0 = d + 1
    src0, dst0 = np.meshgrid(np.arange(s0), np.arange(s0), indexing="ij")
    mask = src0 != dst0
    src_l = [src0[mask].ravel().astype(np.int64)]
    dst_l = [dst0[mask].ravel().astype(np.int64)]
    # pool: every node once (the +1) plus once per in-edge
    pool = np.empty(s0 + (n_nodes * (d + 1)), dtype=np.int64)
    plen = 0
    pool[:s0] = np.arange(s0)
    plen = s0
    tgt0 = dst_l[0]
    pool[plen:plen + tgt0.size] = tgt0
    plen += tgt0.size
    v = s0
    while v < n_nodes:
        b = max(1, min(n_nodes - v, v // 100))
        draws = pool[rng.integers(0, plen, size=(b, d))]
        # redraw duplicates within a node's targets
        while True:
            srt = np.sort(draws, axis=1)
            bad_rows = np.flatnonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))
            if bad_rows.size == 0:
                break
            redraw = pool[rng.integers(0, plen, size=(bad_rows.size, d))]
            draws[bad_rows] = redraw
        new_src = np.repeat(np.arange(v, v + b, dtype=np.int64), d)
        new_dst = draws.ravel()
        src_l.append(new_src)
        dst_l.append(new_dst)
        pool[plen:plen + b] = np.arange(v, v + b)
        plen += b
        pool[plen:plen + new_dst.size] = new_dst
        plen += new_dst.size
        v += b
    return np.concatenate(src_l), np.concatenate(dst_l)


def pagerank_lp(seed: int = 2, n_nodes: int = 5_000_000, out_deg: int = 8, damping: float = 0.85,
                name="PageRank LP") -> LP:
    """PageRank as an LP (Appendix D): with the column-stochastic link matrix S' (entries
    1/out_deg), rows i < N read  x_i - damping (S'x)_i >= (1-damping)/N, row N is sum(x) = 1,
    x >= 0, c = 0.  One column per node, n_eq = 1."""
    src, dst = preferential_attachment_graph(seed, n_nodes, out_deg)
    N = n_nodes
    w = -damping / out_deg
    rows = np.concatenate([dst, np.arange(N, dtype=np.int64), np.full(N, N, dtype=np.int64)])
    cols = np.concatenate([src, np.arange(N, dtype=np.int64), np.arange(N, dtype=np.int64)])
    vals = np.concatenate([np.full(src.size, w), np.ones(N), np.ones(N)])
    del src, dst
    K = sp.coo_matrix((vals, (rows, cols)), shape=(N + 1, N)).tocsr()
    del rows, cols, vals
    K.sort_indices()
    q = np.full(N + 1, (1.0 - damping) / N)
    q[N] = 1.0
    lp = from_csr(K, np.zeros(N), q, np.zeros(N), np.full(N, INF), n_eq=1, name=name)
    lp.extra["damping"] = damping
    lp.extra["out_deg"] = out_deg
    return lp


def pagerank_5m(seed: int = 2) -> LP:
    """PageRank LP on 5e6 nodes, out-degree 8 (nnz 5.0e7)."""
    return pagerank_lp(seed, 5_000_000, name="PageRank LP 5e6 nodes out-degree 8")


def batched_instance(i: int, base_seed: int = 3000) -> LP:
    """Member i of the batched workload: m log-uniform in [50,2000], n = round(U[2,3] m),
    3..8 nonzeros per column, 60% equality rows, otherwise as the tiny plain LP."""
    rng = np.random.default_rng(base_seed + i)
    m = int(round(np.exp(rng.uniform(np.log(50.0), np.log(2000.0)))))
    n = int(round(rng.uniform(2.0, 3.0) * m))
    counts = rng.integers(3, 9, size=n).astype(np.int64)
    counts = np.minimum(counts, m)
    key = _distinct_rows_per_column(rng, counts, m)
    vals = rng.standard_normal(key.shape[0])
    K = _csc_to_lp_csr(key, vals, m, n)
    m_le = m - int(round(0.6 * m))
    x0 = rng.uniform(0.0, 5.0, size=n)
    lp = _finish_plain_lp(rng, K, m_le, x0, np.zeros(n), np.full(n, 10.0), None,
                          name=f"batched member {i} m={m} n={n}")
    return lp


def unroll_lp(seed: int = 4):
    """Unroll workload: m=2e4 (8000 '<=' rows, 12000 equalities), n=5e4, 6 nonzeros per column;
    x_tgt ~ U[0,5]^n drawn from a fresh generator with the same seed after the instance."""
    lp = tiny_plain(seed, 20_000, 50_000, 8_000, 6, name="unroll LP m=2e4 n=5e4 nnz=3e5")
    x_tgt = np.random.default_rng(seed).uniform(0.0, 5.0, size=lp.n)
    return lp, x_tgt


def tiny_box_lp(seed: int, m: int = 4, n: int = 5, n_eq: int = 1, density: float = 0.7) -> LP:
    """Very small dense-ish LP with a finite box [0, U], used for vertex enumeration."""
    rng = np.random.default_rng(seed)
    while True:
        Kd = rng.standard_normal((m, n)) * (rng.random((m, n)) < density)
        if (np.abs(Kd).sum(axis=1) > 0).all():
            break
    x0 = rng.uniform(0.5, 2.5, size=n)
    ub = rng.uniform(3.0, 4.0, size=n)
    q = Kd @ x0
    m1 = m - n_eq
    q[:m1] -= rng.uniform(0.0, 1.0, size=m1)       # G x0 >= h with slack
    c = rng.standard_normal(n)
    lp = from_csr(sp.csr_matrix(Kd), c, q, np.zeros(n), ub, n_eq=n_eq, name=f"tiny box LP seed {seed}")
    lp.x0 = x0
    return lp


def add_empty_row_and_column(lp: LP) -> LP:
    """Same LP with one extra empty '>=' row (0 >= -1) placed first and one extra column
    (bounds [0,1], cost 1) that no row touches, appended last."""
    K = lp.K()
    m, n = K.shape
    K2 = sp.vstack([sp.csr_matrix((1, n)), K]).tocsr()
    K2 = sp.hstack([K2, sp.csr_matrix((m + 1, 1))]).tocsr()
    q2 = np.concatenate([[-1.0], lp.q])
    c2 = np.concatenate([lp.c, [1.0]])
    l2 = np.concatenate([lp.l, [0.0]])
    u2 = np.concatenate([lp.u, [1.0]])
    out = from_csr(K2, c2, q2, l2, u2, n_eq=lp.n_eq, name=lp.name + " +empty row/col")
    if lp.x0 is not None:
        out.x0 = np.concatenate([lp.x0, [0.0]])
    return out
