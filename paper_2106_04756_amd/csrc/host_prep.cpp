// Host-side preparation of an LP for the gfx950 kernels: input validation, the transposed
// CSR copy of K (deterministic counting sort, so no value atomics are ever needed on the
// device) and the row-block schedule that load-balances the CSR products.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pdlp.h"
#include "pdlp_internal.h"
#include "host_prep.h"

namespace pdlp {

namespace {

// smallest p (p <= 6) with len <= emax * 2^p
int lanes_log2_for(int64_t len, int emax = kElemsPerLane) {
  int p = 0;
  while (p < 6 && (int64_t(emax) << p) < len) ++p;
  return p;
}

// entries per lane for rows of at most maxlen nonzeros on 2^p lanes: ceil(maxlen / 2^p), >= 1
int32_t entries_per_lane(int64_t maxlen, int p, int emax = kElemsPerLane) {
  const int64_t L = int64_t(1) << p;
  return int32_t(std::max<int64_t>(1, std::min<int64_t>(emax, (maxlen + L - 1) / L)));
}

}  // namespace

Schedule build_schedule(const int64_t* rp, int64_t nrows) {
  Schedule s;
  std::vector<std::vector<int32_t>> bins(7);
  for (int64_t i = 0; i < nrows; ++i) {
    const int64_t len = rp[i + 1] - rp[i];
    if (len <= kWaveMaxLen) {
      bins[size_t(lanes_log2_for(len))].push_back(int32_t(i));
    } else if (len <= kVectorMax) {
      s.block.push_back(RowDesc{int32_t(i), 0, kVector, 0});
    } else {
      const int32_t id = int32_t(s.split_row.size());
      const int32_t nch = int32_t((len + kChunk - 1) / kChunk);
      s.split_row.push_back(int32_t(i));
      s.split_nchunks.push_back(nch);
      s.split_base.push_back(int32_t(s.total_chunks));
      s.total_chunks += nch;
      for (int32_t c = 0; c < nch; ++c) s.block.push_back(RowDesc{int32_t(i), c, kSplit, id});
    }
  }
  // Rows per lane group in one wavefront task: kRounds when the matrix has enough rows to
  // give every wavefront of a full grid several tasks; fewer (down to 1) on small matrices,
  // which shortens each wavefront's serial chain and spreads the rows over more workgroups.
  int64_t tasks1 = 0;
  for (int p = 0; p <= 6; ++p) tasks1 += (int64_t(bins[size_t(p)].size()) + (64 >> p) - 1) / (64 >> p);
  const int rounds = int(std::min<int64_t>(kRounds, std::max<int64_t>(1, (tasks1 + kFillWaves - 1) / kFillWaves)));
  for (int p = 0; p <= 6; ++p) {
    std::vector<int32_t>& b = bins[size_t(p)];
    // rows of one lane class ordered by length, so a task's rows need about the same number of
    // entries per lane
    std::stable_sort(b.begin(), b.end(), [&](int32_t x, int32_t y) {
      return rp[x + 1] - rp[x] < rp[y + 1] - rp[y];
    });
    const int32_t per_task = int32_t((64 >> p) * rounds);
    for (size_t off = 0; off < b.size(); off += size_t(per_task)) {
      const int32_t cnt = int32_t(std::min<size_t>(size_t(per_task), b.size() - off));
      int64_t maxlen = 0;
      for (int32_t i = 0; i < cnt; ++i) {
        const int32_t r = b[off + size_t(i)];
        maxlen = std::max(maxlen, rp[r + 1] - rp[r]);
      }
      s.wave.push_back(RowDesc{int32_t(s.perm.size() + off), cnt, int32_t(kWaveRows | (p << 8)),
                               entries_per_lane(maxlen, p)});
    }
    s.perm.insert(s.perm.end(), b.begin(), b.end());
  }
  return s;
}

namespace {

// Appends wavefront tasks for the panel rows [k0, k1) (all of one lane class `lg`, ordered by
// length) with offsets prow_ptr.
void push_wave_tasks(Schedule& s, const std::vector<int64_t>& prow_ptr, int64_t k0, int64_t k1, int lg,
                     int emax) {
  const int64_t per_task = int64_t((64 >> lg) * kRounds);
  for (int64_t off = k0; off < k1; off += per_task) {
    const int32_t cnt = int32_t(std::min<int64_t>(per_task, k1 - off));
    int64_t maxlen = 0;
    for (int64_t k = off; k < off + cnt; ++k) maxlen = std::max(maxlen, prow_ptr[size_t(k) + 1] - prow_ptr[size_t(k)]);
    s.wave.push_back(RowDesc{int32_t(off), cnt, int32_t(kWaveRows | (lg << 8)), entries_per_lane(maxlen, lg, emax)});
  }
}

}  // namespace

std::vector<int32_t> panel_cuts(const int32_t* ci, int64_t nnz, int64_t ncols, int P) {
  std::vector<int64_t> colcnt(size_t(ncols) + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) colcnt[size_t(ci[e]) + 1]++;
  for (int64_t j = 0; j < ncols; ++j) colcnt[size_t(j) + 1] += colcnt[size_t(j)];
  std::vector<int32_t> cut(size_t(P) + 1, int32_t(ncols));
  cut[0] = 0;
  for (int p = 1; p < P; ++p) {
    const int64_t target = nnz * p / P;
    cut[size_t(p)] = int32_t(std::lower_bound(colcnt.begin(), colcnt.end(), target) - colcnt.begin());
    cut[size_t(p)] = std::max(cut[size_t(p)], cut[size_t(p) - 1]);
  }
  return cut;
}

std::vector<int32_t> hot_column_order(const int32_t* ci, int64_t nnz, int64_t ncols,
                                      const std::vector<int32_t>& cut) {
  const int P = int(cut.size()) - 1;
  std::vector<int64_t> cnt(size_t(ncols), 0);
  for (int64_t e = 0; e < nnz; ++e) cnt[size_t(ci[e])]++;
  std::vector<int32_t> order(static_cast<size_t>(ncols));
  for (int64_t j = 0; j < ncols; ++j) order[size_t(j)] = int32_t(j);
  for (int p = 0; p < P; ++p)
    std::stable_sort(order.begin() + cut[size_t(p)], order.begin() + cut[size_t(p) + 1],
                     [&](int32_t a, int32_t b) { return cnt[size_t(a)] > cnt[size_t(b)]; });
  return order;
}

bool build_panels(const int64_t* rp, const int32_t* ci, int64_t nrows, int64_t ncols, int P,
                  double max_prow_frac, PanelLayout& L, const std::vector<int32_t>* given_cuts, int emax) {
  const int64_t nnz = rp[nrows];
  L = PanelLayout();
  L.P = P;
  L.cut = given_cuts ? *given_cuts : panel_cuts(ci, nnz, ncols, P);
  const std::vector<int32_t>& cut = L.cut;
  // Layouts for the LDS-staged kernel (emax = kElemsPerLaneLds) hold wavefront tasks: a row's
  // run inside a panel of kWaveMaxLen + 1 .. kVectorMax entries is cut into pieces of
  // kWaveMaxLen entries (the last one shorter), each a panel row of its own, added in order by
  // the combine.  Longer runs stay whole (a workgroup task): the combine adds a row's panel
  // rows one thread at a time, and thousands of pieces would serialize it.
  const bool cut_runs = emax == kElemsPerLaneLds;
  auto pieces = [&](int64_t len) -> int64_t {
    return (cut_runs && len > kWaveMaxLen && len <= kVectorMax) ? (len + kWaveMaxLen - 1) / kWaveMaxLen : 1;
  };
  // Row segments: the panel rows of row r are segments sp[r] .. sp[r + 1], in panel order,
  // with their panel and length (a sparse form of the rows x panels length table).
  std::vector<int64_t> sp(size_t(nrows) + 1, 0);
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t cntr = 0, run = 0;
    int p = -1;
    for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
      int q = p < 0 ? 0 : p;
      while (ci[e] >= cut[size_t(q) + 1]) ++q;
      if (q != p) {
        if (p >= 0) cntr += pieces(run);
        p = q;
        run = 0;
      }
      ++run;
    }
    if (p >= 0) cntr += pieces(run);
    sp[size_t(r) + 1] = sp[size_t(r)] + cntr;
  }
  const int64_t nprow = sp[size_t(nrows)];
  if (double(nprow) > max_prow_frac * double(std::max<int64_t>(nnz, 1))) return false;
  std::vector<int32_t> seg_p(static_cast<size_t>(nprow)), seg_len(static_cast<size_t>(nprow));
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t k = sp[size_t(r)];
    int64_t e = rp[r];
    int q = 0;
    while (e < rp[r + 1]) {
      // the run of panel q starting at e, then its pieces
      while (ci[e] >= cut[size_t(q) + 1]) ++q;
      int64_t e1 = e + 1;
      while (e1 < rp[r + 1] && ci[e1] < cut[size_t(q) + 1]) ++e1;
      const int64_t np = pieces(e1 - e);
      for (int64_t i = 0; i < np; ++i) {
        const int64_t a = e + i * kWaveMaxLen;
        seg_p[size_t(k)] = q;
        seg_len[size_t(k)] = int32_t(np > 1 ? std::min<int64_t>(kWaveMaxLen, e1 - a) : e1 - e);
        ++k;
      }
      e = e1;
    }
  }
  // segments of each panel in row order (counting sort by panel)
  std::vector<int64_t> pp(size_t(P) + 1, 0);
  for (int64_t k = 0; k < nprow; ++k) pp[size_t(seg_p[size_t(k)]) + 1]++;
  for (int p = 0; p < P; ++p) pp[size_t(p) + 1] += pp[size_t(p)];
  std::vector<int64_t> by_panel(static_cast<size_t>(nprow)), fill(pp.begin(), pp.end() - 1);
  std::vector<int32_t> seg_row(static_cast<size_t>(nprow));
  for (int64_t r = 0; r < nrows; ++r)
    for (int64_t k = sp[size_t(r)]; k < sp[size_t(r) + 1]; ++k) {
      seg_row[size_t(k)] = int32_t(r);
      by_panel[size_t(fill[size_t(seg_p[size_t(k)])]++)] = k;
    }
  // order panel rows: panel, then lane class (wavefront rows by p, then long rows), then
  // length (wavefront classes), then row
  L.prow_ptr.reserve(size_t(nprow) + 1);
  L.prow_ptr.push_back(0);
  L.prow_row.reserve(size_t(nprow));
  std::vector<int32_t> prow_of(static_cast<size_t>(nprow), -1);   // panel row id of each segment
  L.wave_begin.push_back(0);
  L.block_begin.push_back(0);
  Schedule& S = L.sched;
  std::vector<int64_t> cls_segs[8];
  for (int p = 0; p < P; ++p) {
    for (auto& v : cls_segs) v.clear();
    for (int64_t i = pp[size_t(p)]; i < pp[size_t(p) + 1]; ++i) {
      const int64_t k = by_panel[size_t(i)];
      const int64_t len = seg_len[size_t(k)];
      cls_segs[(len <= kWaveMaxLen) ? lanes_log2_for(len, emax) : 7].push_back(k);
    }
    for (int cls = 0; cls <= 7; ++cls) {           // 0..6 lane classes, 7 = long rows
      const int64_t k0 = int64_t(L.prow_row.size());
      std::vector<int64_t>& segs = cls_segs[cls];
      if (cls < 7)
        std::stable_sort(segs.begin(), segs.end(), [&](int64_t x, int64_t y) {
          return seg_len[size_t(x)] < seg_len[size_t(y)];
        });
      for (const int64_t k : segs) {
        const int64_t len = seg_len[size_t(k)];
        prow_of[size_t(k)] = int32_t(L.prow_row.size());
        L.prow_row.push_back(seg_row[size_t(k)]);
        L.prow_ptr.push_back(L.prow_ptr.back() + len);
        if (cls == 7) {
          const int32_t kk = int32_t(L.prow_row.size() - 1);
          if (len <= kVectorMax) {
            S.block.push_back(RowDesc{kk, 0, kVector, 0});
          } else {
            const int32_t id = int32_t(S.split_row.size());
            const int32_t nch = int32_t((len + kChunk - 1) / kChunk);
            S.split_row.push_back(kk);
            S.split_nchunks.push_back(nch);
            S.split_base.push_back(int32_t(S.total_chunks));
            S.total_chunks += nch;
            for (int32_t cc = 0; cc < nch; ++cc) S.block.push_back(RowDesc{kk, cc, kSplit, id});
          }
        }
      }
      if (cls < 7) push_wave_tasks(S, L.prow_ptr, k0, int64_t(L.prow_row.size()), cls, emax);
    }
    L.wave_begin.push_back(int32_t(S.wave.size()));
    L.block_begin.push_back(int32_t(S.block.size()));
  }
  // source index of every panel-ordered nonzero, and each row's panel rows in panel order
  L.src.resize(size_t(nnz));
  L.slot_ptr.assign(size_t(nrows) + 1, 0);
  L.slot_idx.reserve(size_t(nprow));
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t e = rp[r];
    for (int64_t k = sp[size_t(r)]; k < sp[size_t(r) + 1]; ++k) {
      const int32_t len = seg_len[size_t(k)];
      const int32_t id = prow_of[size_t(k)];
      const int64_t dst = L.prow_ptr[size_t(id)];
      for (int32_t t = 0; t < len; ++t) L.src[size_t(dst + t)] = e + t;
      e += len;
      L.slot_idx.push_back(id);
    }
    L.slot_ptr[size_t(r) + 1] = int64_t(L.slot_idx.size());
  }
  return true;
}

void build_interleaved(const Schedule& S, const int64_t* rp, const int32_t* ci, const double* v,
                       const int32_t* perm, std::vector<int64_t>& off, std::vector<int32_t>& cis,
                       std::vector<double>& vs) {
  const size_t nt = S.wave.size();
  off.assign(nt + 1, 0);
  for (size_t t = 0; t < nt; ++t) {
    const RowDesc& D = S.wave[t];
    const int lg = D.kind_l >> 8;
    const int64_t per_round = 64 >> lg;
    const int64_t rounds = (int64_t(D.b) + per_round - 1) / per_round;
    off[t + 1] = off[t] + rounds * 64 * int64_t(D.aux);
  }
  cis.assign(size_t(off[nt]), 0);
  vs.assign(size_t(off[nt]), 0.0);
  for (size_t t = 0; t < nt; ++t) {
    const RowDesc& D = S.wave[t];
    const int lg = D.kind_l >> 8, L = 1 << lg, E = D.aux;
    const int per_round = 64 >> lg;
    for (int base = 0, i = 0; base < D.b; base += per_round, ++i) {
      const int64_t blk = off[t] + int64_t(i) * 64 * E;
      for (int j = 0; j < 64; ++j) {
        const int slot = base + (j >> lg), lane = j & (L - 1);
        int64_t q0 = 0, len = 0;
        if (slot < D.b) {
          const int64_t r = perm ? perm[D.a + slot] : D.a + slot;
          q0 = rp[r];
          len = rp[r + 1] - q0;
        }
        const int32_t pad_col = len > 0 ? ci[q0] : 0;
        for (int k = 0; k < E; ++k) {
          const int64_t e = int64_t(k) * L + lane;
          const size_t pos = size_t(blk + int64_t(k) * 64 + j);
          if (e < len) {
            cis[pos] = ci[q0 + e];
            vs[pos] = v[q0 + e];
          } else {
            cis[pos] = pad_col;
          }
        }
      }
    }
  }
}

std::vector<int32_t> lds_segments(const PanelLayout& L, int G, bool aligned, std::vector<LdsSeg>& seg) {
  const std::vector<RowDesc>& W = L.sched.wave;
  const int nt = int(W.size());
  std::vector<double> pre(size_t(nt) + 1, 0.0);
  for (int t = 0; t < nt; ++t) {
    const RowDesc& D = W[size_t(t)];
    const int64_t nz = L.prow_ptr[size_t(D.a + D.b)] - L.prow_ptr[size_t(D.a)];
    pre[size_t(t) + 1] = pre[size_t(t)] + 12.0 * double(nz) + 16.0 * double(D.b) + 64.0;
  }
  // first task of share j of `parts` equal-cost shares of tasks [t0, t1)
  auto share_start = [&](int t0, int t1, int parts, int j) -> int {
    if (j <= 0) return t0;
    if (j >= parts) return t1;
    const double target = pre[size_t(t0)] + (pre[size_t(t1)] - pre[size_t(t0)]) * double(j) / double(parts);
    return int(std::lower_bound(pre.begin() + t0, pre.begin() + t1, target) - pre.begin());
  };
  std::vector<int32_t> seg_ptr(size_t(G) + 1, 0);
  seg.clear();
  for (int b = 0; b < G; ++b) {
    if (aligned) {
      const int p = b % L.P, j = b / L.P, parts = G / L.P;
      const int t0 = L.wave_begin[size_t(p)], t1 = L.wave_begin[size_t(p) + 1];
      const int ta = share_start(t0, t1, parts, j), tb = share_start(t0, t1, parts, j + 1);
      if (tb > ta) seg.push_back(LdsSeg{p, ta, tb, 0});
    } else {
      const int ta = share_start(0, nt, G, b), tb = share_start(0, nt, G, b + 1);
      for (int p = 0; p < L.P && ta < tb; ++p) {
        const int lo = std::max(ta, L.wave_begin[size_t(p)]), hi = std::min(tb, L.wave_begin[size_t(p) + 1]);
        if (hi > lo) seg.push_back(LdsSeg{p, lo, hi, 0});
      }
    }
    seg_ptr[size_t(b) + 1] = int32_t(seg.size());
  }
  return seg_ptr;
}

std::string validate_lp(int64_t m, int64_t n, int64_t n_eq, const double* c, const int64_t* rp,
                        const int32_t* ci, const double* v, const double* q, const double* l,
                        const double* u) {
  if (n < 1) return "n must be at least 1";
  if (m < 0) return "m must be non-negative";
  if (n_eq < 0 || n_eq > m) return "n_eq must lie in [0, m]";
  if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31)) return "m and n must be below 2^31";
  if (rp[0] != 0) return "row_ptr[0] must be 0";
  for (int64_t i = 0; i < m; ++i) {
    if (rp[i + 1] < rp[i]) return "row_ptr must be non-decreasing (row " + std::to_string(i) + ")";
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int32_t j = ci[e];
      if (j < 0 || j >= n) return "column index out of range in row " + std::to_string(i);
      if (e > rp[i] && ci[e - 1] >= j)
        return "column indices must be strictly increasing within row " + std::to_string(i);
      if (!std::isfinite(v[e])) return "non-finite matrix value in row " + std::to_string(i);
    }
  }
  for (int64_t j = 0; j < n; ++j) {
    if (!std::isfinite(c[j])) return "non-finite c[" + std::to_string(j) + "]";
    if (std::isnan(l[j]) || std::isnan(u[j])) return "NaN bound at column " + std::to_string(j);
    if (l[j] > u[j]) return "l > u at column " + std::to_string(j);
    if (l[j] == INFINITY || u[j] == -INFINITY) return "empty box at column " + std::to_string(j);
  }
  for (int64_t i = 0; i < m; ++i)
    if (!std::isfinite(q[i])) return "non-finite q[" + std::to_string(i) + "]";
  return "";
}

void transpose_csr(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* v,
                   std::vector<int64_t>& rpT, std::vector<int32_t>& ciT, std::vector<double>& vT) {
  const int64_t nnz = rp[m];
  rpT.assign(size_t(n) + 1, 0);
  ciT.resize(size_t(nnz));
  vT.resize(size_t(nnz));
  for (int64_t e = 0; e < nnz; ++e) rpT[size_t(ci[e]) + 1]++;
  for (int64_t j = 0; j < n; ++j) rpT[j + 1] += rpT[j];
  std::vector<int64_t> pos(rpT.begin(), rpT.end() - 1);
  for (int64_t i = 0; i < m; ++i) {
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int64_t p = pos[ci[e]]++;
      ciT[size_t(p)] = int32_t(i);
      vT[size_t(p)] = v[e];
    }
  }
}

}  // namespace pdlp

extern "C" int pdlp_build_schedule(const int64_t* row_ptr, int64_t nrows, int32_t* desc,
                                   int64_t cap, int64_t* ndesc, int64_t* nsplit, int32_t* perm) {
  if (!row_ptr || nrows < 0 || !ndesc) return -1;
  pdlp::Schedule s = pdlp::build_schedule(row_ptr, nrows);
  *ndesc = int64_t(s.wave.size() + s.block.size());
  if (nsplit) *nsplit = int64_t(s.split_row.size());
  if (desc) {
    std::vector<pdlp::RowDesc> all(s.wave);
    all.insert(all.end(), s.block.begin(), s.block.end());
    const int64_t nc = std::min<int64_t>(cap, int64_t(all.size()));
    std::memcpy(desc, all.data(), size_t(nc) * sizeof(pdlp::RowDesc));
  }
  if (perm && !s.perm.empty()) std::memcpy(perm, s.perm.data(), s.perm.size() * sizeof(int32_t));
  return 0;
}

extern "C" int pdlp_build_panel_layout(const int64_t* row_ptr, const int32_t* col_idx, const double* val,
                                       int64_t nrows, int64_t ncols, int32_t npanel, const int32_t* cuts,
                                       int32_t emax, int32_t groups, int32_t aligned, pdlp_panel_layout* out) {
  if (!row_ptr || !col_idx || !val || !out || nrows < 0 || ncols < 1 || npanel < 1 || groups < 1 ||
      (aligned && groups % npanel != 0) || (emax != pdlp::kElemsPerLane && emax != pdlp::kElemsPerLaneLds))
    return -1;
  // a valid CSR matrix (offsets from 0, non-decreasing; columns in range, increasing in a row)
  // and valid cuts (0 = cut[0] <= cut[1] <= ... <= cut[npanel] = ncols)
  if (row_ptr[0] != 0) return -1;
  for (int64_t r = 0; r < nrows; ++r) {
    if (row_ptr[r + 1] < row_ptr[r]) return -1;
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
      if (col_idx[e] < 0 || col_idx[e] >= ncols || (e > row_ptr[r] && col_idx[e] <= col_idx[e - 1])) return -1;
  }
  if (cuts) {
    if (cuts[0] != 0 || cuts[npanel] != ncols) return -1;
    for (int p = 0; p < npanel; ++p)
      if (cuts[p + 1] < cuts[p]) return -1;
  }
  std::vector<int32_t> given;
  if (cuts) given.assign(cuts, cuts + npanel + 1);
  pdlp::PanelLayout L;
  if (!pdlp::build_panels(row_ptr, col_idx, nrows, ncols, npanel, 1e300, L, cuts ? &given : nullptr, emax))
    return -1;
  const int64_t nnz = row_ptr[nrows];
  std::vector<int32_t> ciP(static_cast<size_t>(nnz));
  std::vector<double> vP(static_cast<size_t>(nnz));
  for (int64_t k = 0; k < nnz; ++k) {
    ciP[size_t(k)] = col_idx[L.src[size_t(k)]];
    vP[size_t(k)] = val[L.src[size_t(k)]];
  }
  std::vector<int64_t> off;
  std::vector<int32_t> cis;
  std::vector<double> vs;
  pdlp::build_interleaved(L.sched, L.prow_ptr.data(), ciP.data(), vP.data(), nullptr, off, cis, vs);
  std::vector<pdlp::LdsSeg> seg;
  const std::vector<int32_t> seg_ptr = pdlp::lds_segments(L, groups, aligned != 0, seg);
  const bool fill = out->prow_ptr != nullptr;
  if (fill && (out->nprow != int64_t(L.prow_row.size()) || out->nwave != int64_t(L.sched.wave.size()) ||
               out->nslots != off.back() || out->nseg != int64_t(seg.size())))
    return -1;
  out->nprow = int64_t(L.prow_row.size());
  out->nwave = int64_t(L.sched.wave.size());
  out->nblock = int64_t(L.sched.block.size());
  out->nslots = off.back();
  out->nseg = int64_t(seg.size());
  if (!fill) return 0;
  auto put = [](auto* dst, const auto& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  put(out->cut, L.cut);
  put(out->prow_ptr, L.prow_ptr);
  put(out->prow_row, L.prow_row);
  put(out->src, L.src);
  put(out->slot_ptr, L.slot_ptr);
  put(out->slot_idx, L.slot_idx);
  put(out->wave, L.sched.wave);
  put(out->wave_begin, L.wave_begin);
  put(out->task_off, off);
  put(out->cis, cis);
  put(out->vs, vs);
  put(out->seg_ptr, seg_ptr);
  put(out->seg, seg);
  return 0;
}
