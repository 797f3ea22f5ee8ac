// Host-side preparation of an LP for the gfx950 kernels: input validation, the transposed
// CSR copy of K (deterministic counting sort, so no value atomics are ever needed on the
// device) and the row-block schedule that load-balances the CSR products.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <exception>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pdlp.h"
#include "pdlp_internal.h"
#include "host_prep.h"

namespace pdlp {

namespace {

std::atomic<int> g_host_threads{0};

// Matrices below this many nonzeros are prepared on one thread.
constexpr int64_t kParallelNnz = int64_t(1) << 20;

// Stable sort of ids by key(id) in [0, kmax]: a counting sort, which gives the order of a
// stable comparison sort in linear time.
template <class Id, class Key>
void counting_sort_by(std::vector<Id>& ids, int64_t kmax, Key key) {
  std::vector<int64_t> cnt(size_t(kmax) + 2, 0);
  for (const Id& x : ids) cnt[size_t(key(x)) + 1]++;
  for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
  std::vector<Id> out(ids.size());
  for (const Id& x : ids) out[size_t(cnt[size_t(key(x))]++)] = x;
  ids.swap(out);
}

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

int host_threads() {
  const int n = g_host_threads.load();
  if (n > 0) return n;
  const unsigned hw = std::thread::hardware_concurrency();
  return int(std::max(1u, std::min(16u, hw)));
}

void set_host_threads(int n) { g_host_threads.store(std::max(0, n)); }

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f, int64_t min_chunk) {
  if (n <= 0) return;
  const int64_t T = std::max<int64_t>(1, std::min<int64_t>(host_threads(), (n + std::max<int64_t>(min_chunk, 1) - 1) /
                                                                                std::max<int64_t>(min_chunk, 1)));
  if (T == 1) {
    f(0, n);
    return;
  }
  std::exception_ptr err;
  std::mutex mu;
  auto run = [&](int64_t t) {
    try {
      f(n * t / T, n * (t + 1) / T);
    } catch (...) {
      std::lock_guard<std::mutex> g(mu);
      if (!err) err = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  th.reserve(size_t(T - 1));
  try {
    for (int64_t t = 1; t < T; ++t) th.emplace_back(run, t);
  } catch (...) {
    // no more threads: this thread runs the chunks that have none
    for (int64_t t = int64_t(th.size()) + 1; t < T; ++t) run(t);
  }
  run(0);
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

std::vector<int64_t> column_counts(const int32_t* ci, int64_t nnz, int64_t ncols) {
  std::vector<int64_t> cnt(size_t(std::max<int64_t>(ncols, 0)), 0);
  const int64_t T = nnz < kParallelNnz ? 1 : host_threads();
  // thread t counts the columns of its range over all nonzeros
  parallel_for(T, [&](int64_t t0, int64_t t1) {
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t c0 = ncols * t / T, c1 = ncols * (t + 1) / T;
      for (int64_t e = 0; e < nnz; ++e) {
        const int64_t j = ci[e];
        if (j >= c0 && j < c1) cnt[size_t(j)]++;
      }
    }
  }, 1);
  return cnt;
}

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
    counting_sort_by(b, kWaveMaxLen, [&](int32_t x) { return rp[x + 1] - rp[x]; });
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

std::vector<int32_t> panel_cuts(const int32_t* ci, int64_t nnz, int64_t ncols, int P) {
  std::vector<int64_t> colcnt(size_t(ncols) + 1, 0);
  {
    const std::vector<int64_t> cnt = column_counts(ci, nnz, ncols);
    for (int64_t j = 0; j < ncols; ++j) colcnt[size_t(j) + 1] = colcnt[size_t(j)] + cnt[size_t(j)];
  }
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
  const std::vector<int64_t> cnt = column_counts(ci, nnz, ncols);
  std::vector<int32_t> order(static_cast<size_t>(ncols));
  for (int64_t j = 0; j < ncols; ++j) order[size_t(j)] = int32_t(j);
  parallel_for(P, [&](int64_t p0, int64_t p1) {
    for (int64_t p = p0; p < p1; ++p)
      std::stable_sort(order.begin() + cut[size_t(p)], order.begin() + cut[size_t(p) + 1],
                       [&](int32_t a, int32_t b) { return cnt[size_t(a)] > cnt[size_t(b)]; });
  }, 1);
  return order;
}

namespace {

// Layouts for the LDS-staged kernel (emax = kElemsPerLaneLds) hold wavefront tasks: a row's run
// inside a panel of kWaveMaxLen + 1 .. kVectorMax entries is cut into pieces of kWaveMaxLen
// entries (the last one shorter), each a panel row of its own, added in order by the combine.
// Longer runs stay whole (a workgroup task): the combine adds a row's panel rows one thread at
// a time, and thousands of pieces would serialize it.  The panel rows of a run of len entries:
int64_t run_pieces(int64_t len, int emax) {
  return (emax == kElemsPerLaneLds && len > kWaveMaxLen && len <= kVectorMax) ? (len + kWaveMaxLen - 1) / kWaveMaxLen
                                                                             : 1;
}

// The panel rows of each row under the column cuts `cut`, as offsets: row r's are
// sp[r] .. sp[r + 1] (rows in parallel chunks).  Returns their total.
int64_t panel_row_offsets(const int64_t* rp, const int32_t* ci, int64_t nrows, const std::vector<int32_t>& cut,
                          int emax, std::vector<int64_t>& sp) {
  const int64_t nnz = rp[nrows];
  const int64_t row_chunk = nnz < kParallelNnz ? std::max<int64_t>(nrows, 1) : int64_t(1) << 14;
  sp.assign(size_t(nrows) + 1, 0);
  parallel_for(nrows, [&](int64_t r0, int64_t r1) {
    for (int64_t r = r0; r < r1; ++r) {
      int64_t cntr = 0, run = 0;
      int p = -1;
      for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
        int q = p < 0 ? 0 : p;
        while (ci[e] >= cut[size_t(q) + 1]) ++q;
        if (q != p) {
          if (p >= 0) cntr += run_pieces(run, emax);
          p = q;
          run = 0;
        }
        ++run;
      }
      if (p >= 0) cntr += run_pieces(run, emax);
      sp[size_t(r) + 1] = cntr;
    }
  }, row_chunk);
  for (int64_t r = 0; r < nrows; ++r) sp[size_t(r) + 1] += sp[size_t(r)];
  return sp[size_t(nrows)];
}

}  // namespace

int64_t count_panel_rows(const int64_t* rp, const int32_t* ci, int64_t nrows, const std::vector<int32_t>& cut,
                         int emax) {
  std::vector<int64_t> sp;
  return panel_row_offsets(rp, ci, nrows, cut, emax, sp);
}

bool build_panels(const int64_t* rp, const int32_t* ci, int64_t nrows, int64_t ncols, int P,
                  double max_prow_frac, PanelLayout& L, const std::vector<int32_t>* given_cuts, int emax) {
  const int64_t nnz = rp[nrows];
  L = PanelLayout();
  L.P = P;
  L.cut = given_cuts ? *given_cuts : panel_cuts(ci, nnz, ncols, P);
  const std::vector<int32_t>& cut = L.cut;
  auto pieces = [&](int64_t len) -> int64_t { return run_pieces(len, emax); };
  // Row segments: the panel rows of row r are segments sp[r] .. sp[r + 1], in panel order,
  // with their panel and length (a sparse form of the rows x panels length table).
  // (rows in parallel chunks; each writes only its own rows' entries)
  const int64_t row_chunk = nnz < kParallelNnz ? std::max<int64_t>(nrows, 1) : int64_t(1) << 14;
  std::vector<int64_t> sp;
  const int64_t nprow = panel_row_offsets(rp, ci, nrows, cut, emax, sp);
  if (double(nprow) > max_prow_frac * double(std::max<int64_t>(nnz, 1))) return false;
  std::vector<int32_t> seg_p(static_cast<size_t>(nprow)), seg_len(static_cast<size_t>(nprow));
  std::vector<int32_t> seg_row(static_cast<size_t>(nprow));
  parallel_for(nrows, [&](int64_t r0, int64_t r1) {
    for (int64_t r = r0; r < r1; ++r) {
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
          seg_row[size_t(k)] = int32_t(r);
          ++k;
        }
        e = e1;
      }
    }
  }, row_chunk);
  // segments of each panel in row order (counting sort by panel)
  std::vector<int64_t> pp(size_t(P) + 1, 0);
  for (int64_t k = 0; k < nprow; ++k) pp[size_t(seg_p[size_t(k)]) + 1]++;
  for (int p = 0; p < P; ++p) pp[size_t(p) + 1] += pp[size_t(p)];
  std::vector<int64_t> by_panel(static_cast<size_t>(nprow)), fill(pp.begin(), pp.end() - 1);
  for (int64_t k = 0; k < nprow; ++k) by_panel[size_t(fill[size_t(seg_p[size_t(k)])]++)] = k;
  // order panel rows: panel, then lane class (wavefront rows by p, then long rows), then
  // length (wavefront classes), then row.  Each panel is ordered and gets its tasks on its own
  // (panels in parallel, indices relative to the panel), then placed at its offsets.
  struct Part {
    std::vector<int64_t> order;        // the panel's segments in panel-row order
    int64_t nnz = 0;
    std::vector<RowDesc> wave, block;  // .a relative to the panel's first panel row
    std::vector<int32_t> split_prow;   // relative panel row and chunk count of each split row
    std::vector<int32_t> split_nch;
    int64_t nchunks = 0;
  };
  std::vector<Part> part(static_cast<size_t>(P));
  parallel_for(P, [&](int64_t p0, int64_t p1) {
    std::vector<int64_t> cls_segs[8];
    for (int64_t p = p0; p < p1; ++p) {
      Part& W = part[size_t(p)];
      for (auto& v : cls_segs) v.clear();
      for (int64_t i = pp[size_t(p)]; i < pp[size_t(p) + 1]; ++i) {
        const int64_t k = by_panel[size_t(i)];
        const int64_t len = seg_len[size_t(k)];
        cls_segs[(len <= kWaveMaxLen) ? lanes_log2_for(len, emax) : 7].push_back(k);
      }
      W.order.reserve(size_t(pp[size_t(p) + 1] - pp[size_t(p)]));
      for (int cls = 0; cls <= 7; ++cls) {           // 0..6 lane classes, 7 = long rows
        std::vector<int64_t>& segs = cls_segs[cls];
        const int32_t k0 = int32_t(W.order.size());
        if (cls < 7) counting_sort_by(segs, kWaveMaxLen, [&](int64_t x) { return seg_len[size_t(x)]; });
        for (const int64_t k : segs) {
          const int64_t len = seg_len[size_t(k)];
          const int32_t kk = int32_t(W.order.size());
          W.order.push_back(k);
          W.nnz += len;
          if (cls == 7) {
            if (len <= kVectorMax) {
              W.block.push_back(RowDesc{kk, 0, kVector, 0});
            } else {
              const int32_t id = int32_t(W.split_prow.size());
              const int32_t nch = int32_t((len + kChunk - 1) / kChunk);
              W.split_prow.push_back(kk);
              W.split_nch.push_back(nch);
              W.nchunks += nch;
              for (int32_t cc = 0; cc < nch; ++cc) W.block.push_back(RowDesc{kk, cc, kSplit, id});
            }
          }
        }
        if (cls < 7) {
          // wavefront tasks of (64 >> cls) * kRounds rows of this lane class
          const int32_t k1 = int32_t(W.order.size());
          const int32_t per_task = int32_t((64 >> cls) * kRounds);
          for (int32_t off = k0; off < k1; off += per_task) {
            const int32_t cnt = std::min(per_task, k1 - off);
            int64_t maxlen = 0;
            for (int32_t i = off; i < off + cnt; ++i) maxlen = std::max<int64_t>(maxlen, seg_len[size_t(W.order[size_t(i)])]);
            W.wave.push_back(RowDesc{off, cnt, int32_t(kWaveRows | (cls << 8)), entries_per_lane(maxlen, cls, emax)});
          }
        }
      }
    }
  }, 1);
  // offsets of each panel's panel rows, entries, tasks and split rows
  std::vector<int64_t> prow_base(size_t(P) + 1, 0), nnz_base(size_t(P) + 1, 0), split_id_base(size_t(P) + 1, 0),
      chunk_base(size_t(P) + 1, 0);
  Schedule& S = L.sched;
  L.wave_begin.assign(size_t(P) + 1, 0);
  L.block_begin.assign(size_t(P) + 1, 0);
  for (int p = 0; p < P; ++p) {
    const Part& W = part[size_t(p)];
    prow_base[size_t(p) + 1] = prow_base[size_t(p)] + int64_t(W.order.size());
    nnz_base[size_t(p) + 1] = nnz_base[size_t(p)] + W.nnz;
    split_id_base[size_t(p) + 1] = split_id_base[size_t(p)] + int64_t(W.split_prow.size());
    chunk_base[size_t(p) + 1] = chunk_base[size_t(p)] + W.nchunks;
    L.wave_begin[size_t(p) + 1] = L.wave_begin[size_t(p)] + int32_t(W.wave.size());
    L.block_begin[size_t(p) + 1] = L.block_begin[size_t(p)] + int32_t(W.block.size());
  }
  L.prow_ptr.assign(size_t(nprow) + 1, 0);
  L.prow_row.resize(size_t(nprow));
  std::vector<int32_t> prow_of(static_cast<size_t>(nprow));     // panel row id of each segment
  S.wave.resize(size_t(L.wave_begin[size_t(P)]));
  S.block.resize(size_t(L.block_begin[size_t(P)]));
  S.split_row.resize(size_t(split_id_base[size_t(P)]));
  S.split_nchunks.resize(size_t(split_id_base[size_t(P)]));
  S.split_base.resize(size_t(split_id_base[size_t(P)]));
  S.total_chunks = chunk_base[size_t(P)];
  parallel_for(P, [&](int64_t p0, int64_t p1) {
    for (int64_t p = p0; p < p1; ++p) {
      Part& W = part[size_t(p)];
      const int64_t pb = prow_base[size_t(p)];
      int64_t e = nnz_base[size_t(p)];
      for (size_t i = 0; i < W.order.size(); ++i) {
        const int64_t k = W.order[i];
        prow_of[size_t(k)] = int32_t(pb + int64_t(i));
        L.prow_row[size_t(pb) + i] = seg_row[size_t(k)];
        e += seg_len[size_t(k)];
        L.prow_ptr[size_t(pb) + i + 1] = e;
      }
      for (size_t t = 0; t < W.wave.size(); ++t) {
        RowDesc D = W.wave[t];
        D.a += int32_t(pb);
        S.wave[size_t(L.wave_begin[size_t(p)]) + t] = D;
      }
      for (size_t t = 0; t < W.block.size(); ++t) {
        RowDesc D = W.block[t];
        D.a += int32_t(pb);
        if (D.kind_l == kSplit) D.aux += int32_t(split_id_base[size_t(p)]);
        S.block[size_t(L.block_begin[size_t(p)]) + t] = D;
      }
      int64_t cb = chunk_base[size_t(p)];
      for (size_t j = 0; j < W.split_prow.size(); ++j) {
        const size_t id = size_t(split_id_base[size_t(p)]) + j;
        S.split_row[id] = int32_t(pb) + W.split_prow[j];
        S.split_nchunks[id] = W.split_nch[j];
        S.split_base[id] = int32_t(cb);
        cb += W.split_nch[j];
      }
      std::vector<int64_t>().swap(W.order);
    }
  }, 1);
  // source index of every panel-ordered nonzero, and each row's panel rows in panel order (the
  // segments of row r, sp[r] .. sp[r + 1], are its panel rows)
  L.src.resize(size_t(nnz));
  L.slot_ptr = sp;
  L.slot_idx = prow_of;
  parallel_for(nrows, [&](int64_t r0, int64_t r1) {
    for (int64_t r = r0; r < r1; ++r) {
      int64_t e = rp[r];
      for (int64_t k = sp[size_t(r)]; k < sp[size_t(r) + 1]; ++k) {
        const int32_t len = seg_len[size_t(k)];
        const int64_t dst = L.prow_ptr[size_t(prow_of[size_t(k)])];
        for (int32_t t = 0; t < len; ++t) L.src[size_t(dst + t)] = e + t;
        e += len;
      }
    }
  }, row_chunk);
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
  // tasks in parallel chunks (each task owns its slots off[t] .. off[t + 1])
  auto fill_task = [&](size_t t) {
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
  };
  parallel_for(int64_t(nt), [&](int64_t t0, int64_t t1) {
    for (int64_t t = t0; t < t1; ++t) fill_task(size_t(t));
  }, off[nt] < kParallelNnz ? std::max<int64_t>(int64_t(nt), 1) : 1024);
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
  {
    const std::vector<int64_t> cnt = column_counts(ci, nnz, n);
    for (int64_t j = 0; j < n; ++j) rpT[size_t(j) + 1] = rpT[size_t(j)] + cnt[size_t(j)];
  }
  // thread t fills the transposed rows (columns of K) of a range holding about nnz / T
  // entries, scanning the rows of K in order, so each transposed row keeps increasing rows
  const int64_t T = nnz < kParallelNnz ? 1 : host_threads();
  std::vector<int64_t> cut(size_t(T) + 1, n);
  cut[0] = 0;
  for (int64_t t = 1; t < T; ++t)
    cut[size_t(t)] = std::min(n, std::max(cut[size_t(t) - 1],
                                          int64_t(std::lower_bound(rpT.begin(), rpT.end(), nnz * t / T) - rpT.begin())));
  std::vector<int64_t> pos(rpT.begin(), rpT.end() - 1);
  parallel_for(T, [&](int64_t t0, int64_t t1) {
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t c0 = cut[size_t(t)], c1 = cut[size_t(t) + 1];
      if (c0 >= c1) continue;
      for (int64_t i = 0; i < m; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
          const int64_t j = ci[e];
          if (j < c0 || j >= c1) continue;
          const int64_t p = pos[size_t(j)]++;
          ciT[size_t(p)] = int32_t(i);
          vT[size_t(p)] = v[e];
        }
    }
  }, 1);
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
  pdlp::parallel_for(nnz, [&](int64_t k0, int64_t k1) {
    for (int64_t k = k0; k < k1; ++k) {
      ciP[size_t(k)] = col_idx[L.src[size_t(k)]];
      vP[size_t(k)] = val[L.src[size_t(k)]];
    }
  }, int64_t(1) << 20);
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
