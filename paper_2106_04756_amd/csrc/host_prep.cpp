// Host-side preparation of an LP for the gfx950 kernels: input validation, the transposed
// CSR copy of K (deterministic counting sort, so no value atomics are ever needed on the
// device) and the row-block schedule that load-balances the CSR products.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "pdlp_internal.h"
#include "host_prep.h"

namespace pdlp {

namespace {

// smallest p (p <= 6) with len <= kElemsPerLane * 2^p
int lanes_log2_for(int64_t len) {
  int p = 0;
  while (p < 6 && (int64_t(kElemsPerLane) << p) < len) ++p;
  return p;
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
  for (int p = 0; p <= 6; ++p) {
    const std::vector<int32_t>& b = bins[size_t(p)];
    const int32_t per_task = int32_t((64 >> p) * kRounds);
    for (size_t off = 0; off < b.size(); off += size_t(per_task)) {
      const int32_t cnt = int32_t(std::min<size_t>(size_t(per_task), b.size() - off));
      s.wave.push_back(RowDesc{int32_t(s.perm.size() + off), cnt, int32_t(kWaveRows | (p << 8)), 0});
    }
    s.perm.insert(s.perm.end(), b.begin(), b.end());
  }
  return s;
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
