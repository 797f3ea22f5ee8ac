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

int lanes_log2_for(int64_t len) {
  // smallest L = 2^p (p <= 6) with ceil(len / L) <= kPerThread
  int p = 0;
  while (p < 6 && (int64_t(kPerThread) << p) < len) ++p;
  return p;
}

}  // namespace

Schedule build_schedule(const int64_t* rp, int64_t nrows) {
  Schedule s;
  int32_t cur_r0 = 0, cur_rows = 0;
  int64_t cur_nnz = 0;
  int cur_lg = 0;
  auto flush = [&]() {
    if (cur_rows > 0) s.desc.push_back(RowDesc{cur_r0, cur_rows, int32_t(kStream | (cur_lg << 8)), 0});
    cur_rows = 0;
    cur_nnz = 0;
    cur_lg = 0;
  };
  const int64_t stream_max_len = int64_t(kPerThread) * kMaxLanesRow;
  for (int64_t i = 0; i < nrows; ++i) {
    const int64_t len = rp[i + 1] - rp[i];
    if (len > stream_max_len) {
      flush();
      if (len <= kVectorMax) {
        s.desc.push_back(RowDesc{int32_t(i), 0, kVector, 0});
      } else {
        const int32_t id = int32_t(s.split_row.size());
        const int32_t nch = int32_t((len + kChunk - 1) / kChunk);
        s.split_row.push_back(int32_t(i));
        s.split_nchunks.push_back(nch);
        s.split_base.push_back(int32_t(s.total_chunks));
        s.total_chunks += nch;
        for (int32_t c = 0; c < nch; ++c) s.desc.push_back(RowDesc{int32_t(i), c, kSplit, id});
      }
      continue;
    }
    const int lg_new = std::max(cur_lg, lanes_log2_for(len));
    if (cur_rows > 0 &&
        ((int64_t(cur_rows + 1) << lg_new) > kBlock || cur_nnz + len > kStreamNnz)) {
      flush();
    }
    if (cur_rows == 0) {
      cur_r0 = int32_t(i);
      cur_lg = lanes_log2_for(len);
    } else {
      cur_lg = lg_new;
    }
    ++cur_rows;
    cur_nnz += len;
  }
  flush();
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
                                   int64_t cap, int64_t* ndesc, int64_t* nsplit) {
  if (!row_ptr || nrows < 0 || !ndesc) return -1;
  pdlp::Schedule s = pdlp::build_schedule(row_ptr, nrows);
  *ndesc = int64_t(s.desc.size());
  if (nsplit) *nsplit = int64_t(s.split_row.size());
  if (desc) {
    const int64_t nc = std::min<int64_t>(cap, int64_t(s.desc.size()));
    std::memcpy(desc, s.desc.data(), size_t(nc) * sizeof(pdlp::RowDesc));
  }
  return 0;
}
