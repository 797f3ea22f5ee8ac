// Host-side preparation helpers (validation, transpose) of the PDLP solver.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pdlp {

// Returns "" if the LP is well formed, else a description of the first problem found.
std::string validate_lp(int64_t m, int64_t n, int64_t n_eq, const double* c, const int64_t* rp,
                        const int32_t* ci, const double* v, const double* q, const double* l,
                        const double* u);

// CSR of K^T from CSR of K (m x n); entries of each transposed row keep increasing row order.
void transpose_csr(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* v,
                   std::vector<int64_t>& rpT, std::vector<int32_t>& ciT, std::vector<double>& vT);

}  // namespace pdlp
