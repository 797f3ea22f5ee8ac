// Host-side preparation helpers (validation, transpose) of the PDLP solver.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace pdlp {

// Host threads of the preparation work in pdlp_create (default: the hardware threads, at most
// 16).  Every parallel loop below splits its index range into contiguous chunks whose writes
// are disjoint, so the prepared data do not depend on the thread count.
int host_threads();
void set_host_threads(int n);

// f(lo, hi) over contiguous chunks of [0, n) of at least min_chunk indices, on up to
// host_threads() threads; returns when all are done.  An exception thrown by f is rethrown
// here (the first one).
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f, int64_t min_chunk = 1 << 15);

// Nonzeros of each column 0..ncols-1 (each thread counts the columns of its own range).
std::vector<int64_t> column_counts(const int32_t* ci, int64_t nnz, int64_t ncols);

// Returns "" if the LP is well formed, else a description of the first problem found.
std::string validate_lp(int64_t m, int64_t n, int64_t n_eq, const double* c, const int64_t* rp,
                        const int32_t* ci, const double* v, const double* q, const double* l,
                        const double* u);

// CSR of K^T from CSR of K (m x n); entries of each transposed row keep increasing row order.
void transpose_csr(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* v,
                   std::vector<int64_t>& rpT, std::vector<int32_t>& ciT, std::vector<double>& vT);

// Column cuts of the XCD panels: P + 1 offsets splitting columns 0..ncols into ranges of
// about nnz / P nonzeros each (the same cuts build_panels uses).
std::vector<int32_t> panel_cuts(const int32_t* ci, int64_t nnz, int64_t ncols, int P);

// A column order that keeps every column inside its range of `cut` and, within each range, puts
// the columns with the most nonzeros first (ties by index): order[j'] = column at position j'.
// Gathers from the few dense columns of a skewed matrix then hit a small contiguous slice.
// The panels of the reordered matrix must then be built with the same cuts.
std::vector<int32_t> hot_column_order(const int32_t* ci, int64_t nnz, int64_t ncols,
                                      const std::vector<int32_t>& cut);

}  // namespace pdlp
