// Device-side views of the solver's data, shared by the kernels and the host driver.
#pragma once

#include <cstdint>

#include "../../include/pdlp.h"
#include "pdlp_internal.h"

namespace pdlp {

// One CSR copy with its row-block schedule.
struct CsrDev {
  const int64_t* rp;
  const int32_t* ci;
  const double* v;
  int32_t nrows;         // rows of the layout (panel rows in panel mode)
  int32_t nwave;         // wavefront tasks
  int32_t nblock;        // workgroup tasks
  int32_t npanel;        // 1 = plain row layout, else XCD column panels
  const int32_t* perm;   // row of each wavefront slot (nullptr: identity)
  const RowDesc* wave;
  const RowDesc* block;
  const int64_t* task_off;     // interleaved entries of wavefront task t from task_off[t]
  const double* vs;            // (build_interleaved); the CSR arrays serve workgroup tasks
  const int32_t* cis;
  const uint16_t* cis16;       // slices only: the interleaved columns relative to the slice
  const uint16_t* rlen;        // length of each row of the layout (wavefront rows: <= 512)
  const int32_t* wave_begin;   // npanel + 1 task offsets per panel
  const int32_t* block_begin;
  const int32_t* prow_row;     // panel mode: original row of each panel row
  const int64_t* slot_ptr;     // panel mode: panel rows of original row r: slot_idx[slot_ptr[r] ..]
  const int32_t* slot_idx;
  int32_t nrows_orig;
  int32_t emax;          // most entries per lane of a wavefront task (8, or 16 in LDS layouts)
  const int32_t* split_nchunks;
  const int32_t* split_base;
  int32_t nsplit;
  int32_t nsub;          // panel mode: runs of nsub consecutive panels (column ranges), each
                         // run taken by one group of workgroups, one panel after another
  double* split_part;    // partial sums of split-row chunks
  unsigned* split_cnt;   // chunk arrival counters (reset to 0 by the last arrival)
  // LDS-staged products (lds_h > 0, panel mode, wavefront tasks only): lds_grid workgroups of
  // kLdsBlock threads; workgroup b runs segments lds_seg[lds_seg_ptr[b] .. lds_seg_ptr[b + 1]);
  // panel p covers columns col_cut[p] .. col_cut[p + 1], of which the first lds_h are staged.
  int32_t lds_h;
  int32_t lds_grid;
  const int32_t* col_cut;
  const int32_t* lds_seg_ptr;
  const LdsSeg* lds_seg;
};

// Device vectors of a solver.  n-vectors are indexed by column j, m-vectors by row i.
struct Bufs {
  int32_t n, m, m1, pad;
  const double* c;       // c~ = D2 c
  const double* l;       // l~ = l / D2
  const double* u;       // u~ = u / D2
  const double* q;       // q~ = D1 q
  const double* c0;      // the user's c, l, u, q
  const double* l0;
  const double* u0;
  const double* q0;
  const double* D1;
  const double* D2;
  double* X[2];          // current / next primal iterate (parity-selected)
  double* Y[2];
  double* KX[2];         // K~ x of X[.]
  double* KTy;           // K~^T y of the current y (valid when DevState.kty_valid)
  double* KTyH;          // K~^T y^ of the running Malitsky-Pock trial
  double* Sx;            // eta-weighted sums since the last restart
  double* Sy;
  double* XB;            // averages and their products (restart checks)
  double* YB;
  double* KXB;
  double* KTYB;
  double* XA;            // anchor z^{n,0}
  double* YA;
  double* GA[2];         // normalized-gap scratch, n + m each: |a_i| and b_i
  double* GB[2];
  pdlp_attempt_rec* att; // trace logs
  pdlp_check_rec* chk;
  double* tx;
  double* ty;
};

enum Pred : int {
  kPredAlways = 0,
  kPredCheck = 1,
  kPredCheckKty = 2,
  kPredKty = 3,
  kPredCheckRestart = 4,
  kPredAttempt = 5,
  kPredAttemptKty = 6,
  kPredMpNew = 7,        // an attempt runs and starts a Malitsky-Pock iteration
  kPredKtyPeek = 8       // K~^T y is not valid: form it for a KKT evaluation, leave it unmarked
};

}  // namespace pdlp
