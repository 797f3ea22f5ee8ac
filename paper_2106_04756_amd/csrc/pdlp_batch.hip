// Batched PDLP: many independent LPs in one persistent launch, one workgroup per LP.
//
// Each workgroup runs the whole method on its own LP: preconditioning (Section 3.5), the
// initial point, and Algorithm 1 with adaptive steps (Algorithm 2), averages, restart checks
// (Section 3.2), primal-weight updates (Algorithm 3) and the KKT test (Section 4.1), each with
// its own step size, primal weight, restart state, counters and termination.  The scalar state
// lives in LDS (a DevState per workgroup) and is changed only by thread 0 between barriers,
// through the same decision functions the one-LP kernels use; the per-element work uses the
// same element functions.  Products: one thread per row of K~ or K~^T (the member LPs have
// short rows), summing in index order.  No atomics; every sum has a fixed order.
//
// The workgroup size BS (64 .. 1024 threads) is a template parameter: the host launches one
// kernel per size class of the members, with the size its tuner picked for that class.  A
// launch starts from the members' original matrix values (copied into the work arrays it
// scales), so solving again, or timing a candidate size, repeats the same computation.
//
// Included into the solver's translation unit after pdlp_kernels.hip.

namespace pdlp {

struct BatchInst {
  int32_t m, n, m1, pad;
  int64_t rp;     // offset of the member's m + 1 row offsets of K (member-local, from 0)
  int64_t rpT;    // offset of its n + 1 row offsets of K^T
  int64_t nz;     // offset of its nonzeros (same in both copies)
  int64_t xo;     // offset of its n-vectors
  int64_t yo;     // offset of its m-vectors (its (n+m)-vectors start at xo + yo)
};

struct BatchDev {
  const BatchInst* inst;
  const int32_t* order;  // member run by workgroup b (largest members first)
  const int64_t* rp;
  const int32_t* ci;
  double* v;             // work copies of the values, preconditioned in place by each launch
  const double* v0;      // the members' original values
  const int64_t* rpT;
  const int32_t* ciT;
  double* vT;
  const double* vT0;
  double *c, *l, *u, *c0, *l0, *u0, *D2, *X0, *X1, *KTy, *Sx, *XB, *KTYB, *XA;
  double *q, *q0, *D1, *Y0, *Y1, *KX0, *KX1, *Sy, *YB, *KXB, *YA;
  double *GA0, *GA1, *GB0, *GB1;
  DevState* out_state;   // final state of every member
};

__device__ Bufs batch_bufs(const BatchDev& D, const BatchInst& I) {
  Bufs B;
  B.n = I.n;
  B.m = I.m;
  B.m1 = I.m1;
  B.pad = 0;
  const int64_t xo = I.xo, yo = I.yo, zo = I.xo + I.yo;
  B.c = D.c + xo;
  B.l = D.l + xo;
  B.u = D.u + xo;
  B.q = D.q + yo;
  B.c0 = D.c0 + xo;
  B.l0 = D.l0 + xo;
  B.u0 = D.u0 + xo;
  B.q0 = D.q0 + yo;
  B.D1 = D.D1 + yo;
  B.D2 = D.D2 + xo;
  B.X[0] = D.X0 + xo;
  B.X[1] = D.X1 + xo;
  B.Y[0] = D.Y0 + yo;
  B.Y[1] = D.Y1 + yo;
  B.KX[0] = D.KX0 + yo;
  B.KX[1] = D.KX1 + yo;
  B.KTy = D.KTy + xo;
  B.Sx = D.Sx + xo;
  B.Sy = D.Sy + yo;
  B.XB = D.XB + xo;
  B.YB = D.YB + yo;
  B.KXB = D.KXB + yo;
  B.KTYB = D.KTYB + xo;
  B.XA = D.XA + xo;
  B.YA = D.YA + yo;
  B.GA[0] = D.GA0 + zo;
  B.GA[1] = D.GA1 + zo;
  B.GB[0] = D.GB0 + zo;
  B.GB[1] = D.GB1 + zo;
  B.att = nullptr;
  B.chk = nullptr;
  B.tx = nullptr;
  B.ty = nullptr;
  return B;
}

// One member's CSR copy: row offsets from 0, nonzeros at a member offset.
struct LocalCsr {
  const int64_t* rp;
  const int32_t* ci;
  double* v;
  int32_t nrows;
};

// Row r of A times x, summed in index order.  The nonzeros are taken C at a time with the
// index clamped into the row and the extra products masked to +0.0, so the loads of a chunk
// (and then its gathers) are all in flight together; the sum is bit-identical to the plain
// left-to-right loop for any C.
template <int C>
__device__ __forceinline__ double local_row_dot(const LocalCsr& A, int r, const double* __restrict__ x) {
  double s = 0.0;
  const int64_t p0 = A.rp[r], p1 = A.rp[r + 1];
  for (int64_t base = p0; base < p1; base += C) {
    double v[C], xv[C];
    int32_t c[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const int64_t e = (base + k < p1) ? base + k : p1 - 1;
      v[k] = A.v[e];
      c[k] = A.ci[e];
    }
#pragma unroll
    for (int k = 0; k < C; ++k) xv[k] = x[c[k]];
#pragma unroll
    for (int k = 0; k < C; ++k) s = s + ((base + k < p1) ? v[k] * xv[k] : 0.0);
  }
  return s;
}

// Rows r[0..R) of A times x together (r[q] < 0: no row), each summed as local_row_dot sums
// it: the offsets, then each chunk's loads and gathers of all R rows are in flight together.
template <int C, int R>
__device__ __forceinline__ void local_rows_dot(const LocalCsr& A, const int (&r)[R], const double* __restrict__ x,
                                               double (&s)[R]) {
  int64_t p0[R], p1[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    s[q] = 0.0;
    p0[q] = r[q] >= 0 ? A.rp[r[q]] : 0;
    p1[q] = r[q] >= 0 ? A.rp[r[q] + 1] : 0;
  }
  for (int64_t off = 0;; off += C) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < R; ++q) any = any || p0[q] + off < p1[q];
    if (!any) break;
    double v[R][C], xv[R][C];
    int32_t c[R][C];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t last = p1[q] > p0[q] ? p1[q] - 1 : 0;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        const int64_t e = (p0[q] + off + k < p1[q]) ? p0[q] + off + k : last;
        v[q][k] = p1[q] > p0[q] ? A.v[e] : 0.0;
        c[q][k] = p1[q] > p0[q] ? A.ci[e] : 0;
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int k = 0; k < C; ++k) xv[q][k] = (p1[q] > p0[q]) ? x[c[q][k]] : 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int k = 0; k < C; ++k) s[q] = s[q] + ((p0[q] + off + k < p1[q]) ? v[q][k] * xv[q][k] : 0.0);
  }
}

#define PDLP_BLOCK_LOOP(idx, total) for (int64_t idx = threadIdx.x; idx < (total); idx += BS)

// Sum over a workgroup of BS threads of N values per thread, valid in thread 0: wave sums,
// then the waves' sums added in wave order (for BS = 256 the order of block_sum).
template <int N, int BS>
__device__ void bsum(double (&a)[N]) {
  constexpr int NW = BS / 64;
  __shared__ double lds[NW * N];
#pragma unroll
  for (int k = 0; k < N; ++k) a[k] = wave_sum(a[k]);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) lds[w * N + k] = a[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double t = lds[k];
      for (int q = 1; q < NW; ++q) t = t + lds[q * N + k];
      a[k] = t;
    }
  }
  __syncthreads();
}

template <int BS>
__device__ double bmax(double v) {
  constexpr int NW = BS / 64;
  __shared__ double lds[NW];
  v = wave_max(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = lds[0];
    for (int q = 1; q < NW; ++q) t = fmax(t, lds[q]);
    v = t;
  }
  __syncthreads();
  return v;
}

// out = A x, one thread per row.
// Chunk of a row's nonzeros in flight together: 8, or 4 with 1024 threads per member (whose
// 16 waves per CU allow 128 registers per thread).
template <int BS>
constexpr int kRowChunk = BS >= 1024 ? 4 : 8;

template <int BS>
__device__ void local_spmv(const LocalCsr& A, const double* x, double* out) {
  PDLP_BLOCK_LOOP(r, A.nrows) out[r] = local_row_dot<kRowChunk<BS>>(A, int(r), x);
}

template <int BS>
__device__ void batch_gap(DevState& S, const Bufs& B, int mode) {
  PointPtrs pt[2];
  gap_points_of(S, B, mode, pt);
  const int ns = (mode == 0) ? 2 : 1;
  const double sw = sqrt(S.omega);
  const int64_t NM = int64_t(B.n) + B.m;
  {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    PDLP_BLOCK_LOOP(idx, NM) gap_setup_elem(B, pt, ns, sw, idx, acc);
    bsum<6, BS>(acc);
    if (threadIdx.x == 0) gap_setup_decide(S, mode, acc);
    __syncthreads();
  }
  // bisection, one slot at a time, the 32 points of a pass in four groups of 8 (few
  // registers; each point's sum is the one a single group of 32 would form)
  __shared__ double tot[kGapPts];
  for (int pass = 0; pass < 13; ++pass) {
    bool any = false;
    for (int s = 0; s < ns; ++s) {
      if (S.gap_state[s] != 0) continue;
      any = true;
      const uint64_t lo = S.gap_lo[s], hi = S.gap_hi[s];
      const double* GA = s ? B.GA[1] : B.GA[0];
      const double* GB = s ? B.GB[1] : B.GB[0];
      for (int g0 = 0; g0 < kGapPts; g0 += 8) {
        double acc[8];
        double pt8[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          acc[i] = 0.0;
          pt8[i] = __longlong_as_double((long long)gap_point(lo, hi, g0 + i + 1));
        }
        PDLP_BLOCK_LOOP(idx, NM) {
          const double aa = GA[idx], b = GB[idx];
          if (aa != 0.0) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const double e = fmin(pt8[i] * aa, b);
              acc[i] += e * e;
            }
          }
        }
        bsum<8, BS>(acc);
        if (threadIdx.x == 0) {
#pragma unroll
          for (int i = 0; i < 8; ++i) tot[g0 + i] = acc[i];
        }
      }
      if (threadIdx.x == 0) gap_bisect_decide_slot(S, s, tot);
      __syncthreads();
    }
    if (!any) break;
  }
  {
    double sstar[2];
    for (int s = 0; s < 2; ++s)
      sstar[s] = (S.gap_state[s] == 1) ? INFINITY : __longlong_as_double((long long)S.gap_hi[s]);
    double acc[2] = {0.0, 0.0};
    PDLP_BLOCK_LOOP(idx, NM) gap_final_elem(B, S, ns, sstar, idx, acc);
    bsum<2, BS>(acc);
    if (threadIdx.x == 0) gap_final_decide(S, mode, acc, nullptr);
    __syncthreads();
  }
}

template <int BS>
__device__ void batch_kkt(DevState& S, const Bufs& B, int mode) {
  const PointPtrs pt = kkt_point_is_average(S, mode) ? average_point(B) : current_point(B, S.parity);
  double a[7] = {0, 0, 0, 0, 0, 0, 0};
  PDLP_BLOCK_LOOP(idx, int64_t(B.n) + B.m) kkt_elem(B, pt, idx, a);
  bsum<7, BS>(a);
  if (threadIdx.x == 0) kkt_decide(S, mode, a, nullptr);
  __syncthreads();
}

// BS threads per member; the attempt's products take RR rows per thread at a time, CC
// nonzeros of each at a time (the schedule the host's tuner picks per size class).
template <int BS, int CC = kRowChunk<BS>, int RR = 1>
__global__ __launch_bounds__(BS) void k_batch_solve(BatchDev D, DevState tmpl, double tol,
                                                    int64_t iter_limit, int ruiz_iters,
                                                    int pock_chambolle, double primal_importance) {
  __shared__ DevState S;
  // the member's buffers live in LDS (read after each barrier) rather than in registers
  __shared__ Bufs sB;
  const int mb = D.order[blockIdx.x];
  const BatchInst I = D.inst[mb];
  if (threadIdx.x == 0) sB = batch_bufs(D, I);
  __syncthreads();
  const Bufs& B = sB;
  const LocalCsr K{D.rp + I.rp, D.ci + I.nz, D.v + I.nz, I.m};
  const LocalCsr KT{D.rpT + I.rpT, D.ciT + I.nz, D.vT + I.nz, I.n};
  const int n = I.n, m = I.m;
  const int64_t NM = int64_t(n) + m;
  if (threadIdx.x == 0) {
    S = tmpl;
    S.tol = tol;
    S.iter_limit = iter_limit;
  }
  double* D1 = const_cast<double*>(B.D1);
  double* D2 = const_cast<double*>(B.D2);
  PDLP_BLOCK_LOOP(i, m) D1[i] = 1.0;
  PDLP_BLOCK_LOOP(j, n) D2[j] = 1.0;
  {
    const int64_t nnz = K.rp[m];
    const double* v0 = D.v0 + I.nz;
    const double* vT0 = D.vT0 + I.nz;
    PDLP_BLOCK_LOOP(e, nnz) {
      K.v[e] = v0[e];
      KT.v[e] = vT0[e];
    }
  }
  __syncthreads();

  // ---- diagonal preconditioning (Section 3.5): Ruiz passes, then Pock-Chambolle
  const int passes = ruiz_iters + (pock_chambolle ? 1 : 0);
  for (int p = 0; p < passes; ++p) {
    const bool inf_norm = p < ruiz_iters;
    PDLP_BLOCK_LOOP(i, m) {
      double r = 0.0;
      for (int64_t e = K.rp[i]; e < K.rp[i + 1]; ++e) r = inf_norm ? fmax(r, fabs(K.v[e])) : r + fabs(K.v[e]);
      const double d = (r > 0.0) ? 1.0 / sqrt(r) : 1.0;
      B.GB[0][i] = d;
      D1[i] = D1[i] * d;
    }
    PDLP_BLOCK_LOOP(j, n) {
      double r = 0.0;
      for (int64_t e = KT.rp[j]; e < KT.rp[j + 1]; ++e) r = inf_norm ? fmax(r, fabs(KT.v[e])) : r + fabs(KT.v[e]);
      const double d = (r > 0.0) ? 1.0 / sqrt(r) : 1.0;
      B.GB[1][j] = d;
      D2[j] = D2[j] * d;
    }
    __syncthreads();
    const double* dr = B.GB[0];
    const double* dc = B.GB[1];
    PDLP_BLOCK_LOOP(i, m) {
      for (int64_t e = K.rp[i]; e < K.rp[i + 1]; ++e) K.v[e] = (K.v[e] * dr[i]) * dc[K.ci[e]];
    }
    PDLP_BLOCK_LOOP(j, n) {
      for (int64_t e = KT.rp[j]; e < KT.rp[j + 1]; ++e) KT.v[e] = (KT.v[e] * dr[KT.ci[e]]) * dc[j];
    }
    __syncthreads();
  }
  PDLP_BLOCK_LOOP(idx, NM) {
    if (idx < n) {
      const double d = B.D2[idx];
      const_cast<double*>(B.c)[idx] = d * B.c0[idx];
      const_cast<double*>(B.l)[idx] = B.l0[idx] / d;
      const_cast<double*>(B.u)[idx] = B.u0[idx] / d;
    } else {
      const int i = int(idx - n);
      const_cast<double*>(B.q)[i] = B.D1[i] * B.q0[i];
    }
  }
  __syncthreads();

  // ---- initial point and scalars
  {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    double vmax = 0.0;
    PDLP_BLOCK_LOOP(idx, NM) {
      if (idx < n) {
        const int j = int(idx);
        const double x0 = fmin(fmax(0.0, B.l[j]), B.u[j]);
        B.X[0][j] = x0;
        B.X[1][j] = x0;
        B.XA[j] = x0;
        B.Sx[j] = 0.0;
        B.KTy[j] = 0.0;
        a[0] += B.c0[j] * B.c0[j];
        a[2] += B.c[j] * B.c[j];
      } else {
        const int i = int(idx - n);
        B.Y[0][i] = 0.0;
        B.Y[1][i] = 0.0;
        B.YA[i] = 0.0;
        B.Sy[i] = 0.0;
        a[1] += B.q0[i] * B.q0[i];
        a[3] += B.q[i] * B.q[i];
      }
    }
    const int64_t nnz = K.rp[m];
    PDLP_BLOCK_LOOP(e, nnz) vmax = fmax(vmax, fabs(K.v[e]));
    bsum<4, BS>(a);
    vmax = bmax<BS>(vmax);
    if (threadIdx.x == 0) {
      S.c_norm = sqrt(a[0]);
      S.q_norm = sqrt(a[1]);
      const double nc = sqrt(a[2]), nq = sqrt(a[3]);
      S.omega = ((nc > S.eps_zero && nq > S.eps_zero) ? nc / nq : 1.0) * primal_importance;
      S.eta_hat = (vmax > 0.0) ? 1.0 / vmax : 1.0;
      S.eta = S.eta_hat;
    }
    __syncthreads();
    local_spmv<BS>(K, B.X[0], B.KX[0]);
    __syncthreads();
  }

  // ---- termination check before the first step
  batch_kkt<BS>(S, B, 1);

  // ---- Algorithm 1
  while (!S.done) {
    if (!S.check_pending && S.k >= S.iter_limit) {
      if (threadIdx.x == 0) {
        S.done = 1;
        S.status = PDLP_ITERATION_LIMIT;
        S.out_avg = 0;
      }
      __syncthreads();
      break;
    }
    if (!S.check_pending) {
      // one attempt of Algorithm 2
      const int P = S.parity;
      const int kty_valid = S.kty_valid;
      const PrimalEpi pe{B.c, B.l, B.u, pick(B.X, P), pick(B.X, P ^ 1), B.Sx, B.KTy, S.eta / S.omega, S.w_pending, !kty_valid};
      double ax[1] = {0.0};
      double c1[1];
      if constexpr (RR == 1) {
        PDLP_BLOCK_LOOP(j, n) {
          const double s = kty_valid ? B.KTy[j] : local_row_dot<CC>(KT, int(j), pick(B.Y, P));
          pe.row(int(j), s, c1);
          ax[0] += c1[0];
        }
      } else {
        // rows j0, j0 + BS, ..., j0 + (RR - 1) BS together; each thread still updates its rows
        // in the order of the one-row loop
        for (int64_t j0 = threadIdx.x; j0 < n; j0 += int64_t(RR) * BS) {
          int rows[RR];
          double sv[RR];
#pragma unroll
          for (int q = 0; q < RR; ++q) rows[q] = (j0 + int64_t(q) * BS < n) ? int(j0 + int64_t(q) * BS) : -1;
          if (kty_valid) {
#pragma unroll
            for (int q = 0; q < RR; ++q) sv[q] = rows[q] >= 0 ? B.KTy[rows[q]] : 0.0;
          } else {
            local_rows_dot<CC, RR>(KT, rows, pick(B.Y, P), sv);
          }
#pragma unroll
          for (int q = 0; q < RR; ++q) {
            if (rows[q] >= 0) {
              pe.row(rows[q], sv[q], c1);
              ax[0] += c1[0];
            }
          }
        }
      }
      bsum<1, BS>(ax);      // its barriers also publish x' to the whole workgroup
      const DualEpi de{B.q, pick(B.Y, P), pick(B.KX, P), pick(B.Y, P ^ 1), pick(B.KX, P ^ 1), B.Sy, S.eta * S.omega, S.w_pending, B.m1};
      double ay[2] = {0.0, 0.0};
      double c2[2];
      if constexpr (RR == 1) {
        PDLP_BLOCK_LOOP(i, m) {
          de.row(int(i), local_row_dot<CC>(K, int(i), pick(B.X, P ^ 1)), c2);
          ay[0] += c2[0];
          ay[1] += c2[1];
        }
      } else {
        for (int64_t i0 = threadIdx.x; i0 < m; i0 += int64_t(RR) * BS) {
          int rows[RR];
          double sv[RR];
#pragma unroll
          for (int q = 0; q < RR; ++q) rows[q] = (i0 + int64_t(q) * BS < m) ? int(i0 + int64_t(q) * BS) : -1;
          local_rows_dot<CC, RR>(K, rows, pick(B.X, P ^ 1), sv);
#pragma unroll
          for (int q = 0; q < RR; ++q) {
            if (rows[q] >= 0) {
              de.row(rows[q], sv[q], c2);
              ay[0] += c2[0];
              ay[1] += c2[1];
            }
          }
        }
      }
      bsum<2, BS>(ay);
      if (threadIdx.x == 0) {
        if (!kty_valid) S.spmv_KT += 1;
        attempt_decide(S, ax[0], ay[0], ay[1], nullptr);
      }
      __syncthreads();
      continue;
    }
    // ---- restart / termination check
    {
      const int P = S.parity;
      const double w = S.w_pending, se = S.s_eta;
      PDLP_BLOCK_LOOP(idx, NM) prepare_elem(B, P, w, se, idx);
      __syncthreads();
      if (threadIdx.x == 0) S.w_pending = 0.0;
      if (S.restarts_on) {
        local_spmv<BS>(KT, B.YB, B.KTYB);
        local_spmv<BS>(K, B.XB, B.KXB);
      }
      if (!S.kty_valid) local_spmv<BS>(KT, pick(B.Y, P), B.KTy);
      __syncthreads();
      if (threadIdx.x == 0) {
        if (S.restarts_on) {
          S.spmv_K += 1;
          S.spmv_KT += 1;
        }
        if (!S.kty_valid) S.spmv_KT += 1;
        S.kty_valid = 1;
      }
      __syncthreads();
    }
    if (S.restarts_on) batch_gap<BS>(S, B, 0);
    batch_kkt<BS>(S, B, 0);
    if (S.done) break;
    if (S.restarts_on && S.restart) batch_gap<BS>(S, B, 1);
    if (S.restart) {
      const bool avg = S.use_avg != 0;
      const int P = S.parity;
      PDLP_BLOCK_LOOP(idx, NM) apply_elem(B, P, avg, idx);
      __syncthreads();
    }
    if (threadIdx.x == 0) apply_decide(S);
    __syncthreads();
  }

  // ---- KKT error of the returned point when the solve did not end at a passing check
  if (S.status != PDLP_OPTIMAL) {
    if (!S.kty_valid) {
      local_spmv<BS>(KT, pick(B.Y, S.parity), B.KTy);
      __syncthreads();
      if (threadIdx.x == 0) {
        S.kty_valid = 1;
        S.spmv_KT += 1;
      }
      __syncthreads();
    }
    batch_kkt<BS>(S, B, 2);
  }
  if (threadIdx.x == 0) D.out_state[mb] = S;
}

// x = D2 x~, y = D1 y~ of every member's returned point into packed outputs.
__global__ __launch_bounds__(kBlock) void k_batch_output(BatchDev D, double* xo, double* yo) {
  constexpr int BS = kBlock;
  const BatchInst I = D.inst[blockIdx.x];
  const Bufs B = batch_bufs(D, I);
  const DevState& S = D.out_state[blockIdx.x];
  const bool avg = S.out_avg != 0;
  const double* xs = avg ? B.XB : pick(B.X, S.parity);
  const double* ys = avg ? B.YB : pick(B.Y, S.parity);
  PDLP_BLOCK_LOOP(j, I.n) xo[I.xo + j] = B.D2[j] * xs[j];
  PDLP_BLOCK_LOOP(i, I.m) yo[I.yo + i] = B.D1[i] * ys[i];
}

}  // namespace pdlp
