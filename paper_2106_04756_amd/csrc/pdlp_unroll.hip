// Unrolled PDHG and its adjoint: a fixed number T of steps of Eq. (3) with frozen step size
// eta, primal weight omega and preconditioners D1, D2, no restarts and no rejections, and the
// reverse-mode pass that gives d loss / d(c, q) from d loss / d(x_T, y_T).
//
// Forward step t maps (x_t, y_t) to
//     x_{t+1} = proj_[l,u](x_t - tau (c~ - K~^T y_t))                 tau   = eta / omega
//     y_{t+1} = proj_Y(y_t + sigma (q~ - 2 K~ x_{t+1} + K~ x_t))       sigma = eta * omega
// with K~ x_t carried from the previous step, so each step is one K~^T product fused with the
// primal update and one K~ product fused with the dual update.  Each step also records one
// byte per coordinate: whether the projection passes derivatives (1 strictly inside [l, u];
// on ">=" rows 1 where y_{t+1} > 0; equality rows always 1).
//
// The adjoint of step t, with xb, yb the adjoints of x_{t+1}, y_{t+1}, vb = mask_y * yb:
//     g   = K~^T vb
//     ub  = mask_x * (xb - 2 sigma g)        cb -= tau ub
//     xb <- ub + sigma g                     (adjoint of x_t)
//     yb <- vb + tau K~ ub                   (adjoint of y_t)     qb += sigma vb
// which is again one K~^T product (of vb) and one K~ product (of ub) per step, each fused with
// its elementwise update; the K~ kernel applies the mask of y_t at once and stores vb for
// the next (earlier) step.
#pragma once

#include "pdlp_device.h"
#include "pdlp_internal.h"

namespace pdlp {

// x' = proj_[l,u](x - tau (c - K^T y)) in place, mask byte of x'.
struct UFwdPrimal {
  static constexpr int N = 1;
  const double* __restrict__ c;
  const double* __restrict__ l;
  const double* __restrict__ u;
  double* __restrict__ x;
  uint8_t* __restrict__ mx;
  double tau;
  __device__ __forceinline__ void row(int j, double s, double (&out)[1]) const {
    const double lj = l[j], uj = u[j];
    const double g = c[j] - s;
    double xp = x[j] - tau * g;
    xp = fmin(fmax(xp, lj), uj);
    x[j] = xp;
    mx[j] = (xp > lj && xp < uj) ? 1 : 0;
    out[0] = 0.0;
  }
};

// y' = proj_Y(y + sigma (q - (2 K x' - K x))) in place, K x <- K x', mask byte of y'.
struct UFwdDual {
  static constexpr int N = 1;
  const double* __restrict__ q;
  double* __restrict__ y;
  double* __restrict__ kx;
  uint8_t* __restrict__ my;
  double sigma;
  int m1;
  __device__ __forceinline__ void row(int i, double s, double (&out)[1]) const {
    double v = y[i] + sigma * (q[i] - (2.0 * s - kx[i]));
    uint8_t pass = 1;
    if (i < m1) {
      v = fmax(v, 0.0);
      pass = v > 0.0 ? 1 : 0;
    }
    y[i] = v;
    kx[i] = s;
    my[i] = pass;
    out[0] = 0.0;
  }
};

// Adjoint of the primal update: s = (K~^T vb)_j.
struct UBwdPrimal {
  static constexpr int N = 1;
  const uint8_t* __restrict__ mx;
  double* __restrict__ xb;
  double* __restrict__ ub;
  double* __restrict__ cb;
  double tau, sigma;
  __device__ __forceinline__ void row(int j, double s, double (&out)[1]) const {
    const double u = mx[j] ? (xb[j] - 2.0 * sigma * s) : 0.0;
    ub[j] = u;
    cb[j] = cb[j] - tau * u;
    xb[j] = u + sigma * s;
    out[0] = 0.0;
  }
};

// Adjoint of the dual update: s = (K~ ub)_i.  qb += sigma vb, then vb <- mask(y_t) * yb_t,
// the mask read from the recorded bytes (my_prev), or from y_t itself at a segment start
// (y_prev, a checkpoint), or not applied (t = 0: that adjoint is not used).
struct UBwdDual {
  static constexpr int N = 1;
  double* __restrict__ vb;
  double* __restrict__ qb;
  const uint8_t* __restrict__ my_prev;
  const double* __restrict__ y_prev;
  double tau, sigma;
  int m1;
  __device__ __forceinline__ void row(int i, double s, double (&out)[1]) const {
    const double v = vb[i];
    qb[i] = qb[i] + sigma * v;
    const double yb = v + tau * s;
    bool pass = true;
    if (i < m1) {
      if (my_prev) pass = my_prev[i] != 0;
      else if (y_prev) pass = y_prev[i] > 0.0;
    }
    vb[i] = pass ? yb : 0.0;
    out[0] = 0.0;
  }
};

template <class Epi>
__global__ __launch_bounds__(kBlock) void k_unroll_rows(CsrDev A, const double* in, Epi epi) {
  double acc[1] = {0.0};
  csr_rows<kProd>(A, in, epi, acc, nullptr);
}

template <class Epi>
__global__ __launch_bounds__(kBlock) void k_unroll_combine(CsrDev A, const double* part, Epi epi) {
  double acc[1] = {0.0};
  combine_rows<kProd>(A, part, nullptr, epi, acc);
}

// c~ = D2 c, q~ = D1 q (frozen preconditioners); x0 = proj_[l,u](0), y0 = 0.
__global__ __launch_bounds__(kBlock) void k_unroll_start(const double* c_in, const double* q_in,
                                                         const double* D1, const double* D2,
                                                         const double* l, const double* u,
                                                         double* ct, double* qt, double* x, double* y,
                                                         int n, int m) {
  for (int64_t idx = blockIdx.x * int64_t(kBlock) + threadIdx.x; idx < int64_t(n) + m;
       idx += int64_t(gridDim.x) * kBlock) {
    if (idx < n) {
      const int j = int(idx);
      ct[j] = D2[j] * c_in[j];
      x[j] = fmin(fmax(0.0, l[j]), u[j]);
    } else {
      const int i = int(idx - n);
      qt[i] = D1[i] * q_in[i];
      y[i] = 0.0;
    }
  }
}

// dst[k] = src[k] for k < len (checkpoint store and restore).
__global__ __launch_bounds__(kBlock) void k_unroll_copy(const double* __restrict__ src,
                                                        double* __restrict__ dst, int64_t len) {
  for (int64_t k = blockIdx.x * int64_t(kBlock) + threadIdx.x; k < len; k += int64_t(gridDim.x) * kBlock)
    dst[k] = src[k];
}

// Adjoint seeds: xb = D2 gx (d loss / d x~_T), vb = mask(y_T) D1 gy; cb = qb = 0.
// gx or gy may be null (zero).
__global__ __launch_bounds__(kBlock) void k_unroll_seed(const double* gx, const double* gy,
                                                        const double* D1, const double* D2,
                                                        const uint8_t* my_T, double* xb, double* vb,
                                                        double* cb, double* qb, int n, int m, int m1) {
  for (int64_t idx = blockIdx.x * int64_t(kBlock) + threadIdx.x; idx < int64_t(n) + m;
       idx += int64_t(gridDim.x) * kBlock) {
    if (idx < n) {
      const int j = int(idx);
      xb[j] = gx ? D2[j] * gx[j] : 0.0;
      cb[j] = 0.0;
    } else {
      const int i = int(idx - n);
      const bool pass = (i >= m1) || my_T[i] != 0;
      vb[i] = (gy && pass) ? D1[i] * gy[i] : 0.0;
      qb[i] = 0.0;
    }
  }
}

// out = D * v (back to the user's units: x = D2 x~, y = D1 y~, dc = D2 dc~, dq = D1 dq~).
__global__ __launch_bounds__(kBlock) void k_unroll_unscale(const double* a, const double* Da, int na,
                                                           const double* b, const double* Db, int nb,
                                                           double* out) {
  for (int64_t idx = blockIdx.x * int64_t(kBlock) + threadIdx.x; idx < int64_t(na) + nb;
       idx += int64_t(gridDim.x) * kBlock) {
    if (idx < na) out[idx] = Da[idx] * a[idx];
    else out[idx] = Db[idx - na] * b[idx - na];
  }
}

}  // namespace pdlp
