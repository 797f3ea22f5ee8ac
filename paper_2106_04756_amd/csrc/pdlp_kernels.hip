// gfx950 kernels of the PDLP solver (float64 throughout).
//
// Work layout
//  * Both K~ and its transpose are stored in CSR (int64 row offsets, int32 columns, float64
//    values).  Every product is a gather over one CSR copy; no value atomics anywhere.
//  * A host-built schedule cuts the rows of each copy into descriptors: runs of short rows
//    whose nonzeros (<= 2048) are staged through LDS and reduced by 2^p lanes per row, single
//    rows reduced by a whole workgroup, and chunks of giant rows whose partial sums are
//    combined, in chunk order, by the last chunk to arrive.  Workgroups walk the descriptor
//    list with a fixed grid stride, so every sum has a fixed order and two runs are bitwise equal.
//  * Each product carries its per-row epilogue (the PDHG primal or dual update, a norm, a
//    store) so vectors are touched once per product.
//  * Reductions: per-thread registers -> wave64 butterflies -> LDS across the 4 waves ->
//    one partial per workgroup -> the last workgroup to arrive (agent-scope ticket) adds the
//    partials in slot order and applies the scalar logic (step-size rule, restart tests).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/pdlp.h"
#include "pdlp_device.h"

namespace pdlp {

// ------------------------------------------------------------------------------------------
// small device helpers
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True in every thread of the workgroup that arrives last at `ticket` (of `total`).
// Writes made before the call by any workgroup are visible to the last one after it.
__device__ bool arrive_last(unsigned* ticket, unsigned total) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev + 1u == total) ? 1 : 0;
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

__device__ __forceinline__ void reset_ticket(unsigned* ticket) {
  if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum of N per-thread values over the workgroup; the result is valid in thread 0.
template <int N>
__device__ void block_sum(double (&a)[N]) {
  __shared__ double lds[4 * (N > 0 ? N : 1)];
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
    for (int k = 0; k < N; ++k) a[k] = ((lds[k] + lds[N + k]) + lds[2 * N + k]) + lds[3 * N + k];
  }
  __syncthreads();
}

__device__ double block_max(double v) {
  __shared__ double lds[4];
  v = wave_max(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) v = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
  __syncthreads();
  return v;
}

// Sum over `nslot` partial slots of N values each (slot-major), value k in a[k] of thread 0.
// Slots are plain memory: they are read after a kernel boundary (k_tail) or after the acquire
// fence of arrive_last, which pairs with the release fence every writer passed.  Thread t adds
// slots t, t + kBlock, ... in that order, the loads of Q slots (8 values) issued before their
// adds (one slot at a time, the chain of loads set the time of the one-workgroup tail
// kernels); then the workgroup's sums are added in a fixed order.  Many values per slot:
// sum_slots_shared.
template <int N>
__device__ void sum_slots(const double* part, int nslot, double (&a)[N]) {
  static_assert(N < 8, "use sum_slots_shared");
  constexpr int Q = 8 / N;
#pragma unroll
  for (int k = 0; k < N; ++k) a[k] = 0.0;
  for (int sl0 = threadIdx.x; sl0 < nslot; sl0 += Q * kBlock) {
    double v[Q][N];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int sl = sl0 + q * kBlock;
#pragma unroll
      for (int k = 0; k < N; ++k) v[q][k] = sl < nslot ? part[size_t(sl) * N + k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (sl0 + q * kBlock < nslot) {
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] += v[q][k];
      }
    }
  }
  block_sum<N>(a);
}

// Sum over `nslot` slots of N >= 8 values each (N dividing the workgroup size): thread t sums
// value k = t mod N of every (kBlock / N)-th slot, so each pass over the slots is one
// contiguous read, with eight interleaved partial sums keeping eight loads in flight; then
// threads 0 .. N - 1 add the kBlock / N partial sums of their k in a fixed order into out[k] in
// LDS, visible to the whole workgroup on return (no thread holds all N in registers).
template <int N>
__device__ void sum_slots_shared(const double* part, int nslot, double* out) {
  static_assert(N >= 8 && kBlock % N == 0, "N must divide the workgroup size");
  constexpr int G = kBlock / N;
  __shared__ double lds[kBlock];
  const int k = threadIdx.x % N, g = threadIdx.x / N;
  double u8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int sl = g;
  for (; sl + 7 * G < nslot; sl += 8 * G) {
#pragma unroll
    for (int q = 0; q < 8; ++q) u8[q] += part[size_t(sl + q * G) * N + k];
  }
  for (int q = 0; sl < nslot; sl += G, ++q) u8[q] += part[size_t(sl) * N + k];
  const double t = ((u8[0] + u8[1]) + (u8[2] + u8[3])) + ((u8[4] + u8[5]) + (u8[6] + u8[7]));
  __syncthreads();
  lds[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x < N) {
    double u = 0.0;
    for (int gg = 0; gg < G; ++gg) u += lds[gg * N + threadIdx.x];
    out[threadIdx.x] = u;
  }
  __syncthreads();
}

template <int N>
__device__ __forceinline__ void write_slot(double* part, int slot, const double (&a)[N]) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) part[size_t(slot) * N + k] = a[k];
  }
}

// ------------------------------------------------------------------------------------------
// CSR row reductions driven by the schedule
// ------------------------------------------------------------------------------------------

enum ElemMode { kProd = 0, kAbsMax = 1, kAbsSum = 2 };

template <int MODE>
__device__ __forceinline__ double comb(double a, double b) {
  if constexpr (MODE == kAbsMax) return fmax(a, b);
  else return a + b;
}

template <int MODE>
__device__ __forceinline__ double block_comb(double v) {
  if constexpr (MODE == kAbsMax) return block_max(v);
  double a[1] = {v};
  block_sum<1>(a);
  return a[0];
}

// Reduction of one contiguous nonzero range [p0, p1) by the whole workgroup, result in thread 0.
template <int MODE>
__device__ double range_reduce(const CsrDev& A, const double* __restrict__ x, int64_t p0, int64_t p1) {
  double s = 0.0;
  int64_t e = p0 + threadIdx.x;
  for (; e + 3 * kBlock < p1; e += 4 * kBlock) {
    double v0 = A.v[e], v1 = A.v[e + kBlock], v2 = A.v[e + 2 * kBlock], v3 = A.v[e + 3 * kBlock];
    if constexpr (MODE == kProd) {
      const int32_t c0 = A.ci[e], c1 = A.ci[e + kBlock], c2 = A.ci[e + 2 * kBlock], c3 = A.ci[e + 3 * kBlock];
      v0 *= x[c0];
      v1 *= x[c1];
      v2 *= x[c2];
      v3 *= x[c3];
    } else {
      v0 = fabs(v0); v1 = fabs(v1); v2 = fabs(v2); v3 = fabs(v3);
    }
    s = comb<MODE>(comb<MODE>(comb<MODE>(comb<MODE>(s, v0), v1), v2), v3);
  }
  for (; e < p1; e += kBlock) {
    double v = A.v[e];
    if constexpr (MODE == kProd) v *= x[A.ci[e]];
    else v = fabs(v);
    s = comb<MODE>(s, v);
  }
  return block_comb<MODE>(s);
}

// Task range of this workgroup: panel p and the workgroup's index and count among those of p.
// The grid holds npanel / nsub groups (the workgroup's XCD when there are 8) and nsub runs of
// nb workgroups per group: workgroup b belongs to group g = b mod groups, takes run
// q = (b / groups) / nb of that group, and works on panel g nsub + q.  Workgroups start in
// the order of their index, so a group's sub-panels are taken one after another.
struct PanelSlice {
  int p, lb, nb;
};
__device__ __forceinline__ PanelSlice panel_slice(const CsrDev& A) {
  PanelSlice ps;
  const int S = A.nsub > 1 ? A.nsub : 1;
  const int ng = A.npanel / S;
  const int rest = int(blockIdx.x) / ng;
  ps.nb = int(gridDim.x) / A.npanel;
  ps.p = (int(blockIdx.x) % ng) * S + rest / ps.nb;
  ps.lb = rest % ps.nb;
  return ps;
}

// Long rows (kVector) and chunks of giant rows (kSplit), one workgroup each.
template <int MODE, class Epi>
__device__ __forceinline__ void csr_block_tasks(const CsrDev& A, const double* __restrict__ x,
                                                const Epi& epi, double (&acc)[Epi::N], double* part) {
  const PanelSlice ps = panel_slice(A);
  const int d1 = A.block_begin[ps.p + 1];
  for (int d = A.block_begin[ps.p] + ps.lb; d < d1; d += ps.nb) {
    const RowDesc D = A.block[d];
    const int kind = D.kind_l & 0xff;
    const int r = D.a;
    if (kind == kVector) {
      const double s = range_reduce<MODE>(A, x, A.rp[r], A.rp[r + 1]);
      if (threadIdx.x == 0) {
        double c[Epi::N];
        epi.row(r, s, c);
#pragma unroll
        for (int k = 0; k < Epi::N; ++k) acc[k] += c[k];
      }
    } else {
      const int ch = D.b, sid = D.aux;
      const int64_t q0 = A.rp[r] + int64_t(ch) * kChunk;
      const int64_t q1 = min(A.rp[r + 1], q0 + int64_t(kChunk));
      const double s = range_reduce<MODE>(A, x, q0, q1);
      const int base = A.split_base[sid], nch = A.split_nchunks[sid];
      if (threadIdx.x == 0) st_agent(&A.split_part[base + ch], s);
      if (arrive_last(&A.split_cnt[sid], unsigned(nch))) {
        double t = 0.0;
        for (int c = threadIdx.x; c < nch; c += kBlock) t = comb<MODE>(t, ld_agent(&A.split_part[base + c]));
        t = block_comb<MODE>(t);
        if (threadIdx.x == 0) {
          __hip_atomic_store(&A.split_cnt[sid], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          double c[Epi::N];
          epi.row(r, t, c);
          if (part) {
#pragma unroll
            for (int k = 0; k < Epi::N; ++k) st_agent(&part[size_t(gridDim.x + sid) * Epi::N + k], c[k]);
          }
        }
      }
    }
  }
}

// Sources of the gathered operand of a product: device memory, or the LDS stage of a panel
// (its columns c0 .. c0 + h, h >= 1) with device memory for the rest.  Every lane reads the
// stage at its column clamped into it; only lanes whose column lies outside read device
// memory, behind a branch, so served lanes send no request to the caches.
struct GlobalGather {
  const double* __restrict__ x;
};
struct LdsGather {
  const double* stage;
  const double* __restrict__ x;
  int32_t c0;
  uint32_t h;
};
// A slice wholly in LDS, addressed by columns relative to the slice.
struct StageGather {
  const double* stage;
};
template <int E>
__device__ __forceinline__ void gather_all(const StageGather& g, const int32_t (&c)[E], double (&xv)[E]) {
#pragma unroll
  for (int k = 0; k < E; ++k) xv[k] = g.stage[c[k]];
}
template <int E>
__device__ __forceinline__ void gather_all(const GlobalGather& g, const int32_t (&c)[E], double (&xv)[E]) {
#pragma unroll
  for (int k = 0; k < E; ++k) xv[k] = g.x[c[k]];
}
template <int E>
__device__ __forceinline__ void gather_all(const LdsGather& g, const int32_t (&c)[E], double (&xv)[E]) {
  bool far = false;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const uint32_t d = uint32_t(c[k] - g.c0);
    far = far || d >= g.h;
    xv[k] = g.stage[d < g.h ? d : g.h - 1];
  }
  if (far) {
#pragma unroll
    for (int k = 0; k < E; ++k)
      if (uint32_t(c[k] - g.c0) >= g.h) xv[k] = g.x[c[k]];
  }
}

// The interleaved matrix entries are read once per product.  Non-temporal loads mark their
// lines for early eviction, so that the L2 keeps the lines of the gathered vector between
// their uses (on the K~ product of the large LP: 11% less HBM traffic, the K~^T pass 7% faster).
template <class T>
__device__ __forceinline__ T ld_entry(const T* p) {
  return __builtin_nontemporal_load(p);
}

// One wavefront task: rows perm[D.a .. D.a + D.b) (panel rows D.a .. in panel mode), each by a
// group of L = 2^p lanes, E entries per lane (E L >= every row length of the task), read from
// the task's interleaved entries at `off` (each of the E loads covers 64 consecutive slots).
// R rounds of rows at a time: all their loads, then all their gathers, are in flight
// together.  Entries past a row end are masked to +0.0, which leaves each row's sum
// bit-identical for any E and R; rows reach the epilogue in task order for any R.
// LOCAL: columns from the 16-bit slice-relative copy (slices, gathered from the stage).
template <int MODE, int E, int R, bool LOCAL, class Epi, class G>
__device__ __forceinline__ void wave_task(const CsrDev& A, const G& x, const Epi& epi,
                                          double (&acc)[Epi::N], const RowDesc& D, int64_t off, int lane64) {
  const int lg = D.kind_l >> 8, L = 1 << lg;
  const int g = lane64 >> lg, lane = lane64 & (L - 1);
  const int per_round = 64 >> lg;
  int64_t blk = off + lane64;
  if constexpr (R == 1) {
    // one round at a time (fewer live registers than the general form below)
    for (int base = 0; base < D.b; base += per_round, blk += int64_t(64) * E) {
      const int slot = base + g;
      const bool active = slot < D.b;
      int r = 0;
      double s = 0.0;
      if (active) {
        // the entry loads stay inside the task's slots, so they are issued together with the
        // row length; the gathers wait for it (an empty row, e.g. of a copy with no columns,
        // gathers nothing)
        r = A.perm ? A.perm[D.a + slot] : D.a + slot;
        const int len = A.rlen[r];
        double v[E];
        int32_t c[E];
#pragma unroll
        for (int k = 0; k < E; ++k) {
          v[k] = ld_entry(&A.vs[blk + int64_t(k) * 64]);
          if constexpr (MODE == kProd) {
            if constexpr (LOCAL) c[k] = ld_entry(&A.cis16[blk + int64_t(k) * 64]);
            else c[k] = ld_entry(&A.cis[blk + int64_t(k) * 64]);
          }
        }
        if constexpr (MODE == kProd) {
          if (len > 0) {
            double xv[E];
            gather_all<E>(x, c, xv);
#pragma unroll
            for (int k = 0; k < E; ++k) {
              const double t = v[k] * xv[k];
              s = s + ((k * L + lane < len) ? t : 0.0);
            }
          }
        } else {
#pragma unroll
          for (int k = 0; k < E; ++k) s = comb<MODE>(s, (k * L + lane < len) ? fabs(v[k]) : 0.0);
        }
      }
      for (int o = L >> 1; o > 0; o >>= 1) s = comb<MODE>(s, __shfl_xor(s, o, 64));
      if (active && lane == 0) {
        double cc[Epi::N];
        epi.row(r, s, cc);
#pragma unroll
        for (int k = 0; k < Epi::N; ++k) acc[k] += cc[k];
      }
    }
    return;
  }
  for (int base = 0; base < D.b; base += R * per_round, blk += int64_t(R) * 64 * E) {
    int r[R];
    int64_t len[R];
    bool active[R];
    double v[R][E];
    int32_t c[R][E];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int slot = base + q * per_round + g;
      active[q] = slot < D.b;
      r[q] = 0;
      len[q] = 0;
      if (active[q]) {
        r[q] = A.perm ? A.perm[D.a + slot] : D.a + slot;
        len[q] = A.rlen[r[q]];
#pragma unroll
        for (int k = 0; k < E; ++k) {
          v[q][k] = ld_entry(&A.vs[blk + int64_t(q * E + k) * 64]);
          if constexpr (MODE == kProd) {
            if constexpr (LOCAL) c[q][k] = ld_entry(&A.cis16[blk + int64_t(q * E + k) * 64]);
            else c[q][k] = ld_entry(&A.cis[blk + int64_t(q * E + k) * 64]);
          }
        }
      }
    }
    double s[R];
    if constexpr (MODE == kProd) {
      double xv[R][E];
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (active[q] && len[q] > 0) gather_all<E>(x, c[q], xv[q]);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        s[q] = 0.0;
        if (active[q] && len[q] > 0) {
#pragma unroll
          for (int k = 0; k < E; ++k) {
            const double t = v[q][k] * xv[q][k];
            s[q] = s[q] + ((k * L + lane < len[q]) ? t : 0.0);
          }
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        s[q] = 0.0;
        if (active[q]) {
#pragma unroll
          for (int k = 0; k < E; ++k) s[q] = comb<MODE>(s[q], (k * L + lane < len[q]) ? fabs(v[q][k]) : 0.0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      for (int o = L >> 1; o > 0; o >>= 1) s[q] = comb<MODE>(s[q], __shfl_xor(s[q], o, 64));
      if (active[q] && lane == 0) {
        double cc[Epi::N];
        epi.row(r[q], s[q], cc);
#pragma unroll
        for (int k = 0; k < Epi::N; ++k) acc[k] += cc[k];
      }
    }
  }
}

// wave_task with the entries per lane of the task (uniform across the wavefront).
// R: rounds in flight for tasks of 1 or 2 entries per lane (at most 2 from 3 entries, 1 from 5).
// EMAX: the most entries per lane the layout's tasks have (kElemsPerLane or kElemsPerLaneLds).
template <int MODE, int R = 1, bool LOCAL = false, int EMAX = kElemsPerLane, class Epi, class G>
__device__ __forceinline__ void wave_task_e(const CsrDev& A, const G& x, const Epi& epi,
                                            double (&acc)[Epi::N], int t, int lane64) {
  const RowDesc D = A.wave[t];
  const int64_t off = A.task_off[t];
  switch (D.aux) {
    case 1: wave_task<MODE, 1, R, LOCAL>(A, x, epi, acc, D, off, lane64); break;
    case 2: wave_task<MODE, 2, R, LOCAL>(A, x, epi, acc, D, off, lane64); break;
    // at most two rounds at a time from 3 entries per lane
    case 3: wave_task<MODE, 3, (R > 2 ? 2 : R), LOCAL>(A, x, epi, acc, D, off, lane64); break;
    case 4: wave_task<MODE, 4, (R > 2 ? 2 : R), LOCAL>(A, x, epi, acc, D, off, lane64); break;
    // one round at a time above 4 entries per lane (two would exceed the registers)
    case 5: wave_task<MODE, 5, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
    case 6: wave_task<MODE, 6, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
    case 7: wave_task<MODE, 7, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
    case 8: wave_task<MODE, 8, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
    default:
      if constexpr (EMAX > 8) {
        switch (D.aux) {
          case 9: wave_task<MODE, 9, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
          case 10: wave_task<MODE, 10, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
          case 11: wave_task<MODE, 11, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
          case 12: wave_task<MODE, 12, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
          case 13: wave_task<MODE, 13, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
          case 14: wave_task<MODE, 14, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
          case 15: wave_task<MODE, 15, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
          default: wave_task<MODE, 16, 1, LOCAL>(A, x, epi, acc, D, off, lane64); break;
        }
      }
      break;
  }
}

// Visit every row of A once: row value s = sum_j A_rj x_j (kProd) or max/sum |A_rj|, and
// call epi.row(r, s, contrib).  Rows up to kWaveMaxLen long are handled by wavefronts on
// their own (no LDS, no workgroup barrier): a group of L = 2^p lanes per row, each lane
// loading at most kElemsPerLane nonzeros at once, then an xor-butterfly across the group.
// Contributions of ordinary rows go to acc (per thread); those of split rows go straight to
// partial slot gridDim.x + split id (if part != nullptr).
template <int MODE, int EMAX = kElemsPerLane, class Epi>
__device__ void csr_rows(const CsrDev& A, const double* __restrict__ x, const Epi& epi,
                         double (&acc)[Epi::N], double* part) {
  const int lane64 = threadIdx.x & 63;
  const PanelSlice ps = panel_slice(A);
  const int nw = ps.nb * kWaves;
  const int t1 = A.wave_begin[ps.p + 1];
  const int w0 = __builtin_amdgcn_readfirstlane(A.wave_begin[ps.p] + ps.lb * kWaves + (threadIdx.x >> 6));
  const GlobalGather gx{x};
  for (int t = w0; t < t1; t += nw) wave_task_e<MODE, 1, false, EMAX>(A, gx, epi, acc, t, lane64);
  csr_block_tasks<MODE>(A, x, epi, acc, part);
}

// Same visit with the row values read from `stored` instead of recomputed.
template <class Epi>
__device__ void csr_rows_stored(const CsrDev& A, const double* __restrict__ stored, const Epi& epi,
                                double (&acc)[Epi::N], double* part) {
  const int nw = gridDim.x * kWaves;
  const int lane64 = threadIdx.x & 63;
  double c[Epi::N];
  for (int t = blockIdx.x * kWaves + (threadIdx.x >> 6); t < A.nwave; t += nw) {
    const RowDesc D = A.wave[t];
    for (int slot = lane64; slot < D.b; slot += 64) {
      const int r = A.perm ? A.perm[D.a + slot] : D.a + slot;
      epi.row(r, stored[r], c);
#pragma unroll
      for (int k = 0; k < Epi::N; ++k) acc[k] += c[k];
    }
  }
  for (int d = blockIdx.x; d < A.nblock; d += gridDim.x) {
    const RowDesc D = A.block[d];
    const int kind = D.kind_l & 0xff;
    if (threadIdx.x != 0) continue;
    if (kind == kVector) {
      epi.row(D.a, stored[D.a], c);
#pragma unroll
      for (int k = 0; k < Epi::N; ++k) acc[k] += c[k];
    } else if (D.b == 0) {
      epi.row(D.a, stored[D.a], c);
      if (part) {
#pragma unroll
        for (int k = 0; k < Epi::N; ++k) st_agent(&part[size_t(gridDim.x + D.aux) * Epi::N + k], c[k]);
      }
    }
  }
}

// Visit every nonzero of A with its (row, column): f(e, r, col).
// (In panel mode the row passed to f is the original row of the panel row.)
template <class F>
__device__ void csr_elements(const CsrDev& A, F f) {
  const int nw = gridDim.x * kWaves;
  const int lane64 = threadIdx.x & 63;
  for (int t = blockIdx.x * kWaves + (threadIdx.x >> 6); t < A.nwave; t += nw) {
    const RowDesc D = A.wave[t];
    const int lg = D.kind_l >> 8, L = 1 << lg;
    const int g = lane64 >> lg, lane = lane64 & (L - 1);
    const int per_round = 64 >> lg;
    for (int base = 0; base < D.b; base += per_round) {
      const int slot = base + g;
      if (slot < D.b) {
        const int k = A.perm ? A.perm[D.a + slot] : D.a + slot;
        const int r = A.prow_row ? A.prow_row[k] : k;
        for (int64_t e = A.rp[k] + lane; e < A.rp[k + 1]; e += L) f(e, r, A.ci[e]);
      }
    }
  }
  for (int d = blockIdx.x; d < A.nblock; d += gridDim.x) {
    const RowDesc D = A.block[d];
    const int kind = D.kind_l & 0xff;
    const int k = D.a;
    const int r = A.prow_row ? A.prow_row[k] : k;
    int64_t q0 = A.rp[k], q1 = A.rp[k + 1];
    if (kind == kSplit) {
      q0 += int64_t(D.b) * kChunk;
      q1 = min(q1, q0 + int64_t(kChunk));
    }
    for (int64_t e = q0 + threadIdx.x; e < q1; e += kBlock) f(e, r, A.ci[e]);
  }
}

// Panel mode, second pass: the value of original row r is the sum (or max) of its panel
// rows' partial values, taken in panel order; then epi.row(r, s, contrib).
template <int MODE, class Epi>
__device__ void combine_rows(const CsrDev& A, const double* __restrict__ part,
                             const double* __restrict__ stored, const Epi& epi, double (&acc)[Epi::N]) {
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < A.nrows_orig; r += gridDim.x * kBlock) {
    double s = 0.0;
    if (stored) {
      s = stored[r];
    } else {
      // eight partial values at a time: indices clamped into the row, all loads in flight
      // together, then added in slot order; the padding adds +0.0, which leaves s unchanged
      // (s starts at +0.0, so it is never -0.0; the partial values of max are >= 0)
      const int64_t j1 = A.slot_ptr[r + 1];
      for (int64_t j = A.slot_ptr[r]; j < j1; j += 8) {
        int32_t k[8];
        double p[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) k[q] = A.slot_idx[j + q < j1 ? j + q : j1 - 1];
#pragma unroll
        for (int q = 0; q < 8; ++q) p[q] = part[k[q]];
#pragma unroll
        for (int q = 0; q < 8; ++q) s = comb<MODE>(s, j + q < j1 ? p[q] : 0.0);
      }
    }
    double c[Epi::N];
    epi.row(r, s, c);
#pragma unroll
    for (int k = 0; k < Epi::N; ++k) acc[k] += c[k];
  }
}

// Parity-selected buffer without a runtime array index (keeps a local Bufs out of scratch).
__device__ __forceinline__ double* pick(double* const (&a)[2], int P) { return P ? a[1] : a[0]; }

// ------------------------------------------------------------------------------------------
// predicates on the device state
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ bool attempt_runs(const DevState& S) {
  return !S.done && !S.check_pending && S.k < S.iter_limit;
}
// The primal step of an attempt runs unless the attempt retries a Malitsky-Pock dual trial.
__device__ __forceinline__ bool primal_runs(const DevState& S) {
  return attempt_runs(S) && !(S.mp_on && S.mp_stage);
}
__device__ __forceinline__ bool check_runs(const DevState& S) {
  return !S.done && S.check_pending;
}
__device__ bool pred_ok(const DevState& S, int pred) {
  switch (pred) {
    case kPredAlways: return true;
    case kPredCheck: return check_runs(S);
    case kPredCheckKty: return check_runs(S) && !S.kty_valid;
    case kPredKty: return !S.kty_valid;
    case kPredCheckRestart: return check_runs(S) && S.restart;
    case kPredAttempt: return attempt_runs(S);
    case kPredAttemptKty: return primal_runs(S) && !S.kty_valid;
    case kPredMpNew: return primal_runs(S);
    case kPredKtyPeek: return !S.kty_valid;
    default: return false;
  }
}

// ------------------------------------------------------------------------------------------
// the PDHG attempt (Algorithm 2): primal step fused with K~^T y, dual step fused with K~ x'
// ------------------------------------------------------------------------------------------

// x' = proj_[l,u](x - (eta/omega)(c - K^T y))   (Eq. (3), first line)
struct PrimalEpi {
  static constexpr int N = 1;
  const double* __restrict__ c;
  const double* __restrict__ l;
  const double* __restrict__ u;
  const double* __restrict__ x;
  double* __restrict__ xn;
  double* __restrict__ sx;
  double* __restrict__ kty;
  double tau, w;
  int store_kty;
  __device__ __forceinline__ void row(int j, double s, double (&out)[1]) const {
    if (store_kty) kty[j] = s;
    const double xj = x[j];
    if (w != 0.0) sx[j] = sx[j] + w * xj;          // eta-weighted sum of the last accepted iterate
    const double g = c[j] - s;
    double xp = xj - tau * g;
    xp = fmin(fmax(xp, l[j]), u[j]);
    xn[j] = xp;
    const double d = xp - xj;
    out[0] = d * d;
  }
};

// y' = proj_Y(y + eta*omega (q - 2 K x' + K x))   (Eq. (3), second line, with K x cached)
struct DualEpi {
  static constexpr int N = 2;
  const double* __restrict__ q;
  const double* __restrict__ y;
  const double* __restrict__ kx;
  double* __restrict__ yn;
  double* __restrict__ kxn;
  double* __restrict__ sy;
  double sigma, w;
  int m1;
  __device__ __forceinline__ void row(int i, double s, double (&out)[2]) const {
    const double yi = y[i];
    const double kxi = kx[i];
    if (w != 0.0) sy[i] = sy[i] + w * yi;
    double v = yi + sigma * (q[i] - (2.0 * s - kxi));
    if (i < m1) v = fmax(v, 0.0);
    yn[i] = v;
    kxn[i] = s;
    const double dy = v - yi;
    out[0] = dy * dy;
    out[1] = dy * (s - kxi);
  }
};

// "No restart" mode (restarts off; Appendix C): the primal weight is still updated when an
// artificial restart would have fired, i.e. at k = 2, 4, 8, ...  Such a k gets a check of its
// own, which only updates the weight and moves the anchor.
__device__ __forceinline__ void mark_weight_event(DevState& W) {
  if (W.pw_pow2 && W.k >= 2 && (W.k & (W.k - 1)) == 0) {
    W.check_pending = 1;
    W.pw_event = 1;
  }
}

// Algorithm 2 decision for one attempt: the largest step Eq. (5) allows, the next proposal,
// accept or retry, and the bookkeeping of Algorithm 1.  One thread.
__device__ void attempt_decide(DevState& W, double dx2, double dy2, double cross, pdlp_attempt_rec* att) {
  const int P = W.parity;
  const double eta = W.eta, omega = W.omega;
  const double num = omega * dx2 + dy2 / omega;
  const double den = 2.0 * fabs(cross);
  double eta_bar = (den > 0.0) ? num / den : INFINITY;
  const double k2 = double(W.k + 2);   // (k + 1) with a 1-based step counter
  double eta_next = fmin((1.0 - pow(k2, -0.3)) * eta_bar, (1.0 + pow(k2, -0.6)) * eta);
  if (W.constant_step) {               // baseline PDHG: a fixed step, always accepted
    eta_bar = INFINITY;
    eta_next = eta;
  }
  const bool ok = isfinite(dx2) && isfinite(dy2) && isfinite(cross) && isfinite(eta_next);
  const bool accepted = ok && (eta <= eta_bar);
  if (att && W.trace_cap > 0) {
    pdlp_attempt_rec& rec = att[W.n_att_log % W.trace_cap];
    rec.k = W.k;
    rec.eta = eta;
    rec.eta_bar = eta_bar;
    rec.accepted = accepted ? 1 : 0;
    rec.pad = 0;
  }
  W.n_att_log += 1;
  W.attempts += 1;
  W.spmv_K += 1;
  W.w_pending = 0.0;
  if (!ok) {
    W.status = PDLP_NUMERICAL_ERROR;
    W.done = 1;
    return;
  }
  if (accepted) {
    W.parity = P ^ 1;
    W.w_pending = eta;
    W.s_eta += eta;
    W.eta_hat = eta_next;
    W.eta = eta_next;
    W.k += 1;
    W.t += 1;
    W.kty_valid = 0;
    W.retries = 0;
    if (W.k % W.check_every == 0) W.check_pending = 1;
    mark_weight_event(W);
    if (W.k <= W.trace_iters) W.snap_pending = 1;
  } else {
    W.eta = eta_next;
    W.retries += 1;
    W.kty_valid = 1;
    if (W.retries >= W.max_retries) {
      W.status = PDLP_NUMERICAL_ERROR;
      W.done = 1;
    }
  }
}

// Run by the last workgroup of the dual-step kernel.
__device__ void finish_attempt(DevState* st, const Bufs& B, const double* partA, int nslotA,
                               const double* partB, int nslotB) {
  double ax[1], ay[2];
  sum_slots<1>(partA, nslotA, ax);
  sum_slots<2>(partB, nslotB, ay);
  if (threadIdx.x == 0) {
    if (!st->kty_valid) st->spmv_KT += 1;     // the primal step formed K~^T y
    attempt_decide(*st, ax[0], ay[0], ay[1], B.att);
  }
}

// Step of the primal update: the attempt's eta (Algorithm 2, constant step) or, under the
// Malitsky-Pock line search, the step eta_k of the last accepted iteration.
__device__ __forceinline__ double primal_step(const DevState& S) {
  return (S.mp_on ? S.eta_hat : S.eta) / S.omega;
}

__global__ __launch_bounds__(kBlock) void k_primal(CsrDev AT, DevState* st, Bufs B, double* partA) {
  const DevState& S = *st;
  if (!primal_runs(S)) return;
  const int P = S.parity;
  const int kty_valid = S.kty_valid;
  PrimalEpi epi{B.c, B.l, B.u, pick(B.X, P), pick(B.X, P ^ 1), B.Sx, B.KTy, primal_step(S), S.w_pending, !kty_valid};
  double acc[1] = {0.0};
  if (kty_valid) csr_rows_stored(AT, B.KTy, epi, acc, partA);
  else csr_rows<kProd>(AT, pick(B.Y, P), epi, acc, partA);
  block_sum<1>(acc);
  write_slot<1>(partA, blockIdx.x, acc);
}

__global__ __launch_bounds__(kBlock) void k_dual(CsrDev A, DevState* st, Bufs B, const double* partA,
                                                 int nslotA, double* partB, unsigned* ticket) {
  const DevState& S = *st;
  if (!attempt_runs(S)) return;
  const int P = S.parity;
  DualEpi epi{B.q, pick(B.Y, P), pick(B.KX, P), pick(B.Y, P ^ 1), pick(B.KX, P ^ 1), B.Sy, S.eta * S.omega, S.w_pending, B.m1};
  double acc[2] = {0.0, 0.0};
  csr_rows<kProd>(A, pick(B.X, P ^ 1), epi, acc, partB);
  block_sum<2>(acc);
  write_slot<2>(partB, blockIdx.x, acc);
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  finish_attempt(st, B, partA, nslotA, partB, int(gridDim.x) + A.nsplit);
}

// Copy of the accepted iterate for the parity trace.
__global__ __launch_bounds__(kBlock) void k_snapshot(DevState* st, Bufs B, unsigned* ticket) {
  const DevState& S = *st;
  if (!S.snap_pending) return;
  const int P = S.parity;
  const int64_t kk = S.k - 1;
  for (int64_t idx = blockIdx.x * int64_t(kBlock) + threadIdx.x; idx < int64_t(B.n) + B.m;
       idx += int64_t(gridDim.x) * kBlock) {
    if (idx < B.n) B.tx[kk * B.n + idx] = pick(B.X, P)[idx];
    else B.ty[kk * B.m + (idx - B.n)] = pick(B.Y, P)[idx - B.n];
  }
  if (arrive_last(ticket, gridDim.x)) {
    if (threadIdx.x == 0) {
      st->snap_pending = 0;
      st->n_iter_log = S.k;
    }
    reset_ticket(ticket);
  }
}

// ------------------------------------------------------------------------------------------
// Malitsky-Pock line search (Appendix C): x' from the step eta_k of the last iteration, then
// dual trials y^ = proj_Y(y + omega eta^ (q - K~(x' + th (x' - x)))), th = eta_k / eta^,
// accepted when eta^ ||K~^T (y^ - y)|| <= breaking_factor ||y^ - y||, else eta^ is scaled down.
// K~(x' + th (x' - x)) is formed as (1 + th) K~x' - th K~x from the cached K~x.
// ------------------------------------------------------------------------------------------

// First candidate of an iteration from the accepted step eta_k (in W.eta_hat) and theta_k.
__device__ __forceinline__ void mp_first_candidate(DevState& W) {
  W.eta = W.eta_hat + W.mp_ic * (sqrt(1.0 + W.mp_theta) - 1.0) * W.eta_hat;
  W.mp_stage = 0;
}

// Dual trial of row i given s = (K~ x')_i; stores K~ x' when the product was just formed, adds
// the pending average weight of the last accepted y (first trial of an iteration only).
struct MpDualEpi {
  static constexpr int N = 1;
  const double* __restrict__ q;
  const double* __restrict__ y;
  const double* __restrict__ kx;
  double* __restrict__ yn;
  double* __restrict__ kxn;
  double* __restrict__ sy;
  double sigma, th, w;
  int m1, store_kx;
  __device__ __forceinline__ void row(int i, double s, double (&out)[1]) const {
    const double yi = y[i];
    if (store_kx) kxn[i] = s;
    if (w != 0.0) sy[i] = sy[i] + w * yi;
    double v = yi + sigma * (q[i] - ((1.0 + th) * s - th * kx[i]));
    if (i < m1) v = fmax(v, 0.0);
    yn[i] = v;
    const double d = v - yi;
    out[0] = d * d;
  }
};

// K~^T y^ of the trial: stored, and ||K~^T y^ - K~^T y||^2 accumulated.
struct MpKtyEpi {
  static constexpr int N = 1;
  const double* __restrict__ kty;
  double* __restrict__ ktyh;
  __device__ __forceinline__ void row(int j, double s, double (&out)[1]) const {
    ktyh[j] = s;
    const double d = s - kty[j];
    out[0] = d * d;
  }
};

__device__ __forceinline__ MpDualEpi mp_dual_epi(const DevState& S, const Bufs& B, int store_kx) {
  const int P = S.parity;
  return MpDualEpi{B.q, pick(B.Y, P), pick(B.KX, P), pick(B.Y, P ^ 1), pick(B.KX, P ^ 1), B.Sy,
                   S.omega * S.eta, S.eta_hat / S.eta, S.w_pending, B.m1, store_kx};
}

// First trial of an iteration, fused with the product K~ x' (plain layout).
__global__ __launch_bounds__(kBlock) void k_mp_dual(CsrDev A, DevState* st, Bufs B, double* partB) {
  const DevState& S = *st;
  if (!primal_runs(S)) return;
  const MpDualEpi epi = mp_dual_epi(S, B, 1);
  double acc[1] = {0.0};
  csr_rows<kProd>(A, pick(B.X, S.parity ^ 1), epi, acc, partB);
  block_sum<1>(acc);
  write_slot<1>(partB, blockIdx.x, acc);
}

// Same, second pass of the XCD-panel layout.
__global__ __launch_bounds__(kBlock) void k_mp_dual_combine(CsrDev A, DevState* st, Bufs B, const double* part,
                                                            double* partB) {
  const DevState& S = *st;
  if (!primal_runs(S)) return;
  const MpDualEpi epi = mp_dual_epi(S, B, 1);
  double acc[1] = {0.0};
  combine_rows<kProd>(A, part, nullptr, epi, acc);
  block_sum<1>(acc);
  write_slot<1>(partB, blockIdx.x, acc);
}

// A retried trial: the same row update from the stored K~ x'.
__global__ __launch_bounds__(kBlock) void k_mp_retry(DevState* st, Bufs B, double* partB) {
  const DevState& S = *st;
  if (!(attempt_runs(S) && S.mp_stage)) return;
  const MpDualEpi epi = mp_dual_epi(S, B, 0);
  const double* kxn = pick(B.KX, S.parity ^ 1);
  double acc[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < B.m; i += gridDim.x * kBlock) {
    double c[1];
    epi.row(i, kxn[i], c);
    acc[0] += c[0];
  }
  block_sum<1>(acc);
  write_slot<1>(partB, blockIdx.x, acc);
}

// K~^T y^ of every trial (plain layout).
__global__ __launch_bounds__(kBlock) void k_mp_kty(CsrDev AT, DevState* st, Bufs B, double* partA) {
  const DevState& S = *st;
  if (!attempt_runs(S)) return;
  const MpKtyEpi epi{B.KTy, B.KTyH};
  double acc[1] = {0.0};
  csr_rows<kProd>(AT, pick(B.Y, S.parity ^ 1), epi, acc, partA);
  block_sum<1>(acc);
  write_slot<1>(partA, blockIdx.x, acc);
}

__global__ __launch_bounds__(kBlock) void k_mp_kty_combine(CsrDev AT, DevState* st, Bufs B, const double* part,
                                                           double* partA) {
  const DevState& S = *st;
  if (!attempt_runs(S)) return;
  const MpKtyEpi epi{B.KTy, B.KTyH};
  double acc[1] = {0.0};
  combine_rows<kProd>(AT, part, nullptr, epi, acc);
  block_sum<1>(acc);
  write_slot<1>(partA, blockIdx.x, acc);
}

// The line-search test and the bookkeeping of Algorithm 1 for one trial.  One thread.
__device__ void mp_decide(DevState& W, double dy2, double kdy2, pdlp_attempt_rec* att) {
  const double eta = W.eta;
  const double ndy = sqrt(dy2), nkdy = sqrt(kdy2);
  const double eta_bar = (nkdy > 0.0) ? W.mp_bf * ndy / nkdy : INFINITY;
  const bool ok = isfinite(dy2) && isfinite(kdy2);
  const bool accepted = ok && (eta * nkdy <= W.mp_bf * ndy);
  if (att && W.trace_cap > 0) {
    pdlp_attempt_rec& rec = att[W.n_att_log % W.trace_cap];
    rec.k = W.k;
    rec.eta = eta;
    rec.eta_bar = eta_bar;
    rec.accepted = accepted ? 1 : 0;
    rec.pad = 0;
  }
  W.n_att_log += 1;
  W.attempts += 1;
  W.spmv_KT += 1;                         // K~^T y^
  if (W.mp_stage == 0) {
    W.spmv_K += 1;                        // K~ x'
    if (!W.kty_valid) {                   // the primal step formed K~^T y
      W.spmv_KT += 1;
      W.kty_valid = 1;
    }
  }
  W.w_pending = 0.0;
  W.mp_commit = accepted ? 1 : 0;
  if (!ok) {
    W.status = PDLP_NUMERICAL_ERROR;
    W.done = 1;
    return;
  }
  if (accepted) {
    W.parity ^= 1;
    W.w_pending = eta;
    W.s_eta += eta;
    W.mp_theta = W.eta_hat / eta;         // theta_{k+1} = eta_k / eta_{k+1}
    W.eta_hat = eta;
    mp_first_candidate(W);
    W.k += 1;
    W.t += 1;
    W.retries = 0;
    if (W.k % W.check_every == 0) W.check_pending = 1;
    mark_weight_event(W);
    if (W.k <= W.trace_iters) W.snap_pending = 1;
  } else {
    W.eta = W.mp_df * eta;
    W.mp_stage = 1;
    W.retries += 1;
    if (W.retries >= W.max_retries) {
      W.status = PDLP_NUMERICAL_ERROR;
      W.done = 1;
    }
  }
}

// After an accepted trial: K~^T y <- K~^T y^ (the product of the new current y).  The flag is
// the outcome of the latest trial, so a repeated copy (a slot whose attempt did not run) copies
// the same values again; a restart clears it.
__global__ __launch_bounds__(kBlock) void k_mp_commit(DevState* st, Bufs B) {
  if (!st->mp_commit) return;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < B.n; j += gridDim.x * kBlock) B.KTy[j] = B.KTyH[j];
}

// ------------------------------------------------------------------------------------------
// plain products (restart checks, initialisation, the spmv entry point)
// ------------------------------------------------------------------------------------------

struct StoreEpi {
  static constexpr int N = 1;
  double* __restrict__ out;
  __device__ __forceinline__ void row(int r, double s, double (&c)[1]) const {
    out[r] = s;
    c[0] = 0.0;
  }
};

// Bookkeeping after a plain product: counters, and K~^T y of the current y is now valid.
__device__ void spmv_tail(DevState* st, int pred, int count_as) {
  if (threadIdx.x == 0) {
    if (count_as == 1) st->spmv_K += 1;
    if (count_as == 2) st->spmv_KT += 1;
    if (pred == kPredCheckKty || pred == kPredKty) st->kty_valid = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_spmv(CsrDev A, DevState* st, const double* in0,
                                                 const double* in1, int in_parity, double* out0,
                                                 double* out1, int out_parity, int pred,
                                                 int count_as, unsigned* ticket) {
  const DevState& S = *st;
  if (!pred_ok(S, pred)) return;
  const double* in = (in_parity && S.parity) ? in1 : in0;
  double* out = (out_parity && S.parity) ? out1 : out0;
  StoreEpi epi{out};
  double acc[1] = {0.0};
  csr_rows<kProd>(A, in, epi, acc, nullptr);
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  spmv_tail(st, pred, count_as);
}

// ------------------------------------------------------------------------------------------
// XCD column-panel mode: first pass per panel row, second pass per row in panel order
// ------------------------------------------------------------------------------------------

// COPY = 0 for passes over K~, 1 over K~^T (the same code; two symbols so that a kernel trace
// tells the two products apart).
// (EMAX: the most entries per lane of A's tasks; 16 only in the layouts of the LDS kernel.)
template <int COPY, int EMAX>
__global__ __launch_bounds__(kBlock) void k_panel_rows(CsrDev A, DevState* st, const double* in0,
                                                       const double* in1, int in_parity, double* out,
                                                       int pred, int mode) {
  const DevState& S = *st;
  if (!pred_ok(S, pred)) return;
  const double* in = (in_parity && S.parity) ? in1 : in0;
  StoreEpi epi{out};
  double acc[1] = {0.0};
  if (mode == kProd) csr_rows<kProd, EMAX>(A, in, epi, acc, nullptr);
  else if (mode == kAbsMax) csr_rows<kAbsMax, EMAX>(A, nullptr, epi, acc, nullptr);
  else csr_rows<kAbsSum, EMAX>(A, nullptr, epi, acc, nullptr);
}

// First pass of a panel-mode product with the gathered operand staged in LDS: the panel-row
// values of k_panel_rows (mode kProd), summed in the same order.  One workgroup of kLdsBlock
// threads per CU; for each of its segments the workgroup stages the panel's first lds_h
// entries of the operand, then its wavefronts share the segment's tasks.
template <int COPY>
__global__ __launch_bounds__(kLdsBlock) void k_lds_rows(CsrDev A, DevState* st, const double* in0,
                                                        const double* in1, int in_parity, double* out,
                                                        int pred) {
  __shared__ double stage[kLdsEntries];
  const DevState& S = *st;
  if (!pred_ok(S, pred)) return;
  const double* in = (in_parity && S.parity) ? in1 : in0;
  StoreEpi epi{out};
  double acc[1] = {0.0};
  const int lane64 = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int s0 = A.lds_seg_ptr[blockIdx.x], s1 = A.lds_seg_ptr[blockIdx.x + 1];
  for (int sg = s0; sg < s1; ++sg) {
    const LdsSeg G = A.lds_seg[sg];
    const int32_t c0 = A.col_cut[G.p];
    const int32_t h = min(A.lds_h, A.col_cut[G.p + 1] - c0);
    if (sg > s0) __syncthreads();        // every wavefront is done with the previous stage
    {
      // all of a thread's stage loads in flight before its stores (one wait instead of a
      // chain of them; the stage fill holds up every wavefront of the workgroup)
      constexpr int kPer = (kLdsEntries + kLdsBlock - 1) / kLdsBlock;
      double tmp[kPer];
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int i = threadIdx.x + q * kLdsBlock;
        tmp[q] = i < h ? in[c0 + i] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int i = threadIdx.x + q * kLdsBlock;
        if (i < h) stage[i] = tmp[q];
      }
    }
    __syncthreads();
    if (A.cis16) {            // a slice: every column is in the stage
      const StageGather gx{stage};
      for (int t = G.tb + wave; t < G.te; t += kLdsWaves)
        wave_task_e<kProd, 4, true, kElemsPerLaneLds>(A, gx, epi, acc, t, lane64);
    } else {
      const LdsGather gx{stage, in, c0, uint32_t(h)};
      for (int t = G.tb + wave; t < G.te; t += kLdsWaves)
        wave_task_e<kProd, 4, false, kElemsPerLaneLds>(A, gx, epi, acc, t, lane64);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_primal_combine(CsrDev AT, DevState* st, Bufs B,
                                                           const double* part, double* partA) {
  const DevState& S = *st;
  if (!primal_runs(S)) return;
  const int P = S.parity;
  const int kty_valid = S.kty_valid;
  PrimalEpi epi{B.c, B.l, B.u, pick(B.X, P), pick(B.X, P ^ 1), B.Sx, B.KTy, primal_step(S), S.w_pending, !kty_valid};
  double acc[1] = {0.0};
  combine_rows<kProd>(AT, part, kty_valid ? B.KTy : nullptr, epi, acc);
  block_sum<1>(acc);
  write_slot<1>(partA, blockIdx.x, acc);
}

__global__ __launch_bounds__(kBlock) void k_dual_combine(CsrDev A, DevState* st, Bufs B,
                                                         const double* part, const double* partA,
                                                         int nslotA, double* partB, unsigned* ticket) {
  const DevState& S = *st;
  if (!attempt_runs(S)) return;
  const int P = S.parity;
  DualEpi epi{B.q, pick(B.Y, P), pick(B.KX, P), pick(B.Y, P ^ 1), pick(B.KX, P ^ 1), B.Sy, S.eta * S.omega, S.w_pending, B.m1};
  double acc[2] = {0.0, 0.0};
  combine_rows<kProd>(A, part, nullptr, epi, acc);
  block_sum<2>(acc);
  write_slot<2>(partB, blockIdx.x, acc);
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  finish_attempt(st, B, partA, nslotA, partB, int(gridDim.x));
}

__global__ __launch_bounds__(kBlock) void k_spmv_combine(CsrDev A, DevState* st, const double* part,
                                                         double* out0, double* out1, int out_parity,
                                                         int pred, int count_as, unsigned* ticket) {
  const DevState& S = *st;
  if (!pred_ok(S, pred)) return;
  double* out = (out_parity && S.parity) ? out1 : out0;
  StoreEpi epi{out};
  double acc[1] = {0.0};
  combine_rows<kProd>(A, part, nullptr, epi, acc);
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  spmv_tail(st, pred, count_as);
}

__global__ __launch_bounds__(kBlock) void k_norm_combine(CsrDev A, const double* part, double* out,
                                                         int inf_norm) {
  StoreEpi epi{out};
  double acc[1] = {0.0};
  if (inf_norm) combine_rows<kAbsMax>(A, part, nullptr, epi, acc);
  else combine_rows<kAbsSum>(A, part, nullptr, epi, acc);
}

// ------------------------------------------------------------------------------------------
// preconditioning (Section 3.5)
// ------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_row_norms(CsrDev A, double* out, int inf_norm) {
  StoreEpi epi{out};
  double acc[1] = {0.0};
  if (inf_norm) csr_rows<kAbsMax>(A, nullptr, epi, acc, nullptr);
  else csr_rows<kAbsSum>(A, nullptr, epi, acc, nullptr);
}

// d = 1/sqrt(norm) (1 for an empty row or column), D *= d.
__global__ __launch_bounds__(kBlock) void k_scale_factors(const double* norms, double* fac, double* D, int len) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < len; i += gridDim.x * kBlock) {
    const double r = norms[i];
    const double d = (r > 0.0) ? 1.0 / sqrt(r) : 1.0;
    fac[i] = d;
    D[i] = D[i] * d;
  }
}

// K~_ij <- (K~_ij * dr_i) * dc_j, on the row-major copy (transposed = 0) or on the
// transposed copy (transposed = 1, where the CSR row is j and the column is i); the same
// expression keeps the two copies bitwise transposes of each other.
__global__ __launch_bounds__(kBlock) void k_scale_values(CsrDev A, double* v, double* vs, const double* dr,
                                                         const double* dc, int transposed) {
  csr_elements(A, [&](int64_t e, int r, int col) {
    const int i = transposed ? col : r;
    const int j = transposed ? r : col;
    v[e] = (v[e] * dr[i]) * dc[j];
  });
  // the interleaved entries of the wavefront tasks, with the same expression
  const int nw = gridDim.x * kWaves;
  const int lane64 = threadIdx.x & 63;
  for (int t = blockIdx.x * kWaves + (threadIdx.x >> 6); t < A.nwave; t += nw) {
    const RowDesc D = A.wave[t];
    const int lg = D.kind_l >> 8, L = 1 << lg, E = D.aux;
    const int g = lane64 >> lg, lane = lane64 & (L - 1), per_round = 64 >> lg;
    int64_t blk = A.task_off[t] + lane64;
    for (int base = 0; base < D.b; base += per_round, blk += int64_t(64) * E) {
      const int slot = base + g;
      if (slot >= D.b) continue;
      const int k = A.perm ? A.perm[D.a + slot] : D.a + slot;
      const int r = A.prow_row ? A.prow_row[k] : k;
      const int64_t len = A.rp[k + 1] - A.rp[k];
      for (int q = 0; q < E; ++q) {
        if (int64_t(q) * L + lane >= len) break;
        const int64_t pos = blk + int64_t(q) * 64;
        const int col = A.cis[pos];
        const int i = transposed ? col : r;
        const int j = transposed ? r : col;
        vs[pos] = (vs[pos] * dr[i]) * dc[j];
      }
    }
  }
}

// c~ = D2 c, l~ = l / D2, u~ = u / D2, q~ = D1 q
__global__ __launch_bounds__(kBlock) void k_scale_vectors(Bufs B, double* c, double* l, double* u, double* q) {
  for (int64_t idx = blockIdx.x * int64_t(kBlock) + threadIdx.x; idx < int64_t(B.n) + B.m;
       idx += int64_t(gridDim.x) * kBlock) {
    if (idx < B.n) {
      const double d = B.D2[idx];
      c[idx] = d * B.c0[idx];
      l[idx] = B.l0[idx] / d;
      u[idx] = B.u0[idx] / d;
    } else {
      const int i = int(idx - B.n);
      q[i] = B.D1[i] * B.q0[i];
    }
  }
}

// Initial point x0 = proj_X(0), y0 = 0, anchors, sums and the scalars omega, eta_hat,
// ||c||, ||q|| (Algorithm 1 initialisation, Section 3.3 InitializePrimalWeight).
__global__ __launch_bounds__(kBlock) void k_init(CsrDev A, DevState* st, Bufs B, double* part,
                                                 unsigned* ticket, double primal_importance,
                                                 double eps_zero) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};   // ||c||^2, ||q||^2, ||c~||^2, ||q~||^2
  double vmax = 0.0;
  for (int64_t idx = blockIdx.x * int64_t(kBlock) + threadIdx.x; idx < int64_t(B.n) + B.m;
       idx += int64_t(gridDim.x) * kBlock) {
    if (idx < B.n) {
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
      const int i = int(idx - B.n);
      B.Y[0][i] = 0.0;
      B.Y[1][i] = 0.0;
      B.YA[i] = 0.0;
      B.Sy[i] = 0.0;
      a[1] += B.q0[i] * B.q0[i];
      a[3] += B.q[i] * B.q[i];
    }
  }
  const int64_t nnz = A.nrows > 0 ? A.rp[A.nrows] : 0;
  for (int64_t e = blockIdx.x * int64_t(kBlock) + threadIdx.x; e < nnz; e += int64_t(gridDim.x) * kBlock)
    vmax = fmax(vmax, fabs(A.v[e]));
  block_sum<4>(a);
  vmax = block_max(vmax);
  double o[5] = {a[0], a[1], a[2], a[3], vmax};
  write_slot<5>(part, blockIdx.x, o);
  if (!arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  double t[4];
  {
    double s4[4] = {0, 0, 0, 0};
    for (int s = threadIdx.x; s < int(gridDim.x); s += kBlock)
      for (int k = 0; k < 4; ++k) s4[k] += ld_agent(&part[size_t(s) * 5 + k]);
    block_sum<4>(s4);
    for (int k = 0; k < 4; ++k) t[k] = s4[k];
  }
  double mx = 0.0;
  for (int s = threadIdx.x; s < int(gridDim.x); s += kBlock) mx = fmax(mx, ld_agent(&part[size_t(s) * 5 + 4]));
  mx = block_max(mx);
  if (threadIdx.x != 0) return;
  DevState& W = *st;
  W.c_norm = sqrt(t[0]);
  W.q_norm = sqrt(t[1]);
  const double nc = sqrt(t[2]), nq = sqrt(t[3]);
  W.omega = ((nc > eps_zero && nq > eps_zero) ? nc / nq : 1.0) * primal_importance;
  W.eta_hat = (mx > 0.0) ? 1.0 / mx : 1.0;
  W.eta = W.eta_hat;
  if (W.mp_on) {
    W.mp_theta = 1.0;
    mp_first_candidate(W);
  }
}

// ------------------------------------------------------------------------------------------
// restart / termination check (Algorithm 1 every check_every accepted steps)
//
// Each stage is split into a per-element piece and a scalar decision taken by one thread,
// so the multi-workgroup kernels below (grid-stride + last-workgroup ticket) and the batched
// solver (one workgroup per LP) run the very same arithmetic.
// ------------------------------------------------------------------------------------------

struct PointPtrs {
  const double* x;
  const double* y;
  const double* kty;
  const double* kx;
};

__device__ __forceinline__ PointPtrs current_point(const Bufs& B, int P) {
  return PointPtrs{pick(B.X, P), pick(B.Y, P), B.KTy, pick(B.KX, P)};
}
__device__ __forceinline__ PointPtrs average_point(const Bufs& B) {
  return PointPtrs{B.XB, B.YB, B.KTYB, B.KXB};
}

// Add the pending weighted iterate to the sums and form the average x_bar = S_x / S_eta.
__device__ __forceinline__ void prepare_elem(const Bufs& B, int P, double w, double se, int64_t idx) {
  if (idx < B.n) {
    double s = B.Sx[idx];
    if (w != 0.0) {
      s = s + w * pick(B.X, P)[idx];
      B.Sx[idx] = s;
    }
    B.XB[idx] = s / se;
  } else {
    const int i = int(idx - B.n);
    double s = B.Sy[i];
    if (w != 0.0) {
      s = s + w * pick(B.Y, P)[i];
      B.Sy[i] = s;
    }
    B.YB[i] = s / se;
  }
}

// Normalized duality gap (Section 3.2), set-up: the trust-region data |a_i| and b_i (the
// distance to the box along sign(a_i)) of every slot, and the radius sums.
// mode 0: slot 0 = current iterate, slot 1 = average, both against the anchor.
// mode 1: slot 0 = the restart candidate against the old anchor (after the weight update).
__device__ __forceinline__ void gap_points_of(const DevState& S, const Bufs& B, int mode, PointPtrs (&pt)[2]) {
  const int P = S.parity;
  if (mode == 0) {
    pt[0] = current_point(B, P);
    pt[1] = average_point(B);
  } else {
    pt[0] = S.use_avg ? average_point(B) : current_point(B, P);
    pt[1] = pt[0];
  }
}

__device__ __forceinline__ void gap_setup_elem(const Bufs& B, const PointPtrs (&pt)[2], int ns,
                                               double sw, int64_t idx, double (&acc)[6]) {
  for (int s = 0; s < ns; ++s) {
    double a, lo, hi;
    if (idx < B.n) {
      const int j = int(idx);
      const double xj = pt[s].x[j];
      const double d = xj - B.XA[j];
      acc[3 * s] += d * d;
      a = -(B.c[j] - pt[s].kty[j]) / sw;
      lo = sw * (B.l[j] - xj);
      hi = sw * (B.u[j] - xj);
    } else {
      const int i = int(idx - B.n);
      const double yi = pt[s].y[i];
      const double d = yi - B.YA[i];
      acc[3 * s + 1] += d * d;
      a = sw * (B.q[i] - pt[s].kx[i]);
      lo = (i < B.m1) ? -yi / sw : -INFINITY;
      hi = INFINITY;
    }
    lo = fmin(lo, 0.0);
    hi = fmax(hi, 0.0);
    double aa = fabs(a), b = (a > 0.0) ? hi : -lo;
    if (a == 0.0) {
      aa = 0.0;
      b = 0.0;
    }
    B.GA[s][idx] = aa;
    B.GB[s][idx] = b;
    acc[3 * s + 2] += b * b;
  }
}

__device__ void gap_setup_decide(DevState& W, int mode, const double (&t)[6]) {
  const int ns = (mode == 0) ? 2 : 1;
  const double omega = W.omega;
  for (int s = 0; s < ns; ++s) {
    const double r = sqrt(omega * t[3 * s] + t[3 * s + 1] / omega);
    W.gap_r[s] = r;
    W.gap_lo[s] = 0;
    W.gap_hi[s] = 0x7FF0000000000000ull;   // +inf
    if (r == 0.0) W.gap_state[s] = 2;
    else if (t[3 * s + 2] <= r * r) W.gap_state[s] = 1;
    else W.gap_state[s] = 0;
  }
  if (mode == 1) W.gap_state[1] = 2;
}

constexpr int kGapPts = 32;

__device__ __forceinline__ uint64_t gap_point(uint64_t lo, uint64_t hi, int i) {
  const uint64_t d = hi - lo;
  return lo + (d >> 5) * uint64_t(i) + (((d & 31ull) * uint64_t(i)) >> 5);
}

// One bisection pass over the breakpoints of ||e(s)||^2 = sum min(s|a_i|, b_i)^2 of gap slot
// sel: it is evaluated at 32 points splitting [lo, hi] (as bit patterns of positive doubles,
// which order like the values) and the sub-interval where it crosses r^2 is kept.  The two
// slots of a restart check run in one launch on separate workgroups (the first half of the
// grid for slot 0, the second for slot 1): 32 sums per thread instead of 64 keep the pass at
// more wavefronts per SIMD.
__device__ __forceinline__ void gap_bisect_points(const DevState& S, int sel, double (&sp)[kGapPts]) {
#pragma unroll
  for (int i = 0; i < kGapPts; ++i)
    sp[i] = __longlong_as_double((long long)gap_point(S.gap_lo[sel], S.gap_hi[sel], i + 1));
}

__device__ __forceinline__ void gap_bisect_elem(const Bufs& B, int sel, const double (&sp)[kGapPts],
                                                int64_t idx, double (&acc)[kGapPts]) {
  const double aa = (sel ? B.GA[1] : B.GA[0])[idx], b = (sel ? B.GB[1] : B.GB[0])[idx];
  if (aa != 0.0) {
#pragma unroll
    for (int i = 0; i < kGapPts; ++i) {
      const double e = fmin(sp[i] * aa, b);
      acc[i] += e * e;
    }
  }
}

// t[i] holds f at point i + 1 of slot s (point 32 is hi itself; point 0 is lo).
__device__ void gap_bisect_decide_slot(DevState& W, int s, const double* t) {
  const double r2 = W.gap_r[s] * W.gap_r[s];
  const uint64_t lo = W.gap_lo[s], hi = W.gap_hi[s];
  int i = 0;
  while (i < kGapPts && t[i] < r2) ++i;
  if (i == kGapPts) i = kGapPts - 1;
  const uint64_t nlo = (i == 0) ? lo : gap_point(lo, hi, i);
  const uint64_t nhi = gap_point(lo, hi, i + 1);
  W.gap_lo[s] = nlo;
  W.gap_hi[s] = nhi;
  if (nhi - nlo <= 1) W.gap_state[s] = 3;
}

// mu = a^T e(s*) / r with s* the upper end of the final bracket (or +inf).
__device__ __forceinline__ void gap_final_elem(const Bufs& B, const DevState& S, int ns,
                                               const double (&sstar)[2], int64_t idx, double (&acc)[2]) {
  for (int s = 0; s < ns; ++s) {
    if (S.gap_state[s] == 2) continue;
    const double aa = B.GA[s][idx], b = B.GB[s][idx];
    if (aa != 0.0) acc[s] += aa * (isinf(sstar[s]) ? b : fmin(sstar[s] * aa, b));
  }
}

__device__ void gap_final_decide(DevState& W, int mode, const double (&t)[2], pdlp_check_rec* chk) {
  double mu[2];
  for (int s = 0; s < 2; ++s) mu[s] = (W.gap_state[s] == 2) ? 0.0 : t[s] / W.gap_r[s];
  if (mode == 0) {
    W.mu_cur = mu[0];
    W.mu_avg = mu[1];
    W.use_avg = (W.to_current && mu[0] < mu[1]) ? 0 : 1;   // GetRestartCandidate: a tie picks the average
    W.mu_c = W.use_avg ? mu[1] : mu[0];
  } else {
    W.mu_anchor = mu[0];
    if (chk && W.trace_cap > 0 && W.n_chk_log > 0) chk[(W.n_chk_log - 1) % W.trace_cap].mu_anchor = mu[0];
  }
}

// Relative KKT error (Section 4.1, Eq. (6a)-(6c)) of a point on the user's unscaled problem:
// x = D2 x~, K x = (K~ x~) / D1, y = D1 y~, K^T y = (K~^T y~) / D2.  Sums: pobj, dobj (q
// part), dobj (bound part), primal residual^2, dual residual^2, |x~ - xa|^2, |y~ - ya|^2.
__device__ __forceinline__ void kkt_elem(const Bufs& B, const PointPtrs& pt, int64_t idx, double (&a)[7]) {
  if (idx < B.n) {
    const int j = int(idx);
    const double xs = pt.x[j];
    const double x = B.D2[j] * xs;
    const double g = B.c0[j] - pt.kty[j] / B.D2[j];
    const double lj = B.l0[j], uj = B.u0[j];
    const bool lf = isfinite(lj), uf = isfinite(uj);
    double lam = g;
    if (!lf && !uf) lam = 0.0;
    else if (!lf) lam = fmin(g, 0.0);
    else if (!uf) lam = fmax(g, 0.0);
    const double dr = g - lam;
    a[4] += dr * dr;
    a[0] += B.c0[j] * x;
    double bt = 0.0;
    if (lf) bt += lj * fmax(lam, 0.0);
    if (uf) bt += uj * fmin(lam, 0.0);
    a[2] += bt;
    const double d = xs - B.XA[j];
    a[5] += d * d;
  } else {
    const int i = int(idx - B.n);
    const double ys = pt.y[i];
    const double y = B.D1[i] * ys;
    const double kx = pt.kx[i] / B.D1[i];
    const double r = (i < B.m1) ? fmax(B.q0[i] - kx, 0.0) : kx - B.q0[i];
    a[3] += r * r;
    a[1] += B.q0[i] * y;
    const double d = ys - B.YA[i];
    a[6] += d * d;
  }
}

__device__ __forceinline__ bool kkt_point_is_average(const DevState& S, int mode) {
  return (mode == 0) ? (S.use_avg != 0) : (mode == 2 && S.out_avg != 0);
}

// mode 0: the restart candidate of a check, followed by the restart decision (criteria
//         (i)-(iii)) and the primal-weight update (Algorithm 3);
// mode 1: the current point before the first step (termination only);
// mode 2: the returned point after the solve stopped.
// Algorithm 3 from the current iterate's distance to the anchor (t[5], t[6] of the KKT pass).
__device__ __forceinline__ void weight_event_update(DevState& W, const double (&t)[7]) {
  const double dxn = sqrt(t[5]), dyn = sqrt(t[6]);
  W.dx_norm = dxn;
  W.dy_norm = dyn;
  if (W.pw_on && dxn > W.eps_zero && dyn > W.eps_zero)
    W.omega = exp(W.theta * log(dyn / dxn) + (1.0 - W.theta) * log(W.omega));
}

__device__ void kkt_decide(DevState& W, int mode, const double (&t)[7], pdlp_check_rec* chk) {
  const double pobj = t[0], dobj = t[1] + t[2];
  const double e_gap = fabs(dobj - pobj) / (1.0 + fabs(dobj) + fabs(pobj));
  const double e_pri = sqrt(t[3]) / (1.0 + W.q_norm);
  const double e_dual = sqrt(t[4]) / (1.0 + W.c_norm);
  const double kkt = fmax(e_gap, fmax(e_pri, e_dual));
  W.kkt[0] = e_gap;
  W.kkt[1] = e_pri;
  W.kkt[2] = e_dual;
  W.kkt[3] = kkt;
  const bool conv = kkt <= W.tol;   // false for NaN
  if (mode == 1) {
    if (conv) {
      W.done = 1;
      W.status = PDLP_OPTIMAL;
      W.out_avg = 0;
    }
    return;
  }
  if (mode == 2) {
    if (W.status == PDLP_NUMERICAL_ERROR && conv) W.status = PDLP_OPTIMAL;
    return;
  }
  if (W.pw_event && W.k % W.check_every != 0) {
    // only a weight update of the "no restart" mode: no termination test, no record
    weight_event_update(W, t);
    W.mask = 0;
    W.restart = 0;
    return;
  }
  W.checks += 1;
  pdlp_check_rec* rec = nullptr;
  if (chk && W.trace_cap > 0) {
    rec = &chk[W.n_chk_log % W.trace_cap];
    rec->k = W.k;
    rec->mu_cur = W.restarts_on ? W.mu_cur : NAN;
    rec->mu_avg = W.restarts_on ? W.mu_avg : NAN;
    rec->kkt = kkt;
    rec->use_avg = W.use_avg;
    rec->mask = 0;
    rec->terminated = conv ? 1 : 0;
    rec->mu_anchor = NAN;
    rec->pad = 0;
  }
  W.n_chk_log += 1;
  if (conv) {
    W.done = 1;
    W.status = PDLP_OPTIMAL;
    W.out_avg = W.use_avg;
    W.check_pending = 0;
    if (rec) rec->omega_after = W.omega;
    return;
  }
  int mask = 0;
  if (W.restarts_on) {
    if (W.n_outer > 0) {
      if (W.mu_c <= W.beta_suff * W.mu_anchor) mask |= 1;
      if (W.mu_c <= W.beta_nec * W.mu_anchor && W.mu_c > W.mu_prev) mask |= 2;
    }
    if (double(W.t) >= W.beta_art * double(W.k)) mask |= 4;
  }
  W.mask = mask;
  W.restart = mask != 0;
  if (W.restart) {
    const double dxn = sqrt(t[5]), dyn = sqrt(t[6]);
    W.dx_norm = dxn;
    W.dy_norm = dyn;
    if (W.pw_on && dxn > W.eps_zero && dyn > W.eps_zero)
      W.omega = exp(W.theta * log(dyn / dxn) + (1.0 - W.theta) * log(W.omega));
  }
  if (rec) {
    rec->mask = mask;
    rec->omega_after = W.omega;
  }
  // a regular check at k = 2^j (check_every dividing it): the "no restart" weight update
  // follows the check, as it precedes the next step
  if (W.pw_event) weight_event_update(W, t);
}

// Restart (Algorithm 1): z <- z_c, anchor <- z_c, sums cleared; then close the check.
__device__ __forceinline__ void apply_elem(const Bufs& B, int P, bool avg, int64_t idx) {
  if (idx < B.n) {
    const int j = int(idx);
    double xc = pick(B.X, P)[j];
    if (avg) {
      xc = B.XB[j];
      pick(B.X, P)[j] = xc;
      B.KTy[j] = B.KTYB[j];
    }
    B.XA[j] = xc;
    B.Sx[j] = 0.0;
  } else {
    const int i = int(idx - B.n);
    double yc = pick(B.Y, P)[i];
    if (avg) {
      yc = B.YB[i];
      pick(B.Y, P)[i] = yc;
      pick(B.KX, P)[i] = B.KXB[i];
    }
    B.YA[i] = yc;
    B.Sy[i] = 0.0;
  }
}

__device__ void apply_decide(DevState& W) {
  if (W.restart) {
    W.s_eta = 0.0;
    W.t = 0;
    W.n_outer += 1;
    W.mu_prev = INFINITY;
    W.kty_valid = 1;
    if (W.mp_on) {                       // the line search starts afresh: theta = 1
      W.mp_theta = 1.0;
      W.mp_commit = 0;
      mp_first_candidate(W);
    }
  } else if (W.pw_event) {              // anchor moved; iterate, averages and t stay
    W.n_outer += 1;
    W.pw_event = 0;
    if (W.mp_on) {
      W.mp_theta = 1.0;
      W.mp_commit = 0;
      mp_first_candidate(W);
    }
  } else if (W.restarts_on) {
    W.mu_prev = W.mu_c;
  }
  W.restart = 0;
  W.use_avg = 0;
  W.check_pending = 0;
  if (W.k >= W.iter_limit) {
    W.done = 1;
    W.status = PDLP_ITERATION_LIMIT;
    W.out_avg = 0;
  }
}

#define PDLP_GRID_LOOP(idx, total) \
  for (int64_t idx = blockIdx.x * int64_t(kBlock) + threadIdx.x; idx < (total); idx += int64_t(gridDim.x) * kBlock)

// Each check kernel below is an element pass over all n + m coordinates that writes one slot
// per workgroup, then a tail (sums of the slots, the scalar decision) taken either by the last
// workgroup to arrive at `ticket` (small grids) or, with ticket = nullptr, by the
// one-workgroup kernel k_tail launched after it (large grids: there the agent-scope fences
// of the arrival cost more than a launch).  Both run the same tail function on the same slots.

__device__ __forceinline__ bool gap_active(const DevState& S, int mode) {
  return check_runs(S) && (mode == 0 || S.restart);
}
// Gap slot sel still bisects (slot 1, the average, only in the restart check, mode 0).
__device__ __forceinline__ bool gap_bisect_active(const DevState& S, int mode, int sel) {
  return gap_active(S, mode) && S.gap_state[sel] == 0 && (sel == 0 || mode == 0);
}
// Workgroup groups of a bisection pass: one per gap slot the check evaluates.
__device__ __forceinline__ int gap_groups(int mode) { return mode == 0 ? 2 : 1; }

__device__ void prepare_tail(DevState* st) {
  if (threadIdx.x == 0) st->w_pending = 0.0;
}
__device__ void gap_setup_tail(DevState* st, int mode, const double* part, int nslot) {
  double t[6];
  sum_slots<6>(part, nslot, t);
  if (threadIdx.x == 0) gap_setup_decide(*st, mode, t);
}
// nslot: slots of the whole pass, nslot / gap_groups(mode) per gap slot, group by group.
__device__ void gap_bisect_tail(DevState* st, int mode, const double* part, int nslot) {
  __shared__ double t[kGapPts];
  const int ng = gap_groups(mode), per = nslot / ng;
  bool act[2];
  for (int sel = 0; sel < 2; ++sel) act[sel] = sel < ng && gap_bisect_active(*st, mode, sel);
  __syncthreads();
  for (int sel = 0; sel < ng; ++sel) {
    if (!act[sel]) continue;
    sum_slots_shared<kGapPts>(part + size_t(sel) * per * kGapPts, per, t);
    if (threadIdx.x == 0) gap_bisect_decide_slot(*st, sel, t);
  }
}
__device__ void gap_final_tail(DevState* st, const Bufs& B, int mode, const double* part, int nslot) {
  double t[2];
  sum_slots<2>(part, nslot, t);
  if (threadIdx.x == 0) gap_final_decide(*st, mode, t, B.chk);
}
__device__ void kkt_tail(DevState* st, const Bufs& B, int mode, const double* part, int nslot) {
  double t[7];
  sum_slots<7>(part, nslot, t);
  if (threadIdx.x == 0) kkt_decide(*st, mode, t, B.chk);
}
__device__ void apply_tail(DevState* st) {
  if (threadIdx.x == 0) apply_decide(*st);
}

__global__ __launch_bounds__(kBlock) void k_check_prepare(DevState* st, Bufs B, unsigned* ticket) {
  const DevState& S = *st;
  if (!check_runs(S)) return;
  const int P = S.parity;
  const double w = S.w_pending, se = S.s_eta;
  PDLP_GRID_LOOP(idx, int64_t(B.n) + B.m) prepare_elem(B, P, w, se, idx);
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  prepare_tail(st);
}

__global__ __launch_bounds__(kBlock) void k_gap_setup(DevState* st, Bufs B, int mode, double* part,
                                                      unsigned* ticket) {
  const DevState& S = *st;
  if (!gap_active(S, mode)) return;
  PointPtrs pt[2];
  gap_points_of(S, B, mode, pt);
  const int ns = (mode == 0) ? 2 : 1;
  const double sw = sqrt(S.omega);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  PDLP_GRID_LOOP(idx, int64_t(B.n) + B.m) gap_setup_elem(B, pt, ns, sw, idx, acc);
  block_sum<6>(acc);
  write_slot<6>(part, blockIdx.x, acc);
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  gap_setup_tail(st, mode, part, gridDim.x);
}

// Grid: gap_groups(mode) groups of equal size; group sel bisects gap slot sel.
__global__ __launch_bounds__(kBlock) void k_gap_bisect(DevState* st, Bufs B, int mode, double* part,
                                                       unsigned* ticket) {
  const DevState& S = *st;
  if (!gap_bisect_active(S, mode, 0) && !gap_bisect_active(S, mode, 1)) return;
  const int per = int(gridDim.x) / gap_groups(mode);
  const int sel = int(blockIdx.x) / per, lb = int(blockIdx.x) % per;
  double acc[kGapPts];
#pragma unroll
  for (int i = 0; i < kGapPts; ++i) acc[i] = 0.0;
  if (gap_bisect_active(S, mode, sel)) {
    double sp[kGapPts];
    gap_bisect_points(S, sel, sp);
    for (int64_t idx = lb * int64_t(kBlock) + threadIdx.x; idx < int64_t(B.n) + B.m; idx += int64_t(per) * kBlock)
      gap_bisect_elem(B, sel, sp, idx, acc);
  }
  block_sum<kGapPts>(acc);
  write_slot<kGapPts>(part, blockIdx.x, acc);
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  gap_bisect_tail(st, mode, part, gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_gap_final(DevState* st, Bufs B, int mode, double* part,
                                                      unsigned* ticket) {
  const DevState& S = *st;
  if (!gap_active(S, mode)) return;
  const int ns = (mode == 0) ? 2 : 1;
  double sstar[2];
  for (int s = 0; s < 2; ++s)
    sstar[s] = (S.gap_state[s] == 1) ? INFINITY : __longlong_as_double((long long)S.gap_hi[s]);
  double acc[2] = {0.0, 0.0};
  PDLP_GRID_LOOP(idx, int64_t(B.n) + B.m) gap_final_elem(B, S, ns, sstar, idx, acc);
  block_sum<2>(acc);
  write_slot<2>(part, blockIdx.x, acc);
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  gap_final_tail(st, B, mode, part, gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_kkt(DevState* st, Bufs B, int mode, double* part,
                                                unsigned* ticket) {
  const DevState& S = *st;
  if (mode == 0 && !check_runs(S)) return;
  const PointPtrs pt = kkt_point_is_average(S, mode) ? average_point(B) : current_point(B, S.parity);
  double a[7] = {0, 0, 0, 0, 0, 0, 0};
  PDLP_GRID_LOOP(idx, int64_t(B.n) + B.m) kkt_elem(B, pt, idx, a);
  block_sum<7>(a);
  write_slot<7>(part, blockIdx.x, a);
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  kkt_tail(st, B, mode, part, gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_check_apply(DevState* st, Bufs B, unsigned* ticket) {
  const DevState& S = *st;
  if (!check_runs(S)) return;
  const int P = S.parity;
  if (S.restart) {
    const bool avg = S.use_avg != 0;
    PDLP_GRID_LOOP(idx, int64_t(B.n) + B.m) apply_elem(B, P, avg, idx);
  } else if (S.pw_event) {
    PDLP_GRID_LOOP(idx, int64_t(B.n) + B.m) {
      if (idx < B.n) B.XA[idx] = pick(B.X, P)[idx];
      else B.YA[idx - B.n] = pick(B.Y, P)[idx - B.n];
    }
  }
  if (!ticket || !arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  apply_tail(st);
}

enum TailKind : int {
  kTailAttempt = 0, kTailSpmv, kTailPrepare, kTailGapSetup, kTailGapBisect, kTailGapFinal, kTailKkt,
  kTailApply, kTailMp
};

// The tail of a kernel launched without a ticket, in one workgroup after it; it re-evaluates
// the kernel's own entry predicate on the unchanged state, so it runs exactly when the
// kernel's element pass ran.  part/nslot: that kernel's slots (partB for the attempt, whose
// primal slots are partA/nslotA).
__global__ __launch_bounds__(kBlock) void k_tail(DevState* st, Bufs B, int kind, int mode, const double* part,
                                                 int nslot, const double* partA, int nslotA, int pred,
                                                 int count_as) {
  const DevState& S = *st;
  switch (kind) {
    case kTailAttempt:
      if (attempt_runs(S)) finish_attempt(st, B, partA, nslotA, part, nslot);
      break;
    case kTailSpmv:
      if (pred_ok(S, pred)) spmv_tail(st, pred, count_as);
      break;
    case kTailPrepare:
      if (check_runs(S)) prepare_tail(st);
      break;
    case kTailGapSetup:
      if (gap_active(S, mode)) gap_setup_tail(st, mode, part, nslot);
      break;
    case kTailGapBisect:
      if (gap_bisect_active(S, mode, 0) || gap_bisect_active(S, mode, 1)) gap_bisect_tail(st, mode, part, nslot);
      break;
    case kTailGapFinal:
      if (gap_active(S, mode)) gap_final_tail(st, B, mode, part, nslot);
      break;
    case kTailKkt:
      if (!(mode == 0 && !check_runs(S))) kkt_tail(st, B, mode, part, nslot);
      break;
    case kTailApply:
      if (check_runs(S)) apply_tail(st);
      break;
    case kTailMp:   // part: the trial's ||dy||^2 slots (nslot for a first trial, pred for a
                    // retry); partA: the ||K^T dy||^2 slots
      if (attempt_runs(S)) {
        double a[1], b[1];
        sum_slots<1>(part, S.mp_stage ? pred : nslot, a);
        sum_slots<1>(partA, nslotA, b);
        if (threadIdx.x == 0) mp_decide(*st, a[0], b[0], B.att);
      }
      break;
    default:
      break;
  }
}

// Resume from a checkpoint: vectors already copied into X[0], Y[0], XA, YA, Sx, Sy.
__global__ void k_set_state(DevState* st, pdlp_state v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    DevState& W = *st;
    W.k = v.k;
    W.t = v.t;
    W.n_outer = v.n_outer;
    W.eta_hat = v.eta_hat;
    W.eta = v.eta_hat;
    W.omega = v.omega;
    W.s_eta = v.s_eta;
    W.mu_prev = v.mu_prev;
    W.mu_anchor = v.mu_anchor;
    W.w_pending = 0.0;
    W.parity = 0;
    W.kty_valid = 0;
    W.check_pending = 0;
    W.done = 0;
    W.status = PDLP_NOT_SOLVED;
    W.retries = 0;
    W.restart = 0;
    W.use_avg = 0;
    W.out_avg = 0;
    W.snap_pending = 0;
    W.pw_event = 0;
    if (W.mp_on) {
      W.mp_theta = 1.0;
      W.mp_commit = 0;
      mp_first_candidate(W);
    }
  }
}

// Power iteration for ||K~||_2 (constant step policy): w = K~^T K~ v is in `w`; store
// ||w||^2 and v <- w / ||w|| for the next round.
__global__ __launch_bounds__(kBlock) void k_pow_norm(DevState* st, const double* w, int n, double* part,
                                                     unsigned* ticket) {
  double a[1] = {0.0};
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) a[0] += w[j] * w[j];
  block_sum<1>(a);
  write_slot<1>(part, blockIdx.x, a);
  if (!arrive_last(ticket, gridDim.x)) return;
  reset_ticket(ticket);
  double t[1];
  sum_slots<1>(part, gridDim.x, t);
  if (threadIdx.x == 0) st->pow_norm2 = t[0];
}

__global__ __launch_bounds__(kBlock) void k_pow_scale(const DevState* st, const double* w, double* v, int n) {
  const double nw = sqrt(st->pow_norm2);
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock)
    v[j] = (nw > 0.0) ? w[j] / nw : 0.0;
}

// v[j] = value for j < n (start vector of the power iteration).
__global__ __launch_bounds__(kBlock) void k_fill(double* v, double value, int n) {
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) v[j] = value;
}

// eta = 0.9 / ||K~||_2 with ||K~||_2 = sqrt(||K~^T K~ v||) of the last power iteration.
__global__ void k_pow_set_step(DevState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double sigma = sqrt(sqrt(st->pow_norm2));
    st->eta_hat = (sigma > 0.0) ? 0.9 / sigma : 1.0;
    st->eta = st->eta_hat;
  }
}

// Small state edits the host makes between solves.
__global__ void k_set_solve_params(DevState* st, double tol, int64_t iter_limit) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->tol = tol;
    st->iter_limit = iter_limit;
    st->done = 0;
    st->status = PDLP_NOT_SOLVED;
  }
}

__global__ void k_mark_limit(DevState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (!st->done && !st->check_pending && st->k >= st->iter_limit) {
      st->done = 1;
      st->status = PDLP_ITERATION_LIMIT;
      st->out_avg = 0;
    }
  }
}

// dst[i] = src[idx[i]] for i < len (reordering of n-vectors at the interface).
__global__ __launch_bounds__(kBlock) void k_gather(const double* __restrict__ src, const int32_t* __restrict__ idx,
                                                  double* __restrict__ dst, int64_t len) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < len; i += int64_t(gridDim.x) * kBlock)
    dst[i] = src[idx[i]];
}

// x = D2 x~ and y = D1 y~ of the returned point (or the current iterate, scaled = 1).
__global__ __launch_bounds__(kBlock) void k_output(const DevState* st, Bufs B, double* xo, double* yo,
                                                   int which) {
  const DevState& S = *st;
  const int P = S.parity;
  const bool avg = (which == 0) && S.out_avg;
  const double* xs = avg ? B.XB : pick(B.X, P);
  const double* ys = avg ? B.YB : pick(B.Y, P);
  for (int64_t idx = blockIdx.x * int64_t(kBlock) + threadIdx.x; idx < int64_t(B.n) + B.m;
       idx += int64_t(gridDim.x) * kBlock) {
    if (idx < B.n) xo[idx] = (which == 0) ? B.D2[idx] * xs[idx] : xs[idx];
    else {
      const int i = int(idx - B.n);
      yo[i] = (which == 0) ? B.D1[i] * ys[i] : ys[i];
    }
  }
}

}  // namespace pdlp
