// Host driver of the PDLP solver behind the C ABI of include/pdlp.h.
//
// pdlp_create validates the LP, builds the transposed CSR copy and the row schedules on the
// host, uploads everything once, and preconditions on the device.  pdlp_solve enqueues
// blocks of check_every PDHG attempts followed by one restart/termination check; every
// kernel reads its go/no-go from the device state, so the host never waits inside a block.
// Two blocks are kept in flight: the host reads the status record of block b-1 while block b
// runs, and stops when that record says the solve is over.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pdlp.h"
#include "host_prep.h"
#include "pdlp_device.h"
#include "pdlp_internal.h"
#include "pdlp_kernels.hip"
#include "pdlp_batch.hip"
#include "pdlp_unroll.hip"

using namespace pdlp;

namespace {

thread_local std::string g_create_error;

enum Ticket {
  kTkPrimal = 0, kTkDual, kTkSnap, kTkSpmv, kTkInit, kTkPrep, kTkGapSetup, kTkGapBisect,
  kTkGapFinal, kTkKkt, kTkApply, kNumTickets
};

constexpr int kBisectPasses = 13;   // 32-way splits of the 2^63 positive doubles

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.isManaged;
}

// The option ranges pdlp_create accepts (include/pdlp.h).
bool options_valid(const pdlp_options& o) {
  return !(o.ruiz_iters < 0 || o.check_every < 1 || o.max_retries < 1 || o.trace_iters < 0 ||
           o.trace_capacity < 0 || !(o.theta >= 0.0 && o.theta <= 1.0) || !(o.primal_importance > 0.0) ||
           !(o.eps_zero >= 0.0) || !(o.beta_sufficient > 0.0) || !(o.beta_necessary > 0.0) ||
           !(o.beta_artificial > 0.0) || o.step_policy < 0 || o.step_policy > 2 || o.power_iters < 1 ||
           !(o.mp_breaking_factor > 0.0) || !(o.mp_downscaling > 0.0 && o.mp_downscaling < 1.0) ||
           !(o.mp_interpolation >= 0.0 && o.mp_interpolation <= 1.0) || o.column_order < -1 ||
           o.column_order > 1 || (o.pw_power_of_two != 0 && (o.pw_power_of_two != 1 || o.adaptive_restarts)) ||
           o.lds_gather < -1 || o.lds_gather > 2 || o.lds_entries < 0 || o.lds_entries > kLdsEntries ||
           o.xcd_subpanels < -1 || o.xcd_subpanels > kMaxSubpanels);
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct pdlp_solver {
  hipStream_t stream = nullptr;
  int device = 0;                      // the GPU current at pdlp_create
  int64_t m = 0, n = 0, n_eq = 0, nnz = 0;
  pdlp_options opts{};
  std::vector<void*> allocs;
  CsrDev K{}, KT{};
  double* vK = nullptr;
  double* vKT = nullptr;
  double* vsK = nullptr;         // interleaved entries of the wavefront tasks of each copy
  double* vsKT = nullptr;
  Bufs B{};
  DevState* st = nullptr;
  double* partA = nullptr;
  double* partB = nullptr;
  double* partX = nullptr;
  double* partPK = nullptr;           // panel-row partials of the K~ products (panel mode)
  double* partPT = nullptr;           // panel-row partials of the K~^T products (panel mode)
  int gAc = 1, gBc = 1;               // grids of the row-ordered second passes
  unsigned* tickets = nullptr;
  double* outbuf = nullptr;
  int gA = 1, gB = 1, gE = 1, maxG = 1;
  DevState* h_st = nullptr;            // pinned, two records
  hipEvent_t blk_ev[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;    // private stream the block graphs are captured on
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  bool graphs_tried = false;
  // internal order of the primal variables (empty = the user's order): col_user[j'] is the
  // user's index of internal column j', col_int its inverse; device copies for the gathers
  std::vector<int32_t> col_user, col_int;
  const int32_t* d_col_user = nullptr;
  const int32_t* d_col_int = nullptr;
  double* permbuf = nullptr;           // n values of staging for the reordering gathers
  // kernel timing (options.time_kernels): 5 events per attempt slot of a block, around the
  // primal first pass, the primal combine, the dual first pass and the dual combine + tail
  std::vector<hipEvent_t> tev[2];
  int blk_slots[2] = {0, 0};           // attempt slots of the block last enqueued at each parity
  double t_ms[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t t_cnt[4] = {0, 0, 0, 0};
  int64_t timed_attempts = 0;          // attempts counted before the block being timed
  bool kkt_stale = false;              // the returned point's KKT error is not evaluated yet
  std::string err;
  bool solved = false;
  bool initial_checked = false;
  double create_seconds = 0.0, solve_seconds = 0.0;
  int last_status = PDLP_NOT_SOLVED;
  double bytes_A = 0.0, bytes_B = 0.0;
  double omega0 = 0.0;                 // initial primal weight (frozen omega of the unroll)
  double eta_pow = 0.0;                // 0.9 / ||K~||_2 once computed (frozen eta of the unroll)

  // Unrolled PDHG: buffers sized for the last forward call, the checkpoints of its segments
  // and the projection masks of one segment.
  struct Unroll {
    std::vector<void*> allocs;
    int64_t T = 0, S = 1, nseg = 0, cap_seg = -1, cap_S = -1;
    double eta = 0.0, omega = 0.0;
    struct Buf {
      double* ct = nullptr;      // c~, q~ of the forward call
      double* qt = nullptr;
      double* gin = nullptr;     // staging of the caller's c, q (forward) or gx, gy (backward)
      double* z = nullptr;       // x (n) | y (m) | K~ x (m) of the running step
      double* ck = nullptr;      // nseg checkpoints with the layout of z
      double* xb = nullptr;      // adjoints
      double* ub = nullptr;
      double* vb = nullptr;
      double* cb = nullptr;      // cb (n) | qb (m), contiguous
      double* out = nullptr;     // n + m outputs in the user's units
      uint8_t* mask = nullptr;   // S steps x (n + m) bytes
    };
    Buf own;                     // the solver's own buffers (pdlp_unroll_forward)
    Buf b;                       // the buffers of the last forward call: `own`, or carved from
                                 // the per-GPU scratch array (pdlp_unroll_forward_noalloc)
    bool in_scratch = false;     // b lies in the scratch array, claimed with scratch_gen
    uint64_t scratch_gen = 0;
    bool ready = false, masks_last = false;
    double fwd_s = 0.0, bwd_s = 0.0, bytes = 0.0;
    int64_t recomputed = 0;
  } U;

  ~pdlp_solver() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : allocs) (void)hipFree(p);
    for (void* p : U.allocs) (void)hipFree(p);
    if (h_st) (void)hipHostFree(h_st);
    for (int b = 0; b < 2; ++b) {
      if (blk_ev[b]) (void)hipEventDestroy(blk_ev[b]);
      if (gexec[b]) (void)hipGraphExecDestroy(gexec[b]);
      if (graph[b]) (void)hipGraphDestroy(graph[b]);
      for (hipEvent_t e : tev[b]) (void)hipEventDestroy(e);
    }
  }

  template <class T>
  hipError_t alloc(T** p, size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
    if (e == hipSuccess) allocs.push_back(*p);
    return e;
  }
};

#define PDLP_HIP(s, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      (s)->err = std::string(#call) + ": " + hipGetErrorString(e_);                        \
      return e_ == hipErrorOutOfMemory ? PDLP_ERR_OUT_OF_MEMORY : PDLP_ERR_DEVICE;          \
    }                                                                                      \
  } while (0)

#define PDLP_LAUNCH(s) PDLP_HIP(s, hipGetLastError())

// ------------------------------------------------------------------------------------------
// The scratch array of pdlp_unroll_forward_noalloc: device memory for the checkpoints,
// projection masks, adjoints and staging of an unrolled pass, for callers that cannot
// allocate.  Each GPU holds its own copy (at its own address) from the module load until the
// process ends.  Host code never passes `scratch` itself to a kernel or a copy: on the host
// the name only stands in for the symbol.  Its device address on each GPU is looked up once
// (hipGetSymbolAddress, with that GPU current, at the first pdlp_create on it) and every use
// goes through that address.  Every no-alloc call on a GPU shares the array: a call claims
// it by bumping the GPU's generation, and a backward pass checks that its forward still owns
// it.  Calls that overlap on one GPU race.
// ------------------------------------------------------------------------------------------

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxScratchDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct ScratchSlot {
  unsigned char* ptr;      // device address of `scratch` on this GPU (nullptr until looked up)
  uint64_t gen;            // claims so far
  hipError_t err;          // result of the lookup
  bool tried;
};
std::mutex g_scratch_mu;
ScratchSlot g_scratch[kMaxScratchDevices] = {};

// Looks up the scratch array's address on GPU `dev`, which must be current; once per GPU.
void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  ScratchSlot& sl = g_scratch[dev];
  if (sl.tried) return;
  sl.tried = true;
  void* p = nullptr;
  sl.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (sl.err == hipSuccess) sl.ptr = static_cast<unsigned char*>(p);
  else (void)hipGetLastError();
}

}  // namespace

namespace {

template <class T>
int fetch_input(pdlp_solver* s, const T* p, size_t count, std::vector<T>& tmp, const T** out) {
  if (count == 0) {
    *out = p;
    return 0;
  }
  if (is_device_ptr(p)) {
    tmp.resize(count);
    PDLP_HIP(s, hipMemcpy(tmp.data(), p, count * sizeof(T), hipMemcpyDeviceToHost));
    *out = tmp.data();
  } else {
    *out = p;
  }
  return 0;
}

int write_output(pdlp_solver* s, void* dst, const void* src_dev, size_t bytes) {
  if (!dst || bytes == 0) return 0;
  const hipMemcpyKind kind = is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  PDLP_HIP(s, hipMemcpyAsync(dst, src_dev, bytes, kind, s->stream));
  PDLP_HIP(s, hipStreamSynchronize(s->stream));
  return 0;
}

// n values in the solver's column order (device src) to dst in the user's order.
int write_n(pdlp_solver* s, double* dst, const double* src) {
  if (!dst) return 0;
  if (s->col_user.empty()) return write_output(s, dst, src, size_t(s->n) * 8);
  const int g = int(std::max<int64_t>(1, std::min<int64_t>((s->n + kBlock - 1) / kBlock, s->maxG)));
  k_gather<<<g, kBlock, 0, s->stream>>>(src, s->d_col_int, s->permbuf, s->n);
  PDLP_LAUNCH(s);
  return write_output(s, dst, s->permbuf, size_t(s->n) * 8);
}

// n values in the user's order (host or device src) into device dst in the solver's order.
int read_n(pdlp_solver* s, const double* src, double* dst) {
  const size_t bytes = size_t(s->n) * 8;
  const hipMemcpyKind kind = is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (s->col_user.empty()) {
    PDLP_HIP(s, hipMemcpyAsync(dst, src, bytes, kind, s->stream));
    return 0;
  }
  PDLP_HIP(s, hipMemcpyAsync(s->permbuf, src, bytes, kind, s->stream));
  const int g = int(std::max<int64_t>(1, std::min<int64_t>((s->n + kBlock - 1) / kBlock, s->maxG)));
  k_gather<<<g, kBlock, 0, s->stream>>>(s->permbuf, s->d_col_user, dst, s->n);
  PDLP_LAUNCH(s);
  return 0;
}

template <class T>
int upload_vec(pdlp_solver* s, const std::vector<T>& h, const T** out) {
  T* d;
  PDLP_HIP(s, s->alloc(&d, h.size()));
  if (!h.empty()) PDLP_HIP(s, hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = d;
  return 0;
}

int upload_tasks(pdlp_solver* s, const Schedule& sc, CsrDev& A) {
  int rc;
  const RowDesc *w, *b;
  const int32_t *nch, *base;
  if ((rc = upload_vec(s, sc.wave, &w)) || (rc = upload_vec(s, sc.block, &b)) ||
      (rc = upload_vec(s, sc.split_nchunks, &nch)) || (rc = upload_vec(s, sc.split_base, &base)))
    return rc;
  double* part;
  unsigned* cnt;
  PDLP_HIP(s, s->alloc(&part, size_t(sc.total_chunks)));
  PDLP_HIP(s, s->alloc(&cnt, sc.split_row.size()));
  PDLP_HIP(s, hipMemset(cnt, 0, std::max<size_t>(sc.split_row.size(), 1) * sizeof(unsigned)));
  A.nwave = int32_t(sc.wave.size());
  A.nblock = int32_t(sc.block.size());
  A.wave = w;
  A.block = b;
  A.split_nchunks = nch;
  A.split_base = base;
  A.nsplit = int32_t(sc.split_row.size());
  A.split_part = part;
  A.split_cnt = cnt;
  return 0;
}

// Uploads the interleaved entries of a layout's wavefront tasks (build_interleaved), the
// 16-bit length of each of its nrows rows and, for slices (panel cuts `cut`, tasks of panel p
// from wave_begin[p]), the interleaved columns relative to the task's slice.
int upload_interleaved(pdlp_solver* s, const Schedule& sc, const int64_t* rp, int64_t nrows, const int32_t* ci,
                       const double* v, const int32_t* perm, CsrDev& A, double** vsdev,
                       const std::vector<int32_t>* cut = nullptr, const std::vector<int32_t>* wave_begin = nullptr) {
  int rc;
  std::vector<int64_t> off;
  std::vector<int32_t> cis;
  std::vector<double> vs;
  build_interleaved(sc, rp, ci, v, perm, off, cis, vs);
  std::vector<uint16_t> rlen(static_cast<size_t>(nrows));
  for (int64_t r = 0; r < nrows; ++r) rlen[size_t(r)] = uint16_t(std::min<int64_t>(rp[r + 1] - rp[r], 65535));
  A.cis16 = nullptr;
  if (cut) {
    std::vector<uint16_t> cis16(cis.size(), 0);
    const int P = int(cut->size()) - 1;
    for (int p = 0; p < P; ++p) {
      const int32_t c0 = (*cut)[size_t(p)], w = (*cut)[size_t(p) + 1] - c0;
      if (w > 65536) {
        s->err = "internal error: slice wider than 16-bit columns";
        return PDLP_ERR_DEVICE;
      }
      for (int t = (*wave_begin)[size_t(p)]; t < (*wave_begin)[size_t(p) + 1]; ++t)
        for (int64_t q = off[size_t(t)]; q < off[size_t(t) + 1]; ++q) {
          const int32_t d = cis[size_t(q)] - c0;       // slots of missing rows hold column 0
          cis16[size_t(q)] = uint16_t(d >= 0 && d < w ? d : 0);
        }
    }
    const uint16_t* d16;
    if ((rc = upload_vec(s, cis16, &d16))) return rc;
    A.cis16 = d16;
  }
  const double* dvs;
  if ((rc = upload_vec(s, off, &A.task_off)) || (rc = upload_vec(s, cis, &A.cis)) || (rc = upload_vec(s, vs, &dvs)) ||
      (rc = upload_vec(s, rlen, &A.rlen)))
    return rc;
  A.vs = dvs;
  *vsdev = const_cast<double*>(dvs);
  return 0;
}

// Sub-panels per XCD panel: opt >= 1 as given (1 = none); automatic (-1): none while every
// panel's operand slice fits in kSubpanelBytes, else the fewest that keep each within it,
// rounded up to an even count, at most kMaxSubpanels.
int subpanel_count(const std::vector<int32_t>& cut, int opt) {
  if (opt >= 1) return opt;
  if (opt == 0) return 1;
  int64_t widest = 0;
  for (size_t p = 0; p + 1 < cut.size(); ++p) widest = std::max<int64_t>(widest, cut[p + 1] - cut[p]);
  int64_t S = (widest * 8 + kSubpanelBytes - 1) / kSubpanelBytes;
  if (S <= 1) return 1;
  S += S & 1;
  return int(std::min<int64_t>(S, kMaxSubpanels));
}

// Each column range of `cut` cut into S ranges of (nearly) equal width.
std::vector<int32_t> split_cuts(const std::vector<int32_t>& cut, int S) {
  std::vector<int32_t> sc;
  sc.reserve((cut.size() - 1) * size_t(S) + 1);
  for (size_t p = 0; p + 1 < cut.size(); ++p) {
    const int64_t a = cut[p], w = int64_t(cut[p + 1]) - a;
    for (int k = 0; k < S; ++k) sc.push_back(int32_t(a + w * k / S));
  }
  sc.push_back(cut.back());
  return sc;
}

// Uploads one CSR copy (nrows x ncols) in the plain row layout or, when it pays, in XCD
// column panels; *vdev receives the device values (the scaling kernels rewrite them) and
// *prow_part the panel-row partial buffer (panel mode only).
int upload_copy(pdlp_solver* s, int64_t nrows, int64_t ncols, const int64_t* rp, const int32_t* ci,
                const double* v, CsrDev& A, double** vdev, double** vsdev, double** prow_part,
                const std::vector<int32_t>* cuts = nullptr, bool hot_first = false) {
  int rc;
  const int64_t nnz = rp[nrows];
  const int mode = s->opts.xcd_panels;
  const int lmode = s->opts.lds_gather;
  const int W = s->opts.lds_entries > 0 ? s->opts.lds_entries : kLdsEntries;
  const int G = std::max(1, s->maxG / 8);          // one LDS workgroup per CU
  PanelLayout PL;
  bool panel = false;
  bool slices = false;
  int lds_h = 0;
  const bool want = nnz > 0 && (mode == 1 || (mode < 0 && ncols * 8 > (int64_t(4) << 20)));
  if (want && (lmode == 1 || (lmode < 0 && !hot_first))) {
    // one panel per W-wide slice of the gathered vector: every gather from LDS.  Automatic
    // for a copy whose columns keep their order, whose gathers have no hot entries to stage
    // (on the 1e6 x 2e6 LP, K~^T y was fastest this way: 0.80 ms in slices against 0.94 ms in
    // XCD panels and 0.98 ms with a hot stage, measured together)
    const int64_t Pw = (ncols + W - 1) / W;
    if (Pw >= 2 && Pw <= kMaxLdsPanels) {
      std::vector<int32_t> wc(size_t(Pw) + 1);
      for (int64_t p = 0; p <= Pw; ++p) wc[size_t(p)] = int32_t(std::min<int64_t>(p * W, ncols));
      double frac = lmode == 1 ? 1e300 : kLdsRowFrac;
      if (lmode < 0) {
        // with XCD panels as the alternative (forced, or their panel rows below
        // kPanelRowFrac), slices may cost more panel rows
        const std::vector<int32_t> xc = cuts ? *cuts : panel_cuts(ci, nnz, ncols, kMaxPanels);
        if (mode == 1 || double(count_panel_rows(rp, ci, nrows, xc)) <= kPanelRowFrac * double(nnz))
          frac = kLdsRowFracVsPanels;
      }
      panel = build_panels(rp, ci, nrows, ncols, int(Pw), frac, PL, &wc, kElemsPerLaneLds) && PL.sched.block.empty();
      if (panel) {
        lds_h = W;
        slices = true;
      }
    }
  }
  int nsub = 1;
  if (!panel && want) {
    // the first W columns of each panel staged in LDS: its hottest when the columns are
    // ordered hot-first, automatic for such a copy (on the 1e6 x 2e6 LP, K~ x took 0.55 ms
    // with the stage against 0.89 ms without and 1.21 ms in slices, measured together)
    const bool stage = lmode == 2 || (lmode < 0 && hot_first);
    const double frac = mode == 1 ? 1e300 : kPanelRowFrac;
    bool unstaged = !stage;
    if (stage) {
      panel = build_panels(rp, ci, nrows, ncols, kMaxPanels, frac, PL, cuts, kElemsPerLaneLds);
      if (panel && PL.sched.block.empty()) {
        lds_h = W;
      } else if (panel) {     // rows too long for the LDS kernel: the tasks of the other kernels
        panel = false;
        unstaged = true;
      }
    }
    if (unstaged) {
      // operand slices wider than an XCD's L2 share: sub-panels, when their panel rows allow
      const std::vector<int32_t> xc = cuts ? *cuts : panel_cuts(ci, nnz, ncols, kMaxPanels);
      const int S = subpanel_count(xc, s->opts.xcd_subpanels);
      if (S > 1) {
        const std::vector<int32_t> sc = split_cuts(xc, S);
        panel = build_panels(rp, ci, nrows, ncols, kMaxPanels * S, frac, PL, &sc);
        if (panel) nsub = S;
      }
      if (!panel) panel = build_panels(rp, ci, nrows, ncols, kMaxPanels, frac, PL, &xc);
    }
  }
  A.nrows_orig = int32_t(nrows);
  A.emax = (panel && lds_h > 0) ? kElemsPerLaneLds : kElemsPerLane;
  A.lds_h = 0;
  if (panel && lds_h > 0) {
    std::vector<LdsSeg> seg;
    const std::vector<int32_t> seg_ptr = lds_segments(PL, G, G % PL.P == 0, seg);
    bool ok = lds_h <= kLdsEntries;
    for (const LdsSeg& g : seg)
      ok = ok && g.p >= 0 && g.p < PL.P && g.tb >= PL.wave_begin[size_t(g.p)] &&
           g.te <= PL.wave_begin[size_t(g.p) + 1] && g.tb < g.te;
    if (!ok) {
      s->err = "internal error: LDS plan outside the panel layout";
      return PDLP_ERR_DEVICE;
    }
    if ((rc = upload_vec(s, PL.cut, &A.col_cut)) || (rc = upload_vec(s, seg_ptr, &A.lds_seg_ptr)) ||
        (rc = upload_vec(s, seg, &A.lds_seg)))
      return rc;
    A.lds_h = lds_h;
    A.lds_grid = G;
  }
  if (panel) {
    const int64_t nprow = int64_t(PL.prow_row.size());
    std::vector<int32_t> ciP(static_cast<size_t>(nnz));
    std::vector<double> vP(static_cast<size_t>(nnz));
    parallel_for(nnz, [&](int64_t k0, int64_t k1) {
      for (int64_t k = k0; k < k1; ++k) {
        ciP[size_t(k)] = ci[PL.src[size_t(k)]];
        vP[size_t(k)] = v[PL.src[size_t(k)]];
      }
    }, int64_t(1) << 20);
    std::vector<int64_t>().swap(PL.src);
    if ((rc = upload_interleaved(s, PL.sched, PL.prow_ptr.data(), nprow, ciP.data(), vP.data(), nullptr, A, vsdev,
                                 slices ? &PL.cut : nullptr, &PL.wave_begin)))
      return rc;
    if ((rc = upload_vec(s, PL.prow_ptr, &A.rp)) || (rc = upload_vec(s, ciP, &A.ci))) return rc;
    const double* dv;
    if ((rc = upload_vec(s, vP, &dv))) return rc;
    *vdev = const_cast<double*>(dv);
    A.v = dv;
    if ((rc = upload_vec(s, PL.prow_row, &A.prow_row)) || (rc = upload_vec(s, PL.slot_ptr, &A.slot_ptr)) ||
        (rc = upload_vec(s, PL.slot_idx, &A.slot_idx)) ||
        (rc = upload_vec(s, PL.wave_begin, &A.wave_begin)) ||
        (rc = upload_vec(s, PL.block_begin, &A.block_begin)))
      return rc;
    if ((rc = upload_tasks(s, PL.sched, A))) return rc;
    A.perm = nullptr;
    A.nrows = int32_t(nprow);
    A.npanel = PL.P;
    A.nsub = nsub;
    PDLP_HIP(s, s->alloc(prow_part, size_t(nprow)));
    return 0;
  }
  Schedule sc = build_schedule(rp, nrows);
  if ((rc = upload_interleaved(s, sc, rp, nrows, ci, v, sc.perm.empty() ? nullptr : sc.perm.data(), A, vsdev)))
    return rc;
  std::vector<int64_t> hrp(rp, rp + nrows + 1);
  std::vector<int32_t> hci(ci, ci + nnz);
  std::vector<double> hv(v, v + nnz);
  const double* dv;
  if ((rc = upload_vec(s, hrp, &A.rp)) || (rc = upload_vec(s, hci, &A.ci)) || (rc = upload_vec(s, hv, &dv)))
    return rc;
  *vdev = const_cast<double*>(dv);
  A.v = dv;
  if ((rc = upload_vec(s, sc.perm, &A.perm))) return rc;
  const std::vector<int32_t> wb = {0, int32_t(sc.wave.size())}, bb = {0, int32_t(sc.block.size())};
  if ((rc = upload_vec(s, wb, &A.wave_begin)) || (rc = upload_vec(s, bb, &A.block_begin))) return rc;
  if ((rc = upload_tasks(s, sc, A))) return rc;
  A.prow_row = nullptr;
  A.slot_ptr = nullptr;
  A.slot_idx = nullptr;
  A.nrows = int32_t(nrows);
  A.npanel = 1;
  A.nsub = 1;
  return 0;
}

// First pass of a panel-mode product over A (K~ or K~^T).
void launch_panel_rows(pdlp_solver* s, const CsrDev& A, int grid, const double* in0, const double* in1,
                       int in_par, double* out, int pred, int mode) {
  if (A.lds_h > 0 && mode == kProd) {
    if (&A == &s->KT)
      k_lds_rows<1><<<A.lds_grid, kLdsBlock, 0, s->stream>>>(A, s->st, in0, in1, in_par, out, pred);
    else
      k_lds_rows<0><<<A.lds_grid, kLdsBlock, 0, s->stream>>>(A, s->st, in0, in1, in_par, out, pred);
    return;
  }
  const bool wide = A.emax > kElemsPerLane;
  if (&A == &s->KT) {
    if (wide) k_panel_rows<1, kElemsPerLaneLds><<<grid, kBlock, 0, s->stream>>>(A, s->st, in0, in1, in_par, out, pred, mode);
    else k_panel_rows<1, kElemsPerLane><<<grid, kBlock, 0, s->stream>>>(A, s->st, in0, in1, in_par, out, pred, mode);
  } else {
    if (wide) k_panel_rows<0, kElemsPerLaneLds><<<grid, kBlock, 0, s->stream>>>(A, s->st, in0, in1, in_par, out, pred, mode);
    else k_panel_rows<0, kElemsPerLane><<<grid, kBlock, 0, s->stream>>>(A, s->st, in0, in1, in_par, out, pred, mode);
  }
}

// Grid of a CSR pass: a multiple of npanel.  Each panel group (npanel / nsub of them) gets
// maxG / groups workgroups for each of its nsub panels, which run one run after another.
int grid_for(const CsrDev& A, int maxG) {
  if (A.npanel <= 1) {
    const int by_wave = (A.nwave + kWaves - 1) / kWaves;
    return std::max(1, std::min(std::max(by_wave, A.nblock), maxG));
  }
  const int ng = A.npanel / std::max(1, A.nsub);
  return A.npanel * std::max(1, maxG / ng);
}

int grid_rows(int64_t nrows, int maxG) {
  return int(std::max<int64_t>(1, std::min<int64_t>((nrows + kBlock - 1) / kBlock, maxG)));
}

// Grids up to this size end with the last-arrival ticket; larger ones hand their tail to k_tail
// (each arrival costs an agent-scope release, which writes back the XCD's L2).
constexpr int kFuseMaxGrid = 64;

unsigned* ticket_for(pdlp_solver* s, int grid, int which) {
  return grid <= kFuseMaxGrid ? s->tickets + which : nullptr;
}

int launch_tail(pdlp_solver* s, int grid, int kind, int mode, const double* part, int nslot,
                const double* partA = nullptr, int nslotA = 0, int pred = 0, int count_as = 0) {
  if (grid <= kFuseMaxGrid) return 0;
  k_tail<<<1, kBlock, 0, s->stream>>>(s->st, s->B, kind, mode, part, nslot, partA, nslotA, pred, count_as);
  PDLP_LAUNCH(s);
  return 0;
}

int launch_spmv(pdlp_solver* s, const CsrDev& A, const double* in0, const double* in1, int in_par,
                double* out0, double* out1, int out_par, int pred, int count_as) {
  if (A.npanel > 1) {
    double* part = (&A == &s->K) ? s->partPK : s->partPT;
    launch_panel_rows(s, A, grid_for(A, s->maxG), in0, in1, in_par, part, pred, kProd);
    PDLP_LAUNCH(s);
    const int g = grid_rows(A.nrows_orig, s->maxG);
    k_spmv_combine<<<g, kBlock, 0, s->stream>>>(A, s->st, part, out0, out1, out_par, pred, count_as,
                                                ticket_for(s, g, kTkSpmv));
    PDLP_LAUNCH(s);
    return launch_tail(s, g, kTailSpmv, 0, nullptr, 0, nullptr, 0, pred, count_as);
  }
  const int g = grid_for(A, s->maxG);
  k_spmv<<<g, kBlock, 0, s->stream>>>(A, s->st, in0, in1, in_par, out0, out1, out_par, pred, count_as,
                                      ticket_for(s, g, kTkSpmv));
  PDLP_LAUNCH(s);
  return launch_tail(s, g, kTailSpmv, 0, nullptr, 0, nullptr, 0, pred, count_as);
}

// Power iteration on K~^T K~ from the all-ones vector (v, w: n values, t: m values); leaves
// ||K~^T K~ v||^2 of the last round in the device state, so ||K~||_2 ~ its fourth root.
int power_iterate(pdlp_solver* s, double* v, double* t, double* w) {
  int rc;
  const int64_t n = s->n;
  const int gn = grid_rows(n, s->maxG);
  k_fill<<<gn, kBlock, 0, s->stream>>>(v, 1.0 / std::sqrt(double(n)), int(n));
  PDLP_LAUNCH(s);
  for (int it = 0; it < s->opts.power_iters; ++it) {
    if ((rc = launch_spmv(s, s->K, v, nullptr, 0, t, nullptr, 0, kPredAlways, 0))) return rc;
    if ((rc = launch_spmv(s, s->KT, t, nullptr, 0, w, nullptr, 0, kPredAlways, 0))) return rc;
    k_pow_norm<<<gn, kBlock, 0, s->stream>>>(s->st, w, int(n), s->partX, s->tickets + kTkInit);
    PDLP_LAUNCH(s);
    k_pow_scale<<<gn, kBlock, 0, s->stream>>>(s->st, w, v, int(n));
    PDLP_LAUNCH(s);
  }
  return 0;
}

// The normalized-gap passes run on a grid of at most kGapGrid workgroups (per gap slot in the
// bisection, whose workgroups accumulate 32 sums each), so that the tail has fewer slots to add.
constexpr int kGapGrid = 640;

int enqueue_gap(pdlp_solver* s, int mode) {
  int rc;
  const int g = std::min(s->gE, kGapGrid);
  k_gap_setup<<<g, kBlock, 0, s->stream>>>(s->st, s->B, mode, s->partX, ticket_for(s, g, kTkGapSetup));
  PDLP_LAUNCH(s);
  if ((rc = launch_tail(s, g, kTailGapSetup, mode, s->partX, g))) return rc;
  // one group of workgroups per gap slot, at most 2 kGapGrid in all (32 sums each: within the
  // 64 gE values of the slot buffer)
  const int ng = mode == 0 ? 2 : 1;
  const int gb = ng * std::min(s->gE, 2 * kGapGrid / ng);
  for (int p = 0; p < kBisectPasses; ++p) {
    k_gap_bisect<<<gb, kBlock, 0, s->stream>>>(s->st, s->B, mode, s->partX, ticket_for(s, gb, kTkGapBisect));
    PDLP_LAUNCH(s);
    if ((rc = launch_tail(s, gb, kTailGapBisect, mode, s->partX, gb))) return rc;
  }
  k_gap_final<<<g, kBlock, 0, s->stream>>>(s->st, s->B, mode, s->partX, ticket_for(s, g, kTkGapFinal));
  PDLP_LAUNCH(s);
  return launch_tail(s, g, kTailGapFinal, mode, s->partX, g);
}

int enqueue_kkt(pdlp_solver* s, int mode) {
  const int g = s->gE;
  k_kkt<<<g, kBlock, 0, s->stream>>>(s->st, s->B, mode, s->partX, ticket_for(s, g, kTkKkt));
  PDLP_LAUNCH(s);
  return launch_tail(s, g, kTailKkt, mode, s->partX, g);
}

// The dual side of one Malitsky-Pock attempt: the first trial of an iteration (K~ x' and y^)
// or a retried trial (y^ from the stored K~ x'), then K~^T y^, the line-search test, and the
// commit of K~^T y^ after an accepted trial.  Every kernel reads its go/no-go from the state.
int enqueue_mp_trial(pdlp_solver* s) {
  Bufs& B = s->B;
  const bool panT = s->KT.npanel > 1, panK = s->K.npanel > 1;
  if (panK) {
    launch_panel_rows(s, s->K, s->gB, B.X[1], B.X[0], 1, s->partPK, kPredMpNew, kProd);
    PDLP_LAUNCH(s);
    k_mp_dual_combine<<<s->gBc, kBlock, 0, s->stream>>>(s->K, s->st, B, s->partPK, s->partB);
  } else {
    k_mp_dual<<<s->gB, kBlock, 0, s->stream>>>(s->K, s->st, B, s->partB);
  }
  PDLP_LAUNCH(s);
  const int gR = s->gBc;
  k_mp_retry<<<gR, kBlock, 0, s->stream>>>(s->st, B, s->partB);
  PDLP_LAUNCH(s);
  if (panT) {
    launch_panel_rows(s, s->KT, s->gA, B.Y[1], B.Y[0], 1, s->partPT, kPredAttempt, kProd);
    PDLP_LAUNCH(s);
    k_mp_kty_combine<<<s->gAc, kBlock, 0, s->stream>>>(s->KT, s->st, B, s->partPT, s->partA);
  } else {
    k_mp_kty<<<s->gA, kBlock, 0, s->stream>>>(s->KT, s->st, B, s->partA);
  }
  PDLP_LAUNCH(s);
  const int nslotB = panK ? s->gBc : s->gB + s->K.nsplit;
  const int nslotA = panT ? s->gAc : s->gA + s->KT.nsplit;
  k_tail<<<1, kBlock, 0, s->stream>>>(s->st, B, kTailMp, 0, s->partB, nslotB, s->partA, nslotA, gR, 0);
  PDLP_LAUNCH(s);
  k_mp_commit<<<s->gAc, kBlock, 0, s->stream>>>(s->st, B);
  PDLP_LAUNCH(s);
  return 0;
}

int enqueue_block(pdlp_solver* s, int par, int slots) {
  const pdlp_options& o = s->opts;
  unsigned* tk = s->tickets;
  Bufs& B = s->B;
  const bool panT = s->KT.npanel > 1, panK = s->K.npanel > 1;
  const int nslotA = panT ? s->gAc : s->gA + s->KT.nsplit;
  const int gDual = panK ? s->gBc : s->gB;
  const int nslotB = panK ? s->gBc : s->gB + s->K.nsplit;
  unsigned* tkDual = ticket_for(s, gDual, kTkDual);
  int rc;
  hipEvent_t* ev = o.time_kernels ? s->tev[par].data() : nullptr;
  auto mark = [&](int i, int j) -> int {
    if (ev) PDLP_HIP(s, hipEventRecord(ev[5 * i + j], s->stream));
    return 0;
  };
  for (int i = 0; i < slots; ++i) {
    if ((rc = mark(i, 0))) return rc;
    if (panT) {
      launch_panel_rows(s, s->KT, s->gA, B.Y[0], B.Y[1], 1, s->partPT, kPredAttemptKty, kProd);
      PDLP_LAUNCH(s);
      if ((rc = mark(i, 1))) return rc;
      k_primal_combine<<<s->gAc, kBlock, 0, s->stream>>>(s->KT, s->st, B, s->partPT, s->partA);
    } else {
      if ((rc = mark(i, 1))) return rc;
      k_primal<<<s->gA, kBlock, 0, s->stream>>>(s->KT, s->st, B, s->partA);
    }
    PDLP_LAUNCH(s);
    if ((rc = mark(i, 2))) return rc;
    if (o.step_policy == 2) {
      if ((rc = mark(i, 3))) return rc;
      if ((rc = enqueue_mp_trial(s))) return rc;
      if ((rc = mark(i, 4))) return rc;
      if (o.trace_iters > 0) {
        k_snapshot<<<s->gE, kBlock, 0, s->stream>>>(s->st, B, tk + kTkSnap);
        PDLP_LAUNCH(s);
      }
      continue;
    }
    if (panK) {
      launch_panel_rows(s, s->K, s->gB, B.X[1], B.X[0], 1, s->partPK, kPredAttempt, kProd);
      PDLP_LAUNCH(s);
      if ((rc = mark(i, 3))) return rc;
      k_dual_combine<<<s->gBc, kBlock, 0, s->stream>>>(s->K, s->st, B, s->partPK, s->partA, nslotA,
                                                       s->partB, tkDual);
    } else {
      if ((rc = mark(i, 3))) return rc;
      k_dual<<<s->gB, kBlock, 0, s->stream>>>(s->K, s->st, B, s->partA, nslotA, s->partB, tkDual);
    }
    PDLP_LAUNCH(s);
    if ((rc = launch_tail(s, gDual, kTailAttempt, 0, s->partB, nslotB, s->partA, nslotA))) return rc;
    if ((rc = mark(i, 4))) return rc;
    if (o.trace_iters > 0) {
      k_snapshot<<<s->gE, kBlock, 0, s->stream>>>(s->st, B, tk + kTkSnap);
      PDLP_LAUNCH(s);
    }
  }
  // restart / termination check
  const int gE = s->gE;
  if (o.adaptive_restarts) {
    k_check_prepare<<<gE, kBlock, 0, s->stream>>>(s->st, B, ticket_for(s, gE, kTkPrep));
    PDLP_LAUNCH(s);
    if ((rc = launch_tail(s, gE, kTailPrepare, 0, nullptr, 0))) return rc;
    if ((rc = launch_spmv(s, s->KT, B.YB, nullptr, 0, B.KTYB, nullptr, 0, kPredCheck, 2))) return rc;
    if ((rc = launch_spmv(s, s->K, B.XB, nullptr, 0, B.KXB, nullptr, 0, kPredCheck, 1))) return rc;
  }
  if ((rc = launch_spmv(s, s->KT, B.Y[0], B.Y[1], 1, B.KTy, nullptr, 0, kPredCheckKty, 2))) return rc;
  if (o.adaptive_restarts && (rc = enqueue_gap(s, 0))) return rc;
  if ((rc = enqueue_kkt(s, 0))) return rc;
  if (o.adaptive_restarts && (rc = enqueue_gap(s, 1))) return rc;
  k_check_apply<<<gE, kBlock, 0, s->stream>>>(s->st, B, ticket_for(s, gE, kTkApply));
  PDLP_LAUNCH(s);
  if ((rc = launch_tail(s, gE, kTailApply, 0, nullptr, 0))) return rc;
  PDLP_HIP(s, hipMemcpyAsync(&s->h_st[par], s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  return 0;
}

// Captures the launch sequence of a block (parity 0 and 1) as two HIP graphs on a private
// stream.  Every kernel reads its go/no-go and its parity-selected buffers from the device
// state, so a block's launches and arguments never change and one capture serves every
// block of the solve.  On any failure the solver keeps launching kernel by kernel.
void capture_block_graphs(pdlp_solver* s) {
  s->graphs_tried = true;
  if (!s->opts.use_graphs) return;
  if (hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    s->cap_stream = nullptr;
    return;
  }
  hipStream_t user = s->stream;
  bool ok = true;
  for (int par = 0; par < 2 && ok; ++par) {
    s->stream = s->cap_stream;
    ok = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    const int rc = ok ? enqueue_block(s, par, s->opts.check_every) : 0;
    hipGraph_t g = nullptr;
    const bool ended = ok && hipStreamEndCapture(s->cap_stream, &g) == hipSuccess;
    ok = ok && rc == 0 && ended && g &&
         hipGraphInstantiate(&s->gexec[par], g, nullptr, nullptr, 0) == hipSuccess;
    s->graph[par] = g;
  }
  s->stream = user;
  if (!ok) {
    (void)hipGetLastError();
    for (int par = 0; par < 2; ++par) {
      if (s->gexec[par]) (void)hipGraphExecDestroy(s->gexec[par]);
      if (s->graph[par]) (void)hipGraphDestroy(s->graph[par]);
      s->gexec[par] = nullptr;
      s->graph[par] = nullptr;
    }
    s->err.clear();
  }
}

// Enqueues block `par` of `slots` attempt slots and its check (the captured graph when the
// block is whole, else kernel by kernel) and the event the host waits on.
int launch_block(pdlp_solver* s, int par, int slots) {
  s->blk_slots[par] = slots;
  if (s->gexec[par] && slots == s->opts.check_every && !s->opts.time_kernels) {
    PDLP_HIP(s, hipGraphLaunch(s->gexec[par], s->stream));
  } else {
    int rc;
    if ((rc = enqueue_block(s, par, slots))) return rc;
  }
  PDLP_HIP(s, hipEventRecord(s->blk_ev[par], s->stream));
  return 0;
}

// Waits for block `par`.  With kernel timing (blocks run one at a time) it adds the event
// times of the slots whose attempt ran: the first (attempts after - attempts before) slots of
// the block, since a slot that does not run (a check pending, the solve over, the iteration
// limit reached) is followed only by slots that do not run either.
// The events of kernel timing: 5 per attempt slot of each of the two block parities.
int make_timing_events(pdlp_solver* s) {
  for (int b = 0; b < 2; ++b) {
    if (!s->tev[b].empty()) continue;
    s->tev[b].assign(size_t(5 * s->opts.check_every), nullptr);
    for (auto& e : s->tev[b]) PDLP_HIP(s, hipEventCreate(&e));
  }
  return 0;
}

int wait_block(pdlp_solver* s, int par) {
  PDLP_HIP(s, hipEventSynchronize(s->blk_ev[par]));
  if (s->opts.time_kernels) {
    const int64_t ran = std::min<int64_t>(s->h_st[par].attempts - s->timed_attempts, s->blk_slots[par]);
    s->timed_attempts = s->h_st[par].attempts;
    for (int i = 0; i < ran; ++i) {
      for (int j = 0; j < 4; ++j) {
        float t = 0.f;
        PDLP_HIP(s, hipEventElapsedTime(&t, s->tev[par][5 * i + j], s->tev[par][5 * i + j + 1]));
        s->t_ms[j] += t;
      }
    }
    for (int j = 0; j < 4; ++j) s->t_cnt[j] += std::max<int64_t>(ran, 0);
  }
  return 0;
}

bool block_stops(const DevState& h) {
  return h.done || (!h.check_pending && h.k >= h.iter_limit);
}

int read_state(const pdlp_solver* s, DevState* out) {
  pdlp_solver* w = const_cast<pdlp_solver*>(s);
  PDLP_HIP(w, hipMemcpyAsync(&w->h_st[0], s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  PDLP_HIP(w, hipStreamSynchronize(s->stream));
  *out = w->h_st[0];
  return 0;
}

int precondition(pdlp_solver* s) {
  const int gK = grid_for(s->K, s->maxG), gT = grid_for(s->KT, s->maxG);
  const int gm = std::max<int64_t>(1, std::min<int64_t>((s->m + kBlock - 1) / kBlock, s->maxG));
  const int gn = std::max<int64_t>(1, std::min<int64_t>((s->n + kBlock - 1) / kBlock, s->maxG));
  double* rn = s->B.GA[0];
  double* cn = s->B.GA[1];
  double* rf = s->B.GB[0];
  double* cf = s->B.GB[1];
  double* D1 = const_cast<double*>(s->B.D1);
  double* D2 = const_cast<double*>(s->B.D2);
  const int passes = s->opts.ruiz_iters + (s->opts.pock_chambolle ? 1 : 0);
  for (int p = 0; p < passes; ++p) {
    const int inf_norm = (p < s->opts.ruiz_iters) ? 1 : 0;
    for (int which = 0; which < 2; ++which) {
      const CsrDev& A = which ? s->KT : s->K;
      double* out = which ? cn : rn;
      if (A.npanel > 1) {
        double* part = which ? s->partPT : s->partPK;
        launch_panel_rows(s, A, which ? gT : gK, nullptr, nullptr, 0, part,
                                                                kPredAlways, inf_norm ? kAbsMax : kAbsSum);
        PDLP_LAUNCH(s);
        k_norm_combine<<<grid_rows(A.nrows_orig, s->maxG), kBlock, 0, s->stream>>>(A, part, out, inf_norm);
      } else {
        k_row_norms<<<which ? gT : gK, kBlock, 0, s->stream>>>(A, out, inf_norm);
      }
      PDLP_LAUNCH(s);
    }
    if (s->m > 0) {
      k_scale_factors<<<gm, kBlock, 0, s->stream>>>(rn, rf, D1, int(s->m));
      PDLP_LAUNCH(s);
    }
    k_scale_factors<<<gn, kBlock, 0, s->stream>>>(cn, cf, D2, int(s->n));
    PDLP_LAUNCH(s);
    k_scale_values<<<gK, kBlock, 0, s->stream>>>(s->K, s->vK, s->vsK, rf, cf, 0);
    PDLP_LAUNCH(s);
    k_scale_values<<<gT, kBlock, 0, s->stream>>>(s->KT, s->vKT, s->vsKT, rf, cf, 1);
    PDLP_LAUNCH(s);
  }
  k_scale_vectors<<<s->gE, kBlock, 0, s->stream>>>(s->B, const_cast<double*>(s->B.c),
                                                   const_cast<double*>(s->B.l),
                                                   const_cast<double*>(s->B.u),
                                                   const_cast<double*>(s->B.q));
  PDLP_LAUNCH(s);
  return 0;
}

int create_impl(pdlp_solver* s, int64_t m, int64_t n, int64_t n_eq, const double* c,
                const int64_t* row_ptr, const int32_t* col_idx, const double* val, const double* q,
                const double* l, const double* u) {
  if (!c || !row_ptr || !l || !u || (m > 0 && !q)) {
    s->err = "null input pointer";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  if (n < 1 || m < 0 || n_eq < 0 || n_eq > m || m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31)) {
    s->err = "invalid sizes (need n >= 1, m >= 0, 0 <= n_eq <= m, m, n < 2^31)";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  int rc;
  std::vector<int64_t> t_rp;
  std::vector<int32_t> t_ci;
  std::vector<double> t_v, t_c, t_q, t_l, t_u;
  const int64_t* rp;
  if ((rc = fetch_input(s, row_ptr, size_t(m) + 1, t_rp, &rp))) return rc;
  const int64_t nnz = rp[m];
  if (rp[0] != 0 || nnz < 0) {
    s->err = "row_ptr[0] must be 0 and row_ptr[m] >= 0";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  if (nnz > 0 && (!col_idx || !val)) {
    s->err = "null col_idx or val";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  const int32_t* ci;
  const double *v, *hc, *hq, *hl, *hu;
  if ((rc = fetch_input(s, col_idx, size_t(nnz), t_ci, &ci))) return rc;
  if ((rc = fetch_input(s, val, size_t(nnz), t_v, &v))) return rc;
  if ((rc = fetch_input(s, c, size_t(n), t_c, &hc))) return rc;
  if ((rc = fetch_input(s, q, size_t(m), t_q, &hq))) return rc;
  if ((rc = fetch_input(s, l, size_t(n), t_l, &hl))) return rc;
  if ((rc = fetch_input(s, u, size_t(n), t_u, &hu))) return rc;
  const std::string bad = validate_lp(m, n, n_eq, hc, rp, ci, v, hq, hl, hu);
  if (!bad.empty()) {
    s->err = bad;
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  s->m = m;
  s->n = n;
  s->n_eq = n_eq;
  s->nnz = nnz;

  // internal column order: each XCD panel's columns with the most nonzeros first, so the
  // gathers of the K~ x products that hit the dense columns stay in a small slice of x
  const int co = s->opts.column_order;
  const bool reorder = nnz > 0 && (co == 1 || (co < 0 && s->opts.xcd_panels != 0 &&
                                               (s->opts.xcd_panels == 1 || n * 8 > (int64_t(4) << 20))));
  std::vector<int32_t> ci_r, cuts;
  std::vector<double> c_r, l_r, u_r, v_r;
  if (reorder) {
    cuts = panel_cuts(ci, nnz, n, kMaxPanels);     // of the user's order; kept for the panels
    s->col_user = hot_column_order(ci, nnz, n, cuts);
    s->col_int.assign(size_t(n), 0);
    for (int64_t j = 0; j < n; ++j) s->col_int[size_t(s->col_user[size_t(j)])] = int32_t(j);
    // each row's entries in the new column order (hot columns of a panel first); the panel of
    // an entry still never decreases along a row.  Rows in parallel chunks.
    ci_r.resize(static_cast<size_t>(nnz));
    v_r.resize(static_cast<size_t>(nnz));
    parallel_for(m, [&](int64_t i0, int64_t i1) {
      std::vector<std::pair<int32_t, double>> tmp;
      for (int64_t i = i0; i < i1; ++i) {
        const int64_t a = rp[i], b = rp[i + 1];
        tmp.clear();
        for (int64_t e = a; e < b; ++e) tmp.emplace_back(s->col_int[size_t(ci[e])], v[e]);
        std::sort(tmp.begin(), tmp.end());
        for (int64_t e = a; e < b; ++e) {
          ci_r[size_t(e)] = tmp[size_t(e - a)].first;
          v_r[size_t(e)] = tmp[size_t(e - a)].second;
        }
      }
    }, int64_t(1) << 12);
    v = v_r.data();
    c_r.resize(size_t(n));
    l_r.resize(size_t(n));
    u_r.resize(size_t(n));
    for (int64_t j = 0; j < n; ++j) {
      const size_t uj = size_t(s->col_user[size_t(j)]);
      c_r[size_t(j)] = hc[uj];
      l_r[size_t(j)] = hl[uj];
      u_r[size_t(j)] = hu[uj];
    }
    ci = ci_r.data();
    hc = c_r.data();
    hl = l_r.data();
    hu = u_r.data();
    if ((rc = upload_vec(s, s->col_user, &s->d_col_user)) || (rc = upload_vec(s, s->col_int, &s->d_col_int)))
      return rc;
    PDLP_HIP(s, s->alloc(&s->permbuf, size_t(n)));
  }

  std::vector<int64_t> rpT;
  std::vector<int32_t> ciT;
  std::vector<double> vT;
  transpose_csr(m, n, rp, ci, v, rpT, ciT, vT);

  int dev = 0;
  PDLP_HIP(s, hipGetDevice(&dev));
  s->device = dev;
  scratch_setup(dev);
  int ncu = 0;
  PDLP_HIP(s, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  s->maxG = std::max(1, ncu * 8);

  // the two CSR copies (K~ and K~^T), each in the plain or the XCD-panel layout
  if ((rc = upload_copy(s, m, n, rp, ci, v, s->K, &s->vK, &s->vsK, &s->partPK, reorder ? &cuts : nullptr,
                        reorder)))
    return rc;
  if ((rc = upload_copy(s, n, m, rpT.data(), ciT.data(), vT.data(), s->KT, &s->vKT, &s->vsKT, &s->partPT)))
    return rc;
  std::vector<int64_t>().swap(rpT);
  std::vector<int32_t>().swap(ciT);
  std::vector<double>().swap(vT);

  // vectors
  Bufs& B = s->B;
  B.n = int32_t(n);
  B.m = int32_t(m);
  B.m1 = int32_t(m - n_eq);
  const size_t N = size_t(n), M = size_t(m), NM = size_t(n + m);
  double *c_, *l_, *u_, *q_, *c0, *l0, *u0, *q0, *D1, *D2;
  PDLP_HIP(s, s->alloc(&c_, N));
  PDLP_HIP(s, s->alloc(&l_, N));
  PDLP_HIP(s, s->alloc(&u_, N));
  PDLP_HIP(s, s->alloc(&q_, M));
  PDLP_HIP(s, s->alloc(&c0, N));
  PDLP_HIP(s, s->alloc(&l0, N));
  PDLP_HIP(s, s->alloc(&u0, N));
  PDLP_HIP(s, s->alloc(&q0, M));
  PDLP_HIP(s, s->alloc(&D1, M));
  PDLP_HIP(s, s->alloc(&D2, N));
  B.c = c_; B.l = l_; B.u = u_; B.q = q_;
  B.c0 = c0; B.l0 = l0; B.u0 = u0; B.q0 = q0;
  B.D1 = D1; B.D2 = D2;
  for (int p = 0; p < 2; ++p) {
    PDLP_HIP(s, s->alloc(&B.X[p], N));
    PDLP_HIP(s, s->alloc(&B.Y[p], M));
    PDLP_HIP(s, s->alloc(&B.KX[p], M));
    PDLP_HIP(s, s->alloc(&B.GA[p], NM));
    PDLP_HIP(s, s->alloc(&B.GB[p], NM));
  }
  PDLP_HIP(s, s->alloc(&B.KTy, N));
  PDLP_HIP(s, s->alloc(&B.KTyH, N));
  PDLP_HIP(s, s->alloc(&B.Sx, N));
  PDLP_HIP(s, s->alloc(&B.Sy, M));
  PDLP_HIP(s, s->alloc(&B.XB, N));
  PDLP_HIP(s, s->alloc(&B.YB, M));
  PDLP_HIP(s, s->alloc(&B.KXB, M));
  PDLP_HIP(s, s->alloc(&B.KTYB, N));
  PDLP_HIP(s, s->alloc(&B.XA, N));
  PDLP_HIP(s, s->alloc(&B.YA, M));
  PDLP_HIP(s, s->alloc(&s->outbuf, NM));
  const int cap = std::max(0, s->opts.trace_capacity);
  PDLP_HIP(s, s->alloc(&B.att, size_t(std::max(cap, 1))));
  PDLP_HIP(s, s->alloc(&B.chk, size_t(std::max(cap, 1))));
  const size_t ti = size_t(std::max(0, s->opts.trace_iters));
  PDLP_HIP(s, s->alloc(&B.tx, ti * N));
  PDLP_HIP(s, s->alloc(&B.ty, ti * M));
  PDLP_HIP(s, hipMemcpy(c0, hc, N * 8, hipMemcpyHostToDevice));
  PDLP_HIP(s, hipMemcpy(l0, hl, N * 8, hipMemcpyHostToDevice));
  PDLP_HIP(s, hipMemcpy(u0, hu, N * 8, hipMemcpyHostToDevice));
  if (m > 0) PDLP_HIP(s, hipMemcpy(q0, hq, M * 8, hipMemcpyHostToDevice));
  {
    std::vector<double> ones(std::max(N, M), 1.0);
    PDLP_HIP(s, hipMemcpy(D2, ones.data(), N * 8, hipMemcpyHostToDevice));
    if (m > 0) PDLP_HIP(s, hipMemcpy(D1, ones.data(), M * 8, hipMemcpyHostToDevice));
  }

  // grids and reduction scratch
  s->gA = grid_for(s->KT, s->maxG);
  s->gB = grid_for(s->K, s->maxG);
  s->gAc = grid_rows(n, s->maxG);
  s->gBc = grid_rows(m, s->maxG);
  s->gE = int(std::max<int64_t>(1, std::min<int64_t>(int64_t((NM + kBlock - 1) / kBlock), s->maxG)));
  PDLP_HIP(s, s->alloc(&s->partA, size_t(std::max(s->gA + s->KT.nsplit, s->gAc))));
  PDLP_HIP(s, s->alloc(&s->partB, size_t(std::max(s->gB + s->K.nsplit, s->gBc)) * 2));
  PDLP_HIP(s, s->alloc(&s->partX, size_t(s->gE) * 64));
  PDLP_HIP(s, s->alloc(&s->tickets, size_t(kNumTickets)));
  PDLP_HIP(s, hipMemset(s->tickets, 0, kNumTickets * sizeof(unsigned)));

  // device state
  DevState h{};
  h.mu_prev = INFINITY;
  h.mu_anchor = INFINITY;
  h.tol = 0.0;
  h.iter_limit = 0;
  h.kty_valid = 1;
  h.status = PDLP_NOT_SOLVED;
  h.check_every = s->opts.check_every;
  h.max_retries = s->opts.max_retries;
  h.trace_iters = s->opts.trace_iters;
  h.trace_cap = cap;
  h.restarts_on = s->opts.adaptive_restarts;
  h.constant_step = s->opts.step_policy == 1;
  h.mp_on = s->opts.step_policy == 2;
  h.pw_pow2 = s->opts.pw_power_of_two;
  h.mp_theta = 1.0;
  h.mp_bf = s->opts.mp_breaking_factor;
  h.mp_df = s->opts.mp_downscaling;
  h.mp_ic = s->opts.mp_interpolation;
  h.to_current = s->opts.restart_to_current != 0;
  h.pw_on = s->opts.primal_weight_update;
  h.beta_suff = s->opts.beta_sufficient;
  h.beta_nec = s->opts.beta_necessary;
  h.beta_art = s->opts.beta_artificial;
  h.theta = s->opts.theta;
  h.eps_zero = s->opts.eps_zero;
  PDLP_HIP(s, s->alloc(&s->st, 1));
  PDLP_HIP(s, hipMemcpy(s->st, &h, sizeof(DevState), hipMemcpyHostToDevice));
  PDLP_HIP(s, hipHostMalloc(reinterpret_cast<void**>(&s->h_st), 2 * sizeof(DevState), hipHostMallocDefault));
  for (int b = 0; b < 2; ++b) PDLP_HIP(s, hipEventCreate(&s->blk_ev[b]));
  if (s->opts.time_kernels && (rc = make_timing_events(s))) return rc;

  // preconditioning, then x0 = proj_X(0), y0 = 0 and K x0
  if ((rc = precondition(s))) return rc;
  k_init<<<s->gE, kBlock, 0, s->stream>>>(s->K, s->st, B, s->partX, s->tickets + kTkInit,
                                          s->opts.primal_importance, s->opts.eps_zero);
  PDLP_LAUNCH(s);
  if ((rc = launch_spmv(s, s->K, B.X[0], nullptr, 0, B.KX[0], nullptr, 0, kPredAlways, 0))) return rc;
  if (s->opts.step_policy == 1) {
    // baseline PDHG step 0.9 / ||K~||_2, using the gap scratch buffers (free until the first check)
    if ((rc = power_iterate(s, B.GA[0], B.GB[0], B.GA[1]))) return rc;
    k_pow_set_step<<<1, 1, 0, s->stream>>>(s->st);
    PDLP_LAUNCH(s);
  }
  PDLP_HIP(s, hipStreamSynchronize(s->stream));
  PDLP_HIP(s, hipMemcpy(&s->omega0, &s->st->omega, sizeof(double), hipMemcpyDeviceToHost));
  if (s->opts.step_policy == 1) PDLP_HIP(s, hipMemcpy(&s->eta_pow, &s->st->eta, sizeof(double), hipMemcpyDeviceToHost));

  s->bytes_A = 8.0 * double(n + 1) + 12.0 * double(nnz) + 8.0 * double(m) + 64.0 * double(n);
  s->bytes_B = 8.0 * double(m + 1) + 12.0 * double(nnz) + 8.0 * double(n) + 56.0 * double(m);
  return 0;
}

// ------------------------------------------------------------------------------------------
// unrolled PDHG with frozen eta, omega, D1, D2 and its adjoint
// ------------------------------------------------------------------------------------------

template <class T>
int unroll_alloc(pdlp_solver* s, T** p, size_t count) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e != hipSuccess) {
    s->err = std::string("hipMalloc (unroll buffers): ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PDLP_ERR_OUT_OF_MEMORY : PDLP_ERR_DEVICE;
  }
  s->U.allocs.push_back(*p);
  s->U.bytes += double(bytes);
  return 0;
}

// Buffers for nseg checkpoints and segments of S steps; kept while large enough.
int unroll_reserve(pdlp_solver* s, int64_t nseg, int64_t S) {
  auto& U = s->U;
  const size_t N = size_t(s->n), M = size_t(s->m);
  int rc;
  if (U.cap_seg < 0) {
    if ((rc = unroll_alloc(s, &U.own.ct, N)) || (rc = unroll_alloc(s, &U.own.qt, M)) ||
        (rc = unroll_alloc(s, &U.own.gin, N + M)) || (rc = unroll_alloc(s, &U.own.z, N + 2 * M)) ||
        (rc = unroll_alloc(s, &U.own.xb, N)) || (rc = unroll_alloc(s, &U.own.ub, N)) ||
        (rc = unroll_alloc(s, &U.own.vb, M)) || (rc = unroll_alloc(s, &U.own.cb, N + M)) ||
        (rc = unroll_alloc(s, &U.own.out, N + M)))
      return rc;
    U.cap_seg = 0;
    U.cap_S = 0;
  }
  if (nseg > U.cap_seg) {
    if (U.own.ck) {
      PDLP_HIP(s, hipStreamSynchronize(s->stream));
      PDLP_HIP(s, hipFree(U.own.ck));
      U.allocs.erase(std::find(U.allocs.begin(), U.allocs.end(), static_cast<void*>(U.own.ck)));
      U.bytes -= double(std::max<int64_t>(U.cap_seg, 1)) * double(N + 2 * M) * 8.0;
      U.own.ck = nullptr;
    }
    if ((rc = unroll_alloc(s, &U.own.ck, size_t(nseg) * (N + 2 * M)))) return rc;
    U.cap_seg = nseg;
  }
  if (S > U.cap_S) {
    if (U.own.mask) {
      PDLP_HIP(s, hipStreamSynchronize(s->stream));
      PDLP_HIP(s, hipFree(U.own.mask));
      U.allocs.erase(std::find(U.allocs.begin(), U.allocs.end(), static_cast<void*>(U.own.mask)));
      U.bytes -= double(std::max<int64_t>(U.cap_S, 1)) * double(N + M);
      U.own.mask = nullptr;
    }
    if ((rc = unroll_alloc(s, &U.own.mask, size_t(S) * (N + M)))) return rc;
    U.cap_S = S;
  }
  return 0;
}

// The buffers of an unrolled pass with nseg checkpoints and segments of S steps, carved from
// the per-GPU scratch array instead of allocated.  Fails (nothing enqueued, nothing claimed)
// when they exceed the array.
int unroll_carve_scratch(pdlp_solver* s, int64_t nseg, int64_t S) {
  auto& U = s->U;
  const double N = double(s->n), M = double(s->m);
  // 256-byte aligned pieces: nine vectors of n and m values, the checkpoints, the masks
  const double lens[11] = {N, M, N + M, N + 2 * M, N, N, M, N + M, N + M, double(nseg) * (N + 2 * M),
                           0.0};
  double need = 0.0;
  for (int i = 0; i < 10; ++i) need += std::ceil(lens[i] * 8.0 / 256.0) * 256.0;
  need += std::ceil(double(S) * (N + M) / 256.0) * 256.0;
  if (need > double(kScratchBytes)) {
    s->err = "unroll (no-alloc): the buffers need " + std::to_string(int64_t(need)) +
             " bytes, more than the " + std::to_string(kScratchBytes) +
             "-byte scratch array (fewer checkpoints or a shorter segment need less)";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  unsigned char* base = nullptr;
  {
    const int dev = s->device;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchSlot* sl = (dev >= 0 && dev < kMaxScratchDevices) ? &g_scratch[dev] : nullptr;
    if (!sl || !sl->ptr) {
      s->err = std::string("unroll (no-alloc): no scratch array on this GPU: ") +
               (sl && sl->tried ? hipGetErrorString(sl->err) : "device index out of range");
      return PDLP_ERR_DEVICE;
    }
    sl->gen += 1;
    U.scratch_gen = sl->gen;
    base = sl->ptr;
  }
  size_t off = 0;
  auto take = [&](double len_bytes) {
    unsigned char* p = base + off;
    off += size_t(std::ceil(len_bytes / 256.0) * 256.0);
    return p;
  };
  auto takev = [&](double len) { return reinterpret_cast<double*>(take(len * 8.0)); };
  U.b.ct = takev(lens[0]);
  U.b.qt = takev(lens[1]);
  U.b.gin = takev(lens[2]);
  U.b.z = takev(lens[3]);
  U.b.xb = takev(lens[4]);
  U.b.ub = takev(lens[5]);
  U.b.vb = takev(lens[6]);
  U.b.cb = takev(lens[7]);
  U.b.out = takev(lens[8]);
  U.b.ck = takev(lens[9]);
  U.b.mask = take(double(S) * (N + M));
  U.in_scratch = true;
  return 0;
}

// The scratch array still holds the buffers of this solver's last no-alloc forward pass.
bool unroll_scratch_owned(const pdlp_solver* s) {
  const int dev = s->device;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return dev >= 0 && dev < kMaxScratchDevices && g_scratch[dev].gen == s->U.scratch_gen;
}

// One fused CSR pass: out rows of A from the product with `in`, then epi.row per row.
template <class Epi>
int launch_fused(pdlp_solver* s, const CsrDev& A, const double* in, const Epi& epi) {
  if (A.npanel > 1) {
    double* part = (&A == &s->K) ? s->partPK : s->partPT;
    launch_panel_rows(s, A, grid_for(A, s->maxG), in, nullptr, 0, part,
                                                               kPredAlways, kProd);
    PDLP_LAUNCH(s);
    k_unroll_combine<Epi><<<grid_rows(A.nrows_orig, s->maxG), kBlock, 0, s->stream>>>(A, part, epi);
    PDLP_LAUNCH(s);
    return 0;
  }
  k_unroll_rows<Epi><<<grid_for(A, s->maxG), kBlock, 0, s->stream>>>(A, in, epi);
  PDLP_LAUNCH(s);
  return 0;
}

int unroll_copy(pdlp_solver* s, const double* src, double* dst, int64_t len) {
  const int g = int(std::max<int64_t>(1, std::min<int64_t>((len + kBlock - 1) / kBlock, s->maxG)));
  k_unroll_copy<<<g, kBlock, 0, s->stream>>>(src, dst, len);
  PDLP_LAUNCH(s);
  return 0;
}

// Forward step t -> t + 1 on U.b.z, recording the projection masks into `slot` (n + m bytes).
int unroll_fwd_step(pdlp_solver* s, uint8_t* slot) {
  auto& U = s->U;
  int rc;
  double* x = U.b.z;
  double* y = U.b.z + s->n;
  double* kx = U.b.z + s->n + s->m;
  const UFwdPrimal ep{U.b.ct, s->B.l, s->B.u, x, slot, U.eta / U.omega};
  if ((rc = launch_fused(s, s->KT, y, ep))) return rc;
  const UFwdDual ed{U.b.qt, y, kx, slot + s->n, U.eta * U.omega, s->B.m1};
  return launch_fused(s, s->K, x, ed);
}

// Stage a caller's vector (host or device, len values) in device memory.
int stage_in(pdlp_solver* s, const double* src, double* dst, int64_t len) {
  if (len == 0) return 0;
  const hipMemcpyKind kind = is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  PDLP_HIP(s, hipMemcpyAsync(dst, src, size_t(len) * 8, kind, s->stream));
  return 0;
}

int unroll_forward_impl(pdlp_solver* s, const double* c, const double* q, int64_t T, int64_t segment,
                        double eta, double omega, double* x_T, double* y_T, bool noalloc) {
  auto& U = s->U;
  int rc;
  if (T < 0 || segment < 0 || !(std::isfinite(eta) && std::isfinite(omega))) {
    s->err = "unroll: need steps >= 0, segment >= 0 and finite eta, omega";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  const int64_t n = s->n, m = s->m;
  const int64_t S = std::max<int64_t>(1, segment == 0 ? T : std::min(segment, std::max<int64_t>(T, 1)));
  const int64_t nseg = (T + S - 1) / S;
  const double t0 = now_s();
  U.ready = false;
  if (noalloc) {
    if ((rc = unroll_carve_scratch(s, std::max<int64_t>(nseg, 1), S))) return rc;
  } else {
    if ((rc = unroll_reserve(s, std::max<int64_t>(nseg, 1), S))) return rc;
    U.b = U.own;
    U.in_scratch = false;
  }
  if (eta <= 0.0) {
    if (s->eta_pow <= 0.0) {
      if ((rc = power_iterate(s, U.b.xb, U.b.vb, U.b.ub))) return rc;
      double pn2 = 0.0;
      PDLP_HIP(s, hipMemcpyAsync(&pn2, &s->st->pow_norm2, sizeof(double), hipMemcpyDeviceToHost, s->stream));
      PDLP_HIP(s, hipStreamSynchronize(s->stream));
      const double sig = std::sqrt(std::sqrt(pn2));
      s->eta_pow = sig > 0.0 ? 0.9 / sig : 1.0;
    }
    eta = s->eta_pow;
  }
  if (omega <= 0.0) omega = s->omega0;
  U.eta = eta;
  U.omega = omega;
  U.T = T;
  U.S = S;
  U.nseg = nseg;
  // c~ = D2 c, q~ = D1 q (the LP's own c, q when null), z0 = (proj_X(0), 0, K~ proj_X(0))
  if (c) {
    if ((rc = read_n(s, c, U.b.gin))) return rc;
  } else if ((rc = stage_in(s, s->B.c0, U.b.gin, n))) {
    return rc;
  }
  if ((rc = stage_in(s, q ? q : s->B.q0, U.b.gin + n, m))) return rc;
  const int gE = s->gE;
  k_unroll_start<<<gE, kBlock, 0, s->stream>>>(U.b.gin, U.b.gin + n, s->B.D1, s->B.D2, s->B.l, s->B.u, U.b.ct,
                                               U.b.qt, U.b.z, U.b.z + n, int(n), int(m));
  PDLP_LAUNCH(s);
  if ((rc = launch_spmv(s, s->K, U.b.z, nullptr, 0, U.b.z + n + m, nullptr, 0, kPredAlways, 0))) return rc;
  const int64_t zlen = n + 2 * m;
  for (int64_t t = 0; t < T; ++t) {
    if (t % S == 0 && (rc = unroll_copy(s, U.b.z, U.b.ck + (t / S) * zlen, zlen))) return rc;
    if ((rc = unroll_fwd_step(s, U.b.mask + (t % S) * (n + m)))) return rc;
  }
  k_unroll_unscale<<<gE, kBlock, 0, s->stream>>>(U.b.z, s->B.D2, int(n), U.b.z + n, s->B.D1, int(m), U.b.out);
  PDLP_LAUNCH(s);
  if ((rc = write_n(s, x_T, U.b.out))) return rc;
  if ((rc = write_output(s, y_T, U.b.out + n, size_t(m) * 8))) return rc;
  PDLP_HIP(s, hipStreamSynchronize(s->stream));
  U.ready = true;
  U.masks_last = true;
  U.fwd_s = now_s() - t0;
  return 0;
}

int unroll_backward_impl(pdlp_solver* s, const double* gx, const double* gy, double* gc, double* gq) {
  auto& U = s->U;
  int rc;
  if (!U.ready) {
    s->err = "unroll backward: no forward pass to differentiate";
    return PDLP_ERR_INVALID_STATE;
  }
  if (U.in_scratch && !unroll_scratch_owned(s)) {
    U.ready = false;
    s->err = "unroll backward: another pdlp_unroll_forward_noalloc call on this GPU has reused the "
             "scratch array since the forward pass";
    return PDLP_ERR_INVALID_STATE;
  }
  const int64_t n = s->n, m = s->m, nm = n + m, zlen = n + 2 * m;
  const double t0 = now_s();
  const double tau = U.eta / U.omega, sigma = U.eta * U.omega;
  const int gE = s->gE;
  if (gx && (rc = read_n(s, gx, U.b.gin))) return rc;
  if (gy && (rc = stage_in(s, gy, U.b.gin + n, m))) return rc;
  U.recomputed = 0;
  if (U.nseg == 0) {
    // x_0 = proj_X(0) does not depend on (c, q)
    k_unroll_seed<<<gE, kBlock, 0, s->stream>>>(nullptr, nullptr, s->B.D1, s->B.D2, U.b.mask, U.b.xb, U.b.vb,
                                                U.b.cb, U.b.cb + n, int(n), int(m), s->B.m1);
    PDLP_LAUNCH(s);
  }
  for (int64_t seg = U.nseg - 1; seg >= 0; --seg) {
    const int64_t ta = seg * U.S, tb = std::min(U.T, ta + U.S);
    const bool last = seg == U.nseg - 1;
    if (!(last && U.masks_last)) {
      if ((rc = unroll_copy(s, U.b.ck + seg * zlen, U.b.z, zlen))) return rc;
      for (int64_t t = ta; t < tb; ++t)
        if ((rc = unroll_fwd_step(s, U.b.mask + (t - ta) * nm))) return rc;
      U.recomputed += tb - ta;
    }
    if (last) {
      k_unroll_seed<<<gE, kBlock, 0, s->stream>>>(gx ? U.b.gin : nullptr, gy ? U.b.gin + n : nullptr, s->B.D1,
                                                  s->B.D2, U.b.mask + (tb - 1 - ta) * nm + n, U.b.xb, U.b.vb, U.b.cb,
                                                  U.b.cb + n, int(n), int(m), s->B.m1);
      PDLP_LAUNCH(s);
    }
    for (int64_t t = tb - 1; t >= ta; --t) {
      const uint8_t* slot = U.b.mask + (t - ta) * nm;
      const UBwdPrimal ep{slot, U.b.xb, U.b.ub, U.b.cb, tau, sigma};
      if ((rc = launch_fused(s, s->KT, U.b.vb, ep))) return rc;
      const uint8_t* my_prev = (t > ta) ? slot - nm + n : nullptr;
      const double* y_prev = (t == ta && t > 0) ? U.b.ck + seg * zlen + n : nullptr;
      const UBwdDual ed{U.b.vb, U.b.cb + n, my_prev, y_prev, tau, sigma, s->B.m1};
      if ((rc = launch_fused(s, s->K, U.b.ub, ed))) return rc;
    }
  }
  U.masks_last = U.nseg == 1;
  k_unroll_unscale<<<gE, kBlock, 0, s->stream>>>(U.b.cb, s->B.D2, int(n), U.b.cb + n, s->B.D1, int(m), U.b.out);
  PDLP_LAUNCH(s);
  if ((rc = write_n(s, gc, U.b.out))) return rc;
  if ((rc = write_output(s, gq, U.b.out + n, size_t(m) * 8))) return rc;
  PDLP_HIP(s, hipStreamSynchronize(s->stream));
  U.bwd_s = now_s() - t0;
  return 0;
}

// The KKT error of the returned point when the solve ended without a terminating check: the
// current iterate, which needs K~^T y of the current y.  That product is formed for the
// evaluation only: it is not counted as a product of the iteration and leaves K~^T y marked
// as not formed, so the next step of a later solve forms it as if nothing had been asked.
int settle_kkt(pdlp_solver* s) {
  if (!s->kkt_stale) return 0;
  int rc;
  if ((rc = launch_spmv(s, s->KT, s->B.Y[0], s->B.Y[1], 1, s->B.KTy, nullptr, 0, kPredKtyPeek, 0))) return rc;
  if ((rc = enqueue_kkt(s, 2))) return rc;
  s->kkt_stale = false;
  return 0;
}

}  // namespace

extern "C" {

void pdlp_default_options(pdlp_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->ruiz_iters = 10;
  o->pock_chambolle = 1;
  o->adaptive_restarts = 1;
  o->primal_weight_update = 1;
  o->check_every = 40;
  o->max_retries = 100;
  o->trace_iters = 0;
  o->trace_capacity = 4096;
  o->time_kernels = 0;
  o->xcd_panels = -1;
  o->step_policy = 0;
  o->mp_breaking_factor = 1.0;
  o->mp_downscaling = 0.5;
  o->mp_interpolation = 0.4;
  o->restart_to_current = 1;
  o->power_iters = 200;
  o->use_graphs = 1;
  o->column_order = -1;
  o->lds_gather = -1;
  o->lds_entries = 0;
  o->xcd_subpanels = -1;
  o->beta_sufficient = 0.1;
  o->beta_necessary = 0.9;
  o->beta_artificial = 0.5;
  o->theta = 0.5;
  o->primal_importance = 1.0;
  o->eps_zero = 1e-10;
}

int pdlp_create(pdlp_solver** out, int64_t m, int64_t n, int64_t n_eq, const double* c,
                const int64_t* row_ptr, const int32_t* col_idx, const double* val, const double* q,
                const double* l, const double* u, const pdlp_options* opts, void* hip_stream) {
  if (!out) {
    g_create_error = "out is NULL";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  *out = nullptr;
  const double t0 = now_s();
  pdlp_solver* s = nullptr;
  try {
    s = new pdlp_solver();
  } catch (...) {
    g_create_error = "host allocation failed";
    return PDLP_ERR_OUT_OF_MEMORY;
  }
  if (opts) s->opts = *opts;
  else pdlp_default_options(&s->opts);
  if (!options_valid(s->opts)) {
    g_create_error = "invalid options";
    delete s;
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  s->stream = static_cast<hipStream_t>(hip_stream);
  int rc;
  try {
    rc = create_impl(s, m, n, n_eq, c, row_ptr, col_idx, val, q, l, u);
  } catch (const std::bad_alloc&) {
    s->err = "host allocation failed";
    rc = PDLP_ERR_OUT_OF_MEMORY;
  } catch (...) {
    s->err = "unexpected host exception";
    rc = PDLP_ERR_DEVICE;
  }
  if (rc != 0) {
    g_create_error = s->err;
    delete s;
    return rc;
  }
  s->create_seconds = now_s() - t0;
  *out = s;
  return 0;
}

int pdlp_solve(pdlp_solver* s, double tol, int64_t iter_limit) {
  if (!s) return PDLP_ERR_INVALID_ARGUMENT;
  if (!(tol >= 0.0) || iter_limit < 0) {
    s->err = "tol must be >= 0 and iter_limit >= 0";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  const double t0 = now_s();
  int rc;
  k_set_solve_params<<<1, 1, 0, s->stream>>>(s->st, tol, iter_limit);
  PDLP_LAUNCH(s);
  if (!s->initial_checked) {
    if ((rc = enqueue_kkt(s, 1))) return rc;
    s->initial_checked = true;
  }
  DevState h;
  if ((rc = read_state(s, &h))) return rc;
  s->timed_attempts = h.attempts;
  if (!block_stops(h)) {
    if (!s->graphs_tried && !s->opts.time_kernels) capture_block_graphs(s);
    // Blocks of check_every attempt slots, two in flight (one at a time with kernel timing).
    // k_hi bounds k from above once every enqueued slot has run (a slot takes at most one
    // step); a block is cut to iter_limit - k_hi slots when fewer remain, and when k_hi has
    // reached the limit the host waits for the running block before enqueueing another.
    const bool pipelined = !s->opts.time_kernels;
    int64_t k_hi = h.k;
    int inflight = -1;
    for (int b = 0;; ++b) {
      const int par = b & 1;
      if (inflight >= 0 && (!pipelined || k_hi >= iter_limit)) {
        if ((rc = wait_block(s, inflight))) return rc;
        const DevState& hb = s->h_st[inflight];
        inflight = -1;
        if (block_stops(hb)) break;
        k_hi = hb.k;
      }
      const int64_t room = iter_limit - k_hi;
      const int slots = int(std::max<int64_t>(1, std::min<int64_t>(s->opts.check_every, room)));
      if ((rc = launch_block(s, par, slots))) return rc;
      k_hi += slots;
      if (inflight >= 0) {
        if ((rc = wait_block(s, inflight))) return rc;
        if (block_stops(s->h_st[inflight])) {
          inflight = par;
          break;
        }
      }
      inflight = par;
    }
    if (inflight >= 0 && (rc = wait_block(s, inflight))) return rc;
  }
  k_mark_limit<<<1, 1, 0, s->stream>>>(s->st);
  PDLP_LAUNCH(s);
  if ((rc = read_state(s, &h))) return rc;
  // the KKT error of a returned current iterate (not a terminating check's candidate) is
  // evaluated when first asked for (pdlp_get, pdlp_get_info)
  s->kkt_stale = h.status != PDLP_OPTIMAL;
  s->solved = true;
  s->last_status = h.status;
  s->solve_seconds = now_s() - t0;
  return h.status;
}

int pdlp_get(const pdlp_solver* cs, double* x, double* y, double* kkt) {
  if (!cs) return PDLP_ERR_INVALID_ARGUMENT;
  pdlp_solver* s = const_cast<pdlp_solver*>(cs);
  if (!s->solved) {
    s->err = "pdlp_get before pdlp_solve";
    return PDLP_ERR_INVALID_STATE;
  }
  int rc;
  if (x || y) {
    k_output<<<s->gE, kBlock, 0, s->stream>>>(s->st, s->B, s->outbuf, s->outbuf + s->n, 0);
    PDLP_LAUNCH(s);
    if ((rc = write_n(s, x, s->outbuf))) return rc;
    if ((rc = write_output(s, y, s->outbuf + s->n, size_t(s->m) * 8))) return rc;
  }
  if (kkt) {
    DevState h;
    if ((rc = settle_kkt(s))) return rc;
    if ((rc = read_state(s, &h))) return rc;
    if (is_device_ptr(kkt)) PDLP_HIP(s, hipMemcpy(kkt, h.kkt, 4 * 8, hipMemcpyHostToDevice));
    else std::memcpy(kkt, h.kkt, 4 * 8);
  }
  return 0;
}

int pdlp_get_info(const pdlp_solver* cs, pdlp_info* info) {
  if (!cs || !info) return PDLP_ERR_INVALID_ARGUMENT;
  DevState h;
  int rc;
  if ((rc = settle_kkt(const_cast<pdlp_solver*>(cs)))) return rc;
  if ((rc = read_state(cs, &h))) return rc;
  std::memset(info, 0, sizeof(*info));
  info->status = cs->last_status;
  info->output_is_average = h.out_avg;
  info->m = cs->m;
  info->n = cs->n;
  info->n_eq = cs->n_eq;
  info->nnz = cs->nnz;
  info->iterations = h.k;
  info->attempts = h.attempts;
  info->restarts = h.n_outer;
  info->checks = h.checks;
  info->spmv_K = h.spmv_K;
  info->spmv_KT = h.spmv_KT;
  info->omega = h.omega;
  info->eta_hat = h.eta_hat;
  for (int i = 0; i < 4; ++i) info->kkt[i] = h.kkt[i];
  info->create_seconds = cs->create_seconds;
  info->solve_seconds = cs->solve_seconds;
  info->step_bytes = cs->bytes_A + cs->bytes_B;
  auto layout = [](const CsrDev& A) {
    if (A.npanel <= 1) return 0;
    if (A.lds_h <= 0) return 1;
    return A.cis16 ? 2 : 3;
  };
  info->layout_K = layout(cs->K);
  info->layout_KT = layout(cs->KT);
  info->panels_K = std::max(1, cs->K.npanel);
  info->panels_KT = std::max(1, cs->KT.npanel);
  return 0;
}

void pdlp_destroy(pdlp_solver* s) { delete s; }

const char* pdlp_last_error(const pdlp_solver* s) {
  if (!s) return g_create_error.c_str();
  return s->err.c_str();
}

int pdlp_get_state(const pdlp_solver* cs, double* x, double* y, double* xa, double* ya, double* sx,
                   double* sy, pdlp_state* out) {
  if (!cs) return PDLP_ERR_INVALID_ARGUMENT;
  pdlp_solver* s = const_cast<pdlp_solver*>(cs);
  DevState h;
  int rc;
  if ((rc = read_state(s, &h))) return rc;
  const int P = h.parity;
  const size_t N = size_t(s->n), M = size_t(s->m);
  std::vector<double> hx(N), hy(M), hsx(N), hsy(M);
  PDLP_HIP(s, hipMemcpy(hx.data(), s->B.X[P], N * 8, hipMemcpyDeviceToHost));
  if (M) PDLP_HIP(s, hipMemcpy(hy.data(), s->B.Y[P], M * 8, hipMemcpyDeviceToHost));
  PDLP_HIP(s, hipMemcpy(hsx.data(), s->B.Sx, N * 8, hipMemcpyDeviceToHost));
  if (M) PDLP_HIP(s, hipMemcpy(hsy.data(), s->B.Sy, M * 8, hipMemcpyDeviceToHost));
  // the last accepted iterate may still be waiting to enter the sums
  if (h.w_pending != 0.0) {
    for (size_t j = 0; j < N; ++j) hsx[j] = hsx[j] + h.w_pending * hx[j];
    for (size_t i = 0; i < M; ++i) hsy[i] = hsy[i] + h.w_pending * hy[i];
  }
  if (!s->col_user.empty()) {            // to the user's column order
    std::vector<double> t(N);
    for (size_t j = 0; j < N; ++j) t[j] = hx[size_t(s->col_int[j])];
    hx.swap(t);
    for (size_t j = 0; j < N; ++j) t[j] = hsx[size_t(s->col_int[j])];
    hsx.swap(t);
  }
  auto put = [&](double* dst, const double* src, size_t cnt) -> int {
    if (!dst || cnt == 0) return 0;
    if (is_device_ptr(dst)) PDLP_HIP(s, hipMemcpy(dst, src, cnt * 8, hipMemcpyHostToDevice));
    else std::memcpy(dst, src, cnt * 8);
    return 0;
  };
  if ((rc = put(x, hx.data(), N)) || (rc = put(y, hy.data(), M)) || (rc = put(sx, hsx.data(), N)) ||
      (rc = put(sy, hsy.data(), M)))
    return rc;
  if ((rc = write_n(s, xa, s->B.XA))) return rc;
  if ((rc = write_output(s, ya, s->B.YA, M * 8))) return rc;
  if (out) {
    out->k = h.k;
    out->t = h.t;
    out->n_outer = h.n_outer;
    out->eta_hat = h.eta_hat;
    out->omega = h.omega;
    out->s_eta = h.s_eta;
    out->mu_prev = h.mu_prev;
    out->mu_anchor = h.mu_anchor;
  }
  return 0;
}

int pdlp_set_state(pdlp_solver* s, const double* x, const double* y, const double* xa,
                   const double* ya, const double* sx, const double* sy, const pdlp_state* v) {
  if (!s || !x || !xa || !sx || !v || (s->m > 0 && (!y || !ya || !sy))) return PDLP_ERR_INVALID_ARGUMENT;
  if (v->k < 0 || v->t < 0 || v->t > v->k || v->n_outer < 0 || !(v->eta_hat > 0.0) ||
      !(v->omega > 0.0) || !(v->s_eta >= 0.0) || !std::isfinite(v->eta_hat) || !std::isfinite(v->omega)) {
    s->err = "invalid checkpoint scalars";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  {
    const int rc0 = settle_kkt(s);      // the last solve's returned point keeps its KKT error
    if (rc0) return rc0;
  }
  const size_t M = size_t(s->m);
  auto get = [&](double* dst, const double* src, size_t cnt) -> int {
    if (cnt == 0) return 0;
    const hipMemcpyKind kind = is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    PDLP_HIP(s, hipMemcpyAsync(dst, src, cnt * 8, kind, s->stream));
    return 0;
  };
  int rc;
  if ((rc = read_n(s, x, s->B.X[0])) || (rc = get(s->B.Y[0], y, M)) || (rc = read_n(s, xa, s->B.XA)) ||
      (rc = get(s->B.YA, ya, M)) || (rc = read_n(s, sx, s->B.Sx)) || (rc = get(s->B.Sy, sy, M)))
    return rc;
  k_set_state<<<1, 1, 0, s->stream>>>(s->st, *v);
  PDLP_LAUNCH(s);
  if ((rc = launch_spmv(s, s->K, s->B.X[0], nullptr, 0, s->B.KX[0], nullptr, 0, kPredAlways, 0))) return rc;
  PDLP_HIP(s, hipStreamSynchronize(s->stream));
  s->initial_checked = true;
  return 0;
}

int pdlp_get_scaling(const pdlp_solver* cs, double* D1, double* D2) {
  if (!cs) return PDLP_ERR_INVALID_ARGUMENT;
  pdlp_solver* s = const_cast<pdlp_solver*>(cs);
  int rc;
  if ((rc = write_output(s, D1, s->B.D1, size_t(s->m) * 8))) return rc;
  if ((rc = write_n(s, D2, s->B.D2))) return rc;
  return 0;
}

int pdlp_get_iterate(const pdlp_solver* cs, double* xs, double* ys) {
  if (!cs) return PDLP_ERR_INVALID_ARGUMENT;
  pdlp_solver* s = const_cast<pdlp_solver*>(cs);
  int rc;
  k_output<<<s->gE, kBlock, 0, s->stream>>>(s->st, s->B, s->outbuf, s->outbuf + s->n, 1);
  PDLP_LAUNCH(s);
  if ((rc = write_n(s, xs, s->outbuf))) return rc;
  if ((rc = write_output(s, ys, s->outbuf + s->n, size_t(s->m) * 8))) return rc;
  return 0;
}

int pdlp_get_trace(const pdlp_solver* cs, pdlp_attempt_rec* att, int64_t att_cap, int64_t* n_att,
                   pdlp_check_rec* chk, int64_t chk_cap, int64_t* n_chk, double* xs, double* ys,
                   int64_t* n_iter) {
  if (!cs) return PDLP_ERR_INVALID_ARGUMENT;
  pdlp_solver* s = const_cast<pdlp_solver*>(cs);
  DevState h;
  int rc;
  if ((rc = read_state(s, &h))) return rc;
  const int64_t cap = h.trace_cap;
  auto ring = [&](auto* dst, int64_t dcap, const auto* src, int64_t total) -> int {
    using T = std::remove_pointer_t<decltype(dst)>;
    if (!dst || cap == 0) return 0;
    const int64_t have = std::min(total, cap);
    const int64_t first = total - have;     // index of the oldest kept record
    std::vector<T> tmp(static_cast<size_t>(cap));
    PDLP_HIP(s, hipMemcpy(tmp.data(), src, size_t(cap) * sizeof(T), hipMemcpyDeviceToHost));
    const int64_t nout = std::min(have, dcap);
    std::vector<T> ord(size_t(std::max<int64_t>(nout, 1)));
    for (int64_t i = 0; i < nout; ++i) ord[size_t(i)] = tmp[size_t((first + i) % cap)];
    if (nout > 0) {
      if (is_device_ptr(dst)) PDLP_HIP(s, hipMemcpy(dst, ord.data(), size_t(nout) * sizeof(T), hipMemcpyHostToDevice));
      else std::memcpy(dst, ord.data(), size_t(nout) * sizeof(T));
    }
    return 0;
  };
  if ((rc = ring(att, att_cap, s->B.att, h.n_att_log))) return rc;
  if ((rc = ring(chk, chk_cap, s->B.chk, h.n_chk_log))) return rc;
  if (n_att) *n_att = h.n_att_log;
  if (n_chk) *n_chk = h.n_chk_log;
  const int64_t ni = std::min<int64_t>(h.n_iter_log, cs->opts.trace_iters);
  if (n_iter) *n_iter = ni;
  if (ni > 0) {
    if (xs)
      for (int64_t r = 0; r < ni; ++r)
        if ((rc = write_n(s, xs + r * s->n, s->B.tx + r * s->n))) return rc;
    if ((rc = write_output(s, ys, s->B.ty, size_t(ni) * size_t(s->m) * 8))) return rc;
  }
  return 0;
}

int pdlp_spmv(pdlp_solver* s, int transpose, const double* x, double* out) {
  if (!s || !x || !out) return PDLP_ERR_INVALID_ARGUMENT;
  int rc;
  const CsrDev& A = transpose ? s->KT : s->K;
  if (s->col_user.empty()) {
    if ((rc = launch_spmv(s, A, x, nullptr, 0, out, nullptr, 0, kPredAlways, 0))) return rc;
  } else if (!transpose) {               // x in the user's order -> solver's order (gap scratch)
    if ((rc = read_n(s, x, s->B.GA[0]))) return rc;
    if ((rc = launch_spmv(s, A, s->B.GA[0], nullptr, 0, out, nullptr, 0, kPredAlways, 0))) return rc;
  } else {
    if ((rc = launch_spmv(s, A, x, nullptr, 0, s->B.GA[0], nullptr, 0, kPredAlways, 0))) return rc;
    if ((rc = write_n(s, out, s->B.GA[0]))) return rc;
  }
  PDLP_HIP(s, hipStreamSynchronize(s->stream));
  return 0;
}

int pdlp_kernel_times(const pdlp_solver* s, double* times_ms, int64_t* counts) {
  if (!s) return PDLP_ERR_INVALID_ARGUMENT;
  if (times_ms) {
    times_ms[0] = s->t_ms[0] + s->t_ms[1];
    times_ms[1] = s->t_ms[2] + s->t_ms[3];
  }
  if (counts) {
    counts[0] = s->t_cnt[0];
    counts[1] = s->t_cnt[2];
  }
  return 0;
}

int pdlp_set_host_threads(int n) {
  pdlp::set_host_threads(n);
  return pdlp::host_threads();
}

int pdlp_set_kernel_timing(pdlp_solver* s, int on) {
  if (!s) return PDLP_ERR_INVALID_ARGUMENT;
  if (on) {
    const int rc = make_timing_events(s);
    if (rc) return rc;
  }
  s->opts.time_kernels = on ? 1 : 0;
  return 0;
}

int pdlp_pass_times(const pdlp_solver* s, double* times_ms, int64_t* counts) {
  if (!s) return PDLP_ERR_INVALID_ARGUMENT;
  for (int j = 0; j < 4; ++j) {
    if (times_ms) times_ms[j] = s->t_ms[j];
    if (counts) counts[j] = s->t_cnt[j];
  }
  return 0;
}

int pdlp_reset_kernel_times(pdlp_solver* s) {
  if (!s) return PDLP_ERR_INVALID_ARGUMENT;
  for (int j = 0; j < 4; ++j) {
    s->t_ms[j] = 0.0;
    s->t_cnt[j] = 0;
  }
  return 0;
}

int pdlp_unroll_forward(pdlp_solver* s, const double* c, const double* q, int64_t steps,
                        int64_t segment, double eta, double omega, double* x_T, double* y_T) {
  if (!s) return PDLP_ERR_INVALID_ARGUMENT;
  try {
    return unroll_forward_impl(s, c, q, steps, segment, eta, omega, x_T, y_T, false);
  } catch (const std::bad_alloc&) {
    s->err = "host out of memory";
    return PDLP_ERR_OUT_OF_MEMORY;
  } catch (...) {
    s->err = "unexpected host exception";
    return PDLP_ERR_DEVICE;
  }
}

int pdlp_unroll_forward_noalloc(pdlp_solver* s, const double* c, const double* q, int64_t steps,
                                int64_t segment, double eta, double omega, double* x_T, double* y_T) {
  if (!s) return PDLP_ERR_INVALID_ARGUMENT;
  try {
    return unroll_forward_impl(s, c, q, steps, segment, eta, omega, x_T, y_T, true);
  } catch (...) {
    s->err = "unexpected host exception";
    return PDLP_ERR_DEVICE;
  }
}

int pdlp_unroll_backward(pdlp_solver* s, const double* gx_T, const double* gy_T, double* gc,
                         double* gq) {
  if (!s) return PDLP_ERR_INVALID_ARGUMENT;
  try {
    return unroll_backward_impl(s, gx_T, gy_T, gc, gq);
  } catch (const std::bad_alloc&) {
    s->err = "host out of memory";
    return PDLP_ERR_OUT_OF_MEMORY;
  } catch (...) {
    s->err = "unexpected host exception";
    return PDLP_ERR_DEVICE;
  }
}

int pdlp_unroll_get_info(const pdlp_solver* s, pdlp_unroll_info* info) {
  if (!s || !info) return PDLP_ERR_INVALID_ARGUMENT;
  const auto& U = s->U;
  info->steps = U.T;
  info->segment = U.S;
  info->checkpoints = U.nseg;
  info->recomputed_steps = U.recomputed;
  info->eta = U.eta;
  info->omega = U.omega;
  info->forward_seconds = U.fwd_s;
  info->backward_seconds = U.bwd_s;
  info->device_bytes = U.bytes;
  info->ready = U.ready ? 1 : 0;
  info->pad = 0;
  return 0;
}

}  // extern "C"

// The batched solver's host side (pdlp_batch_*).
#include "pdlp_batch_host.hip"
