// Host side of the batched solver behind pdlp_batch_* of include/pdlp.h: packing many LPs,
// their size classes and schedules, the tuner, and the launches of k_batch_solve.
//
// Included at the end of the solver's translation unit (pdlp_solver.hip), after its helpers.
#pragma once

// ------------------------------------------------------------------------------------------
// batched solver
// ------------------------------------------------------------------------------------------

// Size classes of the batched solve, by member nonzeros: [0, 2^11), [2^11, 2^13), [2^13, 2^15),
// [2^15, ..).  Each class runs as one launch with its own workgroup size.
constexpr int kBatchClasses = PDLP_BATCH_CLASSES;
// The schedules a class can run with: threads per member, and rows per thread whose products
// are in flight together (2 with 4 nonzeros of each at a time, else 1 row with 8, or 4 at 1024
// threads, whose 16 waves per CU allow 128 registers per thread).
struct BatchSchedule {
  int threads, rows;
};
constexpr BatchSchedule kBatchSchedules[] = {{64, 1},  {128, 1}, {128, 2}, {256, 1},
                                             {256, 2}, {512, 1}, {512, 2}, {1024, 1}};

int batch_class_of(int64_t nnz) {
  return nnz < (int64_t(1) << 11) ? 0 : nnz < (int64_t(1) << 13) ? 1 : nnz < (int64_t(1) << 15) ? 2 : 3;
}

struct pdlp_batch {
  hipStream_t stream = nullptr;
  int64_t count = 0, total_n = 0, total_m = 0;
  pdlp_options opts{};
  std::vector<void*> allocs;
  std::vector<BatchInst> inst;
  BatchDev D{};
  DevState tmpl{};
  double* xout = nullptr;
  double* yout = nullptr;
  std::string err;
  bool solved = false;
  double create_seconds = 0.0, solve_seconds = 0.0, tune_seconds = 0.0;
  // members of each size class, largest first, and the workgroup size of each class
  int64_t cls_count[kBatchClasses] = {0, 0, 0, 0};
  const int32_t* cls_order[kBatchClasses] = {nullptr, nullptr, nullptr, nullptr};
  int32_t cls_bs[kBatchClasses] = {256, 256, 256, 256};     // threads per member
  int32_t cls_rows[kBatchClasses] = {1, 1, 1, 1};           // rows per thread in flight
  hipStream_t cls_stream[kBatchClasses] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_start = nullptr;
  hipEvent_t cls_ev[kBatchClasses] = {nullptr, nullptr, nullptr, nullptr};

  ~pdlp_batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (int c = 0; c < kBatchClasses; ++c) {
      if (cls_stream[c]) {
        (void)hipStreamSynchronize(cls_stream[c]);
        (void)hipStreamDestroy(cls_stream[c]);
      }
      if (cls_ev[c]) (void)hipEventDestroy(cls_ev[c]);
    }
    if (ev_start) (void)hipEventDestroy(ev_start);
    for (void* p : allocs) (void)hipFree(p);
  }
  template <class T>
  hipError_t alloc(T** p, size_t count_) {
    const size_t bytes = std::max<size_t>(count_, 1) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
    if (e == hipSuccess) allocs.push_back(*p);
    return e;
  }
};

namespace {

thread_local std::string g_batch_error;

bool batch_schedule_valid(int threads, int rows) {
  for (const BatchSchedule& q : kBatchSchedules)
    if (q.threads == threads && q.rows == rows) return true;
  return false;
}

// One launch of the batched kernel over the members of size class c with the schedule
// (bs threads per member, rows per thread).
int batch_launch(pdlp_batch* b, int c, int bs, int rows, double tol, int64_t iter_limit, hipStream_t st) {
  const unsigned g = unsigned(b->cls_count[c]);
  if (g == 0) return 0;
  BatchDev D = b->D;
  D.order = b->cls_order[c];
  const int ri = b->opts.ruiz_iters, pc = b->opts.pock_chambolle;
  const double pi = b->opts.primal_importance;
  const DevState& T = b->tmpl;
  const int key = bs * 10 + rows;
  switch (key) {
    case 641: k_batch_solve<64><<<g, 64, 0, st>>>(D, T, tol, iter_limit, ri, pc, pi); break;
    case 1281: k_batch_solve<128><<<g, 128, 0, st>>>(D, T, tol, iter_limit, ri, pc, pi); break;
    case 1282: k_batch_solve<128, 4, 2><<<g, 128, 0, st>>>(D, T, tol, iter_limit, ri, pc, pi); break;
    case 2561: k_batch_solve<256><<<g, 256, 0, st>>>(D, T, tol, iter_limit, ri, pc, pi); break;
    case 2562: k_batch_solve<256, 4, 2><<<g, 256, 0, st>>>(D, T, tol, iter_limit, ri, pc, pi); break;
    case 5121: k_batch_solve<512><<<g, 512, 0, st>>>(D, T, tol, iter_limit, ri, pc, pi); break;
    case 5122: k_batch_solve<512, 4, 2><<<g, 512, 0, st>>>(D, T, tol, iter_limit, ri, pc, pi); break;
    case 10241: k_batch_solve<1024><<<g, 1024, 0, st>>>(D, T, tol, iter_limit, ri, pc, pi); break;
    default:
      b->err = "internal error: unknown batch schedule";
      return PDLP_ERR_DEVICE;
  }
  PDLP_LAUNCH(b);
  return 0;
}

// Every class's launch on a stream of its own (largest class first), all after the work
// already on the batch's stream and all waited for on it.
int batch_run(pdlp_batch* b, double tol, int64_t iter_limit) {
  PDLP_HIP(b, hipEventRecord(b->ev_start, b->stream));
  for (int c = kBatchClasses - 1; c >= 0; --c) {
    if (b->cls_count[c] == 0) continue;
    PDLP_HIP(b, hipStreamWaitEvent(b->cls_stream[c], b->ev_start, 0));
    int rc;
    if ((rc = batch_launch(b, c, b->cls_bs[c], b->cls_rows[c], tol, iter_limit, b->cls_stream[c]))) return rc;
    PDLP_HIP(b, hipEventRecord(b->cls_ev[c], b->cls_stream[c]));
    PDLP_HIP(b, hipStreamWaitEvent(b->stream, b->cls_ev[c], 0));
  }
  PDLP_HIP(b, hipStreamSynchronize(b->stream));
  return 0;
}

template <class T>
int batch_fetch(pdlp_batch* b, const T* p, size_t count, std::vector<T>& tmp, const T** out) {
  if (count == 0) {
    *out = p;
    return 0;
  }
  if (is_device_ptr(p)) {
    tmp.resize(count);
    PDLP_HIP(b, hipMemcpy(tmp.data(), p, count * sizeof(T), hipMemcpyDeviceToHost));
    *out = tmp.data();
  } else {
    *out = p;
  }
  return 0;
}

template <class T>
int batch_upload(pdlp_batch* b, const T* h, size_t count, T** d) {
  PDLP_HIP(b, b->alloc(d, count));
  if (count) PDLP_HIP(b, hipMemcpy(*d, h, count * sizeof(T), hipMemcpyHostToDevice));
  return 0;
}

int batch_create_impl(pdlp_batch* b, int64_t count, const int64_t* hm, const int64_t* hn,
                      const int64_t* hneq, const double* c, const int64_t* row_ptr,
                      const int32_t* col_idx, const double* val, const double* q, const double* l,
                      const double* u) {
  if (count < 1 || !hm || !hn || !hneq || !c || !row_ptr || !l || !u) {
    b->err = "count must be >= 1 and the size arrays and c, row_ptr, l, u non-null";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  std::vector<int64_t> vm, vn, vneq;
  const int64_t *pm, *pn, *pneq;
  int rc;
  if ((rc = batch_fetch(b, hm, size_t(count), vm, &pm)) || (rc = batch_fetch(b, hn, size_t(count), vn, &pn)) ||
      (rc = batch_fetch(b, hneq, size_t(count), vneq, &pneq)))
    return rc;
  b->inst.resize(size_t(count));
  int64_t rp_total = 0, rpT_total = 0, tn = 0, tm = 0;
  for (int64_t k = 0; k < count; ++k) {
    if (pn[k] < 1 || pm[k] < 0 || pneq[k] < 0 || pneq[k] > pm[k] || pm[k] >= (int64_t(1) << 31) ||
        pn[k] >= (int64_t(1) << 31)) {
      b->err = "invalid sizes of member " + std::to_string(k);
      return PDLP_ERR_INVALID_ARGUMENT;
    }
    BatchInst& I = b->inst[size_t(k)];
    I.m = int32_t(pm[k]);
    I.n = int32_t(pn[k]);
    I.m1 = int32_t(pm[k] - pneq[k]);
    I.pad = 0;
    I.rp = rp_total;
    I.rpT = rpT_total;
    I.xo = tn;
    I.yo = tm;
    rp_total += pm[k] + 1;
    rpT_total += pn[k] + 1;
    tn += pn[k];
    tm += pm[k];
  }
  if (tm > 0 && !q) {
    b->err = "q is NULL";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  b->count = count;
  b->total_n = tn;
  b->total_m = tm;
  std::vector<int64_t> vrp;
  const int64_t* rp;
  if ((rc = batch_fetch(b, row_ptr, size_t(rp_total), vrp, &rp))) return rc;
  int64_t nz_total = 0;
  for (int64_t k = 0; k < count; ++k) {
    BatchInst& I = b->inst[size_t(k)];
    I.nz = nz_total;
    const int64_t nnz_k = rp[I.rp + I.m];
    if (rp[I.rp] != 0 || nnz_k < 0) {
      b->err = "row offsets of member " + std::to_string(k) + " must start at 0";
      return PDLP_ERR_INVALID_ARGUMENT;
    }
    nz_total += nnz_k;
  }
  if (nz_total > 0 && (!col_idx || !val)) {
    b->err = "null col_idx or val";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  std::vector<int32_t> vci;
  std::vector<double> vv, vc, vq, vl, vu;
  const int32_t* ci;
  const double *v, *hc, *hq, *hl, *hu;
  if ((rc = batch_fetch(b, col_idx, size_t(nz_total), vci, &ci)) ||
      (rc = batch_fetch(b, val, size_t(nz_total), vv, &v)) || (rc = batch_fetch(b, c, size_t(tn), vc, &hc)) ||
      (rc = batch_fetch(b, q, size_t(tm), vq, &hq)) || (rc = batch_fetch(b, l, size_t(tn), vl, &hl)) ||
      (rc = batch_fetch(b, u, size_t(tn), vu, &hu)))
    return rc;
  // validate every member and build its transposed copy
  std::vector<int64_t> rpT(static_cast<size_t>(rpT_total));
  std::vector<int32_t> ciT(static_cast<size_t>(nz_total));
  std::vector<double> vT(static_cast<size_t>(nz_total));
  for (int64_t k = 0; k < count; ++k) {
    const BatchInst& I = b->inst[size_t(k)];
    const int64_t* rpk = rp + I.rp;
    const std::string bad = validate_lp(I.m, I.n, I.m - I.m1, hc + I.xo, rpk, ci + I.nz, v + I.nz,
                                        hq + I.yo, hl + I.xo, hu + I.xo);
    if (!bad.empty()) {
      b->err = "member " + std::to_string(k) + ": " + bad;
      return PDLP_ERR_INVALID_ARGUMENT;
    }
    std::vector<int64_t> trp;
    std::vector<int32_t> tci;
    std::vector<double> tv;
    transpose_csr(I.m, I.n, rpk, ci + I.nz, v + I.nz, trp, tci, tv);
    std::copy(trp.begin(), trp.end(), rpT.begin() + I.rpT);
    std::copy(tci.begin(), tci.end(), ciT.begin() + I.nz);
    std::copy(tv.begin(), tv.end(), vT.begin() + I.nz);
  }
  BatchDev& D = b->D;
  BatchInst* dinst;
  int64_t* drp;
  int64_t* drpT;
  int32_t* dci;
  int32_t* dciT;
  double* dv0;
  double* dvT0;
  if ((rc = batch_upload(b, b->inst.data(), b->inst.size(), &dinst)) ||
      (rc = batch_upload(b, rp, size_t(rp_total), &drp)) || (rc = batch_upload(b, rpT.data(), rpT.size(), &drpT)) ||
      (rc = batch_upload(b, ci, size_t(nz_total), &dci)) || (rc = batch_upload(b, ciT.data(), ciT.size(), &dciT)) ||
      (rc = batch_upload(b, v, size_t(nz_total), &dv0)) || (rc = batch_upload(b, vT.data(), vT.size(), &dvT0)) ||
      (rc = batch_upload(b, hc, size_t(tn), &D.c0)) || (rc = batch_upload(b, hl, size_t(tn), &D.l0)) ||
      (rc = batch_upload(b, hu, size_t(tn), &D.u0)) || (rc = batch_upload(b, hq, size_t(tm), &D.q0)))
    return rc;
  D.inst = dinst;
  D.v0 = dv0;
  D.vT0 = dvT0;
  PDLP_HIP(b, b->alloc(&D.v, size_t(nz_total)));
  PDLP_HIP(b, b->alloc(&D.vT, size_t(nz_total)));
  {
    // workgroup order: members with the most nonzeros first (ties by index), so the longest
    // solves start early and the small ones fill in behind them; grouped by size class
    std::vector<int32_t> order(static_cast<size_t>(count));
    for (int64_t k = 0; k < count; ++k) order[size_t(k)] = int32_t(k);
    auto nz_of = [&](int32_t k) {
      const BatchInst& I = b->inst[size_t(k)];
      return rp[I.rp + I.m];
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return nz_of(a) > nz_of(c); });
    int32_t* dorder;
    if ((rc = batch_upload(b, order.data(), order.size(), &dorder))) return rc;
    D.order = dorder;
    // classes are contiguous in this order (largest class first)
    int64_t pos = 0;
    for (int c = kBatchClasses - 1; c >= 0; --c) {
      int64_t cnt = 0;
      while (pos + cnt < count && batch_class_of(nz_of(order[size_t(pos + cnt)])) == c) ++cnt;
      b->cls_count[c] = cnt;
      b->cls_order[c] = dorder + pos;
      pos += cnt;
    }
    if (pos != count) {
      b->err = "internal error: size classes do not cover the members";
      return PDLP_ERR_DEVICE;
    }
  }
  for (int c = 0; c < kBatchClasses; ++c) {
    PDLP_HIP(b, hipStreamCreateWithFlags(&b->cls_stream[c], hipStreamNonBlocking));
    PDLP_HIP(b, hipEventCreateWithFlags(&b->cls_ev[c], hipEventDisableTiming));
  }
  PDLP_HIP(b, hipEventCreateWithFlags(&b->ev_start, hipEventDisableTiming));
  D.rp = drp;
  D.rpT = drpT;
  D.ci = dci;
  D.ciT = dciT;
  for (double** p : {&D.c, &D.l, &D.u, &D.D2, &D.X0, &D.X1, &D.KTy, &D.Sx, &D.XB, &D.KTYB, &D.XA})
    PDLP_HIP(b, b->alloc(p, size_t(tn)));
  for (double** p : {&D.q, &D.D1, &D.Y0, &D.Y1, &D.KX0, &D.KX1, &D.Sy, &D.YB, &D.KXB, &D.YA})
    PDLP_HIP(b, b->alloc(p, size_t(tm)));
  for (double** p : {&D.GA0, &D.GA1, &D.GB0, &D.GB1}) PDLP_HIP(b, b->alloc(p, size_t(tn + tm)));
  PDLP_HIP(b, b->alloc(&D.out_state, size_t(count)));
  PDLP_HIP(b, b->alloc(&b->xout, size_t(tn)));
  PDLP_HIP(b, b->alloc(&b->yout, size_t(tm)));
  // per-member state template (no traces in batched mode)
  DevState& h = b->tmpl;
  h = DevState{};
  h.mu_prev = INFINITY;
  h.mu_anchor = INFINITY;
  h.kty_valid = 1;
  h.status = PDLP_NOT_SOLVED;
  h.check_every = b->opts.check_every;
  h.max_retries = b->opts.max_retries;
  h.trace_iters = 0;
  h.trace_cap = 0;
  h.restarts_on = b->opts.adaptive_restarts;
  h.pw_on = b->opts.primal_weight_update;
  h.constant_step = 0;
  h.to_current = b->opts.restart_to_current != 0;
  h.beta_suff = b->opts.beta_sufficient;
  h.beta_nec = b->opts.beta_necessary;
  h.beta_art = b->opts.beta_artificial;
  h.theta = b->opts.theta;
  h.eps_zero = b->opts.eps_zero;
  return 0;
}

}  // namespace

extern "C" {

int pdlp_batch_create(pdlp_batch** out, int64_t count, const int64_t* m, const int64_t* n,
                      const int64_t* n_eq, const double* c, const int64_t* row_ptr,
                      const int32_t* col_idx, const double* val, const double* q, const double* l,
                      const double* u, const pdlp_options* opts, void* hip_stream) {
  if (!out) {
    g_batch_error = "out is NULL";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  *out = nullptr;
  const double t0 = now_s();
  pdlp_batch* b = nullptr;
  try {
    b = new pdlp_batch();
  } catch (...) {
    g_batch_error = "host allocation failed";
    return PDLP_ERR_OUT_OF_MEMORY;
  }
  if (opts) b->opts = *opts;
  else pdlp_default_options(&b->opts);
  if (!options_valid(b->opts) || b->opts.step_policy != 0 || b->opts.pw_power_of_two != 0) {
    g_batch_error = "invalid options (the batched solver takes the options of pdlp_create with the "
                    "adaptive step policy and pw_power_of_two = 0)";
    delete b;
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  b->stream = static_cast<hipStream_t>(hip_stream);
  int rc;
  try {
    rc = batch_create_impl(b, count, m, n, n_eq, c, row_ptr, col_idx, val, q, l, u);
  } catch (const std::bad_alloc&) {
    b->err = "host allocation failed";
    rc = PDLP_ERR_OUT_OF_MEMORY;
  } catch (...) {
    b->err = "unexpected host exception";
    rc = PDLP_ERR_DEVICE;
  }
  if (rc != 0) {
    g_batch_error = b->err;
    delete b;
    return rc;
  }
  b->create_seconds = now_s() - t0;
  *out = b;
  return 0;
}

int pdlp_batch_solve(pdlp_batch* b, double tol, int64_t iter_limit) {
  if (!b) return PDLP_ERR_INVALID_ARGUMENT;
  if (!(tol >= 0.0) || iter_limit < 0) {
    b->err = "tol must be >= 0 and iter_limit >= 0";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  const double t0 = now_s();
  int rc;
  if ((rc = batch_run(b, tol, iter_limit))) return rc;
  b->solved = true;
  b->solve_seconds = now_s() - t0;
  return 0;
}

int pdlp_batch_tune(pdlp_batch* b, int64_t steps, int32_t* threads, int32_t* rows) {
  if (!b) return PDLP_ERR_INVALID_ARGUMENT;
  if (steps < 1) {
    b->err = "steps must be >= 1";
    return PDLP_ERR_INVALID_ARGUMENT;
  }
  const double t0 = now_s();
  hipEvent_t e0, e1;
  PDLP_HIP(b, hipEventCreate(&e0));
  PDLP_HIP(b, hipEventCreate(&e1));
  int rc = 0;
  for (int c = 0; c < kBatchClasses && rc == 0; ++c) {
    if (b->cls_count[c] == 0) continue;
    float best = 0.f;
    BatchSchedule best_q{b->cls_bs[c], b->cls_rows[c]};
    for (const BatchSchedule& q : kBatchSchedules) {
      const int bs = q.threads;
      // a run of every member of the class for `steps` accepted steps (tol 0: none stops early)
      if ((rc = batch_launch(b, c, bs, q.rows, 0.0, steps, b->stream))) break;        // warm-up
      if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = PDLP_ERR_DEVICE; break; }
      if ((rc = batch_launch(b, c, bs, q.rows, 0.0, steps, b->stream))) break;
      float ms = 0.f;
      if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        b->err = "batch tune: event timing failed";
        rc = PDLP_ERR_DEVICE;
        break;
      }
      if (best == 0.f || ms < best) {
        best = ms;
        best_q = q;
      }
    }
    b->cls_bs[c] = best_q.threads;
    b->cls_rows[c] = best_q.rows;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  b->solved = false;             // the timing runs are not a solve
  for (int c = 0; c < kBatchClasses; ++c) {
    if (threads) threads[c] = b->cls_bs[c];
    if (rows) rows[c] = b->cls_rows[c];
  }
  b->tune_seconds = now_s() - t0;
  return 0;
}

int pdlp_batch_set_schedule(pdlp_batch* b, const int32_t* threads, const int32_t* rows) {
  if (!b || !threads || !rows) return PDLP_ERR_INVALID_ARGUMENT;
  for (int c = 0; c < kBatchClasses; ++c) {
    if (!batch_schedule_valid(threads[c], rows[c])) {
      b->err = "batch schedule must be one of 64x1, 128x1, 128x2, 256x1, 256x2, 512x1, 512x2, "
               "1024x1 (threads x rows per thread)";
      return PDLP_ERR_INVALID_ARGUMENT;
    }
  }
  for (int c = 0; c < kBatchClasses; ++c) {
    b->cls_bs[c] = threads[c];
    b->cls_rows[c] = rows[c];
  }
  return 0;
}

int pdlp_batch_schedule(const pdlp_batch* b, int32_t* threads, int32_t* rows, int64_t* members) {
  if (!b) return PDLP_ERR_INVALID_ARGUMENT;
  for (int c = 0; c < kBatchClasses; ++c) {
    if (threads) threads[c] = b->cls_bs[c];
    if (rows) rows[c] = b->cls_rows[c];
    if (members) members[c] = b->cls_count[c];
  }
  return 0;
}

double pdlp_batch_tune_seconds(const pdlp_batch* b) { return b ? b->tune_seconds : -1.0; }

int pdlp_batch_get(const pdlp_batch* cb, double* x, double* y, int32_t* status, int64_t* iterations,
                   double* kkt) {
  if (!cb) return PDLP_ERR_INVALID_ARGUMENT;
  pdlp_batch* b = const_cast<pdlp_batch*>(cb);
  if (!b->solved) {
    b->err = "pdlp_batch_get before pdlp_batch_solve";
    return PDLP_ERR_INVALID_STATE;
  }
  if (x || y) {
    k_batch_output<<<unsigned(b->count), kBlock, 0, b->stream>>>(b->D, b->xout, b->yout);
    PDLP_LAUNCH(b);
    PDLP_HIP(b, hipStreamSynchronize(b->stream));
    auto put = [&](void* dst, const void* src, size_t bytes) -> int {
      if (!dst || bytes == 0) return 0;
      const hipMemcpyKind kind = is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
      PDLP_HIP(b, hipMemcpy(dst, src, bytes, kind));
      return 0;
    };
    int rc;
    if ((rc = put(x, b->xout, size_t(b->total_n) * 8)) || (rc = put(y, b->yout, size_t(b->total_m) * 8))) return rc;
  }
  if (status || iterations || kkt) {
    std::vector<DevState> h(static_cast<size_t>(b->count));
    PDLP_HIP(b, hipMemcpy(h.data(), b->D.out_state, h.size() * sizeof(DevState), hipMemcpyDeviceToHost));
    std::vector<int32_t> st(h.size());
    std::vector<int64_t> it(h.size());
    std::vector<double> kk(4 * h.size());
    for (size_t k = 0; k < h.size(); ++k) {
      st[k] = h[k].status;
      it[k] = h[k].k;
      for (int q = 0; q < 4; ++q) kk[4 * k + q] = h[k].kkt[q];
    }
    auto put = [&](void* dst, const void* src, size_t bytes) -> int {
      if (!dst) return 0;
      if (is_device_ptr(dst)) PDLP_HIP(b, hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
      else std::memcpy(dst, src, bytes);
      return 0;
    };
    int rc;
    if ((rc = put(status, st.data(), st.size() * 4)) || (rc = put(iterations, it.data(), it.size() * 8)) ||
        (rc = put(kkt, kk.data(), kk.size() * 8)))
      return rc;
  }
  return 0;
}

double pdlp_batch_solve_seconds(const pdlp_batch* b) { return b ? b->solve_seconds : -1.0; }

void pdlp_batch_destroy(pdlp_batch* b) { delete b; }

const char* pdlp_batch_last_error(const pdlp_batch* b) {
  if (!b) return g_batch_error.c_str();
  return b->err.c_str();
}

}  // extern "C"
