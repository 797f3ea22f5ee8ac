// Internal layout shared by the host driver and the gfx950 kernels of the PDLP solver.
#pragma once

#include <cstdint>
#include <vector>

namespace pdlp {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kElemsPerLane = 8;       // a row of length len gets L = min pow2 with len <= 8 L lanes
constexpr int kElemsPerLaneLds = 16;   // the same with 16 in layouts read by the LDS-staged kernel
constexpr int kWaveMaxLen = kElemsPerLane * 64;   // longer rows are reduced by a whole workgroup
constexpr int kRounds = 4;             // rows per lane group in one wavefront task (at most)
constexpr int kFillWaves = 8192;       // wavefronts of a full grid: 256 CUs x 8 workgroups x 4
constexpr int kVectorMax = 16384;      // longest row one workgroup reduces alone
constexpr int kChunk = 16384;          // nonzeros per chunk of a split row
// Automatic panel mode keeps a copy in panels while its panel rows stay below this fraction of
// its nonzeros (each panel row costs an offset, a partial and a combine read, 28 bytes against
// 12 per nonzero; on a 1e6 x 2e6 LP with 2.1e7 nonzeros, ratios 0.35 / 0.29, panels still
// gave +28%).
constexpr double kPanelRowFrac = 0.4;
constexpr int kMaxPanels = 8;          // XCD column panels of a copy (one per XCD of an MI355X)
// XCD panels without an LDS stage gather their operand slice through the XCD's 4 MiB L2.  A
// slice wider than kSubpanelBytes is cut into equal column ranges (sub-panels), which the
// XCD's workgroups take one after another, so that fewer lines of the operand are in use at a
// time next to the streamed entries; an even number of them, at most kMaxSubpanels.  On the
// PageRank LP on 5e6 nodes (4.8 MiB slices) the K~ x' first pass took 640 us whole and 622,
// 580, 505, 548, 475, 516, 508 us in 2 .. 8 sub-panels, while its combine grew from 121 to
// 137 .. 188 us (more panel rows); odd counts were slower in repeated runs.
constexpr int64_t kSubpanelBytes = int64_t(1) << 20;
constexpr int kMaxSubpanels = 8;
// LDS-staged products: one workgroup of kLdsBlock threads per CU holds up to kLdsEntries
// entries of the gathered vector (152 KiB of the CU's 160 KiB of LDS).  A copy whose
// gathered vector, cut into slices of that width, costs at most kLdsRowFrac panel rows per
// nonzero gets one panel per slice and gathers only from LDS; otherwise a copy in XCD panels
// whose columns are ordered hot-first stages each panel's first kLdsEntries columns.
constexpr int kLdsBlock = 1024;
constexpr int kLdsWaves = kLdsBlock / 64;
constexpr int kLdsEntries = 19456;
constexpr int kMaxLdsPanels = 4096;
constexpr double kLdsRowFrac = 0.4;
// ... or at most kLdsRowFracVsPanels when the alternative is XCD panels (the copy's panel rows
// there below kPanelRowFrac): gathers from LDS instead of L2 are then worth a larger combine
// (on the 1e6 x 2e6 LP with 2.1e7 nonzeros, slices at 0.64 against XCD panels at 0.29 gave
// +4.7% PDHG iterations per second; the PageRank LP's transposed copy, at 0.61 against a plain
// layout, lost 29%).
constexpr double kLdsRowFracVsPanels = 0.7;

enum DescKind : int32_t { kWaveRows = 0, kVector = 1, kSplit = 2 };

// One unit of SpMV work.
//  kWaveRows: rows perm[a .. a + b) for one wavefront, 2^(kind_l >> 8) lanes per row,
//             aux entries per lane (aux * lanes >= every row length of the task)
//  kVector:   row a, reduced by one workgroup
//  kSplit:    chunk b of row a (split id aux), reduced by one workgroup, combined by the last
struct RowDesc {
  int32_t a;
  int32_t b;
  int32_t kind_l;   // kind | log2(lanes per row) << 8
  int32_t aux;
};

struct Schedule {
  std::vector<int32_t> perm;           // rows up to kWaveMaxLen long, grouped by lane count
  std::vector<RowDesc> wave;           // wavefront tasks over perm
  std::vector<RowDesc> block;          // workgroup tasks (long rows and chunks of giant rows)
  std::vector<int32_t> split_row;      // per split id: the row
  std::vector<int32_t> split_nchunks;  // per split id: number of chunks
  std::vector<int32_t> split_base;     // per split id: offset into the chunk-partial table
  int64_t total_chunks = 0;
};

Schedule build_schedule(const int64_t* row_ptr, int64_t nrows);

// XCD column panels of one CSR copy.  The gathered dimension (columns) is cut into P ranges of
// about equal nonzero count; the nonzeros of panel p form "panel rows" (row r restricted to
// panel p), stored panel after panel, each panel's rows grouped by lane count.  Workgroup b
// runs on XCD b mod 8 and only works on panel b mod P, so the slice of the gathered vector it
// touches stays in that XCD's L2.  A second, row-ordered pass adds the panel partial sums of
// each row in panel order.
struct PanelLayout {
  int P = 1;
  std::vector<int32_t> cut;            // P + 1 column offsets of the panels
  std::vector<int64_t> prow_ptr;       // total panel rows + 1
  std::vector<int32_t> prow_row;       // original row of each panel row
  std::vector<int64_t> src;            // row-major nonzero index of each panel-ordered nonzero
  std::vector<int64_t> slot_ptr;       // nrows + 1
  std::vector<int32_t> slot_idx;       // panel rows of each row, in panel order
  Schedule sched;                      // tasks over panel rows (perm empty = identity)
  std::vector<int32_t> wave_begin;     // P + 1 offsets of each panel's wavefront tasks
  std::vector<int32_t> block_begin;    // P + 1 offsets of each panel's workgroup tasks
};

// The work of one LDS-staged pass: wavefront tasks wave[tb .. te) of panel p.
struct LdsSeg {
  int32_t p;
  int32_t tb;
  int32_t te;
  int32_t pad;
};

// Builds the layout with P panels; returns false (and leaves `out` unusable) when the panel
// rows would cost more than `max_prow_frac` of the nonzeros.
// given_cuts: the P + 1 column cuts to use (nullptr: about nnz / P nonzeros per panel).
// emax: most entries per lane of a wavefront task (kElemsPerLane, or kElemsPerLaneLds for a
// layout whose products run in the LDS-staged kernel: fewer lanes per row, less padding).
bool build_panels(const int64_t* rp, const int32_t* ci, int64_t nrows, int64_t ncols, int P,
                  double max_prow_frac, PanelLayout& out,
                  const std::vector<int32_t>* given_cuts = nullptr, int emax = kElemsPerLane);

// Number of panel rows build_panels would make under the column cuts `cut` (P + 1 offsets).
int64_t count_panel_rows(const int64_t* rp, const int32_t* ci, int64_t nrows, const std::vector<int32_t>& cut,
                         int emax = kElemsPerLane);

// Interleaved entries of the wavefront tasks (a sliced-ELL form): round i of task t, with E
// entries per lane, owns 64 E slots from off[t] + 64 E i; entry k of lane j (row group
// j >> log2 L, lane j mod L of it) sits at slot 64 k + j and holds entry k L + (j mod L) of
// that row, so each of a wavefront's E loads reads 64 consecutive values.  Slots past a row's
// end, and of row groups past the task's last row, hold the value 0 and the row's first column
// (column 0 for an empty row or a missing row).  Rows of the task: perm[a + slot] when perm is
// given, else a + slot.  rp, ci, v: the copy in CSR form (row order of the layout).
void build_interleaved(const Schedule& S, const int64_t* rp, const int32_t* ci, const double* v,
                       const int32_t* perm, std::vector<int64_t>& off, std::vector<int32_t>& cis,
                       std::vector<double>& vs);

// Splits the wavefront tasks of a panel layout among G workgroups at about equal cost (12
// bytes per nonzero, 16 per panel row, 64 per task): aligned (G a multiple of P): workgroup b
// takes a contiguous share of panel b mod P's tasks, so it stays on that panel's XCD;
// otherwise workgroup b takes the b-th share of all tasks in panel order, cut into one segment
// per panel it touches.  Returns the G + 1 offsets of each workgroup's segments in `seg`.
std::vector<int32_t> lds_segments(const PanelLayout& L, int G, bool aligned, std::vector<LdsSeg>& seg);

// Scalar state of one solve, resident in device memory.  Kernels read it at entry; only the
// last workgroup of a kernel (after every other workgroup has arrived) writes it.
struct DevState {
  double eta;            // step size of the next attempt
  double eta_hat;        // step size proposed by the last accepted attempt
  double omega;          // primal weight
  double w_pending;      // step of the last accepted iterate, not yet added to the averages
  double s_eta;          // sum of steps since the last restart
  double mu_prev;        // candidate gap at the previous check of this outer loop
  double mu_anchor;      // gap of the anchor vs the previous anchor
  double mu_cur, mu_avg, mu_c;
  double tol;
  double kkt[4];         // KKT errors of the last evaluated point
  double dx_norm, dy_norm;
  double q_norm, c_norm; // of the user's (unscaled) q and c
  // normalized-gap solves, three slots
  double gap_r[3];
  double gap_num[3];
  uint64_t gap_lo[3], gap_hi[3];
  int32_t gap_state[3];  // 0 bisecting, 1 s* = inf, 2 r = 0 (mu = 0), 3 converged
  int32_t pad0;
  int64_t k;             // accepted steps
  int64_t t;             // accepted steps since the last restart
  int64_t n_outer;       // restarts
  int64_t attempts;
  int64_t retries;
  int64_t iter_limit;
  int64_t checks;
  int64_t spmv_K, spmv_KT;
  int64_t n_att_log, n_chk_log, n_iter_log;
  int32_t parity;        // which buffer of X, Y, KX holds the current iterate
  int32_t kty_valid;     // KTy holds K~^T y for the current y
  int32_t check_pending; // k is a multiple of check_every and the check has not run
  int32_t done;
  int32_t status;
  int32_t use_avg;       // candidate of the running check is the average
  int32_t restart;       // the running check restarts
  int32_t mask;
  int32_t out_avg;       // the returned point is the average buffers
  int32_t snap_pending;  // an accepted step waits for its trace snapshot
  int32_t check_every;
  int32_t max_retries;
  int32_t trace_iters;
  int32_t trace_cap;
  int32_t restarts_on, pw_on;
  int32_t constant_step;  // constant step policy: eta never changes, every attempt accepted
  int32_t to_current;     // GetRestartCandidate may pick the current iterate
  double pow_norm2;       // power iteration: squared norm of the last K^T K v
  double beta_suff, beta_nec, beta_art, theta, eps_zero;
  // Malitsky-Pock line search (step policy 2): eta_hat is the step of the last accepted
  // iteration (the primal step), eta the candidate of the running trial.
  int32_t mp_on;
  int32_t mp_stage;       // 0: the next attempt starts an iteration; 1: it retries the dual trial
  int32_t mp_commit;      // the last trial was accepted: K~^T y^ is to become K~^T y
  int32_t pw_pow2;        // restarts off, primal weight updated at k = 2, 4, 8, ...
  int32_t pw_event;       // the pending check is such an update only
  int32_t pad1;
  double mp_theta;        // theta_k = eta_{k-1} / eta_k
  double mp_bf, mp_df, mp_ic;   // breaking factor, downscaling factor, interpolation coefficient
};

// Small record the host reads after every enqueued block.
struct HostStatus {
  int64_t k;
  int64_t attempts;
  int32_t done;
  int32_t status;
  int32_t check_pending;
  int32_t pad;
};

}  // namespace pdlp
