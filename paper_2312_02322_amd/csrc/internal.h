// Internal device/host structures of libmqct (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mqct.h"

#include <functional>
#include <utility>
#include <vector>

namespace mqct {

// Storage element kinds (same numbering as the public MQCT_R64 ... MQCT_C64).
enum Dtype { R64 = 0, C128 = 1, R32 = 2, C64 = 3 };

inline bool dtype_complex(int d) { return d == C128 || d == C64; }
inline bool dtype_fp32(int d) { return d == R32 || d == C64; }
inline int dtype_bytes(int d) { return d == C128 ? 16 : (d == R32 ? 4 : 8); }

// A loaded system as the kernels see it.  Tables are stored [K][N][Npad]:
// knot k, stored row m, column n (Npad = N rounded up to a multiple of 16,
// padding columns are zero).  Because every knot's matrix is Hermitian, column n
// of the stored matrix is the complex conjugate of row n, which lets a lane
// that owns output row n stream memory contiguously with its neighbours.
struct DevSystem {
  int32_t N, K, Npad, dtype;
  int32_t jx_w;              // ELL width of J_x (0 when there is no Coriolis term)
  int32_t ell_w;             // sparse tables: kept elements per column (0: dense tables)
  double mu;
  const double* R;           // [K]
  const double* E;           // [N]
  const void* M;             // [K][N][Npad] values
  const void* M2;            // [K][N][Npad] natural-spline second derivatives
  const int32_t* jx_col;     // [N][jx_w], padding entries point at the row itself
  const double* jx_val;      // [N][jx_w], padding entries are 0
  const int32_t* ell_col;    // sparse tables: [ell_w][Npad] stored row of each slot
  const double* drv;         // [K] driving potential U(R_k) of decoupled (AT) dynamics, or null
  const double* drv2;        // [K] its natural-spline second derivatives
  int64_t knot_stride;       // N * Npad elements (CSR tables: the stored elements)
  double R_inv_h;            // 1 / spacing when the R grid is uniform, else 0
  const int32_t* csr_row;    // coordinate-list systems: [N + 1] start of each row's elements
  const int32_t* csr_col;    // [nnz] their columns, ascending within a row (null: other layouts)
};

// Per-trajectory launch record.
struct TrajIn {
  int64_t id;                // index in the caller's batch
  int64_t amp_off;           // offset of this trajectory's amplitudes (sum of N before it)
  int64_t n_steps;           // RK4 steps of this call
  int32_t sys;               // index into the device system table
  int32_t init_channel;
  int32_t flags;             // TRAJ_* bits
  int32_t status0;           // status bits carried from a stored state (TRAJ_RESUME)
  double E_coll, b, R0, t0, dt;
  double c0[6];              // classical0 when flags & TRAJ_HAS_C0
  // continuation of a stored state (TRAJ_RESUME; zero otherwise)
  int64_t step0;             // RK4: time index of the first step, t_j = t0 + (step0 + j) dt
  int64_t steps0, rejects0, attempts0;   // counts carried
  double h0;                 // DP5: size of the next attempt
  double E0, J0, R_exit;     // references of the diagnostics, DP5 exit radius
  int32_t dflags;            // MQCT_S_LAST_REJECTED
  int32_t pad1;
};

// TRAJ_RESUME: the trajectory continues a stored state (amplitudes and classical
// state come as a0 / classical0; the fields after c0 hold the stepper's state);
// TRAJ_FINISHED: a stored adaptive trajectory that has stopped for good (exited,
// step underflow, non-finite): it is returned unchanged.
enum { TRAJ_HAS_A0 = 1, TRAJ_HAS_C0 = 2, TRAJ_AT = 4, TRAJ_RESUME = 8, TRAJ_FINISHED = 16 };

// Where a kernel writes its per-trajectory results (device pointers; any may be
// null except P).
struct TrajOut {
  double* P;
  double* a_final;
  double* classical;
  double* t_final;
  int64_t* steps;
  int64_t* rejects;
  int32_t* status;
  double* norm_err;
  double* energy_err;
  double* angmom_err;
  mqct_traj_state* state;    // [B] the context's state store (by id), or null
  double2* st_amp;           // its amplitudes (by amp_off), or null
};

enum { ST_EXITED = 1, ST_MAX_STEPS = 2, ST_STEP_UNDERFLOW = 4, ST_BELOW_GRID = 8,
       ST_NONFINITE = 16 };

// Optional event timing of the dominant step kernel (HIP events recorded on
// the launch stream around each of its launches), with the algorithmic table
// bytes those launches had to read: known on the host for the per-trajectory
// kernel, counted on the device (occupied knots per stage) for the binned
// product and copied into pinned slots read after the stream has finished.
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev;   // start/stop pairs
  size_t used = 0;
  double bytes = 0.0;           // host-known algorithmic bytes
  unsigned long long* slots = nullptr;   // pinned, device-filled knot counts
  std::vector<double> slot_bytes;        // bytes per counted knot of each used slot
  static constexpr size_t SLOTS = 4096;
  // the next event of the pool (created on demand), or null when off / failed
  hipEvent_t next() {
    if (!on) return nullptr;
    if (used == ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[used++];
  }
  // a pinned slot for a device-side count of occupied knots (null when off / full)
  unsigned long long* knot_slot(double bytes_per_knot) {
    if (!on) return nullptr;
    if (!slots && hipHostMalloc((void**)&slots, SLOTS * sizeof(unsigned long long), 0) != hipSuccess) {
      slots = nullptr;
      return nullptr;
    }
    if (slot_bytes.size() == SLOTS) return nullptr;
    slot_bytes.push_back(bytes_per_knot);
    return slots + (slot_bytes.size() - 1);
  }
  void reset() {
    used = 0;
    bytes = 0.0;
    slot_bytes.clear();
  }
};

inline void prof_mark(Prof* p, hipEvent_t e, hipStream_t s) {
  if (p && e) (void)hipEventRecord(e, s);
}

// knots per accumulation chunk of the coupling fill kernel (v rows are padded to it)
constexpr int CPL_KNOT_CHUNK = 32;

// Device view of a coupling-matrix build (coupling.hip).  Channels n have a
// (j1, j2, j) level chan_J, a rotor-1 state chan_r, total j and projection m;
// terms are sorted by lam (t_user maps back to the caller's order).
struct CouplingDev {
  int N, T, K, n1, nJ, b_stride;
  const int* chan_J;
  const int* chan_r;
  const int* chan_j;
  const int* chan_m;
  const int* jl_j1;
  const int* jl_j2;
  const int* jl_j;
  const int* rot_j;
  const double* b;       // [n1][b_stride], b_k at k + j1
  const int* t_l1;
  const int* t_mu;
  const int* t_l2;
  const int* t_l;
  const int* t_user;
  const double* v;       // [T][KP], sorted order, zero beyond K
  double* lf;            // [256] log-factorials
  double* Kr;            // [n1][n1][T] rotor-1 factors
  double* F;             // [nJ][nJ][T] level factors
  const int* chan_grp;   // [N] the channel's m group
  const int* grp_off;    // [groups + 1] offsets into grp_list
  const int* grp_list;   // [N] channels of each m group, ascending
  const int2* work;      // [n_work] (row, tile of FILL_BLOCK entries of its m group)
  int64_t n_work;
  int KP;                // v row stride: K rounded up to the fill kernel's knot chunk
  int cg_jmax, cg_lmax;  // extent of the C(j' m lam 0 | j'' m) table
  double* cgt;           // that table
};

// ---- launchers (defined in the .hip files) ----------------------------------

// Sparse (ELL) tables: pattern of the elements whose magnitude exceeds thr at
// some knot (amax [N][N] scratch, cnt [N] kept per column), the slot lists
// col [W][Npad], and the gather of dense storage [K][N][Npad] into [K][W][Npad].
hipError_t launch_ell_pattern(const double* M_in, int N, int K, int ncomp, double thr,
                              double* amax, int* cnt, hipStream_t s);
hipError_t launch_ell_fill(const double* amax, int N, int Npad, int W, double thr, int32_t* col,
                           hipStream_t s);
hipError_t launch_ell_gather(const void* D, const void* D2, const int32_t* col, const int* cnt,
                             int N, int Npad, int K, int W, int ncomp, int dtype, void* E,
                             void* E2, hipStream_t s);

// Table preparation: from FP64 input (device, [K][N][N], real or complex
// interleaved) write storage tables and their natural-spline second
// derivatives.  tmp holds tmp_doubles doubles (>= K); columns are processed in
// chunks of tmp_doubles / K.
hipError_t launch_validate(const double* M_in, int N, int K, int ncomp,
                           unsigned long long* stats /*[3], zeroed*/, hipStream_t s);
hipError_t launch_spline_prepare(const double* M_in, const double* R, int N, int K, int Npad,
                                 int ncomp, int dtype, void* M_out, void* M2_out, double* tmp,
                                 int64_t tmp_doubles, hipStream_t s);

// Fixed-step RK4, one workgroup per trajectory.  All trajectories of one launch
// must use systems of the same dtype whose padded column count is <= max_npad.
hipError_t launch_rk4_gemv(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                           const double* d_a0, TrajOut out, int dtype, int max_npad,
                           hipStream_t s, Prof* prof = nullptr);

// Adaptive-step controls.
struct DpCtl {
  double rtol, atol, h_min;
  int64_t max_steps;
};

// ---- work-list schedule (queue_kernels.h, queue.hip) -------------------------

// State of one trajectory between step launches (written by lane 0).
struct QState {
  double t, h;
  double yc[4];        // R, Phi, P_R, P_Phi
  double kc1[4];       // classical derivative at (t, y): first stage of the next attempt
  double E0, J0, R_exit, theta, ptheta;
  int64_t steps, rejects, attempts;
  int64_t n_idx;       // RK4: time index, t = t0 + n_idx h
  int32_t status, flags;
};
// Q_FINISH: a stored trajectory that had stopped for good; the next step launch
// forms its results (through the same code as a step that finishes) and retires it.
enum { Q_DONE = 1, Q_LASTREJ = 2, Q_FINISH = 4 };

// Device workspace of one class (trajectories sharing storage type and Npad).
struct QWS {
  int32_t n, npad;
  const TrajIn* traj;  // [n] records of the class
  QState* st;          // [n]
  double2* amp;        // [n][npad] amplitudes
  double2* kst;        // [n][8][npad] DP5 stage derivatives and fifth-order solution
  int32_t* list;       // [n] work list (class-local indices of unfinished trajectories)
  int32_t* list2;      // [n] scratch of the compaction
  int32_t* count;      // [1] entries on the work list
};

struct QArgs {
  QWS ws;
  const DevSystem* systems;
  const double* a0_all;
  DpCtl ctl;
  int64_t max_attempts;
  TrajOut out;
  int per_launch;        // attempts (steps) of a trajectory per launch of the tail's kernels
};

// Kernels of one workgroup shape: init and step for RK4 [0] and DP5 [1]
// (null when the shape is not built for the storage type).
struct QKernelSet {
  int block, rpt;
  int split_waves;     // 0: rows shared out over the workgroup; W: split-row form with W waves
  const void* init[2];
  const void* step[2];
  const void* step_multi[2];   // up to QArgs::per_launch attempts per launch (the tail)
};
const QKernelSet* queue_kernels(int dtype);   // [QUEUE_SHAPES]
constexpr int QUEUE_SHAPES = 17;

struct QueueClass {
  int dtype, npad;
  int64_t first, n;    // records [first, first + n) of the device record array
};

struct QueueOpts {
  bool graphs = true;  // replay chunks of step launches as HIP graphs
  bool tune = true;    // time the candidate workgroup shapes on the batch
  int tail = 1;        // 1: switch to the tuned split-row shape once few trajectories remain;
                       // 0: never; 2: run every class on a split-row shape (tests)
  int chunk = 16;      // step launches per replay
  int per_launch = 1;  // attempts of a trajectory per step launch once few are left
  int64_t col_ws = 0;  // columns schedule: workspace cap in bytes (0: 80 % of free memory)
};

// Autotuner decisions, kept for the life of a context.
struct QueueTuneEntry {
  int dtype, npad, method, shape;
  bool tuned;
  std::vector<std::pair<int, double>> ms;   // candidate shape -> ms per step launch
  int tail_shape = -1;                      // shape once few trajectories remain (-1: same)
  std::vector<std::pair<int, double>> tail_ms;   // the same, timed on a small sample
};
struct QueueCache {
  std::vector<QueueTuneEntry> entries;
};

size_t queue_workspace_bytes(const std::vector<QueueClass>& cls, int method);
// Runs a batch on the work-list schedule.  `cap` is a non-default stream used
// only to capture graphs; `h_counts` is pinned host memory for cls.size() ints.
// `on_tail` (may be empty) is called once, when the work lists hold at most
// twice as many trajectories as the device has compute units (their
// latency-bound tail), or when they are done: work on another stream started
// there has most of the device beside the tail, and never shares it with the
// autotuner's timing runs.
hipError_t run_queue(const DevSystem* d_systems, const TrajIn* d_traj,
                     const std::vector<QueueClass>& cls, const double* d_a0, TrajOut out,
                     int method, DpCtl ctl, int64_t max_attempts, const QueueOpts& opt,
                     QueueCache& cache, void* ws, hipStream_t s, hipStream_t cap, int* h_counts,
                     Prof* prof, const std::function<void()>& on_tail = {});

// R-binned lockstep RK4 (all trajectories on one system, d_traj in any order).
size_t binned_workspace_bytes(int B, int Npad, int K, bool fp32);
hipError_t run_binned(const DevSystem* d_systems, const DevSystem& hs, const TrajIn* d_traj,
                      int B, int64_t max_steps, const double* d_a0, TrajOut out, void* ws,
                      hipStream_t s, Prof* prof = nullptr);

// Adaptive Dormand-Prince 5(4) on the binned product: one attempt per round for
// every unfinished trajectory (same tableau, error norm, controller and stopping
// rules as the work-list schedule's), single-system batches.
size_t binned_dp5_workspace_bytes(int B, int Npad, int K, bool fp32);
hipError_t run_binned_dp5(const DevSystem* d_systems, const DevSystem& hs, const TrajIn* d_traj,
                          int B, const double* d_a0, TrajOut out, DpCtl ctl,
                          int64_t max_attempts, void* wsp, hipStream_t s, Prof* prof);


// Adjoint (discrete RK4 adjoint with checkpointed recomputation).  The G_t of
// the parametric form enter as nonzero lists: entries goff[t] .. goff[t+1]-1,
// gent = row | col << 16, gval the values (h_goff: the offsets on the host).
// one_segment: every trajectory has at most S steps (the forward and the backward
// pass then run as two launches, nothing recomputed).
int64_t adjoint_scratch_doubles(int Npad, int64_t n_steps, int S);
hipError_t launch_adjoint(const DevSystem* d_systems, bool cplx, bool ell, int Npad,
                          const TrajIn* d_traj, const int* order,
                          int64_t B, const double* dLdP, double* grad_part, double* grad_out,
                          double* P_out, double* scratch, int64_t scratch_stride, int S,
                          const int* goff, const int* h_goff, const uint32_t* gent,
                          const double* gval, const double* rad, const double* rad2,
                          const int* gidx, int P, int nG, bool one_segment, hipStream_t s);
hipError_t launch_build_param_tables(const double* G, const double* rad, const int* gidx,
                                     const double* theta, int P, int nG, int N, int Npad, int K,
                                     double* Mout, hipStream_t s);
hipError_t launch_spline_rows(const double* y, const double* x, int K, int ncol, double* y2,
                              double* tmp, hipStream_t s);

// ---- coordinate-list systems and the columns schedule (columns.hip) ----------

// Columns that share a path: records first .. first + count - 1 (in group order).
constexpr int COL_MAX = 128;
struct ColGroup {
  int32_t first, count;
  int64_t n_steps;
  int64_t stage_off;   // its stage records: 4 per RK4 step
};
hipError_t launch_coo_gather(const double* values, int64_t ld, const int32_t* perm, int64_t nnz,
                             int K, int NC, double* v64, unsigned long long* nonfinite,
                             hipStream_t s);
hipError_t launch_csr_spline(const double* y, const double* x, int K, int64_t ncol, double* y2,
                             hipStream_t s);
hipError_t launch_csr_partner_check(const double* v64, const int32_t* partner, int64_t nnz, int K,
                                    int NC, unsigned long long* maxdiff,
                                    unsigned long long* maxabs, hipStream_t s);
hipError_t launch_csr_cast_f32(const double* in, int64_t n, float* out, hipStream_t s);
size_t columns_workspace_bytes(int G, int N, int CT, int64_t stages, bool fp32);
// All groups on one system (hs); d_traj holds the records in group order.
hipError_t run_columns(const DevSystem* d_systems, const DevSystem& hs, const TrajIn* d_traj,
                       const std::vector<ColGroup>& groups, int CT, const double* d_a0,
                       TrajOut out, void* wsp, hipStream_t s);

// Streaming read of `bytes` (a multiple of 16) at buf (measure.hip).
hipError_t launch_read_probe(const void* buf, int64_t bytes, int n_cu, hipStream_t s);

// Cross sections on the device.
hipError_t launch_xsec(int64_t B, int N, const double* P, const double* b, const int32_t* init_level,
                       const int32_t* level_of_channel, int n_levels, double b_max,
                       double* level_sums /*[B][n_levels]*/, double* sigma, hipStream_t s);

// cross-section post-processing (postproc.hip), device pointers
hipError_t launch_xs_symmetrize(int nE, int L, const double* g, const double* sigma, double* sym,
                                double* ratio, hipStream_t s);
hipError_t launch_xs_rates(int nE, int L, int nT, const double* U, const double* E,
                           const double* g, const double* sym, double mu, const double* beta,
                           double* k, hipStream_t s);

// coupling-matrix build: M [K][N][N] and/or G [T][N][N] (device, either may be null)
hipError_t launch_coupling(const CouplingDev& d, double* M, double* G, Prof* prof,
                           hipStream_t s);
// screened build: factors, then the equal-m elements whose largest |M| over the
// S screening radii (coefficients vs [T][S], sorted term order) exceeds thr,
// counted in *count and listed in rows / cols up to capacity; then their values
// at the K knots, values[k * capacity + i]
constexpr int CPL_MAX_SCREEN = 8;
hipError_t launch_coupling_screen(const CouplingDev& d, int S, const double* vs, double thr,
                                  int64_t capacity, unsigned long long* count, int32_t* rows,
                                  int32_t* cols, hipStream_t s);
hipError_t launch_coupling_values(const CouplingDev& d, int64_t n, const int32_t* rows,
                                  const int32_t* cols, int64_t capacity, double* values,
                                  hipStream_t s);

}  // namespace mqct
