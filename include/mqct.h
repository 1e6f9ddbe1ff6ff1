/*
 * mqct.h -- C ABI of the MI355X (gfx950) batched Ehrenfest mean-field trajectory
 * propagator for mixed quantum/classical collision dynamics (MQCT).
 *
 * Physics (paper Section II): for every trajectory the interaction-picture
 * amplitudes a_n (Eq. 4) obey
 *     da_n/dt = -i sum_m M_nm(R) e^{i(E_n - E_m)t} a_m - i Phidot (J_x a)_n     (Eq. 5)
 * and the classical separation R, angle Phi and momenta P_R, P_Phi obey
 * Eqs. 7-10 in the collision plane Theta = pi/2 (end of Section II).  M(R) is
 * the coupling matrix (Eq. 6) tabulated on an R grid and interpolated with a
 * natural cubic spline (Section III).  J_x is the Coriolis operator: its
 * elements are the square-root factors of Eq. 5; the generator is taken as
 * -i Phidot J_x (the reading that conserves norm and total energy).  The
 * torque dP_Phi/dt = -i<[J_x, V]> is Eq. 10.  Final |a_n|^2 give state-to-state
 * probabilities and cross sections (end of Section II).
 *
 * Units: atomic units everywhere at this interface (hartree, bohr, electron
 * masses, hbar/E_h).
 *
 * Conventions:
 *   - Every function returns mqct_status (0 = success, negative = error) and
 *     never throws or aborts across the interface.  mqct_last_error() gives a
 *     message for the most recent failure on a context.
 *   - Argument and validation errors are reported before any device work.
 *   - Input pointers are borrowed for the duration of the call (tables are
 *     copied); result pointers are caller-owned.
 *   - A context is used from one host thread at a time.
 */
#ifndef MQCT_H
#define MQCT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mqct_context mqct_context;
typedef int32_t mqct_status;

enum {
  MQCT_OK = 0,
  MQCT_ERR_ARG = -1,           /* invalid argument (sizes, pointers, ranges)           */
  MQCT_ERR_NONFINITE = -2,     /* NaN or Inf in an input table                         */
  MQCT_ERR_NOT_HERMITIAN = -3, /* |M - M^H| > 1e-12 max|M| at some knot                */
  MQCT_ERR_OOM = -4,           /* device allocation failed                             */
  MQCT_ERR_DEVICE = -5,        /* a HIP runtime call failed                            */
  MQCT_ERR_UNSUPPORTED = -6,   /* a valid request the library does not implement      */
  MQCT_ERR_STATE = -7          /* call out of order (e.g. unknown system id)           */
};

/* element types of coupling tables */
enum { MQCT_R64 = 0, MQCT_C128 = 1, MQCT_R32 = 2, MQCT_C64 = 3 };
/* time steppers */
enum { MQCT_RK4 = 0, MQCT_DP5 = 1 };
/* table layouts */
enum { MQCT_DENSE = 0, MQCT_SPARSE = 1 };
/* dynamics: Ehrenfest mean field (Eqs. 5, 7-10 coupled), or AT -- the quantum
   equations (Eq. 5) propagated along a trajectory that does not feel the
   quantum state (Section III), driven by the system's driving potential */
enum { MQCT_EHRENFEST = 0, MQCT_AT = 1 };
/* where a caller buffer lives */
enum { MQCT_MEM_HOST = 0, MQCT_MEM_DEVICE = 1 };
/* per-trajectory status bits */
enum {
  MQCT_T_EXITED = 1,          /* DP5: left the interaction region (R >= R0, P_R > 0)   */
  MQCT_T_MAX_STEPS = 2,       /* DP5: accepted-step limit reached                      */
  MQCT_T_STEP_UNDERFLOW = 4,  /* DP5: step size fell below h_min                       */
  MQCT_T_BELOW_GRID = 8,      /* R went below the first knot (linear continuation used) */
  MQCT_T_NONFINITE = 16       /* NaN/Inf appeared; the trajectory was stopped          */
};
/* batch schedules */
enum {
  MQCT_SCHED_AUTO = 0,        /* library chooses                                        */
  MQCT_SCHED_GEMV = 1,        /* one workgroup per trajectory, step loop inside a kernel */
  MQCT_SCHED_BINNED = 2,      /* lockstep stages, trajectories binned by spline knot,
                                 table x amplitude-columns products on matrix cores;
                                 one system per batch; RK4 steps or DP5 attempts    */
  MQCT_SCHED_QUEUE = 3,       /* work list: one step attempt per launch for every
                                 unfinished trajectory, finished ones retired between
                                 chunks of launches (replayed as HIP graphs); mixes
                                 systems of any size; DP5 uses it unless BINNED is
                                 asked for                                          */
  MQCT_SCHED_COLUMNS = 4      /* decoupled (AT) dynamics on a coordinate-list system
                                 (mqct_system_load_coo): the trajectories that share a
                                 path (same start, energy, impact parameter, t0, dt,
                                 n_steps) are amplitude columns of one matrix, stepped
                                 by RK4 as a sparse-table x column-matrix product; the
                                 only schedule for such systems, and AUTO picks it  */
};

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue all work on (NULL: the context creates and owns its own stream). */
mqct_status mqct_create(int32_t device, void* hip_stream, mqct_context** out);
/* Free every device buffer of the context (waits for its stream first). */
void mqct_destroy(mqct_context* ctx);
/* Message of the most recent failure on ctx (static text when ctx is NULL);
 * valid until the next call on ctx. */
const char* mqct_last_error(const mqct_context* ctx);
/* Block until all work enqueued on the context stream has finished. */
mqct_status mqct_synchronize(mqct_context* ctx);

/*
 * A collision system: channel energies, coupling tables on an R grid and the
 * Coriolis operator (Section II, Eqs. 5-6; Section III for the grid + spline).
 *   N, K      channels; grid points (K >= 4).
 *   R_grid    host [K] bohr, strictly increasing.
 *   E         host [N] hartree.
 *   in_dtype  MQCT_R64 or MQCT_C128: element type of M as passed.
 *   M_mem     MQCT_MEM_HOST or MQCT_MEM_DEVICE: where M lives.
 *   M         [K][N][N] row-major, M[k][n][m] = <n|V(R_k)|m> (hartree), Hermitian
 *             per knot.  Copied; the caller may free it after the call.
 *   storage   MQCT_R64/MQCT_C128 (FP64 path) or MQCT_R32/MQCT_C64 (FP32-table
 *             path).  A real storage type requires real input.
 *   jx_*      J_x as a coordinate list (host), real symmetric, at most 8
 *             nonzeros per row; jx_nnz may be 0.
 *   mu        reduced mass, electron masses.
 *   layout    MQCT_DENSE: every element stored.  MQCT_SPARSE: only the elements
 *             whose magnitude exceeds drop_below (hartree, >= 0) at some knot,
 *             in (m, n) or (n, m), are kept -- the paper's truncated coupling
 *             matrices (elements above 1 cm^-1, Section III) and the block
 *             structure of couplings that conserve m.  Each column's kept rows
 *             are stored as a slot list (ELL, width = the largest count), and
 *             the dropped elements are exactly zero in every computation.  The
 *             binned schedule needs dense tables.
 * The natural-spline second derivatives of every element are computed on the
 * device in FP64 and stored with the tables in the storage type.
 */
typedef struct {
  int32_t N, K;
  const double* R_grid;
  const double* E;
  int32_t in_dtype;
  int32_t M_mem;
  const void* M;
  int32_t storage;
  int32_t jx_nnz;
  const int32_t* jx_row;
  const int32_t* jx_col;
  const double* jx_val;
  double mu;
  int32_t layout;
  double drop_below;
} mqct_system_desc;

/* Validate (finite, Hermitian, increasing grid), upload, spline-prepare.
 * Errors: MQCT_ERR_ARG, MQCT_ERR_NONFINITE, MQCT_ERR_NOT_HERMITIAN,
 * MQCT_ERR_OOM, MQCT_ERR_DEVICE.  Synchronous. */
mqct_status mqct_system_load(mqct_context* ctx, const mqct_system_desc* desc,
                             int32_t* system_id);
/*
 * A collision system from a coordinate list of its coupling elements -- the
 * truncated coupling matrices of Section III (elements above a threshold kept,
 * computed on the radial grid only for those), for bases too large for the
 * dense [K][N][N] input (the paper's 206,350 states).  The list is what
 * mqct_coupling_build_sparse writes.
 *   N, K, R_grid, E, mu, jx_*   as in mqct_system_desc.
 *   in_dtype    MQCT_R64 or MQCT_C128: element type of values.
 *   mem         MQCT_MEM_HOST or MQCT_MEM_DEVICE: where rows, cols, values live.
 *   n_el        stored elements, 1 <= n_el < 2^31, both triangles: every
 *               (n, m) must come with its (m, n) partner, equal (real) or
 *               conjugate (complex) at every knot to 1e-12 of the largest
 *               magnitude; no pair twice; any order.
 *   rows, cols  [n_el] row n and column m of element i (0 <= n, m < N).
 *   values      [K][ld] (element i at knot k: values[k * ld + i], hartree;
 *               complex interleaved), ld >= n_el.
 *   storage     MQCT_R64/MQCT_C128 or MQCT_R32/MQCT_C64 (real with real input).
 * The elements are sorted into rows (CSR: each row's columns ascending), the
 * natural-spline second derivative of every element along the grid is computed
 * on the device in FP64, and values and curvatures are stored per knot in the
 * storage type: 2 K n_el elements.  Such a system runs only decoupled (AT)
 * dynamics with RK4 on MQCT_SCHED_COLUMNS and needs mqct_system_set_driver.
 * Copied; the caller may free its arrays after the call.  Errors: MQCT_ERR_ARG
 * (sizes, indices, duplicates, a missing partner, null pointers),
 * MQCT_ERR_NONFINITE, MQCT_ERR_NOT_HERMITIAN (partner values differ),
 * MQCT_ERR_OOM, MQCT_ERR_DEVICE.  Synchronous.
 */
typedef struct {
  int32_t N, K;
  const double* R_grid;
  const double* E;
  double mu;
  int32_t in_dtype;
  int32_t mem;
  int64_t n_el;
  const int32_t* rows;
  const int32_t* cols;
  const double* values;
  int64_t ld;
  int32_t storage;
  int32_t jx_nnz;
  const int32_t* jx_row;
  const int32_t* jx_col;
  const double* jx_val;
} mqct_coo_desc;
mqct_status mqct_system_load_coo(mqct_context* ctx, const mqct_coo_desc* desc,
                                 int32_t* system_id);

/* The driving potential of decoupled (AT) dynamics (Section III: the classical
 * trajectory is propagated apart from the quantum equations): U [K] host,
 * hartree, on the system's grid, interpolated by its natural cubic spline (the
 * same interval, weights and off-grid rule as the coupling tables).  Copied;
 * replaces an earlier driver.  Errors: MQCT_ERR_ARG, MQCT_ERR_STATE,
 * MQCT_ERR_NONFINITE, MQCT_ERR_OOM, MQCT_ERR_DEVICE.  Synchronous. */
mqct_status mqct_system_set_driver(mqct_context* ctx, int32_t system_id, const double* U);
/* Device bytes held by a loaded system's tables (values + second derivatives). */
mqct_status mqct_system_bytes(mqct_context* ctx, int32_t system_id, int64_t* bytes);
/* Release a system's device memory; its id becomes invalid. */
mqct_status mqct_system_free(mqct_context* ctx, int32_t system_id);

/*
 * A batch of trajectories (Section III: Monte-Carlo initial conditions).  All
 * pointers are host arrays.  Per trajectory b:
 *   system_id[b]     a loaded system; trajectories may mix systems.
 *   init_channel[b]  a(0) = e_n; ignored when a0 is given.
 *   a0               optional [sum_b N_b][2] initial amplitudes (complex
 *                    interleaved, concatenated in batch order).
 *   classical0       optional [B][6] initial (R, Theta, Phi, P_R, P_Theta,
 *                    P_Phi).  Without it: R = R0, Theta = pi/2, Phi = 0,
 *                    P_Phi = b sqrt(2 mu E_coll), P_R = -sqrt(2 mu E_coll - P_Phi^2/R0^2).
 *   E_coll, b        [B] hartree, bohr (0 <= b < R0); unused with classical0.
 *   R0               optional [B] start (and DP5 exit) radius; NULL = last knot.
 *   t0               optional [B] start time; NULL = 0.
 *   dt               [B] RK4 step (required for RK4).
 *   n_steps          [B] RK4 step count (exact; no early exit).
 *   rtol, atol, max_steps, h_min   DP5 controls (scaled RMS error norm).
 *   schedule         MQCT_SCHED_*.
 *   dynamics         MQCT_EHRENFEST, or MQCT_AT (every system of the batch needs a
 *                    driving potential, mqct_system_set_driver).  With AT, each
 *                    trajectory's classical equations read
 *                        dP_R/dt = -U'(R) + P_Phi^2/(mu R^3),  dP_Phi/dt = 0,
 *                    (Eq. 5 unchanged, Coriolis term included), so trajectories
 *                    that share (E_coll, b, R0) share the path and differ only in
 *                    their initial amplitudes: many initial states per trajectory.
 *                    energy_err then follows P^2/2mu + P_Phi^2/(2 mu R^2) + U(R)
 *                    and angmom_err follows P_Phi.
 *   resume           0: start as above.  1: continue every trajectory from the
 *                    context's state store (mqct_get_state / mqct_set_state: the
 *                    final state of the previous mqct_run on this context, or
 *                    what mqct_set_state put there).  B and system_id must match
 *                    the store; init_channel, a0, classical0, E_coll, b, R0, t0
 *                    and dt are then ignored.  RK4 takes n_steps[b] further
 *                    steps of the stored h at t = t_origin + (n_origin + j) h, so
 *                    that a run split in two equals the whole run bit for bit;
 *                    DP5 continues with the stored step size, rejection flag
 *                    and counts (max_steps bounds the total), re-evaluating the
 *                    first stage at the stored state (first same as last), and
 *                    returns trajectories whose status holds EXITED,
 *                    STEP_UNDERFLOW or NONFINITE unchanged (MAX_STEPS is
 *                    cleared: the limit may have been raised).
 */
typedef struct {
  int64_t B;
  const int32_t* system_id;
  const int32_t* init_channel;
  const double* a0;
  const double* classical0;
  const double* E_coll;
  const double* b;
  const double* R0;
  const double* t0;
  int32_t integrator;
  const double* dt;
  const int64_t* n_steps;
  double rtol, atol;
  int64_t max_steps;
  double h_min;
  int32_t schedule;
  int32_t dynamics;
  int32_t resume;
} mqct_batch_desc;

/*
 * Results.  `mem` says where ALL arrays below live.  With MQCT_MEM_DEVICE the
 * run is asynchronous on the context stream; with MQCT_MEM_HOST mqct_run
 * returns after the host arrays are filled.  Arrays other than P may be NULL.
 *   P          [sum_b N_b] final |a_n|^2 (batch order, offsets = prefix sums of N_b)
 *   a_final    [sum_b N_b][2]
 *   classical  [B][6] final R, Theta, Phi, P_R, P_Theta, P_Phi
 *   t_final, steps, rejects, status  [B]
 *   norm_err   [B] sum|a|^2 - 1;  energy_err [B] relative change of the total
 *   (classical + rotational + mean-field) energy;  angmom_err [B] change of
 *   P_Phi - <J_x>.
 */
typedef struct {
  int32_t mem;
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
} mqct_batch_result;

/* Propagate a batch.  Errors: MQCT_ERR_ARG, MQCT_ERR_STATE (unknown system),
 * MQCT_ERR_UNSUPPORTED (schedule/integrator combination), MQCT_ERR_OOM,
 * MQCT_ERR_DEVICE.  Per-trajectory problems go to the status bits.
 * DP5 (Dormand & Prince 1980 tableau, first same as last; error = scaled RMS
 * over the 2N+6 real state components with sc = atol + rtol max(|y|, |y_new|);
 * step factor min(5, max(0.2, 0.9 err^-1/5)), no growth right after a
 * rejection; Hairer-Norsett-Wanner starting step) stops at the first accepted
 * step with R >= R0 and P_R > 0 (EXITED), at max_steps accepted steps or
 * 4 max_steps + 256 attempts (MAX_STEPS), when h < h_min (STEP_UNDERFLOW), or on
 * a non-finite error (NONFINITE).  The work-list schedule (MQCT_SCHED_QUEUE, and
 * DP5 batches on any schedule but MQCT_SCHED_BINNED) runs until every trajectory
 * has finished and returns after the results are enqueued; it synchronises with
 * the context stream between chunks of launches.  DP5 on MQCT_SCHED_BINNED makes
 * one attempt per round for every unfinished trajectory of its single system
 * (six knot-binned products per round) with the same tableau, controller and
 * stopping rules, and synchronises with the stream every eight rounds to count
 * the trajectories still running. */
mqct_status mqct_run(mqct_context* ctx, const mqct_batch_desc* batch,
                     mqct_batch_result* result);

/*
 * Full state of one trajectory (Section II: the amplitudes a_n of Eq. 4 and the
 * classical R, Theta, Phi, P_R, P_Theta, P_Phi of Eqs. 7-10), with what the time
 * steppers carry from step to step.  Every mqct_run leaves the final state of
 * each of its trajectories in the context's state store (device memory owned
 * by the context; the amplitudes are kept beside the records, concatenated in
 * batch order), where mqct_run with resume = 1 picks it up.
 *   t              time of the state.
 *   t_origin, n_origin   t = t_origin + n_origin h as fixed-step RK4 computes its
 *                  step times (a DP5 run writes t_origin = t, n_origin = 0).
 *   h              RK4: the step; DP5: the size of the next attempt.
 *   classical      R, Theta, Phi, P_R, P_Theta, P_Phi.
 *   E0, J0         total energy and P_Phi - <J_x> at the trajectory's start (the
 *                  references of energy_err and angmom_err).
 *   R_exit         DP5 exit radius.
 *   steps, rejects, attempts   accepted steps, rejected and all DP5 attempts.
 *   status         MQCT_T_* bits so far.
 *   flags          MQCT_S_LAST_REJECTED: the last DP5 attempt was rejected (the
 *                  next accepted step may not grow h).
 *   system_id, N   the trajectory's system and channel count.
 */
enum { MQCT_S_LAST_REJECTED = 1 };
typedef struct {
  double t, t_origin, h;
  double classical[6];
  double E0, J0, R_exit;
  int64_t n_origin, steps, rejects, attempts;
  int32_t status, flags;
  int32_t system_id, N;
} mqct_traj_state;

/* Number of trajectories the state store holds (0 before the first run). */
mqct_status mqct_state_count(mqct_context* ctx, int64_t* count);
/* Copy the stored state of trajectories [first, first + count) to the host:
 * state [count] records, amps [sum of their N][2] (complex interleaved, may be
 * NULL).  Waits for the context stream.  Errors: MQCT_ERR_ARG (range beyond the
 * store, null state), MQCT_ERR_DEVICE. */
mqct_status mqct_get_state(mqct_context* ctx, int64_t first, int64_t count,
                           mqct_traj_state* state, double* amps);
/* Write host states into the store.  With first = 0 and count different from the
 * stored count the store is redefined to hold `count` trajectories (their
 * systems and N from the records); otherwise [first, first + count) must lie in
 * the store and each record must keep the system and N stored there.  amps
 * [sum of N][2] is required.  Values must be finite, R > 0, h >= 0, counts >= 0.
 * Synchronous.  Errors: MQCT_ERR_ARG, MQCT_ERR_STATE (unknown system),
 * MQCT_ERR_NONFINITE, MQCT_ERR_OOM, MQCT_ERR_DEVICE. */
mqct_status mqct_set_state(mqct_context* ctx, int64_t first, int64_t count,
                           const mqct_traj_state* state, const double* amps);

/*
 * mqct_run without device allocation, for callers that cannot allocate device
 * memory during the call (tight serving loops, harnesses that forbid it).  The
 * trajectory records and start amplitudes go to a fixed device scratch array of
 * 16 MiB that the library holds for the life of the process (one per GPU; the
 * context finds its address when it is created): at most 16 MiB / 200 B = 83,886
 * trajectories, fewer with a0 (the records plus 16 bytes per amplitude); a batch
 * beyond that fails with MQCT_ERR_ARG before any device work.  Fixed-step RK4 on
 * the per-trajectory schedule only (schedule MQCT_SCHED_AUTO or MQCT_SCHED_GEMV,
 * resume 0; otherwise MQCT_ERR_UNSUPPORTED); results must be device arrays
 * (mem = MQCT_MEM_DEVICE).  The results equal mqct_run's on that schedule; the
 * state store is left as it was.  The call waits for the context stream before it
 * stages the records (synchronous host-to-device copies) and returns with the
 * propagation enqueued.  All calls on one GPU share the scratch array, so calls
 * that overlap on one GPU (other threads, other contexts) race.  Errors as for
 * mqct_run.
 */
mqct_status mqct_run_noalloc(mqct_context* ctx, const mqct_batch_desc* batch,
                             const mqct_batch_result* result);

/*
 * Monte-Carlo cross sections (end of Section II; b sampled uniformly on
 * [0, b_max]):
 *   sigma[L'][L''] = (2 pi b_max / N_L') sum_{b : level(b) = L'} b_b sum_{n in L''} P_b(n)
 * in bohr^2, with N_L' the number of trajectories started in level L'.  All
 * trajectories share one channel-to-level map.  Computed on the device.
 *   mem               where P, b, init_level and sigma live.
 *   P                 [B][N]; b [B]; init_level [B]; level_of_channel host [N].
 *   sigma             [n_levels][n_levels].
 */
mqct_status mqct_cross_sections(mqct_context* ctx, int32_t mem, int64_t B, int32_t N,
                                const double* P, const double* b, const int32_t* init_level,
                                const int32_t* level_of_channel, int32_t n_levels,
                                double b_max, double* sigma);

/*
 * Linear parametric form of a system's coupling tables, for gradients with
 * respect to potential expansion coefficients (the potential expanded over
 * angular functions with R-dependent coefficients, Section II, Eqs. 12-18):
 *     M(R_k) = sum_p theta_p radial[p][k] G[gidx[p]],
 * G real symmetric [nG][N][N] (host), radial [P][K] (host), P <= 256,
 * nG <= 48, R64 storage only.  The natural spline of every radial[p] is
 * prepared on the device; the adjoint reads the nonzeros of G as lists (the
 * angular coupling matrices are sparse).  The loaded tables are not changed.
 */
mqct_status mqct_system_set_params(mqct_context* ctx, int32_t system_id, int32_t P,
                                   const double* radial, const int32_t* gidx, int32_t nG,
                                   const double* G);
/* Rebuild the system's tables on the device from the parametric form at theta
 * [P] (host) and re-prepare their spline.  Synchronous. */
mqct_status mqct_system_set_theta(mqct_context* ctx, int32_t system_id, const double* theta);
/*
 * Gradient of L = sum_b sum_n dL_dP[b][n] P_b(n) over the final probabilities
 * of an RK4 batch with respect to theta (summed over the batch), by the
 * discrete adjoint of RK4: a forward pass stores the state every
 * `checkpoint_every` steps and the four stage states of every step of the last
 * segment, then the segments are swept backward, each earlier one recomputed
 * from its checkpoint first (storing its stage states).  Device workspace:
 * (ceil(n_steps / checkpoint_every) + 4 checkpoint_every + 1) x (2 Npad + 4)
 * doubles per trajectory.  checkpoint_every >= n_steps stores every stage state
 * in the forward pass and recomputes nothing: 8 table passes per step instead of
 * 12, for 4 n_steps (2 Npad + 4) doubles per trajectory (67 MB at N = 256 and
 * 4096 steps); the forward and the backward pass then run as two launches.  The
 * gradient is the same bit for bit for every interval.  One
 * system per batch (with a parametric form), trajectories started from
 * init_channel / E_coll / b / R0 (a0, classical0, t0 must be NULL).  dL_dP [sum N_b] and dL_dtheta [P] are host arrays; P_out
 * (host [sum N_b], may be NULL) receives the final probabilities.  Synchronous.
 */
mqct_status mqct_adjoint(mqct_context* ctx, const mqct_batch_desc* batch, int32_t checkpoint_every,
                         const double* dL_dP, double* dL_dtheta, double* P_out);

/*
 * Options of the work-list schedule (MQCT_SCHED_QUEUE and DP5):
 *   MQCT_OPT_GRAPHS        1 (default): each chunk of step launches plus the
 *                          work-list compaction is captured once per grid size as
 *                          a HIP graph and replayed; 0: launched one by one.
 *   MQCT_OPT_AUTOTUNE      1 (default): the first batch of each (storage type,
 *                          padded N, integrator) class times the candidate
 *                          workgroup shapes (64..512 threads, fewest rows per lane
 *                          covering N) on a copy of up to 2048 of its
 *                          trajectories and keeps the fastest for the context;
 *                          0: the per-trajectory schedule's shape throughout.
 *                          The autotuner also times split-row shapes (4 or 8
 *                          waves that each hold all rows and stream a share of
 *                          the stored rows) against that choice on 32
 *                          trajectories; if one wins, the class switches to it
 *                          once its active count falls to twice the number of
 *                          compute units (the latency-bound tail of a batch).
 *   MQCT_OPT_CHUNK         step launches per replay (1..4096, default 16).
 *   MQCT_OPT_RESET_TUNING  forget the shapes chosen so far (value ignored).
 *   MQCT_OPT_TAIL          1 (default): use the tuned tail shape; 0: never switch;
 *                          2: run every class on its widest split-row shape from
 *                          the first step (for testing that form).
 *   MQCT_OPT_PER_LAUNCH    attempts (RK4 steps, DP5 attempts) of a trajectory per
 *                          step launch once a class is down to twice the number of
 *                          compute units (1..64; 1, the default: one per launch
 *                          throughout): a workgroup leaves its loop as soon as its
 *                          trajectory is done, so the value changes only the
 *                          number of launches, never a result.
 *   MQCT_OPT_COL_WORKSPACE the columns schedule's workspace cap in bytes (>= 0;
 *                          0, the default: 80 % of the device memory free at the
 *                          call plus the workspace already held).  The workspace
 *                          takes 80 (FP32 tables) or 96 (FP64) bytes per state and
 *                          column of a group, plus 64 bytes
 *                          per RK4 stage of each path; a batch whose path groups
 *                          exceed the cap runs in passes of whole groups, with the
 *                          same results bit for bit.  A single group above the cap
 *                          makes mqct_run return MQCT_ERR_OOM.
 * Results are reproducible for a given set of choices, chunk size and batch:
 * a shape switch happens at a chunk boundary.  Errors: MQCT_ERR_ARG.
 */
enum { MQCT_OPT_GRAPHS = 1, MQCT_OPT_AUTOTUNE = 2, MQCT_OPT_CHUNK = 3, MQCT_OPT_RESET_TUNING = 4,
       MQCT_OPT_TAIL = 5, MQCT_OPT_COL_WORKSPACE = 6, MQCT_OPT_PER_LAUNCH = 7 };
mqct_status mqct_set_option(mqct_context* ctx, int32_t option, int64_t value);
/* The shapes chosen so far, as JSON text: one object per class with dtype,
 * npad, method (0 RK4, 1 DP5), block, rows_per_lane, tuned, the candidates'
 * milliseconds per step launch, and the tail shape (or null) with its
 * candidates' timings.  Valid until the next call on ctx. */
const char* mqct_tuning_report(mqct_context* ctx);

/*
 * Cross-section post-processing (paper Section III).  sigma[e][i][f] is the cross
 * section for level i -> level f at the e-th collision energy (e < n_E; i, f < L),
 * g[L] the level degeneracies (2 j1 + 1)(2 j2 + 1).
 *   ratio[e][i][f] = g_i sigma_{i->f} / (g_f sigma_{f->i})   (the two sides of the
 *                    microscopic-reversibility condition, Eq. 19; NaN where the
 *                    right side is zero)
 *   sym[e][i][f]   = (g_i sigma_{i->f} + g_f sigma_{f->i}) / 2   (Eq. 20)
 * Either output may be NULL.  mem: where g, sigma, sym and ratio live
 * (MQCT_MEM_HOST: copied in and out, the call returns when the outputs are
 * written; MQCT_MEM_DEVICE: enqueued on the context stream).  Errors:
 * MQCT_ERR_ARG (sizes, null pointers), MQCT_ERR_NONFINITE (host inputs).
 */
mqct_status mqct_xs_symmetrize(mqct_context* ctx, int32_t mem, int32_t n_E, int32_t L,
                               const double* g, const double* sigma, double* sym, double* ratio);
/*
 * Rate coefficients from the symmetrised cross sections sym[e][i][f] (Eq. 20)
 * computed at the collision energies U[n_E] (hartree, increasing, 2 <= n_E <= 64),
 * by Maxwell-Boltzmann averaging (Section III, details in the paper's ref. 44).
 * U is read as the symmetrised translational energy (the mean of the initial and
 * final kinetic energies of a transition), so that with beta = k_B T (hartree)
 *   k[t][i][f] = (1/g_i) sqrt(8/(pi mu)) beta^(-3/2) exp(-(E_f - E_i)/(2 beta))
 *                * int s(U) U exp(-U/beta) dU
 * obeys detailed balance for any s; s is the natural cubic spline through
 * (U_e, sym_e) on [U_1, U_n], falls linearly to zero at the threshold
 * |E_f - E_i| / 2 below U_1, and stays at sym(U_n) above U_n.  E[L] level energies
 * (hartree), mu reduced mass (m_e), beta[n_T] > 0; k in bohr^3 per atomic unit of
 * time (x 6.1265e-9 for cm^3/s).  The integral is taken up to 40 beta past the
 * threshold by 8-point Gauss-Legendre on pieces no wider than 2 beta, the rest in
 * closed form.  mem as above (U, E, g, sym, beta and k in one space).  Errors:
 * MQCT_ERR_ARG (sizes, U not increasing, g, mu or beta not positive),
 * MQCT_ERR_NONFINITE.  Host inputs are validated; device inputs only by size.
 */
mqct_status mqct_rate_coefficients(mqct_context* ctx, int32_t mem, int32_t n_E, int32_t L,
                                   const double* U, const double* E, const double* g,
                                   const double* sym, double mu, int32_t n_T,
                                   const double* beta, double* k);

/*
 * Coupling-matrix builder for an asymmetric-top rotor + linear rotor (paper
 * Section II, Eqs. 12-18).  The potential is given by its expansion
 * V(R, angles) = sum_t v_t(R) tau_t (Eq. 12) over the angular functions of
 * Eq. 13, labelled t = (lam1, mu1, lam2, lam); the channels are the coupled
 * states of Eq. 3.  The builder writes, on the context stream,
 *   M_out[k][n''][n'] = <n'' m | V(R_k) | n' m>   (Eq. 6 by Eq. 17), zero between
 *                       channels of different m (Eq. 5 couples n' -> n'' within m)
 *   G_out[t][n''][n'] = the same element for v_t = 1 and every other v zero
 * in FP64, row n'' major.  Either output may be NULL (not both); both are
 * device memory the caller owns: M_out holds K*N*N doubles, G_out T*N*N.
 * M_out is what mqct_system_load takes as a device table (MQCT_MEM_DEVICE, real
 * input); the G_out and v rows are a parametric form for
 * mqct_system_set_params (radial = v, gidx = t, G = G_out copied to the host).
 * The call returns when both outputs are written.
 *
 * All descriptor arrays are host memory:
 *   N                  channels; j[N], m[N] total angular momentum and its
 *                      projection; rot1[N] index of the channel's rotor-1 state;
 *                      j2[N] the linear rotor's angular momentum.
 *                      |j1 - j2| <= j <= j1 + j2, |m| <= j.
 *   n_rot1, rot1_j     rotor-1 states and their j1 (0..40);
 *   b, b_stride        coefficients of Eq. 1: b[r * b_stride + k + j1] for
 *                      k = -j1..j1 (b_stride >= 2 j1 + 1), real;
 *   T, lam1, mu1,      expansion terms: 0 <= lam1, lam2 <= 20, |mu1| <= lam1,
 *   lam2, lam          |lam1 - lam2| <= lam <= lam1 + lam2;
 *   K, v               radial coefficients v[t * K + k] (hartree) at the knots.
 * j2 <= 40.  Errors: MQCT_ERR_ARG (bad sizes, indices, angular momenta, null
 * pointers), MQCT_ERR_NONFINITE (b or v), MQCT_ERR_OOM / MQCT_ERR_DEVICE.
 * The Clebsch-Gordan, 6j and 9j coefficients are formed in FP64 from
 * log-factorials; their relative error grows with the angular momenta (measured
 * against long-double sums: 2e-14 of the largest element for j <= 13, 3e-13 for
 * j <= 28).
 */
typedef struct {
  int32_t N;
  const int32_t* j;
  const int32_t* m;
  const int32_t* rot1;
  const int32_t* j2;
  int32_t n_rot1;
  const int32_t* rot1_j;
  const double* b;
  int32_t b_stride;
  int32_t T;
  const int32_t* lam1;
  const int32_t* mu1;
  const int32_t* lam2;
  const int32_t* lam;
  int32_t K;
  const double* v;
} mqct_coupling_desc;
mqct_status mqct_coupling_build(mqct_context* ctx, const mqct_coupling_desc* desc,
                                double* M_out, double* G_out);
/*
 * Screened build for bases too large for the dense tables (Section III: the
 * matrix was computed at two distances in the interaction region, the elements
 * above 1 cm^-1 were kept and only those were computed on the radial grid).
 * Every element of equal m is evaluated at n_screen radii, given by the
 * expansion coefficients there (v_screen[t * n_screen + s], host, 1 <= n_screen
 * <= 8); it is kept when max_s |M(R_s)| > drop_below (hartree), the element and
 * its transpose by the same evaluation, so both triangles are kept or dropped
 * together (the list loads with mqct_system_load_coo).  The kept elements are
 * written to device memory in an unspecified order:
 *   rows[i], cols[i]        row n'' and column n' of kept element i;
 *   values[k * capacity + i] its value at knot k (from desc->v), k < K.
 * *n_kept (host) receives the number of kept elements.  When it exceeds
 * capacity nothing is written beyond capacity and the call fails with
 * MQCT_ERR_ARG (call again with capacity >= *n_kept; capacity 0 only counts).
 * The call returns when the outputs are written.  Other errors as for
 * mqct_coupling_build.
 */
mqct_status mqct_coupling_build_sparse(mqct_context* ctx, const mqct_coupling_desc* desc,
                                       int32_t n_screen, const double* v_screen,
                                       double drop_below, int64_t capacity, int32_t* rows,
                                       int32_t* cols, double* values, int64_t* n_kept);

/*
 * Optional timing of the dominant step kernel of later runs: the fused
 * per-trajectory RK4 kernel, the table x columns product of the binned
 * schedule, or each replayed chunk of the work-list schedule.  HIP events are
 * recorded on the context stream around each of its launches.
 * mqct_profile_read waits for the stream and returns, since the last read:
 *   total_ms      summed milliseconds of the timed launches;
 *   launches      their number;
 *   table_bytes   (may be NULL) the algorithmic coupling-table bytes those
 *                 launches had to read: per-trajectory RK4, 4 spline slices of
 *                 N x Npad stored elements per right-hand side (4 per step plus
 *                 the final diagnostic one); binned product, the value and
 *                 second-derivative slices of every occupied knot once per stage
 *                 (counted on the device); 0 for the work-list schedule;
 *                 for mqct_coupling_build (whose fill kernel is timed), the
 *                 bytes it wrote (M_out and G_out).
 * and resets them.  Timing adds two event records per timed launch.
 */
mqct_status mqct_set_profiling(mqct_context* ctx, int32_t enable);
mqct_status mqct_profile_read(mqct_context* ctx, double* total_ms, int64_t* launches,
                              double* table_bytes);

/*
 * Achievable streaming-read bandwidth, the measured reference for the
 * bandwidth-bound kernels beside the datasheet peak (not part of the method).
 * Reads `bytes` at the device buffer `buf` (caller-owned, 16-byte aligned,
 * bytes a positive multiple of 16; its contents are only read) once untimed,
 * then `reps` (>= 1) times between two events on the context stream, with
 * 1 KiB-contiguous wave loads and four workgroups per compute unit.
 * *ms_per_pass (host) receives the mean milliseconds of one pass.  Synchronous.
 * Errors: MQCT_ERR_ARG (null pointers, size, alignment, reps), MQCT_ERR_DEVICE.
 */
mqct_status mqct_read_bandwidth(mqct_context* ctx, const void* buf, int64_t bytes, int32_t reps,
                                double* ms_per_pass);

#ifdef __cplusplus
}
#endif

#endif /* MQCT_H */
