// Kernels of the work-list schedule: batches of trajectories of uneven size
// and length (different systems, collision energies, impact parameters),
// advanced by short kernels that each perform ONE step attempt for every
// trajectory still on the work list.
//
//   init    one workgroup per trajectory: initial state (end of Section II),
//           first right-hand side (and, for the adaptive stepper, the starting
//           step size), work-list entry.
//   step    one workgroup per work-list entry: one fixed RK4 step, or one
//           Dormand-Prince 5(4) attempt (six right-hand sides, the embedded
//           error estimate and the accept/reject decision).  A trajectory that
//           finishes evaluates its end state once more for the diagnostics and
//           writes its results.
//   compact one workgroup: removes finished trajectories from the work list,
//           orders the rest by R (counting sort over 1/4-bohr buckets, so that
//           concurrent workgroups read the same table slices) and updates the
//           active count.
//
// The launches read the active count from device memory, so a fixed grid can
// be replayed (HIP graph) while the list shrinks: workgroups past the count
// return at once.  The right-hand side is rhs.h; the per-trajectory state
// lives in global memory between launches.
#pragma once

#include "rhs.h"

namespace mqct {
namespace queue {

using namespace rhs;

// Dormand-Prince 5(4) tableau (Dormand & Prince 1980): nodes, stage
// coefficients, and fifth-order minus embedded fourth-order weights.
static __constant__ double QC[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static __constant__ double QA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static __constant__ double QE[7] = {71.0 / 57600, 0.0, -71.0 / 16695, 71.0 / 1920,
                                    -17253.0 / 339200, 22.0 / 525, -1.0 / 40};

template <int DT, int BLOCK, int RPT, bool SPLIT>
struct QK : Rhs<DT, BLOCK, RPT, SPLIT> {
  using Base = Rhs<DT, BLOCK, RPT, SPLIT>;
  using Base::NR;
  using Base::NW;
  using Base::row;
  using Base::eval;
  using Base::energy;
  using Base::classical_rhs;
  using Base::init_state;
  using Base::write_out;

  __device__ static void put_state(QState* p, const QState& s) {
    if (threadIdx.x == 0) *p = s;
  }

  // The stored state of a trajectory at the end of the call; rk4: the time is
  // t0 + n_idx h of fixed steps, else an adaptive time (origin = t).
  __device__ static void store_state(const DevSystem& sy, const TrajIn& tj, const TrajOut& out,
                                     const QState& s, bool rk4) {
    if (threadIdx.x == 0)
      put_traj_state(out, tj, sy.N, s.t, rk4 ? tj.t0 : s.t, rk4 ? s.n_idx : 0, s.h, s.yc,
                     s.theta, s.ptheta, s.E0, s.J0, s.R_exit, s.steps, s.rejects, s.attempts,
                     s.status, (s.flags & Q_LASTREJ) ? MQCT_S_LAST_REJECTED : 0);
  }

  // Results of a finished trajectory: one more right-hand side at its end
  // state gives the norm, energy and J_x diagnostics.  Each step kernel calls it
  // from one place only (a stored trajectory that had stopped for good comes
  // back through the same place, see Q_FINISH), so the results of a trajectory
  // are formed by the same instructions whichever call it finished in (inlined
  // copies may contract multiply-adds differently).
  __device__ static void finish(const DevSystem& sy, const TrajIn& tj, const TrajOut& out,
                                const double2 (&a)[NR], const QState& s, const Lds<DT>& lds,
                                bool rk4) {
    double2 cur[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) cur[r] = a[r];
    Sums tot;
    bool b2 = false;
    eval(sy, s.t, s.yc[0], s.yc[3], cur, tot, b2, lds, (tj.flags & TRAJ_AT) != 0);
    write_out(sy, tj, out, a, s.yc, s.theta, s.ptheta, s.t, s.steps, s.rejects, s.status, tot,
              s.E0, s.J0);
    if (out.P) store_state(sy, tj, out, s, rk4);
  }

  __device__ static void load_rows(const double2* __restrict__ v, int N, double2 (&a)[NR]) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      a[r] = n < N ? v[n] : make_double2(0.0, 0.0);
    }
  }

  __device__ static void store_rows(double2* __restrict__ v, int N, const double2 (&a)[NR]) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n < N) v[n] = a[r];
    }
  }

  // ---- fixed-step RK4 -------------------------------------------------------

  __device__ static void init_rk4(const QArgs& q, int i, const Lds<DT>& lds) {
    const TrajIn tj = q.ws.traj[i];
    const DevSystem sy = q.systems[tj.sys];
    double2 a[NR], cur[NR];
    QState s{};
    init_state(sy, tj, q.a0_all, a, s.yc, s.theta, s.ptheta);
    const bool resume = (tj.flags & TRAJ_RESUME) != 0;
    s.n_idx = tj.step0;
    s.t = tj.t0 + (double)s.n_idx * tj.dt;
    s.h = tj.dt;
    s.R_exit = start_exit_radius(tj, s.yc[0]);
    s.steps = tj.steps0;
    s.rejects = tj.rejects0;
    s.attempts = tj.attempts0;
    s.status = tj.status0;
    s.flags = (tj.dflags & MQCT_S_LAST_REJECTED) ? Q_LASTREJ : 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) cur[r] = a[r];
    Sums tot;
    bool below = false;
    eval(sy, s.t, s.yc[0], s.yc[3], cur, tot, below, lds, (tj.flags & TRAJ_AT) != 0);
    s.E0 = resume ? tj.E0 : energy(sy.mu, s.yc, tot);
    s.J0 = resume ? tj.J0 : s.yc[3] - tot.jx;
    store_rows(q.ws.amp + (int64_t)i * q.ws.npad, sy.N, a);
    if (tj.n_steps <= 0) {
      s.flags |= Q_DONE;
      write_out(sy, tj, q.out, a, s.yc, s.theta, s.ptheta, s.t, s.steps, s.rejects, s.status,
                tot, s.E0, s.J0);
      if (q.out.P) store_state(sy, tj, q.out, s, true);
    }
    put_state(q.ws.st + i, s);
  }

  // One classical RK4 step, t_j = t0 + j h (j counted from the start of the
  // trajectory, also across a stored state); exactly n_steps steps per call.
  __device__ static void step_rk4(const QArgs& q, int i, QState& s, const Lds<DT>& lds) {
    const TrajIn tj = q.ws.traj[i];
    const DevSystem sy = q.systems[tj.sys];
    const double mu = sy.mu, h = tj.dt;
    double2* amp = q.ws.amp + (int64_t)i * q.ws.npad;
    double2 a0[NR], kk[NR], acc[NR];
    load_rows(amp, sy.N, a0);
    double y[4], ky[4] = {0.0, 0.0, 0.0, 0.0}, ay[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = s.yc[k];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      kk[r] = make_double2(0.0, 0.0);
      acc[r] = make_double2(0.0, 0.0);
    }
    const double t = tj.t0 + (double)s.n_idx * h;
    bool below = false;
    Sums tot;
    for (int st = 0; st < 4; ++st) {
      const double cf = st == 0 ? 0.0 : (st == 3 ? h : 0.5 * h);
      const double wgt = (st == 0 || st == 3) ? 1.0 : 2.0;
      double ys[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) ys[k] = fma(cf, ky[k], y[k]);
#pragma unroll
      for (int r = 0; r < NR; ++r)
        kk[r] = make_double2(fma(cf, kk[r].x, a0[r].x), fma(cf, kk[r].y, a0[r].y));
      eval(sy, t + cf, ys[0], ys[3], kk, tot, below, lds, (tj.flags & TRAJ_AT) != 0);
      classical_rhs(mu, ys, tot, ky);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        acc[r].x = fma(wgt, kk[r].x, acc[r].x);
        acc[r].y = fma(wgt, kk[r].y, acc[r].y);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) ay[k] = fma(wgt, ky[k], ay[k]);
    }
    const double h6 = h / 6.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      a0[r].x += h6 * acc[r].x;
      a0[r].y += h6 * acc[r].y;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) s.yc[k] = uni(y[k] + h6 * ay[k]);
    s.steps += 1;
    s.attempts += 1;
    s.n_idx += 1;
    s.t = tj.t0 + (double)s.n_idx * h;
    if (below) s.status |= ST_BELOW_GRID;
    if (!isfinite(tot.force) || !isfinite(tot.torque) || !isfinite(tot.norm) ||
        !isfinite(s.yc[0]) || !isfinite(s.yc[2]) || !isfinite(s.yc[3])) {
      s.status |= ST_NONFINITE;
      s.flags |= Q_DONE;
    }
    if (s.n_idx - tj.step0 >= tj.n_steps) s.flags |= Q_DONE;
    store_rows(amp, sy.N, a0);
    if (s.flags & Q_DONE) finish(sy, tj, q.out, a0, s, lds, true);
  }

  // ---- adaptive Dormand-Prince 5(4) -----------------------------------------
  //
  // Error: scaled RMS over the 2N+6 real state components (Theta and P_Theta
  // are constant and contribute zero error), sc_i = atol + rtol max(|y_i|,
  // |y_new,i|).  Step factor min(5, max(0.2, 0.9 err^-1/5)), no growth right
  // after a rejection.  Starting step: Hairer, Norsett & Wanner, Solving ODEs I,
  // Sec. II.4.  Stop after the first accepted step with R >= R0 and P_R > 0, or
  // when h < h_min, the accepted-step limit or the attempt limit is reached, or
  // on a non-finite error.  Stage derivatives (first same as last) live in the
  // trajectory's global slice kst[8][npad] (slots 0..6 = k1..k7, slot 7 = the
  // fifth-order solution); every lane touches only its own rows.  The classical
  // stage derivatives of one attempt live in LDS (written by lane 0, then a
  // barrier).

  __device__ static void init_dp5(const QArgs& q, int i, const Lds<DT>& lds) {
    const TrajIn tj = q.ws.traj[i];
    const DevSystem sy = q.systems[tj.sys];
    const int N = sy.N;
    const double mu = sy.mu, rtol = q.ctl.rtol, atol = q.ctl.atol;
    const double ncomp = 2.0 * N + 6.0;
    double2* ks = q.ws.kst + (int64_t)i * 8 * q.ws.npad;
    double2 a[NR], f0[NR], st[NR];
    QState s{};
    init_state(sy, tj, q.a0_all, a, s.yc, s.theta, s.ptheta);
    const bool resume = (tj.flags & TRAJ_RESUME) != 0;
    s.t = tj.t0;
    s.R_exit = start_exit_radius(tj, s.yc[0]);
#pragma unroll
    for (int r = 0; r < NR; ++r) f0[r] = a[r];
    Sums tot;
    bool below = false;
    eval(sy, s.t, s.yc[0], s.yc[3], f0, tot, below, lds, (tj.flags & TRAJ_AT) != 0);
    s.E0 = resume ? tj.E0 : energy(mu, s.yc, tot);
    s.J0 = resume ? tj.J0 : s.yc[3] - tot.jx;
    classical_rhs(mu, s.yc, tot, s.kc1);
    store_rows(ks, N, f0);
    store_rows(q.ws.amp + (int64_t)i * q.ws.npad, N, a);
    if (resume) {
      // a stored state: its step size, rejection flag and counts continue (the
      // first stage above is f at the stored state, first same as last)
      s.h = tj.h0;
      s.steps = tj.steps0;
      s.rejects = tj.rejects0;
      s.attempts = tj.attempts0;
      s.status = tj.status0;
      s.flags = (tj.dflags & MQCT_S_LAST_REJECTED) ? Q_LASTREJ : 0;
      if (below) s.status |= ST_BELOW_GRID;
      // stopped for good: the first step launch forms the results as the
      // finishing step gave them, without an attempt
      if (tj.flags & TRAJ_FINISHED) s.flags |= Q_FINISH;
      put_state(q.ws.st + i, s);
      return;
    }
    const double yfull[6] = {s.yc[0], s.theta, s.yc[1], s.yc[2], s.ptheta, s.yc[3]};
    // d0 = ||y||, d1 = ||f(t0, y0)||
    double s2[2] = {0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (row(r) >= N) continue;
      const double sx = atol + rtol * fabs(a[r].x), sy_ = atol + rtol * fabs(a[r].y);
      s2[0] += (a[r].x / sx) * (a[r].x / sx) + (a[r].y / sy_) * (a[r].y / sy_);
      s2[1] += (f0[r].x / sx) * (f0[r].x / sx) + (f0[r].y / sy_) * (f0[r].y / sy_);
    }
    Base::template reduce<2>(s2, lds.red1);
    const double kf[6] = {s.kc1[0], 0.0, s.kc1[1], s.kc1[2], 0.0, s.kc1[3]};
    for (int k = 0; k < 6; ++k) {
      const double sc = atol + rtol * fabs(yfull[k]);
      s2[0] += (yfull[k] / sc) * (yfull[k] / sc);
      s2[1] += (kf[k] / sc) * (kf[k] / sc);
    }
    const double d0 = sqrt(s2[0] / ncomp), d1 = sqrt(s2[1] / ncomp);
    const double h0 = uni((d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1);
    // d2 = ||f(t0 + h0, y0 + h0 f0) - f0|| / h0
#pragma unroll
    for (int r = 0; r < NR; ++r)
      st[r] = make_double2(fma(h0, f0[r].x, a[r].x), fma(h0, f0[r].y, a[r].y));
    double ys[4], kc[4];
    for (int k = 0; k < 4; ++k) ys[k] = uni(fma(h0, s.kc1[k], s.yc[k]));
    eval(sy, s.t + h0, ys[0], ys[3], st, tot, below, lds, (tj.flags & TRAJ_AT) != 0);
    classical_rhs(mu, ys, tot, kc);
    double s1[1] = {0.0};
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (row(r) >= N) continue;
      const double sx = atol + rtol * fabs(a[r].x), sy_ = atol + rtol * fabs(a[r].y);
      const double ex = (st[r].x - f0[r].x) / sx, ey = (st[r].y - f0[r].y) / sy_;
      s1[0] += ex * ex + ey * ey;
    }
    Base::template reduce<1>(s1, lds.red1);
    const double dk[6] = {kc[0] - s.kc1[0], 0.0, kc[1] - s.kc1[1], kc[2] - s.kc1[2], 0.0,
                          kc[3] - s.kc1[3]};
    for (int k = 0; k < 6; ++k) {
      const double sc = atol + rtol * fabs(yfull[k]);
      s1[0] += (dk[k] / sc) * (dk[k] / sc);
    }
    const double d2 = sqrt(s1[0] / ncomp) / h0;
    const double dm = fmax(d1, d2);
    const double h1 = dm <= 1e-15 ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 1.0 / 5.0);
    s.h = uni(fmin(100.0 * h0, h1));
    if (below) s.status |= ST_BELOW_GRID;
    put_state(q.ws.st + i, s);
  }

  __device__ static void step_dp5(const QArgs& q, int i, QState& s, const Lds<DT>& lds) {
    const TrajIn tj = q.ws.traj[i];
    const DevSystem sy = q.systems[tj.sys];
    const int N = sy.N, np = q.ws.npad;
    const double mu = sy.mu, rtol = q.ctl.rtol, atol = q.ctl.atol;
    const double ncomp = 2.0 * N + 6.0;
    double2* amp = q.ws.amp + (int64_t)i * np;
    double2* ks = q.ws.kst + (int64_t)i * 8 * np;
    double* kcl = lds.kcl;   // [7][4]: slot q = classical derivative of stage q (q >= 1)
    bool done = false;
    if (s.flags & Q_FINISH) {
      s.flags &= ~Q_FINISH;
      done = true;
    } else {
    const double h = s.h;
    double2 st[NR];
    double y5c[4] = {0.0, 0.0, 0.0, 0.0};
    Sums tot;
    bool below = false;
    for (int sg = 1; sg < 7; ++sg) {
      // stage input y + h sum_{p < sg} a_{sg,p} k_p
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int n = row(r);
        double2 acc = make_double2(0.0, 0.0);
        if (n < N) {
          acc = amp[n];
          for (int p = 0; p < sg; ++p) {
            const double2 kp = ks[(int64_t)p * np + n];
            const double c = h * QA[sg][p];
            acc.x = fma(c, kp.x, acc.x);
            acc.y = fma(c, kp.y, acc.y);
          }
          if (sg == 6) ks[(int64_t)7 * np + n] = acc;
        }
        st[r] = acc;
      }
      double ys[4];
      for (int k = 0; k < 4; ++k) {
        double acc = fma(h * QA[sg][0], s.kc1[k], s.yc[k]);
        for (int p = 1; p < sg; ++p) acc = fma(h * QA[sg][p], kcl[p * 4 + k], acc);
        ys[k] = uni(acc);
        if (sg == 6) y5c[k] = ys[k];
      }
      eval(sy, s.t + QC[sg] * h, ys[0], ys[3], st, tot, below, lds, (tj.flags & TRAJ_AT) != 0);
      double kc[4];
      classical_rhs(mu, ys, tot, kc);
      if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) kcl[sg * 4 + k] = kc[k];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int n = row(r);
        if (n < N) ks[(int64_t)sg * np + n] = st[r];
      }
      __syncthreads();   // kcl[sg] visible to every wave
    }
    // scaled RMS error of h sum_q e_q k_q
    double e2[1] = {0.0};
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n >= N) continue;
      double ex = 0.0, ey = 0.0;
      for (int p = 0; p < 7; ++p) {
        const double2 kp = ks[(int64_t)p * np + n];
        ex = fma(QE[p], kp.x, ex);
        ey = fma(QE[p], kp.y, ey);
      }
      ex *= h; ey *= h;
      const double2 y0 = amp[n], y5 = ks[(int64_t)7 * np + n];
      const double sx = atol + rtol * fmax(fabs(y0.x), fabs(y5.x));
      const double sy_ = atol + rtol * fmax(fabs(y0.y), fabs(y5.y));
      e2[0] += (ex / sx) * (ex / sx) + (ey / sy_) * (ey / sy_);
    }
    double ecl = 0.0;
    for (int k = 0; k < 4; ++k) {
      double e = QE[0] * s.kc1[k];
      for (int p = 1; p < 7; ++p) e = fma(QE[p], kcl[p * 4 + k], e);
      e *= h;
      const double sc = atol + rtol * fmax(fabs(s.yc[k]), fabs(y5c[k]));
      ecl += (e / sc) * (e / sc);
    }
    Base::template reduce<1>(e2, lds.red1);
    const double en = uni(sqrt((e2[0] + ecl) / ncomp));
    if (below) s.status |= ST_BELOW_GRID;
    s.attempts += 1;
    if (!isfinite(en)) {
      s.status |= ST_NONFINITE;
      done = true;
    } else if (en <= 1.0) {
      s.t += h;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int n = row(r);
        if (n < N) {
          amp[n] = ks[(int64_t)7 * np + n];
          ks[n] = ks[(int64_t)6 * np + n];
        }
      }
      for (int k = 0; k < 4; ++k) {
        s.yc[k] = y5c[k];
        s.kc1[k] = kcl[6 * 4 + k];
      }
      s.steps += 1;
      double fac = en == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(en, -0.2)));
      if (s.flags & Q_LASTREJ) fac = fmin(1.0, fac);
      s.flags &= ~Q_LASTREJ;
      if (s.yc[0] >= s.R_exit && s.yc[2] > 0.0) {
        s.status |= ST_EXITED;
        done = true;
      } else {
        s.h = uni(h * fac);
      }
    } else {
      s.rejects += 1;
      s.h = uni(h * fmax(0.2, 0.9 * pow(en, -0.2)));
      s.flags |= Q_LASTREJ;
    }
    if (!done && s.h < q.ctl.h_min) { s.status |= ST_STEP_UNDERFLOW; done = true; }
    if (!done && s.steps >= q.ctl.max_steps) { s.status |= ST_MAX_STEPS; done = true; }
    if (!done && s.attempts >= q.max_attempts) { s.status |= ST_MAX_STEPS; done = true; }
    }
    if (done) {
      s.flags |= Q_DONE;
      double2 a[NR];
      load_rows(amp, N, a);
      finish(sy, tj, q.out, a, s, lds, false);
    }
  }
};

template <int DT, int BLOCK, int RPT, bool SPLIT, int METHOD>
__global__ void __launch_bounds__(BLOCK) q_init(QArgs q) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int i = blockIdx.x;
  Lds<DT> lds(smem, q.ws.npad);
  if (METHOD == 0) QK<DT, BLOCK, RPT, SPLIT>::init_rk4(q, i, lds);
  else QK<DT, BLOCK, RPT, SPLIT>::init_dp5(q, i, lds);
  if (threadIdx.x == 0) q.ws.list[i] = i;
  if (i == 0 && threadIdx.x == 0) *q.ws.count = q.ws.n;
}

// One attempt (MULTI = false), or up to q.per_launch attempts of one trajectory
// (MULTI = true, for the latency-bound tail of a batch; a separate kernel
// because the loop costs registers that the one-attempt form keeps for
// occupancy), leaving the loop when the trajectory is done.  Every thread holds
// the same state (its fields come from workgroup reductions and LDS) and the exit
// is taken from one workgroup vote, so all waves leave together; each attempt
// reads back only the rows its own threads wrote, and its LDS areas are separated
// from the next attempt's writes by the barriers of the stage evaluations.
template <int DT, int BLOCK, int RPT, bool SPLIT, int METHOD, bool MULTI>
__global__ void __launch_bounds__(BLOCK) q_step(QArgs q) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int cnt = *q.ws.count;
  if ((int)blockIdx.x >= cnt) return;
  const int i = q.ws.list[blockIdx.x];
  QState s = q.ws.st[i];
  if (s.flags & Q_DONE) return;
  Lds<DT> lds(smem, q.ws.npad);
  const int na = MULTI ? q.per_launch : 1;
  for (int a = 0; a < na; ++a) {
    if (METHOD == 0) QK<DT, BLOCK, RPT, SPLIT>::step_rk4(q, i, s, lds);
    else QK<DT, BLOCK, RPT, SPLIT>::step_dp5(q, i, s, lds);
    if (!MULTI || __syncthreads_or((s.flags & Q_DONE) != 0)) break;
  }
  if (threadIdx.x == 0) q.ws.st[i] = s;
}

// Workgroup shapes (threads, 16-byte row groups per lane, split-row form) the
// schedule can use: row-split 0..10, split-row 11..16.
constexpr int QSHAPES = QUEUE_SHAPES;
__host__ __device__ constexpr int qshape_block(int k) {
  return k < 2 ? 64 : k < 4 ? 128 : k < 7 ? 256 : k < 11 ? 512 : k < 14 ? 256 : 512;
}
__host__ __device__ constexpr int qshape_rpt(int k) {
  return k == 0 ? 1 : k == 1 ? 2 : k == 2 ? 1 : k == 3 ? 2 : k == 4 ? 1 : k == 5 ? 2
       : k == 6 ? 4 : k == 7 ? 1 : k == 8 ? 2 : k == 9 ? 4 : k == 10 ? 8
       : k == 11 || k == 14 ? 1 : k == 12 || k == 15 ? 2 : 4;
}
__host__ __device__ constexpr bool qshape_split(int k) { return k >= 11; }

template <int DT, int K>
void fill_one(QKernelSet& ks) {
  constexpr int BL = qshape_block(K), RP = qshape_rpt(K);
  constexpr bool SP = qshape_split(K);
  ks.block = BL;
  ks.rpt = RP;
  ks.split_waves = SP ? BL / 64 : 0;
  // rows per workgroup (per wave for the split-row form) beyond the largest
  // supported column count are not built
  if constexpr ((SP ? 64 : BL) * RP * Tr<DT>::VEC > 4096) {
    ks.init[0] = ks.init[1] = ks.step[0] = ks.step[1] = ks.step_multi[0] = ks.step_multi[1] =
        nullptr;
    return;
  } else {
    ks.init[0] = (const void*)q_init<DT, BL, RP, SP, 0>;
    ks.init[1] = (const void*)q_init<DT, BL, RP, SP, 1>;
    ks.step[0] = (const void*)q_step<DT, BL, RP, SP, 0, false>;
    ks.step[1] = (const void*)q_step<DT, BL, RP, SP, 1, false>;
    ks.step_multi[0] = (const void*)q_step<DT, BL, RP, SP, 0, true>;
    ks.step_multi[1] = (const void*)q_step<DT, BL, RP, SP, 1, true>;
  }
}

template <int DT, int K>
void fill_all(QKernelSet* t) {
  if constexpr (K < QSHAPES) {
    fill_one<DT, K>(t[K]);
    fill_all<DT, K + 1>(t);
  }
}

}  // namespace queue
}  // namespace mqct
