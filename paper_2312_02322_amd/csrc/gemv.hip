// Fixed-step RK4 propagation with one workgroup per trajectory and the whole
// step loop inside the kernel (the right-hand side is rhs.h).
#include "rhs.h"

#include <math.h>

namespace mqct {

namespace {

using namespace rhs;

template <int DT, int BLOCK, int RPT>
struct Kern : Rhs<DT, BLOCK, RPT> {
  using Base = Rhs<DT, BLOCK, RPT>;
  using Base::NR;
  using Base::eval;
  using Base::energy;
  using Base::classical_rhs;
  using Base::init_state;
  using Base::write_out;

  // Fixed-step classical RK4: exactly n_steps steps, t_j = t0 + (j0 + j) h, where
  // j0 > 0 continues a stored state.
  __device__ static void run_rk4(const DevSystem& sy, const TrajIn& tj,
                                 const double* __restrict__ a0_all, TrajOut& out,
                                 const Lds<DT>& lds) {
    const double mu = sy.mu;
    double2 a0[NR], kk[NR], acc[NR];   // kk: stage input, then its derivative
    double y[4], ky[4] = {0.0, 0.0, 0.0, 0.0}, ay[4], theta, ptheta;
    init_state(sy, tj, a0_all, a0, y, theta, ptheta);
    const double R_exit = start_exit_radius(tj, y[0]);
#pragma unroll
    for (int r = 0; r < NR; ++r) kk[r] = make_double2(0.0, 0.0);
    const double h = tj.dt, t0 = tj.t0;
    const bool resume = (tj.flags & TRAJ_RESUME) != 0;
    const int64_t j0 = tj.step0;
    bool below = false;
    int32_t status = tj.status0;
    double E0 = tj.E0, J0 = tj.J0;
    bool first = !resume;
    const bool at = (tj.flags & TRAJ_AT) != 0;
    Sums tot;
    int64_t j = 0;
    for (; j < tj.n_steps; ++j) {
      const double t = t0 + (double)(j0 + j) * h;
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < 4; ++i) ay[i] = 0.0;
      for (int st = 0; st < 4; ++st) {
        const double cf = st == 0 ? 0.0 : (st == 3 ? h : 0.5 * h);
        const double wgt = (st == 0 || st == 3) ? 1.0 : 2.0;
        double ys[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) ys[i] = fma(cf, ky[i], y[i]);
#pragma unroll
        for (int r = 0; r < NR; ++r)
          kk[r] = make_double2(fma(cf, kk[r].x, a0[r].x), fma(cf, kk[r].y, a0[r].y));
        eval(sy, t + cf, ys[0], ys[3], kk, tot, below, lds, at);
        if (first) {
          E0 = energy(mu, ys, tot);
          J0 = ys[3] - tot.jx;
          first = false;
        }
        classical_rhs(mu, ys, tot, ky);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          acc[r].x = fma(wgt, kk[r].x, acc[r].x);
          acc[r].y = fma(wgt, kk[r].y, acc[r].y);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) ay[i] = fma(wgt, ky[i], ay[i]);
      }
      const double h6 = h / 6.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        a0[r].x += h6 * acc[r].x;
        a0[r].y += h6 * acc[r].y;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) y[i] = uni(y[i] + h6 * ay[i]);
      if (!isfinite(tot.force) || !isfinite(tot.torque) || !isfinite(tot.norm) ||
          !isfinite(y[0]) || !isfinite(y[2]) || !isfinite(y[3])) {
        status |= ST_NONFINITE;
        ++j;
        break;
      }
    }
    // diagnostics at the final state (one more evaluation; its derivative is unused)
    const double tend = t0 + (double)(j0 + j) * h;
    bool b2 = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = a0[r];
    eval(sy, tend, y[0], y[3], acc, tot, b2, lds, at);
    if (first) {
      E0 = energy(mu, y, tot);
      J0 = y[3] - tot.jx;
    }
    if (below) status |= ST_BELOW_GRID;
    const int64_t steps = tj.steps0 + j;
    write_out(sy, tj, out, a0, y, theta, ptheta, tend, steps, tj.rejects0, status, tot, E0, J0);
    if (threadIdx.x == 0)
      put_traj_state(out, tj, sy.N, tend, t0, j0 + j, h, y, theta, ptheta, E0, J0, R_exit, steps,
                     tj.rejects0, tj.attempts0 + j, status, tj.dflags);
  }
};

// One workgroup per trajectory (grid = number of trajectories), RK4.
template <int DT, int BLOCK, int RPT>
__global__ void __launch_bounds__(BLOCK)
rk4_gemv_kernel(const DevSystem* __restrict__ systems, const TrajIn* __restrict__ trajs,
                const double* __restrict__ a0_all, TrajOut out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const TrajIn tj = trajs[blockIdx.x];
  const DevSystem sy = systems[tj.sys];
  Lds<DT> lds(smem, sy.Npad);
  Kern<DT, BLOCK, RPT>::run_rk4(sy, tj, a0_all, out, lds);
}

template <int DT, int BLOCK, int RPT>
hipError_t launch_one(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                      const double* d_a0, TrajOut out, int max_npad, hipStream_t s) {
  const bool fp32 = DT == C64 || DT == R32;
  size_t lds = lds_bytes(max_npad, fp32);
  auto kern = rk4_gemv_kernel<DT, BLOCK, RPT>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  for (int64_t first = 0; first < n_traj; first += 1 << 30) {
    int64_t cnt = n_traj - first < (1 << 30) ? n_traj - first : (1 << 30);
    kern<<<(unsigned)cnt, BLOCK, lds, s>>>(d_systems, d_traj + first, d_a0, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int DT>
hipError_t launch_dt(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                     const double* d_a0, TrajOut out, int max_npad, hipStream_t s) {
  const int groups = max_npad / Tr<DT>::VEC;
  if (groups <= 64) return launch_one<DT, 64, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 128) return launch_one<DT, 128, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 256) return launch_one<DT, 256, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 512) return launch_one<DT, 512, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 1024) return launch_one<DT, 512, 2>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 2048) return launch_one<DT, 512, 4>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 4096) return launch_one<DT, 512, 8>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_rk4_gemv_t(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                             const double* d_a0, TrajOut out, int dtype, int max_npad,
                             hipStream_t s);

hipError_t launch_rk4_gemv(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                           const double* d_a0, TrajOut out, int dtype, int max_npad,
                           hipStream_t s, Prof* prof) {
  hipEvent_t e0 = prof ? prof->next() : nullptr, e1 = prof ? prof->next() : nullptr;
  prof_mark(prof, e0, s);
  hipError_t r = launch_rk4_gemv_t(d_systems, d_traj, n_traj, d_a0, out, dtype, max_npad, s);
  prof_mark(prof, e1, s);
  return r;
}

hipError_t launch_rk4_gemv_t(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                             const double* d_a0, TrajOut out, int dtype, int max_npad,
                             hipStream_t s) {
  switch (dtype) {
    case C128: return launch_dt<C128>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
    case C64: return launch_dt<C64>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
    case R64: return launch_dt<R64>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
    case R32: return launch_dt<R32>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mqct
