// Propagation of Ehrenfest mean-field trajectories with the whole step loop
// inside the kernel: fixed-step RK4 with one workgroup per trajectory, and a
// persistent form (RK4 or adaptive Dormand-Prince 5(4)) in which workgroups
// drain a queue of trajectories of uneven size and length.
//
// Right-hand side (paper Section II, Eqs. 5 and 7-10, collision plane
// Theta = pi/2):
//   c_m   = e^{-i E_m t} a_m                      (Eq. 4 phase, factorised per channel)
//   u     = M(R) c,  v = M'(R) c                  (one pass over the four spline slices
//                                                  M_k, M_{k+1}, M2_k, M2_{k+1})
//   y_n   = e^{+i E_n t} u_n                      (= sum_m M_nm e^{i(E_n - E_m)t} a_m)
//   x     = J_x a
//   da/dt = -i y - i Phidot x                     (Eq. 5, Coriolis generator -i Phidot J_x)
//   dR/dt = P_R/mu,  dPhi/dt = Phidot = P_Phi/(mu R^2)                 (Eqs. 7, 8)
//   dP_R/dt   = -Re(c^H v) + P_Phi^2/(mu R^3)                           (Eq. 9)
//   dP_Phi/dt = 2 Im(x^H y) = -i <[J_x, V]>                             (Eq. 10)
//
// Work split: lane n of the workgroup owns output rows n (16-byte column
// groups of the stored tables).  Because every knot's matrix is Hermitian,
// column n of the stored matrix is conj(row n), so all lanes of a wave stream
// one stored row m contiguously while each keeps its own row sums in registers;
// no cross-lane reduction is needed for the matvec.  c lives in LDS and is read
// as a broadcast.  Only the two mean-field scalars (force, torque) and the
// diagnostics are reduced across the workgroup (wave shuffles, then LDS).
//
// Precision: the FP64 tables use FP64 throughout.  The FP32 tables (R32/C64)
// multiply in FP32 and accumulate in FP32 over chunks of 64 stored rows, then
// add the chunk sums into FP64; phases (E t), spline weights, the classical
// state and every RK accumulator stay FP64.
#include "device.h"

#include <math.h>

namespace mqct {

namespace {

template <int DT> struct Tr;
template <> struct Tr<C128> {
  using S = double; using L = double2; using CS = double2;
  static constexpr int VEC = 1; static constexpr bool CPLX = true;
};
template <> struct Tr<C64> {
  using S = float; using L = float4; using CS = float2;
  static constexpr int VEC = 2; static constexpr bool CPLX = true;
};
template <> struct Tr<R64> {
  using S = double; using L = double2; using CS = double2;
  static constexpr int VEC = 2; static constexpr bool CPLX = false;
};
template <> struct Tr<R32> {
  using S = float; using L = float2; using CS = float2;
  static constexpr int VEC = 2; static constexpr bool CPLX = false;
};

constexpr int CHUNK = 64;   // stored rows per FP32 partial sum

// Dormand-Prince 5(4) tableau (Dormand & Prince 1980): nodes, stage
// coefficients, and fifth-order minus embedded fourth-order weights.
__constant__ double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
__constant__ double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
__constant__ double DP_E[7] = {71.0 / 57600, 0.0, -71.0 / 16695, 71.0 / 1920,
                               -17253.0 / 339200, 22.0 / 525, -1.0 / 40};


// Sums produced by one right-hand-side evaluation.
struct Sums {
  double force;    // Re(c^H v)
  double torque;   // Im((J_x c)^H u)  = Im(x^H y)
  double vexp;     // Re(c^H u) = <V>
  double erot;     // sum E_n |a_n|^2
  double norm;     // sum |a_n|^2
  double jx;       // Re(c^H J_x c) = Re(a^H J_x a)
};

// Complex accumulation of u += conj(val) c and v += conj(der) c for one element
// (complex tables) or u += val c, v += der c (real tables).
template <bool CPLX, typename F, typename F2>
__device__ __forceinline__ void elem(F2& u, F2& v, F s0r, F s0i, F s1r, F s1i, F s2r, F s2i,
                                     F s3r, F s3i, const F (&w)[4], const F (&d)[4], F2 c) {
  if constexpr (CPLX) {
    F vr = w[0] * s0r + w[1] * s1r + w[2] * s2r + w[3] * s3r;
    F vi = w[0] * s0i + w[1] * s1i + w[2] * s2i + w[3] * s3i;
    F dr = d[0] * s0r + d[1] * s1r + d[2] * s2r + d[3] * s3r;
    F di = d[0] * s0i + d[1] * s1i + d[2] * s2i + d[3] * s3i;
    u.x += vr * c.x + vi * c.y;
    u.y += vr * c.y - vi * c.x;
    v.x += dr * c.x + di * c.y;
    v.y += dr * c.y - di * c.x;
  } else {
    F vr = w[0] * s0r + w[1] * s1r + w[2] * s2r + w[3] * s3r;
    F dr = d[0] * s0r + d[1] * s1r + d[2] * s2r + d[3] * s3r;
    u.x += vr * c.x;
    u.y += vr * c.y;
    v.x += dr * c.x;
    v.y += dr * c.y;
  }
}


// LDS layout shared by the kernels (bytes):
//   c     [Npad] in the matvec precision (float2 or double2)
//   c64   [Npad] double2 (aliases c on the FP64 path)
//   red0  [16][8] doubles, red1 [16][8] doubles  (two reduction areas)
//   kcl   [8][4] doubles                        (DP5 classical stages and y5)
__host__ __device__ inline size_t lds_bytes(int npad, bool fp32) {
  size_t c = fp32 ? (((size_t)npad * 8 + 15) & ~(size_t)15) : 0;
  return c + (size_t)npad * 16 + 2 * 16 * 8 * 8 + 8 * 4 * 8;
}

template <int DT>
struct Lds {
  typename Tr<DT>::CS* c;
  double2* c64;
  double* red0;
  double* red1;
  double* kcl;
  __device__ Lds(unsigned char* smem, int npad) {
    constexpr bool fp32 = (DT == C64 || DT == R32);
    c = (typename Tr<DT>::CS*)smem;
    c64 = fp32 ? (double2*)(smem + (((size_t)npad * 8 + 15) & ~(size_t)15)) : (double2*)smem;
    red0 = (double*)(c64 + npad);
    red1 = red0 + 16 * 8;
    kcl = red1 + 16 * 8;
  }
};

template <int DT, int BLOCK, int RPT>
struct Kern {
  using T = Tr<DT>;
  using S = typename T::S;
  using L = typename T::L;
  using CS = typename T::CS;
  static constexpr int VEC = T::VEC;
  static constexpr int NR = RPT * VEC;
  static constexpr int NW = BLOCK / 64;
  static constexpr bool FP32 = (DT == C64 || DT == R32);
  static constexpr bool CPLX = T::CPLX;
  static constexpr int NCOMP = CPLX ? 2 : 1;
  static constexpr int UNR = RPT >= 4 ? 1 : 4 / RPT;   // stored rows in flight per lane
  using F = typename std::conditional<FP32, float, double>::type;
  using F2 = typename std::conditional<FP32, float2, double2>::type;

  __device__ static int row(int r) { return (threadIdx.x + (r / VEC) * BLOCK) * VEC + (r % VEC); }

  // The VEC elements of one 16-byte load, as (re, im) pairs.
  __device__ static void split(const L& v, F (&re)[VEC], F (&im)[VEC]) {
    if constexpr (DT == C128) { re[0] = v.x; im[0] = v.y; }
    else if constexpr (DT == C64) { re[0] = v.x; im[0] = v.y; re[1] = v.z; im[1] = v.w; }
    else if constexpr (DT == R64) { re[0] = v.x; re[1] = v.y; im[0] = im[1] = 0.0; }
    else { re[0] = v.x; re[1] = v.y; im[0] = im[1] = 0.f; }
  }

  // One evaluation of the right-hand side at time ts for the stage amplitudes
  // cur (this lane's rows) and classical stage values R, P_Phi.  Overwrites
  // cur with da/dt of this lane's rows and returns the workgroup sums in tot.
  __device__ static void eval(const DevSystem& sy, double ts, double R, double pphi,
                              double2 (&cur)[NR], Sums& tot, bool& below, const Lds<DT>& lds) {
    const int N = sy.N, Npad = sy.Npad;
    const Spl sp = spline_at(sy.R, sy.K, R);
    below |= sp.below;
    const double phidot = uni(pphi / (sy.mu * R * R));

#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n < N) {
        double sn, cs;
        sincos(sy.E[n] * ts, &sn, &cs);
        const double2 c = make_double2(cs * cur[r].x + sn * cur[r].y,
                                       cs * cur[r].y - sn * cur[r].x);
        if constexpr (FP32) lds.c[n] = make_float2((float)c.x, (float)c.y);
        lds.c64[n] = c;
      }
    }
    __syncthreads();

    // fused spline-evaluate + complex matvec over the four slices
    const int64_t ks = sy.knot_stride;
    const uint32_t sbytes = (uint32_t)(ks * NCOMP * (int64_t)sizeof(S));
    const auto rs0 = slice_rsrc((const S*)sy.M + (int64_t)sp.k * ks * NCOMP, sbytes);
    const auto rs1 = slice_rsrc((const S*)sy.M + (int64_t)(sp.k + 1) * ks * NCOMP, sbytes);
    const auto rs2 = slice_rsrc((const S*)sy.M2 + (int64_t)sp.k * ks * NCOMP, sbytes);
    const auto rs3 = slice_rsrc((const S*)sy.M2 + (int64_t)(sp.k + 1) * ks * NCOMP, sbytes);
    const int ngroups = Npad / VEC;   // 16-byte groups per stored row
    const F w[4] = {(F)uni(sp.w0), (F)uni(sp.w1), (F)uni(sp.w2), (F)uni(sp.w3)};
    const F d[4] = {(F)uni(sp.d0), (F)uni(sp.d1), (F)uni(sp.d2), (F)uni(sp.d3)};

    double2 U[NR], V[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) { U[r] = make_double2(0.0, 0.0); V[r] = make_double2(0.0, 0.0); }

    for (int m0 = 0; m0 < N; m0 += (FP32 ? CHUNK : N)) {
      const int m1 = FP32 ? min(N, m0 + CHUNK) : N;
      F2 pu[NR], pv[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        pu[r].x = pu[r].y = pv[r].x = pv[r].y = (F)0;
      }
#pragma unroll UNR
      for (int m = m0; m < m1; ++m) {
        const CS cm = lds.c[m];
        const uint32_t rowoff = (uint32_t)m * (uint32_t)ngroups * (uint32_t)sizeof(L);
        // No lane guard: a lane whose column group lies past the last one reads
        // into the next stored row (or past the slice, which returns zero) and
        // its sums are never used, so the loads of consecutive m stay in flight
        // together.
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const uint32_t off = rowoff + (uint32_t)(threadIdx.x + j * BLOCK) * (uint32_t)sizeof(L);
          const L v0 = load16<L>(rs0, off);
          const L v1 = load16<L>(rs1, off);
          const L v2 = load16<L>(rs2, off);
          const L v3 = load16<L>(rs3, off);
          F r0[VEC], i0[VEC], r1[VEC], i1[VEC], r2[VEC], i2[VEC], r3[VEC], i3[VEC];
          split(v0, r0, i0); split(v1, r1, i1); split(v2, r2, i2); split(v3, r3, i3);
#pragma unroll
          for (int q = 0; q < VEC; ++q)
            elem<CPLX, F, F2>(pu[j * VEC + q], pv[j * VEC + q], r0[q], i0[q], r1[q], i1[q],
                              r2[q], i2[q], r3[q], i3[q], w, d, cm);
        }
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        U[r].x += (double)pu[r].x; U[r].y += (double)pu[r].y;
        V[r].x += (double)pv[r].x; V[r].y += (double)pv[r].y;
      }
    }

    // epilogue.  J_x couples only channels of equal energy, so
    // J_x a = e^{iE_n t} (J_x c) row by row, and with y = e^{iE t} u:
    //   Re(c^H v), Im(x^H y) = Im((J_x c)^H u), Re(c^H u), Re(a^H J_x a) = Re(c^H J_x c).
    double sums[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n >= N) { cur[r] = make_double2(0.0, 0.0); continue; }
      double sn, cs;
      sincos(sy.E[n] * ts, &sn, &cs);
      const double2 c = make_double2(cs * cur[r].x + sn * cur[r].y,
                                     cs * cur[r].y - sn * cur[r].x);
      double2 xc = make_double2(0.0, 0.0);
      for (int q = 0; q < sy.jx_w; ++q) {
        const int col = sy.jx_col[(int64_t)n * sy.jx_w + q];
        const double jv = sy.jx_val[(int64_t)n * sy.jx_w + q];
        const double2 cm = lds.c64[col];
        xc.x = fma(jv, cm.x, xc.x);
        xc.y = fma(jv, cm.y, xc.y);
      }
      const double2 u = U[r], v = V[r];
      sums[0] += c.x * v.x + c.y * v.y;
      sums[1] += xc.x * u.y - xc.y * u.x;
      sums[2] += c.x * u.x + c.y * u.y;
      const double pn = cur[r].x * cur[r].x + cur[r].y * cur[r].y;
      sums[3] += sy.E[n] * pn;
      sums[4] += pn;
      sums[5] += c.x * xc.x + c.y * xc.y;
      // da/dt = -i e^{iE_n t} (u + Phidot J_x c)
      const double gx = u.x + phidot * xc.x, gy = u.y + phidot * xc.y;
      const double yx = cs * gx - sn * gy, yy = cs * gy + sn * gx;
      cur[r] = make_double2(yy, -yx);
    }
    block_sum<6, NW>(sums, lds.red0);
    tot.force = sums[0]; tot.torque = sums[1]; tot.vexp = sums[2];
    tot.erot = sums[3]; tot.norm = sums[4]; tot.jx = sums[5];
  }

  // classical derivatives of (R, Phi, P_R, P_Phi), Eqs. 7-10
  __device__ static void classical_rhs(double mu, const double (&ys)[4], const Sums& tot,
                                       double (&ky)[4]) {
    const double R = ys[0];
    ky[0] = ys[2] / mu;
    ky[1] = ys[3] / (mu * R * R);
    ky[2] = -tot.force + ys[3] * ys[3] / (mu * R * R * R);
    ky[3] = 2.0 * tot.torque;
  }

  __device__ static double energy(double mu, const double (&ys)[4], const Sums& s) {
    return ys[2] * ys[2] / (2.0 * mu) + ys[3] * ys[3] / (2.0 * mu * ys[0] * ys[0]) + s.erot +
           s.vexp;
  }

  // initial amplitudes and classical state of a trajectory
  __device__ static void init_state(const DevSystem& sy, const TrajIn& tj,
                                    const double* __restrict__ a0_all, double2 (&a)[NR],
                                    double (&y)[4], double& theta, double& ptheta) {
    const int N = sy.N;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      double2 v = make_double2(0.0, 0.0);
      if (n < N) {
        if (tj.flags & TRAJ_HAS_A0) v = ((const double2*)a0_all)[tj.amp_off + n];
        else if (n == tj.init_channel) v = make_double2(1.0, 0.0);
      }
      a[r] = v;
    }
    theta = 0.5 * M_PI;
    ptheta = 0.0;
    if (tj.flags & TRAJ_HAS_C0) {
      y[0] = tj.c0[0]; theta = tj.c0[1]; y[1] = tj.c0[2]; y[2] = tj.c0[3]; ptheta = tj.c0[4];
      y[3] = tj.c0[5];
    } else {
      // end of Section II / Section III: P_Phi = b k, P_R = -sqrt(k^2 - P_Phi^2/R0^2)
      const double k = sqrt(2.0 * sy.mu * tj.E_coll);
      const double pphi = tj.b * k;
      y[0] = tj.R0; y[1] = 0.0;
      y[2] = -sqrt(2.0 * sy.mu * tj.E_coll - pphi * pphi / (tj.R0 * tj.R0));
      y[3] = pphi;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = uni(y[i]);
  }

  __device__ static void write_out(const DevSystem& sy, const TrajIn& tj, TrajOut& out,
                                   const double2 (&a)[NR], const double (&y)[4], double theta,
                                   double ptheta, double tend, int64_t steps, int64_t rejects,
                                   int32_t status, const Sums& tot, double E0, double J0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n < sy.N) {
        out.P[tj.amp_off + n] = a[r].x * a[r].x + a[r].y * a[r].y;
        if (out.a_final) ((double2*)out.a_final)[tj.amp_off + n] = a[r];
      }
    }
    if (threadIdx.x == 0) {
      const int64_t id = tj.id;
      if (out.classical) {
        double* o = out.classical + id * 6;
        o[0] = y[0]; o[1] = theta; o[2] = y[1]; o[3] = y[2]; o[4] = ptheta; o[5] = y[3];
      }
      if (out.t_final) out.t_final[id] = tend;
      if (out.steps) out.steps[id] = steps;
      if (out.rejects) out.rejects[id] = rejects;
      if (out.status) out.status[id] = status;
      if (out.norm_err) out.norm_err[id] = tot.norm - 1.0;
      if (out.energy_err) out.energy_err[id] = (energy(sy.mu, y, tot) - E0) / fabs(E0);
      if (out.angmom_err) out.angmom_err[id] = (y[3] - tot.jx) - J0;
    }
  }

  // Fixed-step classical RK4: exactly n_steps steps, t_j = t0 + j h.
  __device__ static void run_rk4(const DevSystem& sy, const TrajIn& tj,
                                 const double* __restrict__ a0_all, TrajOut& out,
                                 const Lds<DT>& lds) {
    const double mu = sy.mu;
    double2 a0[NR], kk[NR], acc[NR];   // kk: stage input, then its derivative
    double y[4], ky[4] = {0.0, 0.0, 0.0, 0.0}, ay[4], theta, ptheta;
    init_state(sy, tj, a0_all, a0, y, theta, ptheta);
#pragma unroll
    for (int r = 0; r < NR; ++r) kk[r] = make_double2(0.0, 0.0);
    const double h = tj.dt, t0 = tj.t0;
    bool below = false;
    int32_t status = 0;
    double E0 = 0.0, J0 = 0.0;
    bool first = true;
    Sums tot;
    int64_t j = 0;
    for (; j < tj.n_steps; ++j) {
      const double t = t0 + (double)j * h;
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
        eval(sy, t + cf, ys[0], ys[3], kk, tot, below, lds);
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
    const double tend = t0 + (double)j * h;
    bool b2 = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = a0[r];
    eval(sy, tend, y[0], y[3], acc, tot, b2, lds);
    if (first) {
      E0 = energy(mu, y, tot);
      J0 = y[3] - tot.jx;
    }
    if (below) status |= ST_BELOW_GRID;
    write_out(sy, tj, out, a0, y, theta, ptheta, tend, j, 0, status, tot, E0, J0);
  }

  // Adaptive Dormand-Prince 5(4) (Dormand & Prince 1980 tableau) with
  // first-same-as-last, the scaled RMS error over the 2N+6 real state
  // components (sc_i = atol + rtol max(|y_i|, |y_new,i|); Theta and P_Theta
  // are constant and contribute zero error), the step factor
  // min(5, max(0.2, 0.9 err^-1/5)) with no growth right after a rejection, and
  // the Hairer-Norsett-Wanner starting step.  Stops after the first accepted
  // step with R >= R0 and P_R > 0, or on max_steps / h < h_min / non-finite.
  // Amplitude stage derivatives live in this workgroup's slice ks[7][Npad] of
  // global scratch (each lane touches only its own rows); the classical ones
  // live in LDS (every lane writes the same values, then reads its own).
  __device__ static void run_dp5(const DevSystem& sy, const TrajIn& tj,
                                 const double* __restrict__ a0_all, TrajOut& out,
                                 const Lds<DT>& lds, double2* __restrict__ ks, int npad_max,
                                 const DpCtl& ctl) {
    const int N = sy.N;
    const double mu = sy.mu;
    const double rtol = ctl.rtol, atol = ctl.atol;
    const double ncomp = 2.0 * N + 6.0;
    double2 y[NR], st[NR];     // solution; stage input, then its derivative
    double yc[4], theta, ptheta;
    init_state(sy, tj, a0_all, y, yc, theta, ptheta);
    const double R_exit = yc[0];
    double* kcl = lds.kcl;     // [8][4]: classical stage derivatives, then slot 7 = y5
    // ks[q][n], q = 0..6 stage derivatives, q = 7 the fifth-order solution
    auto kidx = [&](int q, int r) { return (int64_t)q * npad_max + row(r); };
    bool below = false;
    int32_t status = 0;
    Sums tot;
    double t = tj.t0;
    // first evaluation k1 = f(t0, y0)
#pragma unroll
    for (int r = 0; r < NR; ++r) st[r] = y[r];
    eval(sy, t, yc[0], yc[3], st, tot, below, lds);
    const double E0 = energy(mu, yc, tot), J0 = yc[3] - tot.jx;
    {
      double kc[4];
      classical_rhs(mu, yc, tot, kc);
#pragma unroll
      for (int i = 0; i < 4; ++i) kcl[i] = kc[i];
#pragma unroll
      for (int r = 0; r < NR; ++r) if (row(r) < N) ks[kidx(0, r)] = st[r];
    }
    const double yfull[6] = {yc[0], theta, yc[1], yc[2], ptheta, yc[3]};
    // starting step (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4)
    double h;
    {
      double s2[2] = {0.0, 0.0};
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (row(r) >= N) continue;
        const double sx = atol + rtol * fabs(y[r].x), sy_ = atol + rtol * fabs(y[r].y);
        s2[0] += (y[r].x / sx) * (y[r].x / sx) + (y[r].y / sy_) * (y[r].y / sy_);
        s2[1] += (st[r].x / sx) * (st[r].x / sx) + (st[r].y / sy_) * (st[r].y / sy_);
      }
      block_sum<2, NW>(s2, lds.red1);
      const double kf[6] = {kcl[0], 0.0, kcl[1], kcl[2], 0.0, kcl[3]};
      for (int i = 0; i < 6; ++i) {
        const double sc = atol + rtol * fabs(yfull[i]);
        s2[0] += (yfull[i] / sc) * (yfull[i] / sc);
        s2[1] += (kf[i] / sc) * (kf[i] / sc);
      }
      const double d0 = sqrt(s2[0] / ncomp), d1 = sqrt(s2[1] / ncomp);
      const double h0 = uni((d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1);
#pragma unroll
      for (int r = 0; r < NR; ++r)
        st[r] = make_double2(fma(h0, st[r].x, y[r].x), fma(h0, st[r].y, y[r].y));
      double ys[4];
      for (int i = 0; i < 4; ++i) ys[i] = uni(fma(h0, kcl[i], yc[i]));
      eval(sy, t + h0, ys[0], ys[3], st, tot, below, lds);
      double kc1[4];
      classical_rhs(mu, ys, tot, kc1);
      double s1[1] = {0.0};
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (row(r) >= N) continue;
        const double2 f0 = ks[kidx(0, r)];
        const double sx = atol + rtol * fabs(y[r].x), sy_ = atol + rtol * fabs(y[r].y);
        const double ex = (st[r].x - f0.x) / sx, ey = (st[r].y - f0.y) / sy_;
        s1[0] += ex * ex + ey * ey;
      }
      block_sum<1, NW>(s1, lds.red1);
      const double dk[6] = {kc1[0] - kcl[0], 0.0, kc1[1] - kcl[1], kc1[2] - kcl[2], 0.0,
                            kc1[3] - kcl[3]};
      for (int i = 0; i < 6; ++i) {
        const double sc = atol + rtol * fabs(yfull[i]);
        s1[0] += (dk[i] / sc) * (dk[i] / sc);
      }
      const double d2 = sqrt(s1[0] / ncomp) / h0;
      const double dm = fmax(d1, d2);
      const double h1 = dm <= 1e-15 ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 1.0 / 5.0);
      h = uni(fmin(100.0 * h0, h1));
    }
    int64_t steps = 0, rejects = 0;
    bool last_rejected = false;
    for (;;) {
      if (steps >= ctl.max_steps) { status |= ST_MAX_STEPS; break; }
      for (int s = 1; s < 7; ++s) {
        // stage input y + h sum_q a_sq k_q
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          double2 acc = y[r];
          if (row(r) < N) {
            for (int q = 0; q < s; ++q) {
              const double2 kq = ks[kidx(q, r)];
              const double c = h * DP_A[s][q];
              acc.x = fma(c, kq.x, acc.x);
              acc.y = fma(c, kq.y, acc.y);
            }
            if (s == 6) ks[kidx(7, r)] = acc;
          }
          st[r] = acc;
        }
        double ys[4];
        for (int i = 0; i < 4; ++i) {
          double acc = yc[i];
          for (int q = 0; q < s; ++q) acc = fma(h * DP_A[s][q], kcl[q * 4 + i], acc);
          ys[i] = uni(acc);
          if (s == 6) kcl[28 + i] = ys[i];
        }
        eval(sy, t + DP_C[s] * h, ys[0], ys[3], st, tot, below, lds);
        double kc[4];
        classical_rhs(mu, ys, tot, kc);
        for (int i = 0; i < 4; ++i) kcl[s * 4 + i] = kc[i];
#pragma unroll
        for (int r = 0; r < NR; ++r) if (row(r) < N) ks[kidx(s, r)] = st[r];
      }
      // scaled RMS error of h sum_q e_q k_q
      double e2[1] = {0.0};
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (row(r) >= N) continue;
        double ex = 0.0, ey = 0.0;
        for (int q = 0; q < 7; ++q) {
          const double2 kq = ks[kidx(q, r)];
          ex = fma(DP_E[q], kq.x, ex);
          ey = fma(DP_E[q], kq.y, ey);
        }
        ex *= h; ey *= h;
        const double2 y5 = ks[kidx(7, r)];
        const double sx = atol + rtol * fmax(fabs(y[r].x), fabs(y5.x));
        const double sy_ = atol + rtol * fmax(fabs(y[r].y), fabs(y5.y));
        e2[0] += (ex / sx) * (ex / sx) + (ey / sy_) * (ey / sy_);
      }
      // The classical part reads kcl[0..3] (k1), which the accept branch below
      // overwrites with k7: it must be read before the reduction's barrier, or
      // a wave that is already past the barrier can replace k1 under a slower
      // wave and the waves would disagree on accept/reject.
      double ecl = 0.0;
      for (int i = 0; i < 4; ++i) {
        double e = 0.0;
        for (int q = 0; q < 7; ++q) e = fma(DP_E[q], kcl[q * 4 + i], e);
        e *= h;
        const double sc = atol + rtol * fmax(fabs(yc[i]), fabs(kcl[28 + i]));
        ecl += (e / sc) * (e / sc);
      }
      block_sum<1, NW>(e2, lds.red1);
      const double en = uni(sqrt((e2[0] + ecl) / ncomp));
      if (!isfinite(en)) { status |= ST_NONFINITE; break; }
      if (en <= 1.0) {
        t += h;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (row(r) < N) {
            y[r] = ks[kidx(7, r)];
            ks[kidx(0, r)] = ks[kidx(6, r)];
          }
        }
        for (int i = 0; i < 4; ++i) { yc[i] = uni(kcl[28 + i]); kcl[i] = kcl[24 + i]; }
        ++steps;
        double fac = en == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(en, -0.2)));
        if (last_rejected) fac = fmin(1.0, fac);
        last_rejected = false;
        if (yc[0] >= R_exit && yc[2] > 0.0) { status |= ST_EXITED; break; }
        h = uni(h * fac);
      } else {
        ++rejects;
        h = uni(h * fmax(0.2, 0.9 * pow(en, -0.2)));
        last_rejected = true;
      }
      if (h < ctl.h_min) { status |= ST_STEP_UNDERFLOW; break; }
    }
    bool b2 = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) st[r] = y[r];
    eval(sy, t, yc[0], yc[3], st, tot, b2, lds);
    if (below) status |= ST_BELOW_GRID;
    write_out(sy, tj, out, y, yc, theta, ptheta, t, steps, rejects, status, tot, E0, J0);
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

// Persistent workgroups draining a trajectory queue.  Each workgroup takes the
// next index from a global counter (so long trajectories never hold up the
// rest of the batch) and runs it to completion with the storage type of its
// system (any of the types in TYPES, chosen at run time); it exits once the
// queue is empty, so every wave reaches the end.
template <int T0, int T1, int BLOCK, int RPT>
__global__ void __launch_bounds__(BLOCK)
persistent_kernel(const DevSystem* __restrict__ systems, const TrajIn* __restrict__ trajs,
                  int64_t n_traj, const double* __restrict__ a0_all, TrajOut out,
                  unsigned long long* __restrict__ counter, double2* __restrict__ kscratch,
                  int npad_max, int method, DpCtl ctl) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ long long next;
  double2* ks = kscratch + (int64_t)blockIdx.x * 8 * npad_max;
  for (;;) {
    if (threadIdx.x == 0) next = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const long long idx = next;
    __syncthreads();
    if (idx >= n_traj) break;
    const TrajIn tj = trajs[idx];
    const DevSystem sy = systems[tj.sys];
    if (sy.dtype == T0) {
      Lds<T0> lds(smem, npad_max);
      if (method == 0) Kern<T0, BLOCK, RPT>::run_rk4(sy, tj, a0_all, out, lds);
      else Kern<T0, BLOCK, RPT>::run_dp5(sy, tj, a0_all, out, lds, ks, npad_max, ctl);
    } else if (T1 != T0 && sy.dtype == T1) {
      Lds<T1> lds(smem, npad_max);
      if (method == 0) Kern<T1, BLOCK, RPT>::run_rk4(sy, tj, a0_all, out, lds);
      else Kern<T1, BLOCK, RPT>::run_dp5(sy, tj, a0_all, out, lds, ks, npad_max, ctl);
    }
  }
}

__global__ void zero_counter(unsigned long long* c) { *c = 0ull; }

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

template <int T0, int T1, int RPT>
hipError_t launch_persistent_t(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                               const double* d_a0, TrajOut out, int max_npad, int method,
                               DpCtl ctl, unsigned long long* counter, double2* kscratch,
                               int64_t slots, hipStream_t s) {
  constexpr int BLOCK = 512;
  const bool fp32 = T0 == C64 || T0 == R32 || T1 == C64 || T1 == R32;
  size_t lds = lds_bytes(max_npad, fp32) + 16;
  auto kern = persistent_kernel<T0, T1, BLOCK, RPT>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  zero_counter<<<1, 1, 0, s>>>(counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t grid = slots < n_traj ? slots : n_traj;
  kern<<<(unsigned)grid, BLOCK, lds, s>>>(d_systems, d_traj, n_traj, d_a0, out, counter,
                                          kscratch, max_npad, method, ctl);
  return hipGetLastError();
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

int64_t persistent_slots(bool fp32_family, int max_groups, int max_npad) {
  int dev = 0, cus = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const bool two = max_groups > 512;
  const size_t lds = lds_bytes(max_npad, fp32_family) + 16;
  const void* k;
  if (fp32_family) k = two ? (const void*)persistent_kernel<C64, R32, 512, 2>
                           : (const void*)persistent_kernel<C64, R32, 512, 1>;
  else k = two ? (const void*)persistent_kernel<C128, R64, 512, 2>
               : (const void*)persistent_kernel<C128, R64, 512, 1>;
  if (lds > 65536 &&
      hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 512, lds) != hipSuccess) return 0;
  return (int64_t)cus * (nb > 0 ? nb : 1);
}

hipError_t launch_persistent(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                             const double* d_a0, TrajOut out, bool fp32_family, int max_npad,
                             int max_groups, int method, DpCtl ctl, unsigned long long* counter,
                             double2* kscratch, int64_t slots, hipStream_t s) {
  if (max_groups > 1024) return hipErrorInvalidValue;
  const bool two = max_groups > 512;
  if (fp32_family) {
    if (two) return launch_persistent_t<C64, R32, 2>(d_systems, d_traj, n_traj, d_a0, out, max_npad, method, ctl, counter, kscratch, slots, s);
    return launch_persistent_t<C64, R32, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, method, ctl, counter, kscratch, slots, s);
  }
  if (two) return launch_persistent_t<C128, R64, 2>(d_systems, d_traj, n_traj, d_a0, out, max_npad, method, ctl, counter, kscratch, slots, s);
  return launch_persistent_t<C128, R64, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, method, ctl, counter, kscratch, slots, s);
}

}  // namespace mqct
